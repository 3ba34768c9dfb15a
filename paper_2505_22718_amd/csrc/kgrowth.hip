// Scale-dependent growth D(k, z) (paper Sec. 3.2).  The power spectrum factorises as
// P(k, z_fid) D(k, z(chi)) D(k, z(chi')), so the FFTLog coefficients of f(chi) D(k, chi) depend on k.
// They are computed at N_interp nodes kappa_a, uniform in ln k from k_min to k_max, and continued to
// every k node by the natural cubic spline in ln k through the node values:
//   c_n(k_j) = (1 - t) c_n^a + t c_n^{a+1} + h^2/6 [((1-t)^3 - (1-t)) M_n^a + (t^3 - t) M_n^{a+1}],
// M the spline's second derivatives, a and t the node interval and offset of k_j.  The window
//   W_l(k_j) = c(l) k_j^{-1-b} [k_j^-2 for lensing] Re sum_{n<N/2} h_n U_l(n) c_n(k_j) e^{-2 pi i n j / N}
// (h_0 = 1, else 2) is then no longer a transform over j.  Per (point, tracer, band) it is the real
// GEMM [multipoles x N] . [N x N_k] of the interleaved (Re, Im) parts of U and of
// X_{n,j} = c_n(k_j) e^{-2 pi i n j / N}; it runs on the 16x16x4 f32 MFMA with X generated in LDS
// from the node coefficients, and writes sqrt(s) W to the workspace for the projection kernel.
//
// Stages per chunk of points:
//   k_kg_slots    multipole slots of every point grouped by band, cut into tiles of <= 64
//   k_kg_fft      per (point, node): D(kappa_a, z) splined in z and sampled on the chi nodes, every
//                 (tracer, band) row of kernel samples (assembled with D = 1) times it, r2c
//   k_kg_cspline  per (point, tracer, band, n): the node spline along ln k (Thomas, FP32)
//   k_kg_windows  the GEMM above, one workgroup per (point, tracer, slot tile, 64 k nodes)
//   k_contract    C = V V^T per (point, multipole) from the workspace (forward.hip)
#include "common.h"
#include "geometry.h"
#include "internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int clamp_i(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

constexpr int KG_TILE = 64;   // slots and k nodes per GEMM workgroup
constexpr int KG_KC = 16;     // coefficients n per K chunk (32 real K rows)
constexpr int KG_AS = 2 * KG_KC + 1;  // padded row of the U tile
constexpr int KG_BS = KG_TILE + 4;    // padded row of the X tile

// One thread per point: slot permutation (stable, grouped by band) and the tile list.
__global__ void k_kg_slots(plan_dev P, swiftcl_inputs in, int b0, int nbp) {
  const int bl = blockIdx.x * blockDim.x + threadIdx.x;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  const int Lm = P.max_ell, nb = P.n_bands;
  const int Lb = clamp_i(in.n_ell[b], 0, Lm);
  int cnt[SWIFTCL_MAX_BANDS] = {0, 0, 0, 0};
  bool bad = false;
  for (int li = 0; li < Lb; ++li) {
    int ei = in.ell_idx[(size_t)b * Lm + li];
    if (ei < 0 || ei >= P.n_ell) { bad = true; ei = 0; }
    ++cnt[P.ell_band[ei]];
  }
  if (bad) atomicOr(P.flags, FLAG_BAD_INDEX);
  int off[SWIFTCL_MAX_BANDS];
  int acc = 0;
  for (int bi = 0; bi < nb; ++bi) { off[bi] = acc; acc += cnt[bi]; }
  int* perm = P.kg_perm + (size_t)bl * Lm;
  int pos[SWIFTCL_MAX_BANDS];
  for (int bi = 0; bi < nb; ++bi) pos[bi] = off[bi];
  for (int li = 0; li < Lb; ++li) {
    int ei = in.ell_idx[(size_t)b * Lm + li];
    if (ei < 0 || ei >= P.n_ell) ei = 0;
    perm[pos[P.ell_band[ei]]++] = li;
  }
  int4* tile = (int4*)P.kg_tile + (size_t)bl * P.kg_ntile;
  int nt = 0;
  for (int bi = 0; bi < nb; ++bi)
    for (int s = 0; s < cnt[bi]; s += KG_TILE)
      tile[nt++] = make_int4(bi, off[bi] + s, cnt[bi] - s < KG_TILE ? cnt[bi] - s : KG_TILE, 0);
  for (; nt < P.kg_ntile; ++nt) tile[nt] = make_int4(0, 0, 0, 0);
}

// One workgroup (4 wavefronts) per (point, node).  Dynamic LDS: twiddles [2M], FFT scratch
// [4][fft_lds_size], growth on the chi nodes [2M] float, D(kappa_a, z) samples and their spline
// moments [2][n_zg] double.
template <int M>
__global__ __launch_bounds__(256) void k_kg_fft(plan_dev P, swiftcl_inputs in, const double* __restrict__ Dkz,
                                                int b0, int nbp) {
  extern __shared__ __align__(16) unsigned char smem[];
  typedef float R;
  constexpr int N = 2 * M;
  constexpr int RL = M / SWIFTCL_WAVE;
  constexpr int FL = fft_lds_size(M, sizeof(R));
  C2<R>* stw = (C2<R>*)smem;
  C2<R>* fbuf = stw + N;
  float* Dk = (float*)(fbuf + 4 * FL);
  double* y = (double*)(Dk + N);
  const int nzg = P.n_zg;
  double* Mo = y + nzg;
  const int A = P.n_interp;
  const int bl = blockIdx.x / A, a = blockIdx.x % A;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  const int T = P.max_tracers, nb = P.n_bands;
  const int Tb = clamp_i(in.n_tracers[b], 0, T);
  const int wave = threadIdx.x / SWIFTCL_WAVE, lane = threadIdx.x % SWIFTCL_WAVE;
  for (int i = threadIdx.x; i < N; i += blockDim.x) stw[i] = ((const C2<R>*)P.tw)[i];
  const double* src = Dkz + ((size_t)b * A + a) * nzg;
  bool bad = false;
  for (int i = threadIdx.x; i < nzg; i += blockDim.x) {
    const double v = src[i];
    bad |= !isfinite(v);
    y[i] = v;
  }
  if (bad) atomicOr(P.flags, FLAG_NONFINITE);
  __syncthreads();
  if (wave == 0) wave_spline(y, P.lu_geom, nzg, Mo, lane);
  __syncthreads();
  // growth of node a at every active chi node (zero outside the support, where g is zero)
  const double* pt = P.pt + (size_t)b * PT_STRIDE;
  const int m0 = P.m0, m1 = (int)pt[PT_M1];
  const double* zg = P.z_geom;
  const double* zgih = P.lu_geom + 3 * (size_t)nzg;
  for (int m = threadIdx.x; m < N; m += blockDim.x) {
    float v = 0.f;
    if (m >= m0 && m <= m1) {
      const double z = P.node_f[(size_t)b * 4 * N + m];
      const int ig = P.node_i[(size_t)b * 3 * N + m];
      v = (float)spline_w(zg, zgih, ig, z).at(y, Mo, ig);
    }
    Dk[m] = v;
  }
  __syncthreads();
  const C2<R>* dk2 = (const C2<R>*)Dk;
  C2<R>* mine = fbuf + (size_t)wave * FL;
  const double2* ph = (const double2*)P.phase + (size_t)b * M;
  for (int r = wave; r < Tb * nb; r += 4) {
    const int t = r / nb, bi = r % nb;
    const C2<R>* g2 = (const C2<R>*)((const R*)P.g + (((size_t)b * T + t) * nb + bi) * N);
    C2<R> v[RL];
#pragma unroll
    for (int e = 0; e < RL; ++e) {
      const int q = lane + SWIFTCL_WAVE * e;
      const C2<R> gv = g2[q], dv = dk2[q];
      v[e] = mk<R>(gv.x * dv.x, gv.y * dv.y);
    }
    int ln = lane;  // opaque copy: keeps the FFT's per-lane LDS addresses out of the row loop
    asm volatile("" : "+v"(ln));
    ln &= SWIFTCL_WAVE - 1;
    wave_sync();
    wave_r2c<R, M>(v, mine, stw, ln);
    const int kind = in.kind[(size_t)b * T + t] & 1;
    const double scale = pt[PT_CHI0B + kind * SWIFTCL_MAX_BANDS + bi] / (double)N;
    C2<R>* out = (C2<R>*)P.kg_c + ((((size_t)bl * T + t) * nb + bi) * A + a) * M;
#pragma unroll
    for (int e = 0; e < RL; ++e) {
      const int n = lane + SWIFTCL_WAVE * e;
      const double2 pv = ph[n];
      out[n] = cmul(v[e], mk<R>((R)(pv.x * scale), (R)(pv.y * scale)));
    }
  }
}

// Natural cubic spline of the node coefficients along ln k: one thread per (row, n), the
// tridiagonal system M_{a-1} + 4 M_a + M_{a+1} = 6/h^2 (c_{a+1} - 2 c_a + c_{a-1}), M_0 = M_{A-1} = 0,
// by the Thomas recurrences (1/pivots in kg_ip).
__global__ __launch_bounds__(256) void k_kg_cspline(plan_dev P, swiftcl_inputs in, int b0, int nbp, float s6) {
  const int M = P.M, A = P.n_interp, T = P.max_tracers, nb = P.n_bands;
  const int n = blockIdx.y * blockDim.x + threadIdx.x;
  const long row = blockIdx.x;
  if (n >= M) return;
  const int bl = (int)(row / ((long)T * nb));
  const int t = (int)((row / nb) % T);
  if (bl >= nbp || t >= clamp_i(in.n_tracers[b0 + bl], 0, T)) return;
  const float2* c = (const float2*)P.kg_c + (size_t)row * A * M + n;
  float2* m = (float2*)P.kg_m + (size_t)row * A * M + n;
  m[0] = make_float2(0.f, 0.f);
  m[(size_t)(A - 1) * M] = make_float2(0.f, 0.f);
  float2 cm = c[0], c0 = c[(size_t)M];
  float2 d = make_float2(0.f, 0.f);
  for (int a = 1; a + 1 < A; ++a) {
    const float2 cp = c[(size_t)(a + 1) * M];
    const float ip = P.kg_ip[a];
    d.x = (s6 * (cp.x - 2.f * c0.x + cm.x) - d.x) * ip;
    d.y = (s6 * (cp.y - 2.f * c0.y + cm.y) - d.y) * ip;
    m[(size_t)a * M] = d;
    cm = c0;
    c0 = cp;
  }
  float2 mn = make_float2(0.f, 0.f);
  for (int a = A - 2; a >= 1; --a) {
    const float2 da = m[(size_t)a * M];
    const float ip = P.kg_ip[a];
    mn = make_float2(da.x - ip * mn.x, da.y - ip * mn.y);
    m[(size_t)a * M] = mn;
  }
}

__device__ __forceinline__ unsigned short bf16_rne_kg(float x) {
  const unsigned int u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// W tile [<= 64 slots of one band] x [64 k nodes] of one (point, tracer) by 4 wavefronts: wave w
// owns k nodes 16w..16w+15 and every 16-row tile of slots.  Per K chunk the block writes U (A
// operand, [slot][2n + {0,1}] = h_n (Re U, -Im U)) and X (B operand, [2n + {0,1}][k] = (Re X, Im X))
// to LDS, then each wave runs 8 k-steps of 16x16x4 f32 MFMAs.  Blocks of one (point, tracer) share
// an XCD, so its node coefficients are read into one L2.
template <bool SPLIT>
__global__ __launch_bounds__(256) void k_kg_windows(plan_dev P, swiftcl_inputs in, int b0, int nbp) {
  __shared__ float As[KG_TILE][KG_AS];
  __shared__ float Bs[2 * KG_KC][KG_BS];
  __shared__ float2 stw[1024];
  __shared__ float4 wts[KG_TILE];
  __shared__ int ias[KG_TILE];
  __shared__ int eis[KG_TILE];
  __shared__ int lis[KG_TILE];
  const int T = P.max_tracers, Lm = P.max_ell, nk = P.n_k, nb = P.n_bands, M = P.M, A = P.n_interp;
  const int NJ = (nk + KG_TILE - 1) / KG_TILE, NT = P.kg_ntile;
  const int xcd = blockIdx.x % SWIFTCL_NXCD;
  const int rest = blockIdx.x / SWIFTCL_NXCD;
  const int item = rest % (NT * NJ);
  const int pair = (rest / (NT * NJ)) * SWIFTCL_NXCD + xcd;
  const int bl = pair / T, t = pair % T;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  if (t >= clamp_i(in.n_tracers[b], 0, T)) return;
  const int tile = item / NJ, jt = item % NJ;
  const int4 td = ((const int4*)P.kg_tile)[(size_t)bl * NT + tile];
  const int band = td.x, s0 = td.y, cnt = td.z;
  if (cnt <= 0) return;
  const int kind = in.kind[(size_t)b * T + t] & 1;
  const int tid = threadIdx.x, wave = tid / SWIFTCL_WAVE, lane = tid % SWIFTCL_WAVE;
  const int j0 = jt * KG_TILE;
  for (int i = tid; i < M; i += 256) stw[i] = ((const float2*)P.tw)[i];
  if (tid < KG_TILE) {
    const int r = tid;
    int li = -1, ei = 0;
    if (r < cnt) {
      li = P.kg_perm[(size_t)bl * Lm + s0 + r];
      ei = in.ell_idx[(size_t)b * Lm + li];
      if (ei < 0 || ei >= P.n_ell) ei = 0;  // flagged by k_kg_slots
    }
    lis[r] = li;
    eis[r] = ei;
    const int j = j0 + r;
    ias[r] = j < nk ? P.kg_ia[j] : 0;
    wts[r] = j < nk ? ((const float4*)P.kg_w)[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  const float2* U = (const float2*)P.U + (size_t)kind * P.n_ell * M;
  const size_t cbase = (((size_t)bl * T + t) * nb + band) * A;
  const float2* kc = (const float2*)P.kg_c + cbase * M;
  const float2* km = (const float2*)P.kg_m + cbase * M;
  const int nrt = (cnt + 15) / 16;
  const int Nmask = 2 * M - 1;
  v4f acc[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) acc[rt] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int n0 = 0; n0 < M; n0 += KG_KC) {
    // A operand: 64 slots x 16 coefficients; lanes run along n (coalesced rows of U)
    {
      const int nl = tid & (KG_KC - 1);
      const int n = n0 + nl;
      const float h = n == 0 ? 1.f : 2.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = (tid >> 4) + 16 * q;
        float2 u = make_float2(0.f, 0.f);
        if (r < cnt) u = U[(size_t)eis[r] * M + n];
        As[r][2 * nl] = h * u.x;
        As[r][2 * nl + 1] = -h * u.y;
      }
    }
    // B operand: 16 coefficients x 64 k nodes; lanes run along k
    {
      const int jj = tid & (KG_TILE - 1);
      const int j = j0 + jj;
      const int a = ias[jj];
      const float4 w = wts[jj];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int nl = (tid >> 6) + 4 * q;
        const int n = n0 + nl;
        float2 x = make_float2(0.f, 0.f);
        if (j < nk) {
          const float2 ca = kc[(size_t)a * M + n], cb = kc[(size_t)(a + 1) * M + n];
          const float2 ma = km[(size_t)a * M + n], mb = km[(size_t)(a + 1) * M + n];
          float2 c;
          c.x = w.x * ca.x + w.y * cb.x + w.z * ma.x + w.w * mb.x;
          c.y = w.x * ca.y + w.y * cb.y + w.z * ma.y + w.w * mb.y;
          const int qq = (n * j) & Nmask;
          float2 e = stw[qq & (M - 1)];
          if (qq >= M) { e.x = -e.x; e.y = -e.y; }
          x = cmul(c, e);
        }
        Bs[2 * nl][jj] = x.x;
        Bs[2 * nl + 1][jj] = x.y;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 2 * KG_KC / 4; ++ks) {
      const float bv = Bs[4 * ks + (lane >> 4)][16 * wave + (lane & 15)];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
        if (rt < nrt) {
          const float av = As[16 * rt + (lane & 15)][4 * ks + (lane >> 4)];
          acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[rt], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // V = F(l) kscale sqrt(s) W into the workspace rows (point, slot, tracer)
  const int j = j0 + 16 * wave + (lane & 15);
  if (j >= nk) return;
  const float kq = ((const float*)P.kss)[(((size_t)b * 2 + kind) * nb + band) * nk + j];
  const size_t lo_off = (size_t)P.vchunk * Lm * 32 * nk;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    if (rt >= nrt) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * rt + 4 * (lane >> 4) + q;
      if (r >= cnt) continue;
      const int li = lis[r];
      const float F = kind ? (float)P.fell[eis[r]] : 1.f;
      const float x = F * kq * acc[rt][q];
      const size_t o = (((size_t)bl * Lm + li) * 32 + t) * nk + j;
      if (SPLIT) {
        const unsigned short hi = bf16_rne_kg(x);
        const unsigned short lo = bf16_rne_kg(x - __uint_as_float((unsigned int)hi << 16));
        ((unsigned short*)P.vbuf)[o] = hi;
        ((unsigned short*)P.vbuf)[lo_off + o] = lo;
      } else {
        ((float*)P.vbuf)[o] = x;
      }
    }
  }
}

template <int M>
size_t kg_fft_lds(int n_zg) {
  return sizeof(float2) * (size_t)(2 * M + 4 * fft_lds_size(M, sizeof(float))) + sizeof(float) * 2 * M +
         sizeof(double) * 2 * (size_t)n_zg;
}

template <int M>
hipError_t launch_kg_t(const plan_dev& p, const swiftcl_inputs* in, const double* D_kz, void* C, hipStream_t s) {
  const int T = p.max_tracers, nb = p.n_bands, A = p.n_interp;
  const double h = (double)(p.n_k - 1) * p.delta / (double)(A - 1);
  const float s6 = (float)(6.0 / (h * h));
  const int NJ = (p.n_k + KG_TILE - 1) / KG_TILE;
  const bool split = p.precision == SWIFTCL_SPLIT_BF16;
  for (int b0 = 0; b0 < in->batch; b0 += p.vchunk) {
    const int nbp = in->batch - b0 < p.vchunk ? in->batch - b0 : p.vchunk;
    hipLaunchKernelGGL(k_kg_slots, dim3((nbp + 63) / 64), dim3(64), 0, s, p, *in, b0, nbp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kg_fft<M>, dim3((unsigned)((size_t)nbp * A)), dim3(256), kg_fft_lds<M>(p.n_zg), s, p, *in,
                       D_kz, b0, nbp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_kg_cspline, dim3((unsigned)((size_t)nbp * T * nb), (M + 255) / 256), dim3(256), 0, s, p,
                       *in, b0, nbp, s6);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t pairs = (size_t)nbp * T;
    const size_t groups = (pairs + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD;
    const dim3 gw((unsigned)(groups * p.kg_ntile * NJ * SWIFTCL_NXCD));
    if (split) hipLaunchKernelGGL(k_kg_windows<true>, gw, dim3(256), 0, s, p, *in, b0, nbp);
    else hipLaunchKernelGGL(k_kg_windows<false>, gw, dim3(256), 0, s, p, *in, b0, nbp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_contract(p, in, C, b0, nbp, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t kgrowth_fft_lds(int M, int n_zg) {
  switch (M) {
    case 128: return kg_fft_lds<128>(n_zg);
    case 256: return kg_fft_lds<256>(n_zg);
    case 512: return kg_fft_lds<512>(n_zg);
    case 1024: return kg_fft_lds<1024>(n_zg);
  }
  return 0;
}

hipError_t launch_kgrowth(const plan_dev& p, const swiftcl_inputs* in, const double* D_kz, void* C, hipStream_t s) {
  switch (p.M) {
    case 128: return launch_kg_t<128>(p, in, D_kz, C, s);
    case 256: return launch_kg_t<256>(p, in, D_kz, C, s);
    case 512: return launch_kg_t<512>(p, in, D_kz, C, s);
    case 1024: return launch_kg_t<1024>(p, in, D_kz, C, s);
  }
  return hipErrorInvalidValue;
}
