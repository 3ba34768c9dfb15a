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
//   k_kg_cspline  per (point, tracer, band, n): the node spline along ln k (Thomas, FP32,
//                 one pass, the back substitution restarted per 16-node segment)
//   k_kg_windows  the GEMM above, one workgroup per (point, tracer, slot tile, 64 k nodes)
//   k_contract    C = V V^T per (point, multipole) from the workspace (forward.hip)
#include <type_traits>

#include "common.h"
#include "geometry.h"
#include "internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int clamp_i(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

constexpr int KG_TILE = 64;   // slots and k nodes per GEMM workgroup
constexpr int KG_KC = 16;     // coefficients n per K chunk (32 real K rows)

// One wavefront per point: slot permutation (stable, grouped by band) and the tile list.  The
// slots are taken 64 at a time, one per lane; a ballot per band counts them and places each at its
// band's running offset plus the number of lower lanes of the same band.
__global__ __launch_bounds__(SWIFTCL_WAVE) void k_kg_slots(plan_dev P, swiftcl_inputs in, int b0, int nbp) {
  const int bl = blockIdx.x, lane = threadIdx.x;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  const int Lm = P.max_ell, nb = P.n_bands;
  const int Lb = clamp_i(in.n_ell[b], 0, Lm);
  const unsigned long long below = (1ull << lane) - 1ull;
  // band of slot li (-1 past the point's slots); a bad index is flagged and read as 0
  auto band_of = [&](int li) {
    if (li >= Lb) return -1;
    int ei = in.ell_idx[(size_t)b * Lm + li];
    if (ei < 0 || ei >= P.n_ell) {
      atomicOr(P.flags, FLAG_BAD_INDEX);
      ei = 0;
    }
    return P.ell_band[ei];
  };
  int cnt[SWIFTCL_MAX_BANDS] = {0, 0, 0, 0};
  for (int l0 = 0; l0 < Lb; l0 += SWIFTCL_WAVE) {
    const int bd = band_of(l0 + lane);
    for (int bi = 0; bi < nb; ++bi) cnt[bi] += __popcll(__ballot(bd == bi));
  }
  int off[SWIFTCL_MAX_BANDS], pos[SWIFTCL_MAX_BANDS];
  int acc = 0;
  for (int bi = 0; bi < nb; ++bi) {
    off[bi] = acc;
    pos[bi] = acc;
    acc += cnt[bi];
  }
  int* perm = P.kg_perm + (size_t)bl * Lm;
  for (int l0 = 0; l0 < Lb; l0 += SWIFTCL_WAVE) {
    const int li = l0 + lane;
    int bd = -1;
    if (li < Lb) {
      const int ei = in.ell_idx[(size_t)b * Lm + li];
      bd = P.ell_band[ei < 0 || ei >= P.n_ell ? 0 : ei];
    }
    for (int bi = 0; bi < nb; ++bi) {
      const unsigned long long mask = __ballot(bd == bi);
      if (bd == bi) perm[pos[bi] + __popcll(mask & below)] = li;
      pos[bi] += __popcll(mask);
    }
  }
  if (lane != 0) return;
  int4* tile = (int4*)P.kg_tile + (size_t)bl * P.kg_ntile;
  int nt = 0;
  for (int bi = 0; bi < nb; ++bi)
    for (int s = 0; s < cnt[bi]; s += KG_TILE)
      tile[nt++] = make_int4(bi, off[bi] + s, cnt[bi] - s < KG_TILE ? cnt[bi] - s : KG_TILE, 0);
  for (; nt < P.kg_ntile; ++nt) tile[nt] = make_int4(0, 0, 0, 0);
}

// One workgroup (4 wavefronts) per (point, node).  Dynamic LDS: twiddles [2M], growth on the chi
// nodes [2M] float, then the D(kappa_a, z) samples and their spline moments [2][n_zg] double, which
// are dead once the growth is sampled and share their space with the FFT scratch [4][fft_lds_size].
template <int M>
__global__ __launch_bounds__(256) void k_kg_fft(plan_dev P, swiftcl_inputs in, const double* __restrict__ Dkz,
                                                int b0, int nbp) {
  extern __shared__ __align__(16) unsigned char smem[];
  typedef float R;
  constexpr int N = 2 * M;
  constexpr int RL = M / SWIFTCL_WAVE;
  constexpr int FL = fft_lds_size(M, sizeof(R));
  C2<R>* stw = (C2<R>*)smem;
  float* Dk = (float*)(stw + N);
  C2<R>* fbuf = (C2<R>*)(Dk + N);
  double* y = (double*)(Dk + N);  // same space as fbuf
  const int nzg = P.n_zg;
  double* Mo = y + nzg;
  const int A = P.n_interp;
  const int bl = blockIdx.x / A, a = blockIdx.x % A;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  const int T = P.max_tracers, nb = P.n_bands;
  const int Tb = clamp_i(in.n_tracers[b], 0, T);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / SWIFTCL_WAVE), lane = threadIdx.x % SWIFTCL_WAVE;
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
    const int kind = tracer_kind(in, T, b, t);
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
// by the Thomas recurrences (1/pivots in kg_ip), in one pass over the coefficient rows.  The
// elimination d_a = (r_a - d_{a-1}) / p_a runs forward in registers, 16 nodes at a time, one
// segment ahead of the back substitution M_a = d_a - M_{a+1} / p_a.  That substitution starts
// afresh for every segment from M = 0 at the far end of the next segment: the 1/pivots rise from
// 1/4 to 2 - sqrt(3) and no further, so a moment computed at least 17 nodes before the restart
// differs from the full sweep's by at most (2 - sqrt(3))^17 < 2e-10 times the true moment at the
// restart node, and the moments of the last two segments are exact (the sweep then starts at
// M_{A-1} = 0).  The coefficient rows are read once and the moments written once (the two full
// sweeps read c, wrote d, read d, wrote M).
constexpr int KG_SEG = 16;

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
  const float* ip = P.kg_ip;
  m[0] = make_float2(0.f, 0.f);
  m[(size_t)(A - 1) * M] = make_float2(0.f, 0.f);
  // elimination state: c_{a-1}, c_a and d_{a-1} for the next node a
  float2 cm = c[0], c0 = c[(size_t)M];
  float2 d = make_float2(0.f, 0.f);
  // d of the interior nodes a0 .. a0 + 15 (0 past A - 2); the segment's 16 loads are issued together
  auto eliminate = [&](int a0, float2(&out)[KG_SEG]) {
    float2 cps[KG_SEG];
#pragma unroll
    for (int i = 0; i < KG_SEG; ++i)
      cps[i] = a0 + i + 1 < A ? c[(size_t)(a0 + i + 1) * M] : make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < KG_SEG; ++i) {
      const int a = a0 + i;
      if (a + 1 < A) {
        const float2 cp = cps[i];
        const float ipa = ip[a];
        d.x = (s6 * (cp.x - 2.f * c0.x + cm.x) - d.x) * ipa;
        d.y = (s6 * (cp.y - 2.f * c0.y + cm.y) - d.y) * ipa;
        cm = c0;
        c0 = cp;
        out[i] = d;
      } else {
        out[i] = make_float2(0.f, 0.f);
      }
    }
  };
  float2 dcur[KG_SEG], dnext[KG_SEG];
  eliminate(1, dcur);
  for (int a0 = 1; a0 + 1 < A; a0 += KG_SEG) {
    eliminate(a0 + KG_SEG, dnext);
    // back substitution through the next segment from M = 0 past its end (moments discarded) ...
    float2 mn = make_float2(0.f, 0.f);
#pragma unroll
    for (int i = KG_SEG - 1; i >= 0; --i) {
      const int a = a0 + KG_SEG + i;
      if (a + 1 < A) {
        const float ipa = ip[a];
        mn = make_float2(dnext[i].x - ipa * mn.x, dnext[i].y - ipa * mn.y);
      }
    }
    // ... then through this one, storing its moments
#pragma unroll
    for (int i = KG_SEG - 1; i >= 0; --i) {
      const int a = a0 + i;
      if (a + 1 < A) {
        const float ipa = ip[a];
        mn = make_float2(dcur[i].x - ipa * mn.x, dcur[i].y - ipa * mn.y);
        m[(size_t)a * M] = mn;
      }
    }
#pragma unroll
    for (int i = 0; i < KG_SEG; ++i) dcur[i] = dnext[i];
  }
}

__device__ __forceinline__ unsigned short bf16_rne_kg(float x) {
  const unsigned int u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// U in the A-operand order of the GEMM: for every (kind, multipole) and chunk c of 16 coefficients,
// 4 groups k of 8 consecutive K steps; entry [k][s] is h_n Re U(n) (k even) or -h_n Im U(n) (k odd)
// with n = 16 c + 8 (k / 2) + s.  Lane (row, k) of a 16x16x4 MFMA then loads its A values for the
// chunk's 8 K steps as 8 consecutive floats.  Built once per plan.
__global__ void k_kg_utab(plan_dev P) {
  const int M = P.M;
  const size_t total = (size_t)SWIFTCL_NKINDS * P.n_ell * 2 * M;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(i & 7), k = (int)((i >> 3) & 3);
    const size_t row_c = i >> 5;  // (kind, multipole, chunk)
    const int c = (int)(row_c % (M / KG_KC));
    const size_t row = row_c / (M / KG_KC);
    const int n = KG_KC * c + 8 * (k >> 1) + s;
    const float2 u = ((const float2*)P.U)[row * M + n];
    const float h = n == 0 ? 1.f : 2.f;
    P.kg_uh[i] = (k & 1) ? -h * u.y : h * u.x;
  }
}

// W tile [<= 64 slots of one band] x [64 k nodes] of one (point, tracer) by 4 wavefronts.  Wave w
// owns k nodes 16w..16w+15.  Per chunk of 16 coefficients the block copies the slots' rows of the
// operand-ordered U table into a double-buffered LDS tile (the next chunk's rows are loaded during
// this chunk's MFMAs; one block barrier per chunk), and each wave builds its own 16 columns of X in a
// private LDS strip laid out so that each lane then reads its 8 B values (and, per row tile, its 8
// A values) as two 16-byte loads.  Blocks of one (point, tracer) share an XCD, so its node
// coefficients are read into one L2.
constexpr int KG_XP = 36;  // floats per k-node row of the X strip: [4 groups][8 steps] + 4 (banks)
constexpr int KG_UP = 36;  // floats per slot row of the U tile: [4 groups][8 steps] + 4 (banks)

constexpr int KG_NA = 16;  // node rows a staged 64-node k tile may span (its intervals + 1)

// W_ONLY (the adjoint's recompute, FP32 rows): the rows hold W = F(l) kscale (...) itself, not
// sqrt(s) W.  STAGE (plans whose 64-node k tiles span <= KG_NA node rows): the node coefficients
// and moments of the tile's node rows for each chunk of 16 coefficients are staged in LDS by the
// whole block, one chunk ahead with the U rows, instead of being gathered by every lane when it
// builds X (the gathered loads' latency was exposed once per chunk).
template <bool SPLIT, bool W_ONLY = false, bool STAGE = false>
__global__ __launch_bounds__(256) void k_kg_windows(plan_dev P, swiftcl_inputs in, int b0, int nbp) {
  __shared__ __align__(16) float Xs[4][16][KG_XP];
  __shared__ __align__(16) float Us[2][KG_TILE][KG_UP];
  // node coefficients and moments; rows of 17 entries, so that the rows a half-wave reads (a few
  // consecutive node intervals, two coefficients) fall on distinct 8-byte LDS slots
  __shared__ __align__(16) float2 Cs[STAGE ? 2 : 1][STAGE ? KG_NA : 1][KG_KC + 1];
  __shared__ __align__(16) float2 Ms[STAGE ? 2 : 1][STAGE ? KG_NA : 1][KG_KC + 1];
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
  const int kind = tracer_kind(in, T, b, t);
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid / SWIFTCL_WAVE), lane = tid % SWIFTCL_WAVE;
  if (tid < KG_TILE) {
    int li = -1, ei = 0;
    if (tid < cnt) {
      li = P.kg_perm[(size_t)bl * Lm + s0 + tid];
      ei = in.ell_idx[(size_t)b * Lm + li];
      if (ei < 0 || ei >= P.n_ell) ei = 0;  // flagged by k_kg_slots
    }
    lis[tid] = li;
    eis[tid] = ei;
  }
  __syncthreads();
  const int nrt = (cnt + 15) / 16;
  const int Nmask = 2 * M - 1;
  const float2* tw = (const float2*)P.tw;
  auto twid = [&](int v) {
    const int qq = v & Nmask;
    float2 e = tw[qq & (M - 1)];
    if (qq >= M) { e.x = -e.x; e.y = -e.y; }
    return e;
  };
  const int jl = lane & 15, kq = lane >> 4;
  const int j = KG_TILE * jt + 16 * wave + jl;  // this lane's k node
  const bool jok = j < nk;
  // A: the block stages the operand-ordered U rows of its slots, one chunk ahead, in LDS; thread
  // tid copies 16 bytes (4 k steps) of slots tid / 8 and tid / 8 + 32
  const float* uh = P.kg_uh + (size_t)kind * P.n_ell * 2 * M;
  const int ur = tid >> 3, uc = 4 * (tid & 7);
  const int uoff0 = eis[ur] * 2 * M + uc, uoff1 = eis[ur + 32] * 2 * M + uc;
  const bool ul1 = ur + 32 < cnt;
  // B generation: coefficients nl = kq + 4 q of k node j from its node interval
  const int jc = jok ? j : nk - 1;
  const int ia = P.kg_ia[jc];
  const float4 wb = ((const float4*)P.kg_w)[jc];
  const size_t cbase = (((size_t)bl * T + t) * nb + band) * A;
  const float2* kc = (const float2*)P.kg_c + (cbase + ia) * M + kq;
  const float2* km = (const float2*)P.kg_m + (cbase + ia) * M + kq;
  // STAGE: the tile's first node row, this lane's row in the staged rows, and the entry thread tid
  // stages (node row ia0 + tid / 16, coefficient tid % 16 of the chunk)
  const int ia0 = P.kg_ia[min(KG_TILE * jt, nk - 1)];
  const int na = P.kg_ia[min(KG_TILE * jt + KG_TILE - 1, nk - 1)] - ia0 + 2;
  const int irow = ia - ia0;
  const int sa = tid >> 4, sn = tid & 15;
  const bool sok = STAGE && sa < na;
  const float2* sc = (const float2*)P.kg_c + (cbase + ia0 + (sok ? sa : 0)) * M + sn;
  const float2* sm = (const float2*)P.kg_m + (cbase + ia0 + (sok ? sa : 0)) * M + sn;
  float2 eq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) eq[q] = twid((kq + 4 * q) * j);
  float* xs = &Xs[wave][0][0];
  v4f acc[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) acc[rt] = (v4f){0.f, 0.f, 0.f, 0.f};
  // the K loop, instantiated for the number of 16-slot row tiles so that no MFMA sits behind a branch
  auto kloop = [&](auto nrt_c) {
    constexpr int NRT = decltype(nrt_c)::value;
    {
      *(float4*)&Us[0][ur][uc] = *(const float4*)(uh + uoff0);
      if (NRT > 2) *(float4*)&Us[0][ur + 32][uc] = ul1 ? *(const float4*)(uh + uoff1) : make_float4(0.f, 0.f, 0.f, 0.f);
      if (sok) {
        Cs[0][sa][sn] = sc[0];
        Ms[0][sa][sn] = sm[0];
      }
    }
    __syncthreads();
    int buf = 0;
    // e^{-2 pi i n0 j / N} of the chunk, advanced by one chunk's rotation in FP64 (no table load
    // inside the loop, where its wait would also wait for the prefetches above; 32 FP64 steps stay
    // far below FP32 rounding)
    double2 ed = make_double2(1.0, 0.0);
    double2 wd;
    sincospi(2.0 * (double)((KG_KC * j) & Nmask) / (double)(2 * M), &wd.y, &wd.x);
    wd.y = -wd.y;
    for (int n0 = 0; n0 < M; n0 += KG_KC) {
      // next chunk's U rows (and staged node rows), in flight during this chunk
      float4 un0 = make_float4(0.f, 0.f, 0.f, 0.f), un1 = un0;
      float2 cn = make_float2(0.f, 0.f), mn = cn;
      const bool more = n0 + KG_KC < M;
      if (more) {
        un0 = *(const float4*)(uh + uoff0 + 2 * (n0 + KG_KC));
        if (NRT > 2 && ul1) un1 = *(const float4*)(uh + uoff1 + 2 * (n0 + KG_KC));
        if (sok) {
          cn = sc[n0 + KG_KC];
          mn = sm[n0 + KG_KC];
        }
      }
      const float2 e0 = make_float2((float)ed.x, (float)ed.y);
      ed = make_double2(ed.x * wd.x - ed.y * wd.y, ed.x * wd.y + ed.y * wd.x);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int nl = kq + 4 * q;
        float2 ca, cb, ma, mb;
        if constexpr (STAGE) {
          ca = Cs[buf][irow][nl];
          cb = Cs[buf][irow + 1][nl];
          ma = Ms[buf][irow][nl];
          mb = Ms[buf][irow + 1][nl];
        } else {
          ca = kc[n0 + 4 * q];
          cb = kc[M + n0 + 4 * q];
          ma = km[n0 + 4 * q];
          mb = km[M + n0 + 4 * q];
        }
        float2 c;
        c.x = wb.x * ca.x + wb.y * cb.x + wb.z * ma.x + wb.w * mb.x;
        c.y = wb.x * ca.y + wb.y * cb.y + wb.z * ma.y + wb.w * mb.y;
        const float2 x = cmul(c, cmul(e0, eq[q]));
        // K order of the chunk: group 2 (nl / 8) + {0: Re, 1: Im}, step nl % 8
        xs[jl * KG_XP + 16 * (nl >> 3) + (nl & 7)] = jok ? x.x : 0.f;
        xs[jl * KG_XP + 16 * (nl >> 3) + 8 + (nl & 7)] = jok ? x.y : 0.f;
      }
      wave_sync();
      const float4 b0v = *(const float4*)(xs + jl * KG_XP + 8 * kq);
      const float4 b1v = *(const float4*)(xs + jl * KG_XP + 8 * kq + 4);
      wave_sync();
      const float bf[8] = {b0v.x, b0v.y, b0v.z, b0v.w, b1v.x, b1v.y, b1v.z, b1v.w};
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt) {
        const float4 a0 = *(const float4*)&Us[buf][16 * rt + jl][8 * kq];
        const float4 a1 = *(const float4*)&Us[buf][16 * rt + jl][8 * kq + 4];
        const float af[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[s], bf[s], acc[rt], 0, 0, 0);
      }
      if (more) {
        *(float4*)&Us[buf ^ 1][ur][uc] = un0;
        if (NRT > 2) *(float4*)&Us[buf ^ 1][ur + 32][uc] = un1;
        if constexpr (STAGE) {
          if (sok) {
            Cs[buf ^ 1][sa][sn] = cn;
            Ms[buf ^ 1][sa][sn] = mn;
          }
        }
      }
      __syncthreads();
      buf ^= 1;
    }
  };
  switch (nrt) {
    case 1: kloop(std::integral_constant<int, 1>{}); break;
    case 2: kloop(std::integral_constant<int, 2>{}); break;
    case 3: kloop(std::integral_constant<int, 3>{}); break;
    default: kloop(std::integral_constant<int, 4>{}); break;
  }
  // V = F(l) kscale sqrt(s) W into the workspace rows (point, slot, tracer)
  if (!jok) return;
  static_assert(!(SPLIT && W_ONLY), "the recompute writes FP32 rows");
  const float kqv = W_ONLY ? ((const float*)P.kscale)[((size_t)kind * nb + band) * nk + j]
                           : ((const float*)P.kss)[(((size_t)b * SWIFTCL_NKINDS + kind) * nb + band) * nk + j];
  const size_t lo_off = (size_t)P.vchunk * Lm * 32 * nk;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    if (rt >= nrt) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * rt + 4 * kq + q;
      if (r >= cnt) continue;
      const int li = lis[r];
      const float x = kqv * acc[rt][q];  // (F(l) is folded into U, hence into the operand table)
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

// The adjoint's recompute leaves the workspace rows of absent tracers (t >= T_b, up to the 16 or
// 32 rows the Gram tiles read) as they were: zero them, so that Y = G W reads no stale value.  One
// workgroup per (point, multipole slot < L_b) of the chunk.
__global__ __launch_bounds__(256) void k_kg_zero(plan_dev P, swiftcl_inputs in, int b0, int nbp) {
  const int Lm = P.max_ell, nk = P.n_k, T = P.max_tracers;
  const int bl = blockIdx.x / Lm, li = blockIdx.x % Lm;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  if (li >= clamp_i(in.n_ell[b], 0, Lm)) return;
  const int Tb = clamp_i(in.n_tracers[b], 0, T), rows = T > 16 ? 32 : 16;
  float* w = (float*)P.vbuf + ((size_t)bl * Lm + li) * 32 * nk;
  for (size_t i = (size_t)Tb * nk + threadIdx.x; i < (size_t)rows * nk; i += blockDim.x) w[i] = 0.f;
}

// dL/db_t of the scale-dependent growth path from the forward output: the windows of a clustering
// tracer are linear in its bias (every k node's kernel is b_t n_t dz/dchi D(k, z)), so
// dC^{ij}/db_t = C^{ij} (delta_it + delta_jt) / b_t, summed against dC over the point's multipoles
// and the pairs holding t (in a fixed order: reproducible).  One wavefront per (point, tracer).
__global__ __launch_bounds__(64) void k_kg_dbias(plan_dev P, swiftcl_inputs in, const float* __restrict__ C,
                                                 const float* __restrict__ dC, double* __restrict__ dbias) {
  const int T = P.max_tracers, Lm = P.max_ell, npair = T * (T + 1) / 2;
  const int b = blockIdx.x / T, t = blockIdx.x % T, lane = threadIdx.x;
  if (b >= in.batch) return;
  const int Tb = clamp_i(in.n_tracers[b], 0, T), Lb = clamp_i(in.n_ell[b], 0, Lm);
  double acc = 0.0;
  if (t < Tb && in.kind[(size_t)b * T + t] == SWIFTCL_CLUSTERING) {
    for (int q = lane; q < Lb * Tb; q += SWIFTCL_WAVE) {
      const int li = q / Tb, j = q % Tb;
      const int a = t < j ? t : j, c = t < j ? j : t;
      const size_t at = ((size_t)b * Lm + li) * npair + (size_t)a * T - a * (a - 1) / 2 + (c - a);
      acc += (double)dC[at] * (double)C[at] * (j == t ? 2.0 : 1.0);
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    acc /= in.bias[(size_t)b * T + t];
  }
  if (lane == 0) dbias[(size_t)b * T + t] = acc;
}

template <int M>
size_t kg_fft_lds(int n_zg) {
  const size_t fft = sizeof(float2) * 4 * (size_t)fft_lds_size(M, sizeof(float));
  const size_t spl = sizeof(double) * 2 * (size_t)n_zg;
  return sizeof(float2) * 2 * (size_t)M + sizeof(float) * 2 * M + (fft > spl ? fft : spl);
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
    hipLaunchKernelGGL(k_kg_slots, dim3(nbp), dim3(SWIFTCL_WAVE), 0, s, p, *in, b0, nbp);
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
    if (p.kg_stage) {
      if (split) hipLaunchKernelGGL((k_kg_windows<true, false, true>), gw, dim3(256), 0, s, p, *in, b0, nbp);
      else hipLaunchKernelGGL((k_kg_windows<false, false, true>), gw, dim3(256), 0, s, p, *in, b0, nbp);
    } else {
      if (split) hipLaunchKernelGGL(k_kg_windows<true>, gw, dim3(256), 0, s, p, *in, b0, nbp);
      else hipLaunchKernelGGL(k_kg_windows<false>, gw, dim3(256), 0, s, p, *in, b0, nbp);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_contract(p, in, C, b0, nbp, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Adjoint (dL/dP, dL/db): the windows recomputed as W rows, then Y = G W with the dP partials
// (the workspace adjoint's kernels), their reduction, and dL/db from the forward output C.
template <int M>
hipError_t launch_kg_bwd_t(const plan_dev& p, const swiftcl_inputs* in, const double* D_kz, const void* C,
                           const void* dC, double* dpk, double* dbias, hipStream_t s) {
  const int T = p.max_tracers, nb = p.n_bands, A = p.n_interp;
  const double h = (double)(p.n_k - 1) * p.delta / (double)(A - 1);
  const float s6 = (float)(6.0 / (h * h));
  const int NJ = (p.n_k + KG_TILE - 1) / KG_TILE;
  hipError_t e;
  if (dpk) {
    for (int b0 = 0; b0 < in->batch; b0 += p.vchunk) {
      const int nbp = in->batch - b0 < p.vchunk ? in->batch - b0 : p.vchunk;
      hipLaunchKernelGGL(k_kg_slots, dim3(nbp), dim3(SWIFTCL_WAVE), 0, s, p, *in, b0, nbp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_kg_fft<M>, dim3((unsigned)((size_t)nbp * A)), dim3(256), kg_fft_lds<M>(p.n_zg), s, p,
                         *in, D_kz, b0, nbp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_kg_cspline, dim3((unsigned)((size_t)nbp * T * nb), (M + 255) / 256), dim3(256), 0, s, p,
                         *in, b0, nbp, s6);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_kg_zero, dim3((unsigned)((size_t)nbp * p.max_ell)), dim3(256), 0, s, p, *in, b0, nbp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const size_t groups = ((size_t)nbp * T + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD;
      const dim3 gw((unsigned)(groups * p.kg_ntile * NJ * SWIFTCL_NXCD));
      if (p.kg_stage) hipLaunchKernelGGL((k_kg_windows<false, true, true>), gw, dim3(256), 0, s, p, *in, b0, nbp);
      else hipLaunchKernelGGL((k_kg_windows<false, true>), gw, dim3(256), 0, s, p, *in, b0, nbp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = launch_bwd_gv(p, in, dC, b0, nbp, s)) != hipSuccess) return e;
    }
    if ((e = launch_bwd_dpk(p, in, dpk, s)) != hipSuccess) return e;
  }
  if (dbias) {
    hipLaunchKernelGGL(k_kg_dbias, dim3((unsigned)((size_t)in->batch * T)), dim3(64), 0, s, p, *in,
                       (const float*)C, (const float*)dC, dbias);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_kgrowth_backward(const plan_dev& p, const swiftcl_inputs* in, const double* D_kz, const void* C,
                                   const void* dC, double* dpk, double* dbias, hipStream_t s) {
  switch (p.M) {
    case 128: return launch_kg_bwd_t<128>(p, in, D_kz, C, dC, dpk, dbias, s);
    case 256: return launch_kg_bwd_t<256>(p, in, D_kz, C, dC, dpk, dbias, s);
    case 512: return launch_kg_bwd_t<512>(p, in, D_kz, C, dC, dpk, dbias, s);
    case 1024: return launch_kg_bwd_t<1024>(p, in, D_kz, C, dC, dpk, dbias, s);
  }
  return hipErrorInvalidValue;
}

size_t kgrowth_fft_lds(int M, int n_zg) {
  switch (M) {
    case 128: return kg_fft_lds<128>(n_zg);
    case 256: return kg_fft_lds<256>(n_zg);
    case 512: return kg_fft_lds<512>(n_zg);
    case 1024: return kg_fft_lds<1024>(n_zg);
  }
  return 0;
}

hipError_t launch_kgrowth_tables(const plan_dev& p, hipStream_t s) {
  hipLaunchKernelGGL(k_kg_utab, dim3(256), dim3(256), 0, s, p);
  return hipGetLastError();
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
