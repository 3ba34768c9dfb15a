// Forward hot path: FFTLog coefficients (r2c), multiplication by the power-law Bessel table,
// inverse FFT to the k-windows and the projection C = W diag(s) W^T on MFMA.
//
// Notation (paper Sec. 3.1-3.2, with the readings stated in swiftcl.h):
//   g_m   = w_m f(chi_m) (chi_m / chi_0)^-b                     (assembled in FP64, assemble.hip)
//   c_n   = (1/N) sum_m g_m e^{-2 pi i n m / N} (k_0 chi_0)^{-i eta_n} chi_0^{-b},  n < N/2
//   d_n   = c_n U_l(n),   U_l(n) = sqrt(pi) 2^{p-1} Gamma((1+l+p)/2) / Gamma((2+l-p)/2)
//   x_j   = Re( d_0 + 2 sum_{n=1}^{N/2-1} d_n e^{-2 pi i n j / N} )
//   W_j   = c(l) k_j^{-1-b} [k_j^-2 for lensing] x_j              (Delta_l(k_j) of Sec. 2.1)
//   C_l^{ij} = sum_j s_j W_i(k_j) W_j(k_j),  s_j = (2/pi) w_j k_j^3 P_j
// One wavefront runs one length-N real transform as a length-N/2 complex FFT in registers and
// LDS; one workgroup owns one (point, multipole) and keeps sqrt(s) W of all its tracers in LDS,
// so the windows never touch HBM on the C_l path.
#include "common.h"
#include "internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename R> struct mfma_acc;
// Output layout of the 16x16x4 MFMAs: lane l, accumulator register r holds D[row][l % 16] with
// row = 4 (l / 16) + r for f32 and row = l / 16 + 4 r for f64.
template <> struct mfma_acc<float> {
  typedef v4f type;
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane / 16) + r; }
  static __device__ __forceinline__ type step(float a, float b, type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct mfma_acc<double> {
  typedef v4d type;
  static __device__ __forceinline__ int row(int lane, int r) { return lane / 16 + 4 * r; }
  static __device__ __forceinline__ type step(double a, double b, type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Split precision: v = hi + lo with hi = bf16(v) and lo = bf16(v - hi), both rounded to nearest
// even; hi + lo carries 16 significant bits.  Products accumulate in FP32 on the
// 16x16x32 bf16 MFMA as hi.hi + hi.lo + lo.hi (lo.lo, below 2^-16 relative, is dropped).
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  const unsigned int u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
__device__ __forceinline__ void split_bf16(float x, unsigned short* hi, unsigned short* lo) {
  *hi = bf16_rne(x);
  *lo = bf16_rne(x - bf16_to_float(*hi));
}
__device__ __forceinline__ v4f mfma_bf16(v8us a, v8us b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

template <typename R>
__global__ void k_sqrt_s(plan_dev P, swiftcl_inputs in) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= in.batch || j >= P.n_k) return;
  const double v = P.kw[j] * in.pk[(size_t)b * P.n_k + j];
  if (!(v >= 0.0) || !isfinite(v)) atomicOr(P.flags, FLAG_NONFINITE);
  const R sq = (R)sqrt(fmax(v, 0.0));
  ((R*)P.sqrt_s)[(size_t)b * P.n_k + j] = sq;
  // kscale * sqrt(s) for every kind and band: the projection scales its windows once
  for (int kb = 0; kb < SWIFTCL_NKINDS * P.n_bands; ++kb)
    ((R*)P.kss)[((size_t)b * SWIFTCL_NKINDS * P.n_bands + kb) * P.n_k + j] = ((const R*)P.kscale)[(size_t)kb * P.n_k + j] * sq;
}

// FFTLog coefficients: one wavefront per (point, tracer, band) row.  SET 0: the kernels; 1: the RSD
// kernels; 2: the magnification kernels (tilted with the bias b - 2, hence the extra chi_0^2).
template <typename R, int M, int SET = 0>
__global__ __launch_bounds__(256) void k_forward_fft(plan_dev P, swiftcl_inputs in) {
  __shared__ C2<R> lds[4][fft_lds_size(M, sizeof(R))];
  // FP32: the twiddle table staged in LDS by the block (FP64 reads it through the cache)
  constexpr bool TWS = sizeof(R) == 4;
  __shared__ C2<R> stw_s[TWS ? 2 * M : 1];
  if constexpr (TWS) {
    for (int i = threadIdx.x; i < 2 * M; i += blockDim.x) stw_s[i] = ((const C2<R>*)P.tw)[i];
    __syncthreads();
  }
  const C2<R>* twp = TWS ? (const C2<R>*)stw_s : (const C2<R>*)P.tw;
  constexpr int RL = M / SWIFTCL_WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / SWIFTCL_WAVE), lane = threadIdx.x % SWIFTCL_WAVE;
  const int T = P.max_tracers, nb = P.n_bands, N = P.N;
  const long rows = (long)in.batch * T * nb;
  const long row = (long)blockIdx.x * 4 + wave;
  if (row >= rows) return;  // whole wavefront leaves; no block barrier below
  const int bi = (int)(row % nb);
  const int t = (int)((row / nb) % T);
  const int b = (int)(row / ((long)nb * T));
  C2<R>* out = (C2<R>*)(SET == 1 ? P.chat_r : (SET == 2 ? P.chat_mu : P.chat)) + row * M;
  const int Tb = clampi(in.n_tracers[b], 0, T);
  if (t >= Tb) {
#pragma unroll
    for (int e = 0; e < RL; ++e) out[lane + SWIFTCL_WAVE * e] = mk<R>(0, 0);
    return;
  }
  const C2<R>* g2 = (const C2<R>*)((const R*)(SET == 1 ? P.g_r : (SET == 2 ? P.g_mu : P.g)) + row * N);
  const C2<R>* tw = twp;
  C2<R> v[RL];
#pragma unroll
  for (int e = 0; e < RL; ++e) v[e] = g2[lane + SWIFTCL_WAVE * e];
  wave_r2c<R, M>(v, lds[wave], tw, lane);
  const double* pt = P.pt + (size_t)b * PT_STRIDE;
  const int kind = tracer_kind(in, T, b, t);
  double scale = pt[PT_CHI0B + kind * SWIFTCL_MAX_BANDS + bi] / (double)N;
  if (SET == 2) scale *= pt[PT_CHI0] * pt[PT_CHI0];
  const double2* ph = (const double2*)P.phase + (size_t)b * M;
#pragma unroll
  for (int e = 0; e < RL; ++e) {
    const int n = lane + SWIFTCL_WAVE * e;
    const double2 a = ph[n];
    out[n] = cmul(v[e], mk<R>((R)(a.x * scale), (R)(a.y * scale)));
  }
}

// Windows and / or C_l of one (point, multipole slot) by a workgroup of NW wavefronts (wave t
// handles tracer t); stw: twiddles (LDS or global), fbuf: per-wave FFT scratch, V: sqrt(s) W.
// COMPACT (FP32 projection): the FFT scratch of tracer t lives in V's row t (the wavefront writes
// the row only after its transform): twiddles + 16 x compact_vs_fwd floats of LDS, which for
// n_chi <= 1024 and n_k <= 1024 is 72 KiB, so two 1024-thread workgroups share a CU.
// PACK (C_l only): a second item (b2, li2), b2 >= 0, takes the rows T_b .. T_b + T_b2 - 1 of the
// same 16-row Gram tile; its spectra are the tile's diagonal block at that offset (the two items'
// cross block is computed and dropped).  The packed work list guarantees T_b + T_b2 <= 16.
template <typename R, int M, int NW, bool WRITE_W, bool DO_CL, bool SPLIT, bool COMPACT, bool PACK = false>
__device__ __forceinline__ void windows_cl_item(const plan_dev& P, const swiftcl_inputs& in, R* __restrict__ Wout,
                                                R* __restrict__ Cout, int b, int li, const C2<R>* stw, C2<R>* fbuf,
                                                R* V, int b2 = -1, int li2 = 0) {
  constexpr int RL = M / SWIFTCL_WAVE;
  constexpr int FL = fft_lds_size(M, sizeof(R));
  // W and V = sqrt(s) W take different k scales (kscale, kss); one call produces one of them
  static_assert(!(WRITE_W && DO_CL), "windows and C_l come from separate instantiations");
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / SWIFTCL_WAVE), lane = threadIdx.x % SWIFTCL_WAVE;
  const int T = P.max_tracers, Lm = P.max_ell, nk = P.n_k, nb = P.n_bands;
  const int Tb = clampi(in.n_tracers[b], 0, T);
  const int Lb = clampi(in.n_ell[b], 0, Lm);
  const int npair = T * (T + 1) / 2;
  if (li >= Lb) {
    if (WRITE_W) {
      R* w = Wout + ((size_t)b * Lm + li) * T * nk;
      for (int i = threadIdx.x; i < T * nk; i += NW * 64) w[i] = (R)0;
    }
    if (DO_CL) {
      R* c = Cout + ((size_t)b * Lm + li) * npair;
      for (int i = threadIdx.x; i < npair; i += NW * 64) c[i] = (R)0;
    }
    return;
  }
  static_assert(!PACK || (DO_CL && !WRITE_W), "packing applies to the C_l projection");
  auto ell_index = [&](int pb, int pl) {
    int e = in.ell_idx[(size_t)pb * Lm + pl];
    if (e < 0 || e >= P.n_ell) {
      if (threadIdx.x == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
      e = 0;
    }
    return e;
  };
  const int ei1 = ell_index(b, li);
  // the second item's rows start at o2 (no second item: o2 = 16, no row is its)
  int o2 = 16, Tb2 = 0, ei2 = 0;
  if (PACK && b2 >= 0) {
    Tb2 = clampi(in.n_tracers[b2], 0, T);
    ei2 = ell_index(b2, li2);
    o2 = Tb;
    if (o2 + Tb2 > 16) {  // not produced by the list builder
      if (threadIdx.x == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
      o2 = 16;
      Tb2 = 0;
      b2 = -1;
    }
  }
  const int vs = COMPACT ? compact_vs_fwd(nk, M) : nk + 2;  // row stride of V: rows start on distinct banks
  const int trows = DO_CL ? 16 : T;
  for (int r = wave; r < trows; r += NW) {
    const bool sec = PACK && r >= o2;  // row of the second item
    const int t = sec ? r - o2 : r, bt = sec ? b2 : b, ei = sec ? ei2 : ei1;
    if (t >= (sec ? Tb2 : Tb)) {
      for (int j = lane; j < nk; j += SWIFTCL_WAVE) {
        if (DO_CL) V[r * vs + j] = (R)0;
        if (WRITE_W && t < T) Wout[(((size_t)b * Lm + li) * T + t) * nk + j] = (R)0;
      }
      continue;
    }
    const int band = P.ell_band[ei];
    const int kind = tracer_kind(in, T, bt, t);
    const C2<R>* ch = (const C2<R>*)P.chat + (((size_t)bt * T + t) * nb + band) * M;
    const C2<R>* Ur = (const C2<R>*)P.U + ((size_t)kind * P.n_ell + ei) * M;
    C2<R>* mine = COMPACT ? (C2<R>*)(V + (size_t)r * vs) : fbuf + (size_t)wave * FL;
    C2<R> v[RL];
    wave_sync();
#pragma unroll
    for (int e = 0; e < RL; ++e) {
      const int n = lane + SWIFTCL_WAVE * e;
      v[e] = cconj(cmul(ch[n], Ur[n]));  // X_n = conj(c_n U_l(n))
    }
    int ln = lane;  // opaque copy: keeps the FFT's per-lane LDS addresses from being hoisted
    asm volatile("" : "+v"(ln));
    ln &= SWIFTCL_WAVE - 1;  // the compiler may assume 0 <= ln < 64 again
    wave_c2r<R, M>(v, mine, stw, ln);
    wave_sync();
    // the k scale of the output pairs, loads issued in groups of KG (the index is clamped into
    // the row, nk is even; only the stores are guarded)
    const R* kscl = DO_CL ? (const R*)P.kss + (((size_t)bt * SWIFTCL_NKINDS + kind) * nb + band) * nk
                          : (const R*)P.kscale + ((size_t)kind * nb + band) * nk;
    constexpr int KG = RL < 4 ? RL : 4;  // (the prefactor F(l) is folded into U)
#pragma unroll
    for (int e0 = 0; e0 < RL; e0 += KG) {
      C2<R> kk[KG];
#pragma unroll
      for (int e = 0; e < KG; ++e) kk[e] = *(const C2<R>*)(kscl + min(2 * (ln + SWIFTCL_WAVE * (e0 + e)), nk - 2));
#pragma unroll
      for (int e = 0; e < KG; ++e) {
        const int k0 = 2 * (ln + SWIFTCL_WAVE * (e0 + e));
        if (k0 < nk) {
          const C2<R> x = mk<R>(kk[e].x * v[e0 + e].x, kk[e].y * v[e0 + e].y);
          if (WRITE_W) *(C2<R>*)(Wout + (((size_t)b * Lm + li) * T + t) * nk + k0) = x;
          if (DO_CL) *(C2<R>*)(V + r * vs + k0) = x;  // V = sqrt(s) W
        }
      }
    }
  }
  if (!DO_CL) return;
  __syncthreads();
  // C = V V^T over k on MFMA 16x16x4: lane feeds V[lane % 16][k] as both A and B operand.
  using acc_t = typename mfma_acc<R>::type;
  acc_t acc = {0, 0, 0, 0};
  if constexpr (SPLIT) {
    // 16x16x32 bf16: lane feeds 8 consecutive k of row lane % 16, split into hi + lo
    const int nsteps = (nk + 31) / 32;
    for (int s = wave; s < nsteps; s += NW) {
      const int k0 = 32 * s + 8 * (lane / 16);
      v8us hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        unsigned short h = 0, l = 0;
        if (k0 + e < nk) split_bf16((float)V[(lane & 15) * vs + k0 + e], &h, &l);
        hi[e] = h;
        lo[e] = l;
      }
      acc = mfma_bf16(hi, hi, acc);
      acc = mfma_bf16(hi, lo, acc);
      acc = mfma_bf16(lo, hi, acc);
    }
  } else {
    const int nsteps = (nk + 3) / 4;
    for (int s = wave; s < nsteps; s += NW) {
      const int kk = 4 * s + lane / 16;
      const R a = kk < nk ? V[(lane & 15) * vs + kk] : (R)0;
      acc = mfma_acc<R>::step(a, a, acc);
    }
  }
  R* red = COMPACT ? V : (R*)fbuf;  // [NW][256]: the FFT scratch, or V once every wave has read it
  if (COMPACT) __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave * 256 + mfma_acc<R>::row(lane, r) * 16 + (lane & 15)] = acc[r];
  __syncthreads();
  const int nout = (PACK && b2 >= 0) ? 2 * npair : npair;
  for (int idx = threadIdx.x; idx < nout; idx += NW * 64) {
    const bool sec = PACK && idx >= npair;
    const int o = sec ? o2 : 0, tb = sec ? Tb2 : Tb;
    int i = 0, rem = sec ? idx - npair : idx;
    const int at = rem;
    while (rem >= T - i) { rem -= T - i; ++i; }
    const int j = i + rem;
    R val = (R)0;
    if (i < tb && j < tb) {
#pragma unroll
      for (int w = 0; w < NW; ++w) val += red[w * 256 + (o + i) * 16 + o + j];
    }
    Cout[((size_t)(sec ? b2 : b) * Lm + (sec ? li2 : li)) * npair + at] = val;
  }
}

// Launch modes.  MODE 0: one workgroup per (point, multipole slot), blocks mapped so that all
// multipoles of one point run on one XCD (block = ((b / 8) * Lm + l) * 8 + b % 8); padded slots
// write zeros.  MODE 1: a grid sized to the chip; the blocks of XCD x walk the compact list of
// (point b = 8 i + x, multipole) items built by k_schedule with the grid stride (ragged multipole
// counts leave no idle workgroup, and every block loads the twiddles once).  MODE 2: as MODE 1 over
// the packed list of k_schedule_packed, whose tasks hold one or two items of the XCD's points with
// at most 16 tracers between them (points of few tracers leave no idle wavefronts).  Persistent
// modes: padded slots are zeroed by k_zero_padded.
template <typename R, int M, int NW, bool TW_LDS, bool WRITE_W, bool DO_CL, int MODE, bool SPLIT>
__global__ __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu((sizeof(R) == 4 && DO_CL && M <= 512) ? 8 : 1))) void k_windows_cl(
    plan_dev P, swiftcl_inputs in, R* __restrict__ Wout, R* __restrict__ Cout) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool COMPACT = sizeof(R) == 4 && DO_CL;
  constexpr int N = 2 * M;
  constexpr int FL = fft_lds_size(M, sizeof(R));
  constexpr int NTW = TW_LDS ? N : 0;
  C2<R>* stw_l = (C2<R>*)smem;  // [N] twiddles (TW_LDS)
  C2<R>* fbuf = stw_l + NTW;    // [NW][FL] (not COMPACT)
  R* V = (R*)(smem + ((size_t)NTW + (COMPACT ? 0 : (size_t)NW * FL)) * sizeof(C2<R>));  // [16][vs]
  const int xcd = blockIdx.x % SWIFTCL_NXCD;
  const int rest = blockIdx.x / SWIFTCL_NXCD;
  const C2<R>* stw = TW_LDS ? stw_l : (const C2<R>*)P.tw;
  if constexpr (MODE == 0) {
    const int li = rest % P.max_ell;
    const int b = (rest / P.max_ell) * SWIFTCL_NXCD + xcd;
    if (b >= in.batch) return;
    if constexpr (TW_LDS) {
      const C2<R>* gtw = (const C2<R>*)P.tw;
      for (int i = threadIdx.x; i < N; i += NW * 64) stw_l[i] = gtw[i];
      __syncthreads();
    }
    windows_cl_item<R, M, NW, WRITE_W, DO_CL, SPLIT, COMPACT>(P, in, Wout, Cout, b, li, stw, fbuf, V);
  } else {
    const int stride = P.sched_stride;
    const int* offs = P.sched + sched_list_index(stride, xcd, 0);
    const int total = P.sched[sched_total_index(stride, xcd)];
    const int nx = (in.batch - xcd + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD;
    const int g8 = gridDim.x / SWIFTCL_NXCD;
    if (rest >= total) return;
    if constexpr (TW_LDS) {
      const C2<R>* gtw = (const C2<R>*)P.tw;
      for (int i = threadIdx.x; i < N; i += NW * 64) stw_l[i] = gtw[i];
      __syncthreads();
    }
    // largest i with offs[i] <= q: the position of the point holding stream item q
    auto locate = [&](int q) {
      int i = 0, hi = nx;
      while (hi - i > 1) {
        const int mid = (i + hi) >> 1;
        if (offs[mid] <= q) i = mid; else hi = mid;
      }
      return i;
    };
    if constexpr (MODE == 1) {
      // items rest, rest + g8, ...: the blocks of an XCD work on neighbouring items at any time, so
      // the coefficients of the few points in flight stay in that XCD's L2
      int i = locate(rest);
      for (int k = rest; k < total; k += g8) {
        windows_cl_item<R, M, NW, WRITE_W, DO_CL, SPLIT, COMPACT>(P, in, Wout, Cout, i * SWIFTCL_NXCD + xcd,
                                                                  k - offs[i], stw, fbuf, V);
        __syncthreads();
        while (i + 1 < nx && offs[i + 1] <= k + g8) ++i;  // the point holding item k + g8
      }
    } else {
      static_assert(MODE != 2 || (DO_CL && !WRITE_W), "the packed list serves the C_l projection");
      // tasks of uneven cost: after its first task (rest) a block takes the next one from the XCD's
      // counter (zeroed by the list builder), requested one task ahead; next[] alternates so that
      // the slot written during task i was last read before the barrier that ended task i - 1
      __shared__ int next[2];
      int* ctr = P.sched + sched_ctr_index(stride, xcd);
      const int* pts = P.sched + sched_pts_index(stride, xcd, 0);
      const int* seg = P.sched + sched_seg_index(stride, xcd, 0);
      const int nseg = min(seg[0], SCHED_MAXSEG);
      int sg = 0, par = 0;
      for (int k = rest; k < total; par ^= 1) {
        if (threadIdx.x == 0) next[par] = g8 + atomicAdd(ctr, 1);
        while (sg + 1 < nseg && seg[1 + 3 * (sg + 1)] <= k) ++sg;  // the segment holding task k
        const int d = k - seg[1 + 3 * sg];
        const int qa = seg[2 + 3 * sg] + d, qb0 = seg[3 + 3 * sg];
        const int ia = locate(qa);
        int b2 = -1, l2 = 0;
        if (qb0 >= 0) {
          const int ib = locate(qb0 + d);
          b2 = pts[ib];
          l2 = qb0 + d - offs[ib];
        }
        windows_cl_item<R, M, NW, false, true, SPLIT, COMPACT, true>(P, in, Wout, Cout, pts[ia], qa - offs[ia], stw,
                                                                     fbuf, V, b2, l2);
        __syncthreads();
        k = next[par];  // increasing: the counter only grows and starts above every first task
      }
    }
  }
}

// Per-XCD compact work lists: offs[x][i] = sum of the multipole counts of points 8 j + x, j < i;
// the totals follow the eight lists (layout: sched_layout.h).
__global__ void k_schedule(plan_dev P, swiftcl_inputs in) {
  const int x = threadIdx.x;
  if (x >= SWIFTCL_NXCD) return;
  int* offs = P.sched + sched_list_index(P.sched_stride, x, 0);
  int acc = 0, i = 0;
  for (int b = x; b < in.batch; b += SWIFTCL_NXCD, ++i) {
    offs[i] = acc;
    acc += clampi(in.n_ell[b], 0, P.max_ell);
  }
  offs[i] = acc;
  P.sched[sched_total_index(P.sched_stride, x)] = acc;
}

// Packed per-XCD work lists (layout: sched_layout.h): XCD x's points ordered by descending
// tracer count (a counting sort, stable within a count), the multipole prefix offsets over that
// order, the pairing segments of sched_pack, and the XCD's task counter zeroed.  One 64-thread
// workgroup per XCD: the lanes stage the points' tracer and multipole counts in LDS, lane 0 builds
// the list from there.
__global__ __launch_bounds__(64) void k_schedule_packed(plan_dev P, swiftcl_inputs in) {
  constexpr int NC = SCHED_ROWS + 1;
  __shared__ int s_t[SCHED_PACK_MAXNX], s_l[SCHED_PACK_MAXNX];
  __shared__ int cnt[NC], rem[NC], cur[NC];
  const int x = blockIdx.x, lane = threadIdx.x;
  const int st = P.sched_stride, Tm = min(P.max_tracers, SCHED_ROWS), Lm = P.max_ell;
  const int nx = min((in.batch - x + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD, SCHED_PACK_MAXNX);
  for (int i = lane; i < nx; i += 64) {
    const int b = i * SWIFTCL_NXCD + x;
    s_t[i] = clampi(in.n_tracers[b], 0, Tm);
    s_l[i] = clampi(in.n_ell[b], 0, Lm);
  }
  __syncthreads();
  if (lane != 0) return;
  for (int c = 0; c < NC; ++c) cnt[c] = rem[c] = 0;
  for (int i = 0; i < nx; ++i) {
    ++cnt[s_t[i]];
    rem[s_t[i]] += s_l[i];
  }
  // first position of each count in the point order, and first stream index of its items
  int pos = 0, items = 0;
  for (int c = SCHED_ROWS; c >= 0; --c) {
    const int n = cnt[c];
    cnt[c] = pos;
    cur[c] = items;
    pos += n;
    items += rem[c];
  }
  // place the points; offs over the new order from the position of each point's first item
  int* pts = P.sched + sched_pts_index(st, x, 0);
  int* offs = P.sched + sched_list_index(st, x, 0);
  for (int i = 0; i < nx; ++i) {
    const int c = s_t[i], at = cnt[c]++;
    pts[at] = i * SWIFTCL_NXCD + x;
    offs[at] = cur[c];
    cur[c] += s_l[i];
  }
  offs[pos] = items;
  for (int c = SCHED_ROWS, at = 0; c >= 0; --c) {  // rewind: cur[c] = first item of count c
    cur[c] = at;
    at += rem[c];
  }
  int* seg = P.sched + sched_seg_index(st, x, 0);
  int total = sched_pack(rem, cur, seg);
  if (seg[0] > SCHED_MAXSEG) {  // cannot happen (at most 43 segments); run nothing rather than misread
    atomicOr(P.flags, FLAG_BAD_INDEX);
    total = 0;
  }
  P.sched[sched_total_index(st, x)] = total;
  P.sched[sched_ctr_index(st, x)] = 0;
}

// Zeros of the padded multipole slots (l >= n_ell[b]) for the persistent launch.
template <typename R>
__global__ void k_zero_padded(plan_dev P, swiftcl_inputs in, R* __restrict__ Cout) {
  const int b = blockIdx.y, li = blockIdx.x;
  if (b >= in.batch || li < clampi(in.n_ell[b], 0, P.max_ell)) return;
  const int npair = P.max_tracers * (P.max_tracers + 1) / 2;
  R* c = Cout + ((size_t)b * P.max_ell + li) * npair;
  for (int i = threadIdx.x; i < npair; i += blockDim.x) c[i] = (R)0;
}

template <typename R, int M>
static hipError_t launch_fwd_t(const plan_dev& p, const swiftcl_inputs* in, hipStream_t s) {
  hipLaunchKernelGGL(k_sqrt_s<R>, dim3((p.n_k + 255) / 256, in->batch), dim3(256), 0, s, p, *in);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long rows = (long)in->batch * p.max_tracers * p.n_bands;
  hipLaunchKernelGGL((k_forward_fft<R, M>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, p, *in);
  if (p.rsd) hipLaunchKernelGGL((k_forward_fft<R, M, 1>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, p, *in);
  if (p.mag && in->mag)
    hipLaunchKernelGGL((k_forward_fft<R, M, 2>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, p, *in);
  return hipGetLastError();
}

hipError_t launch_forward_fft(const plan_dev& p, const swiftcl_inputs* in, hipStream_t s) {
  const bool dp = p.precision == SWIFTCL_FP64;
  switch (p.M) {
    case 128: return dp ? launch_fwd_t<double, 128>(p, in, s) : launch_fwd_t<float, 128>(p, in, s);
    case 256: return dp ? launch_fwd_t<double, 256>(p, in, s) : launch_fwd_t<float, 256>(p, in, s);
    case 512: return dp ? launch_fwd_t<double, 512>(p, in, s) : launch_fwd_t<float, 512>(p, in, s);
    case 1024: return dp ? launch_fwd_t<double, 1024>(p, in, s) : launch_fwd_t<float, 1024>(p, in, s);
  }
  return hipErrorInvalidValue;
}

// LDS bytes of the fused kernel (twiddles, per-wave FFT scratch, V)
size_t windows_cl_lds(int M, int NW, bool tw_lds, bool do_cl, size_t rs, int n_k) {
  return ((tw_lds ? 2 * (size_t)M : 0) + (size_t)NW * fft_lds_size(M, (int)rs)) * 2 * rs +
         (do_cl ? (size_t)16 * (n_k + 2) * rs : 0);
}

// Workgroup shape: FP32 16 wavefronts (one tracer each), twiddles in LDS up to N = 1024; FP64 2
// wavefronts with twiddles read through the cache (V alone is 8 bytes x 16 x n_k).
template <typename R, int M> struct wcl_shape;
template <int M> struct wcl_shape<float, M> {
  static constexpr int NW = 16;
  static constexpr bool TW = M <= 512;
};
template <int M> struct wcl_shape<double, M> {
  static constexpr int NW = 2;
  static constexpr bool TW = false;
};

int windows_nw(int precision) { return precision == SWIFTCL_FP64 ? 2 : 16; }
bool windows_tw_lds(int precision, int M) { return precision != SWIFTCL_FP64 && M <= 512; }
// the unfused FP32 windows kernel (no V rows in LDS) stages the twiddles up to n_chi = 2048
constexpr bool unfused_tw(int M) { return M <= 1024; }
bool unfused_tw_lds(int M) { return unfused_tw(M); }

// ---------------------------------------------------------------------------------------------
// Unfused projection for more than 16 tracers or windows too large for LDS (FP32 / split):
// k_windows_v writes V = sqrt(s) W of up to 32 tracer slots per (point, multipole) to the
// workspace, k_contract forms the 32 x 32 Gram matrix from three 16 x 16 MFMA tile pairs
// (0,0), (0,1), (1,1).  Points are processed in chunks of P.vchunk.
// ---------------------------------------------------------------------------------------------
// EXTRA bit 1: the plan carries RSD, bit 2: magnification (used when the inputs give C_g).
// w_only = 1 (FP32, the adjoint's recompute): the rows hold W = F(l) kscale c2r(...) itself, not
// sqrt(s) W.
template <int M, int NW, bool TW_LDS, bool SPLIT, int EXTRA>
__global__ __launch_bounds__(NW * 64) void k_windows_v(plan_dev P, swiftcl_inputs in, int b0, int nbp, int w_only) {
  extern __shared__ __align__(16) unsigned char smem[];
  typedef float R;
  constexpr int RL = M / SWIFTCL_WAVE;
  constexpr int N = 2 * M;
  constexpr int FL = fft_lds_size(M, sizeof(R));
  constexpr int NTW = TW_LDS ? N : 0;
  C2<R>* stw_l = (C2<R>*)smem;
  C2<R>* fbuf = stw_l + NTW;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / SWIFTCL_WAVE), lane = threadIdx.x % SWIFTCL_WAVE;
  const int T = P.max_tracers, Lm = P.max_ell, nk = P.n_k, nb = P.n_bands;
  const int xcd = blockIdx.x % SWIFTCL_NXCD;
  const int rest = blockIdx.x / SWIFTCL_NXCD;
  const int li = rest % Lm;
  const int bl = (rest / Lm) * SWIFTCL_NXCD + xcd;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  const int Tb = clampi(in.n_tracers[b], 0, T);
  const int Lb = clampi(in.n_ell[b], 0, Lm);
  const size_t row0 = ((size_t)bl * Lm + li) * 32;
  const size_t lo_off = (size_t)P.vchunk * Lm * 32 * nk;  // split: lo parts after all hi parts
  float* vf = (float*)P.vbuf;
  unsigned short* vh = (unsigned short*)P.vbuf;
  if (li >= Lb) {
    for (size_t i = threadIdx.x; i < (size_t)32 * nk; i += NW * 64) {
      if (SPLIT) { vh[row0 * nk + i] = 0; vh[lo_off + row0 * nk + i] = 0; }
      else vf[row0 * nk + i] = 0.f;
    }
    return;
  }
  int ei = in.ell_idx[(size_t)b * Lm + li];
  if (ei < 0 || ei >= P.n_ell) {
    if (threadIdx.x == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
    ei = 0;
  }
  const C2<R>* stw = TW_LDS ? stw_l : (const C2<R>*)P.tw;
  if constexpr (TW_LDS) {
    const C2<R>* gtw = (const C2<R>*)P.tw;
    for (int i = threadIdx.x; i < N; i += NW * 64) stw_l[i] = gtw[i];
    __syncthreads();
  }
  const int band = P.ell_band[ei];
  C2<R>* mine = fbuf + (size_t)wave * FL;
  for (int t = wave; t < 32; t += NW) {
    const size_t rb = (row0 + t) * nk;
    if (t >= Tb) {
      for (int j = lane; j < nk; j += SWIFTCL_WAVE) {
        if (SPLIT) { vh[rb + j] = 0; vh[lo_off + rb + j] = 0; }
        else vf[rb + j] = 0.f;
      }
      continue;
    }
    const int kind = tracer_kind(in, T, b, t);
    const C2<R>* ch = (const C2<R>*)P.chat + (((size_t)b * T + t) * nb + band) * M;
    const C2<R>* Ur = (const C2<R>*)P.U + ((size_t)kind * P.n_ell + ei) * M;
    C2<R> v[RL];
    wave_sync();
#pragma unroll
    for (int e = 0; e < RL; ++e) {
      const int n = lane + SWIFTCL_WAVE * e;
      v[e] = cconj(cmul(ch[n], Ur[n]));
    }
    if ((EXTRA & 1) && kind == SWIFTCL_CLUSTERING) {
      // the RSD window of a clustering tracer shares its prefactor and k scale: add its term
      const C2<R>* chr = (const C2<R>*)P.chat_r + (((size_t)b * T + t) * nb + band) * M;
      const C2<R>* URr = (const C2<R>*)P.UR + (size_t)ei * M;
#pragma unroll
      for (int e = 0; e < RL; ++e) {
        const int n = lane + SWIFTCL_WAVE * e;
        v[e] = cadd(v[e], cconj(cmul(chr[n], URr[n])));
      }
    }
    if ((EXTRA & 2) && in.mag && kind == SWIFTCL_CLUSTERING) {
      // magnification: l(l+1) U at the bias b - 2 shares the density window's k scale
      const C2<R>* chm = (const C2<R>*)P.chat_mu + (((size_t)b * T + t) * nb + band) * M;
      const C2<R>* Umr = (const C2<R>*)P.Umu + (size_t)ei * M;
#pragma unroll
      for (int e = 0; e < RL; ++e) {
        const int n = lane + SWIFTCL_WAVE * e;
        v[e] = cadd(v[e], cconj(cmul(chm[n], Umr[n])));
      }
    }
    int ln = lane;  // opaque copy: keeps the FFT's per-lane LDS addresses out of the tracer loop
    asm volatile("" : "+v"(ln));
    ln &= SWIFTCL_WAVE - 1;
    wave_c2r<R, M>(v, mine, stw, ln);
    const R* kq = w_only ? (const R*)P.kscale + ((size_t)kind * nb + band) * nk
                         : (const R*)P.kss + (((size_t)b * SWIFTCL_NKINDS + kind) * nb + band) * nk;  // kscale sqrt(s)
    constexpr int KG = RL < 4 ? RL : 4;  // loads issued in groups (index clamped into the row, nk even)
#pragma unroll
    for (int e0 = 0; e0 < RL; e0 += KG) {
    C2<R> kk[KG];
#pragma unroll
    for (int e = 0; e < KG; ++e) kk[e] = *(const C2<R>*)(kq + min(2 * (ln + SWIFTCL_WAVE * (e0 + e)), nk - 2));
#pragma unroll
    for (int e = 0; e < KG; ++e) {
      const int k0 = 2 * (ln + SWIFTCL_WAVE * (e0 + e));
      if (k0 < nk) {
        const float x0 = kk[e].x * v[e0 + e].x, x1 = kk[e].y * v[e0 + e].y;
        if (SPLIT) {
          unsigned short h0, l0, h1, l1;
          split_bf16(x0, &h0, &l0);
          split_bf16(x1, &h1, &l1);
          *(unsigned int*)(vh + rb + k0) = (unsigned int)h0 | ((unsigned int)h1 << 16);
          *(unsigned int*)(vh + lo_off + rb + k0) = (unsigned int)l0 | ((unsigned int)l1 << 16);
        } else {
          *(C2<R>*)(vf + rb + k0) = mk<R>(x0, x1);
        }
      }
    }
    }
  }
}

// C of one (point, multipole) from the workspace: 4 wavefronts split k; tile pairs (0,0), (0,1),
// (1,1) of the 32 x 32 Gram matrix.
template <bool SPLIT>
__global__ __launch_bounds__(256) void k_contract(plan_dev P, swiftcl_inputs in, float* __restrict__ Cout, int b0,
                                                  int nbp) {
  // [wave][tile][col][row] partial Gram tiles: lane (p, r) stores its accumulator (rows 4p..4p+3 of
  // column r) as one 16-byte LDS store
  __shared__ __align__(16) float red[4][3][256];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / SWIFTCL_WAVE), lane = threadIdx.x % SWIFTCL_WAVE;
  const int T = P.max_tracers, Lm = P.max_ell, nk = P.n_k;
  const int bl = blockIdx.x / Lm, li = blockIdx.x % Lm;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  const int Tb = clampi(in.n_tracers[b], 0, T);
  const int Lb = clampi(in.n_ell[b], 0, Lm);
  const int npair = T * (T + 1) / 2;
  float* c = Cout + ((size_t)b * Lm + li) * npair;
  if (li >= Lb) {
    for (int i = threadIdx.x; i < npair; i += 256) c[i] = 0.f;
    return;
  }
  const size_t row0 = ((size_t)bl * Lm + li) * 32;
  const size_t lo_off = (size_t)P.vchunk * Lm * 32 * nk;
  v4f a00 = {0, 0, 0, 0}, a01 = {0, 0, 0, 0}, a11 = {0, 0, 0, 0};
  const int r = lane & 15, q = lane / 16;
  // the k loop, instantiated for one or two 16-row tracer tiles so that no branch separates the MFMAs
  auto kloop = [&](auto two_c) {
    constexpr bool TWO = decltype(two_c)::value;
    if constexpr (SPLIT) {
      // 16x16x32 bf16: lane (r, q) feeds k = 32 s + 8 q .. + 7 of row r, split into hi + lo; 8
      // consecutive k of a row are one 16-byte load when nk is a multiple of 8
      const unsigned short* vh = (const unsigned short*)P.vbuf;
      const int nsteps = (nk + 31) / 32;
      const bool vec = (nk & 7) == 0;
      auto load8 = [&](size_t at, int k0) {
        v8us x;
        if (vec && k0 + 8 <= nk) {
          x = *(const v8us*)(vh + at);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = k0 + e < nk ? vh[at + e] : (unsigned short)0;
        }
        return x;
      };
      for (int s = wave; s < nsteps; s += 4) {
        const int k0 = 32 * s + 8 * q;
        const v8us h0 = load8((row0 + r) * nk + k0, k0);
        const v8us l0 = load8(lo_off + (row0 + r) * nk + k0, k0);
        a00 = mfma_bf16(h0, h0, a00);
        a00 = mfma_bf16(h0, l0, a00);
        a00 = mfma_bf16(l0, h0, a00);
        if constexpr (TWO) {
          const v8us h1 = load8((row0 + 16 + r) * nk + k0, k0);
          const v8us l1 = load8(lo_off + (row0 + 16 + r) * nk + k0, k0);
          a01 = mfma_bf16(h0, h1, a01);
          a01 = mfma_bf16(h0, l1, a01);
          a01 = mfma_bf16(l0, h1, a01);
          a11 = mfma_bf16(h1, h1, a11);
          a11 = mfma_bf16(h1, l1, a11);
          a11 = mfma_bf16(l1, h1, a11);
        }
      }
    } else {
      // 16x16x4 f32 with V as both operands, so the order in which the k nodes enter the sum is
      // free: lane (r, q) feeds k = 16 s + 4 q + j at step j of block s, four consecutive floats
      // of its row per load
      const float* vf = (const float*)P.vbuf;
      const int nblk = (nk + 15) / 16;
      const bool vec = (nk & 3) == 0;
      auto load4 = [&](size_t at, int k0) {
        float4 x;
        if (vec && k0 + 4 <= nk) {
          x = *(const float4*)(vf + at);
        } else {
          x.x = k0 < nk ? vf[at] : 0.f;
          x.y = k0 + 1 < nk ? vf[at + 1] : 0.f;
          x.z = k0 + 2 < nk ? vf[at + 2] : 0.f;
          x.w = k0 + 3 < nk ? vf[at + 3] : 0.f;
        }
        return x;
      };
      for (int s = wave; s < nblk; s += 4) {
        const int k0 = 16 * s + 4 * q;
        const float4 x0 = load4((row0 + r) * nk + k0, k0);
        const float a0[4] = {x0.x, x0.y, x0.z, x0.w};
        if constexpr (TWO) {
          const float4 x1 = load4((row0 + 16 + r) * nk + k0, k0);
          const float a1[4] = {x1.x, x1.y, x1.z, x1.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            a00 = mfma_acc<float>::step(a0[j], a0[j], a00);
            a01 = mfma_acc<float>::step(a0[j], a1[j], a01);
            a11 = mfma_acc<float>::step(a1[j], a1[j], a11);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) a00 = mfma_acc<float>::step(a0[j], a0[j], a00);
        }
      }
    }
  };
  const bool two = Tb > 16;
  if (two) kloop(std::true_type{});
  else kloop(std::false_type{});
  // rows 4q..4q+3 of column r: red[wave][tile][16 r + 4 q + 0..3]
  *(v4f*)&red[wave][0][16 * r + 4 * q] = a00;
  *(v4f*)&red[wave][1][16 * r + 4 * q] = a01;
  *(v4f*)&red[wave][2][16 * r + 4 * q] = a11;
  __syncthreads();
  for (int idx = threadIdx.x; idx < npair; idx += 256) {
    int i = 0, rem = idx;
    while (rem >= T - i) { rem -= T - i; ++i; }
    const int j = i + rem;
    float val = 0.f;
    if (i < Tb && j < Tb) {
      const int tile = (i < 16) ? (j < 16 ? 0 : 1) : 2;
      const int e = (j % 16) * 16 + (i % 16);  // row i, column j of the tile
#pragma unroll
      for (int w = 0; w < 4; ++w) val += red[w][tile][e];
    }
    c[idx] = val;
  }
}

hipError_t launch_contract(const plan_dev& p, const swiftcl_inputs* in, void* C, int b0, int nbp, hipStream_t s) {
  const dim3 g2((unsigned)((size_t)nbp * p.max_ell));
  if (p.precision == SWIFTCL_SPLIT_BF16) hipLaunchKernelGGL(k_contract<true>, g2, dim3(256), 0, s, p, *in, (float*)C, b0, nbp);
  else hipLaunchKernelGGL(k_contract<false>, g2, dim3(256), 0, s, p, *in, (float*)C, b0, nbp);
  return hipGetLastError();
}

hipError_t launch_sqrt_s(const plan_dev& p, const swiftcl_inputs* in, hipStream_t s) {
  if (p.precision == SWIFTCL_FP64)
    hipLaunchKernelGGL(k_sqrt_s<double>, dim3((p.n_k + 255) / 256, in->batch), dim3(256), 0, s, p, *in);
  else
    hipLaunchKernelGGL(k_sqrt_s<float>, dim3((p.n_k + 255) / 256, in->batch), dim3(256), 0, s, p, *in);
  return hipGetLastError();
}

template <int M>
static hipError_t launch_unfused(const plan_dev& p, const swiftcl_inputs* in, void* C, hipStream_t s) {
  constexpr int NW = 16;
  constexpr bool TW = unfused_tw(M);
  const bool split = p.precision == SWIFTCL_SPLIT_BF16;
  const size_t lds = windows_cl_lds(M, NW, TW, false, sizeof(float), p.n_k);
  for (int b0 = 0; b0 < in->batch; b0 += p.vchunk) {
    const int nbp = in->batch - b0 < p.vchunk ? in->batch - b0 : p.vchunk;
    const size_t groups = (size_t)(nbp + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD;
    const dim3 g1((unsigned)(groups * p.max_ell * SWIFTCL_NXCD));
#define SWIFTCL_WV(SP, EX) hipLaunchKernelGGL((k_windows_v<M, NW, TW, SP, EX>), g1, dim3(NW * 64), lds, s, p, *in, b0, nbp, 0)
    switch ((p.rsd ? 1 : 0) | (p.mag ? 2 : 0)) {
      case 0: if (split) SWIFTCL_WV(true, 0); else SWIFTCL_WV(false, 0); break;
      case 1: if (split) SWIFTCL_WV(true, 1); else SWIFTCL_WV(false, 1); break;
      case 2: if (split) SWIFTCL_WV(true, 2); else SWIFTCL_WV(false, 2); break;
      default: if (split) SWIFTCL_WV(true, 3); else SWIFTCL_WV(false, 3); break;
    }
#undef SWIFTCL_WV
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2((unsigned)((size_t)nbp * p.max_ell));
    if (split) hipLaunchKernelGGL(k_contract<true>, g2, dim3(256), 0, s, p, *in, (float*)C, b0, nbp);
    else hipLaunchKernelGGL(k_contract<false>, g2, dim3(256), 0, s, p, *in, (float*)C, b0, nbp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int M>
static hipError_t launch_ww_t(const plan_dev& p, const swiftcl_inputs* in, int b0, int nbp, hipStream_t s) {
  constexpr int NW = 16;
  constexpr bool TW = unfused_tw(M);
  const size_t lds = windows_cl_lds(M, NW, TW, false, sizeof(float), p.n_k);
  const size_t groups = (size_t)(nbp + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD;
  const dim3 g1((unsigned)(groups * p.max_ell * SWIFTCL_NXCD));
  // the recomputed W carries the RSD and magnification terms of plans built with them
  switch ((p.rsd ? 1 : 0) | (p.mag ? 2 : 0)) {
    case 0: hipLaunchKernelGGL((k_windows_v<M, NW, TW, false, 0>), g1, dim3(NW * 64), lds, s, p, *in, b0, nbp, 1); break;
    case 1: hipLaunchKernelGGL((k_windows_v<M, NW, TW, false, 1>), g1, dim3(NW * 64), lds, s, p, *in, b0, nbp, 1); break;
    case 2: hipLaunchKernelGGL((k_windows_v<M, NW, TW, false, 2>), g1, dim3(NW * 64), lds, s, p, *in, b0, nbp, 1); break;
    default: hipLaunchKernelGGL((k_windows_v<M, NW, TW, false, 3>), g1, dim3(NW * 64), lds, s, p, *in, b0, nbp, 1); break;
  }
  return hipGetLastError();
}

hipError_t launch_windows_w(const plan_dev& p, const swiftcl_inputs* in, int b0, int nbp, hipStream_t s) {
  switch (p.M) {
    case 128: return launch_ww_t<128>(p, in, b0, nbp, s);
    case 256: return launch_ww_t<256>(p, in, b0, nbp, s);
    case 512: return launch_ww_t<512>(p, in, b0, nbp, s);
    case 1024: return launch_ww_t<1024>(p, in, b0, nbp, s);
  }
  return hipErrorInvalidValue;
}

template <typename R, int M, bool WRITE_W, bool DO_CL>
static hipError_t launch_wcl_t(const plan_dev& p, const swiftcl_inputs* in, void* W, void* C, hipStream_t s) {
  constexpr int NW = wcl_shape<R, M>::NW;
  constexpr bool TW = wcl_shape<R, M>::TW;
  const size_t lds = (sizeof(R) == 4 && DO_CL)
                         ? (TW ? 2 * (size_t)M * sizeof(C2<R>) : 0) + (size_t)16 * compact_vs_fwd(p.n_k, M) * sizeof(R)
                         : windows_cl_lds(M, NW, TW, DO_CL, sizeof(R), p.n_k);
  const bool split = p.precision == SWIFTCL_SPLIT_BF16;
  if (DO_CL && !WRITE_W && p.fwd_mode >= 1) {
    // (the packed builder stages up to SCHED_PACK_MAXNX points per XCD; larger batches run mode 1)
    const bool packed = p.fwd_mode == 2 && in->batch <= SCHED_PACK_MAXNX * SWIFTCL_NXCD;
    if (packed) hipLaunchKernelGGL(k_schedule_packed, dim3(SWIFTCL_NXCD), dim3(64), 0, s, p, *in);
    else hipLaunchKernelGGL(k_schedule, dim3(1), dim3(64), 0, s, p, *in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_padded<R>, dim3(p.max_ell, in->batch), dim3(128), 0, s, p, *in, (R*)C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the FP32 projection runs two workgroups per CU
    const dim3 pgrid((unsigned)(p.persist_blocks * ((sizeof(R) == 4 && M <= 512) ? 2 : 1)));
    if (packed) {
      if constexpr (sizeof(R) == 4) {
        if (split) {
          hipLaunchKernelGGL((k_windows_cl<R, M, NW, TW, false, true, 2, true>), pgrid, dim3(NW * 64), lds, s, p,
                             *in, (R*)W, (R*)C);
          return hipGetLastError();
        }
      }
      hipLaunchKernelGGL((k_windows_cl<R, M, NW, TW, false, true, 2, false>), pgrid, dim3(NW * 64), lds, s, p, *in,
                         (R*)W, (R*)C);
      return hipGetLastError();
    }
    if constexpr (sizeof(R) == 4) {
      if (split) {
        hipLaunchKernelGGL((k_windows_cl<R, M, NW, TW, false, true, 1, true>), pgrid, dim3(NW * 64), lds, s, p,
                           *in, (R*)W, (R*)C);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_windows_cl<R, M, NW, TW, false, true, 1, false>), pgrid, dim3(NW * 64), lds, s, p, *in,
                       (R*)W, (R*)C);
    return hipGetLastError();
  }
  const size_t groups = (size_t)(in->batch + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD;
  const dim3 grid((unsigned)(groups * p.max_ell * SWIFTCL_NXCD));
  if constexpr (sizeof(R) == 4 && DO_CL) {
    if (split) {
      hipLaunchKernelGGL((k_windows_cl<R, M, NW, TW, WRITE_W, DO_CL, 0, true>), grid, dim3(NW * 64), lds, s, p,
                         *in, (R*)W, (R*)C);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_windows_cl<R, M, NW, TW, WRITE_W, DO_CL, 0, false>), grid, dim3(NW * 64), lds, s, p, *in,
                     (R*)W, (R*)C);
  return hipGetLastError();
}

template <typename R, int M>
static hipError_t launch_wcl_m(const plan_dev& p, const swiftcl_inputs* in, void* W, void* C, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (W) e = launch_wcl_t<R, M, true, false>(p, in, W, nullptr, s);
  if (e == hipSuccess && C) {
    if (p.fused) e = launch_wcl_t<R, M, false, true>(p, in, nullptr, C, s);
    else if constexpr (sizeof(R) == 4) e = launch_unfused<M>(p, in, C, s);
    else e = hipErrorNotSupported;
  }
  return e;
}

hipError_t launch_windows_cl(const plan_dev& p, const swiftcl_inputs* in, void* W, void* C, hipStream_t s) {
  const bool dp = p.precision == SWIFTCL_FP64;
  switch (p.M) {
    case 128: return dp ? launch_wcl_m<double, 128>(p, in, W, C, s) : launch_wcl_m<float, 128>(p, in, W, C, s);
    case 256: return dp ? launch_wcl_m<double, 256>(p, in, W, C, s) : launch_wcl_m<float, 256>(p, in, W, C, s);
    case 512: return dp ? launch_wcl_m<double, 512>(p, in, W, C, s) : launch_wcl_m<float, 512>(p, in, W, C, s);
    case 1024: return dp ? launch_wcl_m<double, 1024>(p, in, W, C, s) : launch_wcl_m<float, 1024>(p, in, W, C, s);
  }
  return hipErrorInvalidValue;
}

