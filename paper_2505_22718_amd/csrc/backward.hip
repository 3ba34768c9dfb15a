// Hand-written adjoint of the hot path: dL/dP(k), dL/db, dL/dn(z samples), dL/dD(z samples) for
// L = sum_{b,l} sum_{i<=j} dC^{ij} C^{ij}.  Windows are recomputed, never stored.
//
// With G the symmetrised cotangent (G_ii = dC^{ii}, G_ij = G_ji = dC^{ij}/2) and
// C = W diag(s) W^T, s = (2/pi) w k^3 P:
//   Y = G W,   dP_k = sum_l (2/pi) w_k k_k^3 sum_t W_tk Y_tk,   dW = 2 s Y                (a5)
//   W = c(l) k^{-1-b} x, x = c2r(conj(c U)) -> dc_n = sum_l h_n conj(r2c(dx)_n) conj(U_l(n))  (a6)
//      (the real prefactor c(l) is folded into the U table, so dx carries 2 s k^{-1-b} Y only)
//      (h_0 = 1, h_n = 2: the Hermitian half counts every n > 0 twice)
//   c_n = alpha_n r2c(g)_n, alpha_n = (k_0 chi_0)^{-i eta_n} chi_0^{-b} / N
//      -> dg_m = Re sum_{n<N/2} conj(alpha_n) dc_n e^{+2 pi i n m / N}
//   g_band = w f e^{-b m Delta} -> df = sum_band w e^{-b m Delta} dg_band, then the chain through
//   the kernels (bias, n(z) spline, lensing integrals, D(z) spline) in FP64                 (a7)
#include "common.h"
#include "geometry.h"
#include "internal.h"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename R> struct bmfma;
template <> struct bmfma<float> {
  typedef v4f type;
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane / 16) + r; }
  static __device__ __forceinline__ type step(float a, float b, type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct bmfma<double> {
  typedef v4d type;
  static __device__ __forceinline__ int row(int lane, int r) { return lane / 16 + 4 * r; }
  static __device__ __forceinline__ type step(double a, double b, type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ int clampb(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// number of multipole chunks per point: about 256 x bwd_chunk_mul workgroups (one 1024-thread
// workgroup fills a CU; uniform batches run best with one round, ragged ones with more, smaller
// chunks dispatched heaviest first)
int backward_chunks(const plan_dev& p, int batch) {
  const int mul = p.bwd_chunk_mul > 0 ? p.bwd_chunk_mul : 1;
  int c = (256 * mul + batch - 1) / batch;
  if (c > p.max_ell) c = p.max_ell;
  return c < 1 ? 1 : c;
}

// Work items of the fused adjoint: item j = (rest = j / 8, XCD j % 8) is point
// b = (rest / nchunk) * 8 + j % 8 and multipole chunk rest % nchunk (the chunks of a point share an
// XCD's L2).  With ragged tracer and multipole counts their costs differ several-fold, and one
// 1024-thread workgroup fills a CU, so the workgroups are dispatched heaviest first (longest
// processing time first keeps the last CUs from idling): k_bwd_order writes order[w] = the item of
// workgroup w, a stable counting sort on a cost bucket of T_b x (multipoles of the chunk), so
// that uniform batches keep the natural order.  Buckets: lane l of each wavefront counts bucket l
// over its segment of items; 63 cost levels, highest first, and a last bucket for items past the
// batch.
constexpr int BWD_ORDER_MAX = 32768;  // items sorted in LDS (one byte each); larger grids run unsorted

__global__ __launch_bounds__(1024) void k_bwd_order(plan_dev P, swiftcl_inputs in, int nchunk, int n) {
  __shared__ unsigned int bk4[BWD_ORDER_MAX / 4];  // four item buckets per word; 255 pads the tail
  __shared__ int cnt[16][64];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int T = P.max_tracers, Lm = P.max_ell, n4 = (n + 3) / 4;
  const int maxcost = T * ((Lm + nchunk - 1) / nchunk);
  for (int w = tid; w < n4; w += 1024) {
    unsigned int word = 0;
    for (int q = 0; q < 4; ++q) {
      const int j = 4 * w + q;
      int key = 255;
      if (j < n) {
        const int rest = j / SWIFTCL_NXCD, chunk = rest % nchunk;
        const int b = (rest / nchunk) * SWIFTCL_NXCD + j % SWIFTCL_NXCD;
        key = 63;
        if (b < in.batch) {
          const int Tb = clampb(in.n_tracers[b], 0, T), Lb = clampb(in.n_ell[b], 0, Lm);
          const int cost = Tb * ((chunk + 1) * Lb / nchunk - chunk * Lb / nchunk);
          key = 62 - (maxcost > 0 ? cost * 62 / maxcost : 0);
        }
      }
      word |= (unsigned int)key << (8 * q);
    }
    bk4[w] = word;
  }
  __syncthreads();
  // wave w scans words [w0, w1); lane l counts (then places) the items of bucket l
  const int seg = (n4 + 15) / 16, w0 = wave * seg, w1 = min(n4, w0 + seg);
  int c = 0;
  for (int w = w0; w < w1; ++w) {
    const unsigned int u = bk4[w];
    c += ((u & 255u) == (unsigned)lane) + (((u >> 8) & 255u) == (unsigned)lane) +
         (((u >> 16) & 255u) == (unsigned)lane) + ((u >> 24) == (unsigned)lane);
  }
  cnt[wave][lane] = c;
  __syncthreads();
  if (wave == 0) {
    // first position of (bucket lane, segment w): the earlier buckets, then earlier segments
    int tot = 0;
    for (int w = 0; w < 16; ++w) tot += cnt[w][lane];
    int incl = tot;  // inclusive prefix over the buckets up to this lane
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    int at = incl - tot;
    for (int w = 0; w < 16; ++w) {
      const int k = cnt[w][lane];
      cnt[w][lane] = at;
      at += k;
    }
  }
  __syncthreads();
  int pos = cnt[wave][lane];
  for (int w = w0; w < w1; ++w) {
    const unsigned int u = bk4[w];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (((u >> (8 * q)) & 255u) == (unsigned)lane) P.bwd_order[pos++] = 4 * w + q;
  }
}

// (a5, a6) One workgroup per (point, chunk of multipole slots), NW wavefronts, wave t = tracer t.
// Per multipole: recompute W (forward FFT), Y = G W on MFMA, dP partial, dx, r2c, accumulate dc.
// Partial dc per (point, chunk, tracer, band) and partial sum_t W Y per (point, chunk, k) go to
// the workspace; k_bwd_coeffs and k_bwd_point reduce them.
// LDS: twiddles, then (FP32, COMPACT) WY[16][compact_vs] whose row t is also the FFT scratch of
// wavefront t and the workgroup's dP partial dps[n_k] (~77 KiB for n_chi = n_k = 1024); or (FP64)
// per-wave scratch [NW][FL] and WY[16][n_k + 2].  The dc accumulators held in registers across the
// multipole loop need ~126 VGPRs, so one 1024-thread workgroup runs per CU (forcing two costs more
// in spills than the occupancy gains).
// PACK (FP32, one wavefront per tracer slot): the chunk's slots form two sub-chunks [l0, lm) and
// [lm, l1) with partial rows of their own (the reduction then sums 2 nchunk rows per point).  A
// point of at most 8 tracers runs the two side by side, waves 0-7 on the first and waves 8-15 on
// the second: rows 0-7 of the W tile hold the tracers of the first sub-chunk's multipole, rows
// 8-15 those of the second's, and G is block-diagonal, so one Y = G W product serves both and all
// 16 wavefronts transform.  Any other point runs the two sub-chunks one after the other.
template <typename R, int M, int NW, bool TW_LDS, bool PACK = false>
__global__ __launch_bounds__(NW * 64) void k_bwd_windows(plan_dev P, swiftcl_inputs in, const R* __restrict__ dC,
                                                         int nchunk, int ordered) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool COMPACT = sizeof(R) == 4 && NW == 16;
  static_assert(!PACK || COMPACT, "sub-chunk packing needs one wavefront per tracer slot");
  constexpr int RL = M / SWIFTCL_WAVE;
  constexpr int N = 2 * M;
  constexpr int FL = fft_lds_size(M, sizeof(R));
  constexpr int NTW = TW_LDS ? N : 0;
  const int T = P.max_tracers, Lm = P.max_ell, nk = P.n_k, nb = P.n_bands;
  const int vs = COMPACT ? compact_vs(nk, M) : nk + 2;
  C2<R>* stw_l = (C2<R>*)smem;
  C2<R>* fbuf = stw_l + NTW;                                                              // [NW][FL]
  R* WY = (R*)(smem + ((size_t)NTW + (COMPACT ? 0 : (size_t)NW * FL)) * sizeof(C2<R>));  // [16][vs]
  R* dps = WY + (size_t)16 * vs;                                                          // [nk] (COMPACT)
  R* kss = dps + nk;                          // [kind][nb][nk] k scale tables (COMPACT)
  R* sq2 = kss + SWIFTCL_NKINDS * nb * nk;     // [nk] 2 s of this point: dW = 2 s Y (COMPACT)
  // G in MFMA operand order: Gp[s][l] = G[l % 16][4 (l / 16) + s] is what lane l feeds at
  // reduction step s (the step covers tracers s, s + 4, s + 8, s + 12, so the W operand reads of
  // 4 rows x 16 k touch distinct banks with the row stride == 4 mod 64)
  __shared__ R Gp[4][64];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / SWIFTCL_WAVE), lane = threadIdx.x % SWIFTCL_WAVE;
  const int item = ordered ? P.bwd_order[blockIdx.x] : (int)blockIdx.x;
  const int xcd = item % SWIFTCL_NXCD;
  const int rest = item / SWIFTCL_NXCD;
  const int chunk = rest % nchunk;
  const int b = (rest / nchunk) * SWIFTCL_NXCD + xcd;
  if (b >= in.batch) return;
  const int Tb = clampb(in.n_tracers[b], 0, T);
  const int Lb = clampb(in.n_ell[b], 0, Lm);
  const int l0 = (int)(((long)chunk * Lb) / nchunk), l1 = (int)(((long)(chunk + 1) * Lb) / nchunk);
  const int npair = T * (T + 1) / 2;
  // PACK: the sub-chunk split; this wavefront's half, tracer and slots
  const int lm = PACK ? l0 + (l1 - l0) / 2 : l1;
  const bool pk = PACK && Tb <= 8;
  const int hh = pk ? wave >> 3 : 0;
  const int tt = pk ? (wave & 7) : wave;
  const int ml0 = (pk && hh) ? lm : l0, ml1 = (pk && !hh) ? lm : l1;
  const int nsteps = pk ? (lm - l0 > l1 - lm ? lm - l0 : l1 - lm) : l1 - l0;
  const C2<R>* stw = TW_LDS ? stw_l : (const C2<R>*)P.tw;
  if constexpr (TW_LDS) {
    const C2<R>* gtw = (const C2<R>*)P.tw;
    for (int i = threadIdx.x; i < N; i += NW * 64) stw_l[i] = gtw[i];
  }
  const size_t slot = (size_t)b * nchunk + chunk;
  C2<R>* part = (C2<R>*)P.dchat_part + slot * (PACK ? 2 : 1) * T * nb * M;
  if (!COMPACT)  // (COMPACT: every (tracer, band) row of the slot is stored once, below)
    for (size_t i = threadIdx.x; i < (size_t)T * nb * M; i += NW * 64) part[i] = mk<R>(0, 0);
  const R* sq = (const R*)P.sqrt_s + (size_t)b * nk;
  if (COMPACT) {
    for (int i = threadIdx.x; i < SWIFTCL_NKINDS * nb * nk; i += NW * 64) kss[i] = ((const R*)P.kscale)[i];
    for (int i = threadIdx.x; i < nk; i += NW * 64) sq2[i] = (R)2 * sq[i] * sq[i];
  }
  const R* kscale = COMPACT ? (const R*)kss : (const R*)P.kscale;
  const int ntiles = (nk + 15) / 16;
  // this workgroup's slice of the dP partials: column k is owned by one lane of one wavefront
  R* dpp = (R*)P.dpk_part + slot * nk;
  for (int k = threadIdx.x; k < nk; k += NW * 64) {
    if (COMPACT) dps[k] = (R)0;
    else dpp[k] = (R)0;
  }
  C2<R> acc[RL];
#pragma unroll
  for (int e = 0; e < RL; ++e) acc[e] = mk<R>(0, 0);
  int cur_band = -1;
  int cur_sub = 0;       // (PACK) sub-chunk of the accumulators
  unsigned flushed = 0;  // bands (PACK: sub-chunk x 4 + band) whose partial rows this wavefront has written
  // add the accumulators of band cur_band to the partial rows (store on the first visit)
  auto flush = [&]() {
    if constexpr (PACK) {
      const int bit = cur_sub * SWIFTCL_MAX_BANDS + cur_band;
      const bool again = (flushed >> bit) & 1u;
      if (tt < Tb) {
        C2<R>* dst = part + (((size_t)cur_sub * T + tt) * nb + cur_band) * M;
#pragma unroll
        for (int e = 0; e < RL; ++e)
          dst[lane + SWIFTCL_WAVE * e] = again ? cadd(dst[lane + SWIFTCL_WAVE * e], acc[e]) : acc[e];
      }
      flushed |= 1u << bit;
    } else {
      const bool again = (flushed >> cur_band) & 1u;
      for (int t = wave; t < Tb; t += NW) {
        C2<R>* dst = part + ((size_t)t * nb + cur_band) * M;
#pragma unroll
        for (int e = 0; e < RL; ++e)
          dst[lane + SWIFTCL_WAVE * e] = again ? cadd(dst[lane + SWIFTCL_WAVE * e], acc[e]) : acc[e];
      }
      flushed |= 1u << cur_band;
    }
  };
  __syncthreads();

  // multipole slot -> (union index, band); a bad index is flagged and read as 0
  auto ell_of = [&](int li, int& ei, int& band) {
    ei = in.ell_idx[(size_t)b * Lm + li];
    if (ei < 0 || ei >= P.n_ell) {
      if (PACK ? lane == 0 : threadIdx.x == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
      ei = 0;
    }
    band = P.ell_band[ei];
  };
  // G of multipole slot li (symmetrised cotangent)
  auto load_G = [&](int li) {
    for (int gi = threadIdx.x; gi < 256; gi += NW * 64) {
      const int i = gi / 16, j = gi % 16;
      R gv = (R)0;
      if (i < Tb && j < Tb) {
        const int a = i < j ? i : j, c = i < j ? j : i;
        const int p = a * T - a * (a - 1) / 2 + (c - a);
        gv = dC[((size_t)b * Lm + li) * npair + p];
        if (i != j) gv *= (R)0.5;
      }
      Gp[j & 3][16 * (j >> 2) + i] = gv;
    }
  };
  // (PACK) G of step s: block-diagonal over the halves of a packed point
  auto load_G_pk = [&](int s) {
    for (int gi = threadIdx.x; gi < 256; gi += NW * 64) {
      const int i = gi / 16, j = gi % 16;
      int li = -1, ii = i, jj = j;
      if (pk) {
        if ((i >> 3) == (j >> 3)) {
          const int a0 = (i >> 3) ? lm : l0, a1 = (i >> 3) ? l1 : lm;
          if (a0 + s < a1) li = a0 + s;
          ii = i & 7;
          jj = j & 7;
        }
      } else {
        li = l0 + s;
      }
      R gv = (R)0;
      if (li >= 0 && ii < Tb && jj < Tb) {
        const int a = ii < jj ? ii : jj, c = ii < jj ? jj : ii;
        const int p = a * T - a * (a - 1) / 2 + (c - a);
        gv = dC[((size_t)b * Lm + li) * npair + p];
        if (ii != jj) gv *= (R)0.5;
      }
      Gp[j & 3][16 * (j >> 2) + i] = gv;
    }
  };
  // (1) W of tracer t of multipole (ei, band) into LDS row `row`
  auto win_row = [&](int row, int t, int ei, int band) {
    {
      const int kind = tracer_kind(in, T, b, t);
      const C2<R>* ch = (const C2<R>*)P.chat + (((size_t)b * T + t) * nb + band) * M;
      const C2<R>* Ur = (const C2<R>*)P.U + ((size_t)kind * P.n_ell + ei) * M;
      C2<R>* mine = COMPACT ? (C2<R>*)(WY + (size_t)row * vs) : fbuf + (size_t)wave * FL;
      C2<R> v[RL];
      wave_sync();
#pragma unroll
      for (int e = 0; e < RL; ++e) {
        const int n = lane + SWIFTCL_WAVE * e;
        v[e] = cconj(cmul(ch[n], Ur[n]));
      }
      int ln = lane;  // opaque copy: keeps the FFT's per-lane LDS addresses out of the multipole loop
      asm volatile("" : "+v"(ln));
      ln &= SWIFTCL_WAVE - 1;  // the compiler may assume 0 <= ln < 64 again
      wave_c2r<R, M>(v, mine, stw, ln);
      wave_sync();
      const R* ks = kscale + ((size_t)kind * nb + band) * nk;  // (F(l) is folded into U)
      auto w_pair = [&](int k0, int e) {
        const C2<R> kk = *(const C2<R>*)(ks + k0);
        *(C2<R>*)(WY + row * vs + k0) = mk<R>(kk.x * v[e].x, kk.y * v[e].y);
      };
      if (2 * M <= nk) {  // every pair inside the row: no guard between the loads
#pragma unroll
        for (int e = 0; e < RL; ++e) w_pair(2 * (lane + SWIFTCL_WAVE * e), e);
      } else {
#pragma unroll
        for (int e = 0; e < RL; ++e) {
          const int k0 = 2 * (lane + SWIFTCL_WAVE * e);
          if (k0 < nk) w_pair(k0, e);
        }
      }
    }
  };
  // (1) W of every tracer of multipole (ei, band) into its LDS row
  auto windows = [&](int ei, int band) {
    for (int t = wave; t < 16; t += NW) {
      if (t >= Tb) {
        for (int j = lane; j < nk; j += SWIFTCL_WAVE) WY[t * vs + j] = (R)0;
        continue;
      }
      win_row(t, t, ei, band);
    }
  };
  // (PACK) this wavefront's row at step s; its slot's multipole and band go to (nei, nband)
  int nei = 0, nband = 0;
  auto windows_pk = [&](int s) {
    const int li = ml0 + s;
    if (li >= ml1 || tt >= Tb) {
      for (int j = lane; j < nk; j += SWIFTCL_WAVE) WY[wave * vs + j] = (R)0;
      return;
    }
    ell_of(li, nei, nband);
    win_row(wave, tt, nei, nband);
  };

  // (2) Y = G W on MFMA, tile by tile of 16 k (each tile owned by one wavefront, in place)
  auto products = [&]() {
    using acc_t = typename bmfma<R>::type;
    for (int tile = wave; tile < ntiles; tile += NW) {
      const int col = tile * 16 + (lane & 15);
      acc_t y = {0, 0, 0, 0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const R a = Gp[s4][lane];
        const R bo = col < nk ? WY[(4 * (lane / 16) + s4) * vs + col] : (R)0;
        y = bmfma<R>::step(a, bo, y);
      }
      R s = (R)0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bmfma<R>::row(lane, r);
        if (col < nk) s += WY[row * vs + col] * y[r];
      }
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      if (lane < 16 && col < nk) {
        if (COMPACT) dps[col] += s;
        else dpp[col] += s;
      }
      wave_sync();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bmfma<R>::row(lane, r);
        if (col < nk) WY[row * vs + col] = y[r];
      }
    }
  };
  // (3) dx = 2 s F k^{-1-b} Y of LDS row `row` (tracer t, multipole (ei, band)), r2c,
  // dc += h_n conj(X_n) conj(U_l(n))
  auto adj_row = [&](int row, int t, int ei, int band) {
    const int kind = tracer_kind(in, T, b, t);
    const R* ks = kscale + ((size_t)kind * nb + band) * nk;
    C2<R>* mine = COMPACT ? (C2<R>*)(WY + (size_t)row * vs) : fbuf + (size_t)wave * FL;
    C2<R> v[RL];
    // 2 s F k^{-1-b} Y per output pair; when every pair lies inside the row (N <= nk) the loads
    // carry no guard, so they are issued together
    auto dx_pair = [&](int k0) {
      const C2<R> y2 = *(const C2<R>*)(WY + row * vs + k0);
      const C2<R> kk = *(const C2<R>*)(ks + k0);
      if constexpr (COMPACT) {
        const C2<R> s2 = *(const C2<R>*)(sq2 + k0);
        return mk<R>(kk.x * s2.x * y2.x, kk.y * s2.y * y2.y);
      } else {
        const C2<R> s2 = *(const C2<R>*)(sq + k0);
        return mk<R>((R)2 * s2.x * s2.x * kk.x * y2.x, (R)2 * s2.y * s2.y * kk.y * y2.y);
      }
    };
    if (2 * M <= nk) {
#pragma unroll
      for (int e = 0; e < RL; ++e) v[e] = dx_pair(2 * (lane + SWIFTCL_WAVE * e));
    } else {
#pragma unroll
      for (int e = 0; e < RL; ++e) {
        const int k0 = 2 * (lane + SWIFTCL_WAVE * e);
        v[e] = k0 < nk ? dx_pair(k0) : mk<R>(0, 0);
      }
    }
    const C2<R>* Ur = (const C2<R>*)P.U + ((size_t)kind * P.n_ell + ei) * M;
    C2<R> ur[NW >= 16 ? RL : 1];
    if constexpr (NW >= 16) {
      // issued before the transform, used after it
#pragma unroll
      for (int e = 0; e < RL; ++e) ur[e] = Ur[lane + SWIFTCL_WAVE * e];
    }
    wave_sync();
    int ln = lane;
    asm volatile("" : "+v"(ln));
    ln &= SWIFTCL_WAVE - 1;  // the compiler may assume 0 <= ln < 64 again
    wave_r2c<R, M>(v, mine, stw, ln);
    if constexpr (NW >= 16) {
      // one tracer per wavefront: accumulate in registers, flushed when the band changes
#pragma unroll
      for (int e = 0; e < RL; ++e) {
        const int n = lane + SWIFTCL_WAVE * e;
        const R h = n == 0 ? (R)1 : (R)2;
        acc[e] = cadd(acc[e], cscale(cmul(cconj(v[e]), cconj(ur[e])), h));
      }
    } else {
      // a wavefront serves several tracers: add into this workgroup's partial slot directly
      C2<R>* dst = part + ((size_t)t * nb + band) * M;
#pragma unroll
      for (int e = 0; e < RL; ++e) {
        const int n = lane + SWIFTCL_WAVE * e;
        const R h = n == 0 ? (R)1 : (R)2;
        dst[n] = cadd(dst[n], cscale(cmul(cconj(v[e]), cconj(Ur[n])), h));
      }
    }
  };

  if constexpr (PACK) {
    // the same pipeline over the steps of the two sub-chunks; each wavefront keeps its own band,
    // sub-chunk and accumulators
    if (nsteps > 0) {
      load_G_pk(0);
      windows_pk(0);
    }
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
      products();
      __syncthreads();
      const int li = ml0 + s;
      if (li < ml1 && tt < Tb) {
        const int ei = nei, band = nband;  // set by windows_pk(s)
        const int sub = pk ? hh : (li >= lm ? 1 : 0);
        if (band != cur_band || sub != cur_sub) {
          if (cur_band >= 0) flush();
#pragma unroll
          for (int e = 0; e < RL; ++e) acc[e] = mk<R>(0, 0);
          cur_band = band;
          cur_sub = sub;
        }
        adj_row(wave, tt, ei, band);
      }
      if (s + 1 < nsteps) {
        load_G_pk(s + 1);
        windows_pk(s + 1);
      }
      __syncthreads();
    }
    if (cur_band >= 0) flush();
    // (sub-chunk, band) rows this wavefront never wrote: zeros (the reduction sums every row)
    if (tt < Tb) {
      for (int sb = 0; sb < 2; ++sb) {
        if (pk && sb != hh) continue;
        for (int bi = 0; bi < nb; ++bi) {
          if ((flushed >> (sb * SWIFTCL_MAX_BANDS + bi)) & 1u) continue;
          C2<R>* dst = part + (((size_t)sb * T + tt) * nb + bi) * M;
#pragma unroll
          for (int e = 0; e < RL; ++e) dst[lane + SWIFTCL_WAVE * e] = mk<R>(0, 0);
        }
      }
    }
  } else {
    // Software pipeline over the multipoles of this chunk, two barriers per multipole: the adjoint
    // transforms of slot li share a barrier interval with the windows of slot li + 1 (each wavefront
    // only touches its own LDS rows there).
    int ei = 0, band = 0;
    if (l0 < l1) {
      ell_of(l0, ei, band);
      load_G(l0);
      windows(ei, band);
    }
    __syncthreads();
    for (int li = l0; li < l1; ++li) {
      products();
      __syncthreads();
      if (NW >= 16 && band != cur_band) {
        if (cur_band >= 0) flush();
#pragma unroll
        for (int e = 0; e < RL; ++e) acc[e] = mk<R>(0, 0);
        cur_band = band;
      }
      // (3) the adjoint transforms
      for (int t = wave; t < Tb; t += NW) adj_row(t, t, ei, band);
      // (1) for the next slot
      if (li + 1 < l1) {
        ell_of(li + 1, ei, band);
        load_G(li + 1);
        windows(ei, band);
      }
      __syncthreads();
    }
    if (NW >= 16) {
      if (cur_band >= 0) flush();
      // bands this chunk never reached: zero rows (the reduction sums every chunk's row)
      for (int bi = 0; bi < nb; ++bi) {
        if ((flushed >> bi) & 1u) continue;
        for (int t = wave; t < Tb; t += NW) {
          C2<R>* dst = part + ((size_t)t * nb + bi) * M;
#pragma unroll
          for (int e = 0; e < RL; ++e) dst[lane + SWIFTCL_WAVE * e] = mk<R>(0, 0);
        }
      }
    }
  }
  if (COMPACT)
    for (int k = threadIdx.x; k < nk; k += NW * 64) dpp[k] = dps[k];  // the loop ended on a barrier
}

// ---------------------------------------------------------------------------------------------
// Adjoint through the workspace (more than 16 tracers, windows too large for LDS, split plans
// whose fused adjoint does not fit): for a chunk of points the FP32 rows W of every (point,
// multipole, tracer slot) are recomputed into the workspace (k_windows_v, w_only), k_bwd_gv
// replaces them by Y = G W and sums W Y into the dP partials, and k_bwd_adj runs the adjoint
// transforms of each tracer over a chunk of multipoles.  The partial rows have the layout of the
// fused kernel's with nchunk = bwd_nlc, so k_bwd_coeffs, k_bwd_tracer and k_bwd_point follow
// unchanged.
// ---------------------------------------------------------------------------------------------

// (a5) Y = G W on MFMA 16x16x4 for one (point, multipole chunk, 64-wide k tile); wave w owns
// the columns 64 tile + 16 w + (0..15) of every multipole's 32 workspace rows.  G (symmetrised
// cotangent, 32 x 32 with zeros past the point's tracers) is staged in LDS, double-buffered, the
// next multipole's entries loaded during this one's products.  Y overwrites W in place: each lane
// stores only after the MFMAs (which consumed every W read of the wave) and after its own reads
// of the same addresses.  TWO: a second 16-row tracer tile (more than 16 tracers).
template <bool TWO>
__global__ __launch_bounds__(256) void k_bwd_gv(plan_dev P, swiftcl_inputs in, const float* __restrict__ dC,
                                                 int b0, int nbp, int nlc) {
  __shared__ float Gs[2][32][33];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / SWIFTCL_WAVE), lane = tid % SWIFTCL_WAVE;
  const int T = P.max_tracers, Lm = P.max_ell, nk = P.n_k;
  const int ntile = (nk + 63) / 64;
  const int tile = blockIdx.x % ntile;
  const int rest = blockIdx.x / ntile;
  const int c = rest % nlc;
  const int bl = rest / nlc;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  const int Tb = clampb(in.n_tracers[b], 0, T);
  const int Lb = clampb(in.n_ell[b], 0, Lm);
  const int l0 = (int)(((long)c * Lb) / nlc), l1 = (int)(((long)(c + 1) * Lb) / nlc);
  const int npair = T * (T + 1) / 2;
  const int q = lane >> 4, r = lane & 15;
  const int col = 64 * tile + 16 * wave + r;
  const bool cok = col < nk;
  // entry e = tid + 256 m of the 32 x 32 G of multipole slot li
  auto gval = [&](int li, int e) -> float {
    const int i = e >> 5, j = e & 31;
    if (i >= Tb || j >= Tb) return 0.f;
    const int a = i < j ? i : j, cc = i < j ? j : i;
    const float g = dC[((size_t)b * Lm + li) * npair + (a * T - a * (a - 1) / 2 + (cc - a))];
    return i == j ? g : 0.5f * g;
  };
  float gn[4] = {0.f, 0.f, 0.f, 0.f};
  if (l0 < l1)
#pragma unroll
    for (int m = 0; m < 4; ++m) gn[m] = gval(l0, tid + 256 * m);
  float dp = 0.f;  // sum over the chunk of sum_t W Y at column col, over this lane's rows
  for (int li = l0; li < l1; ++li) {
    const int buf = (li - l0) & 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = tid + 256 * m;
      Gs[buf][e >> 5][e & 31] = gn[m];
    }
    __syncthreads();  // (the other buffer was last read before the previous iteration's barrier)
    if (li + 1 < l1)
#pragma unroll
      for (int m = 0; m < 4; ++m) gn[m] = gval(li + 1, tid + 256 * m);
    float* w = (float*)P.vbuf + ((size_t)bl * Lm + li) * 32 * nk;
    v4f y0 = {0.f, 0.f, 0.f, 0.f}, y1 = {0.f, 0.f, 0.f, 0.f};
    constexpr int NJ = TWO ? 8 : 4;  // steps of 4 tracer rows j
#pragma unroll
    for (int st = 0; st < NJ; ++st) {
      const float bv = cok ? w[(size_t)(4 * st + q) * nk + col] : 0.f;  // B: W[4 st + q][col]
      y0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Gs[buf][r][4 * st + q], bv, y0, 0, 0, 0);
      if constexpr (TWO) y1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Gs[buf][16 + r][4 * st + q], bv, y1, 0, 0, 0);
    }
    // y0[m] = Y[4 q + m][col], y1[m] = Y[16 + 4 q + m][col]
    if (cok) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        float* a0 = w + (size_t)(4 * q + m) * nk + col;
        dp += *a0 * y0[m];
        *a0 = y0[m];
        if constexpr (TWO) {
          float* a1 = w + (size_t)(16 + 4 * q + m) * nk + col;
          dp += *a1 * y1[m];
          *a1 = y1[m];
        }
      }
    }
  }
  dp += __shfl_xor(dp, 16);
  dp += __shfl_xor(dp, 32);
  if (q == 0 && cok) ((float*)P.dpk_part)[((size_t)b * nlc + c) * nk + col] = dp;
}

// k_bwd_gv with 16-byte accesses (n_k a multiple of 4): one workgroup per (point, multipole chunk,
// 256-wide k tile); lane (r, q) of wave w owns the columns 256 tile + 64 w + 4 r + (0..3) and reads
// 4 consecutive W values of a row per load.  Column j of the four is the B operand of MFMA tile j,
// so tile j holds the columns {4 r + j}, and every lane stores its 4 columns of a Y row as one
// 16-byte store.  Same in-place order as k_bwd_gv.
template <bool TWO>
__global__ __launch_bounds__(256) void k_bwd_gv4(plan_dev P, swiftcl_inputs in, const float* __restrict__ dC,
                                                  int b0, int nbp, int nlc) {
  __shared__ float Gs[2][32][33];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / SWIFTCL_WAVE), lane = tid % SWIFTCL_WAVE;
  const int T = P.max_tracers, Lm = P.max_ell, nk = P.n_k;
  const int ntile = (nk + 255) / 256;
  const int tile = blockIdx.x % ntile;
  const int rest = blockIdx.x / ntile;
  const int c = rest % nlc;
  const int bl = rest / nlc;
  if (bl >= nbp) return;
  const int b = b0 + bl;
  const int Tb = clampb(in.n_tracers[b], 0, T);
  const int Lb = clampb(in.n_ell[b], 0, Lm);
  const int l0 = (int)(((long)c * Lb) / nlc), l1 = (int)(((long)(c + 1) * Lb) / nlc);
  const int npair = T * (T + 1) / 2;
  const int q = lane >> 4, r = lane & 15;
  const int col = 256 * tile + 64 * wave + 4 * r;  // first of this lane's 4 columns
  const bool cok = col < nk;                       // (nk % 4 == 0: all four or none)
  auto gval = [&](int li, int e) -> float {
    const int i = e >> 5, j = e & 31;
    if (i >= Tb || j >= Tb) return 0.f;
    const int a = i < j ? i : j, cc = i < j ? j : i;
    const float g = dC[((size_t)b * Lm + li) * npair + (a * T - a * (a - 1) / 2 + (cc - a))];
    return i == j ? g : 0.5f * g;
  };
  float gn[4] = {0.f, 0.f, 0.f, 0.f};
  if (l0 < l1)
#pragma unroll
    for (int m = 0; m < 4; ++m) gn[m] = gval(l0, tid + 256 * m);
  float4 dp = make_float4(0.f, 0.f, 0.f, 0.f);
  constexpr int NI = TWO ? 2 : 1;  // 16-row tracer tiles
  for (int li = l0; li < l1; ++li) {
    const int buf = (li - l0) & 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = tid + 256 * m;
      Gs[buf][e >> 5][e & 31] = gn[m];
    }
    __syncthreads();
    if (li + 1 < l1)
#pragma unroll
      for (int m = 0; m < 4; ++m) gn[m] = gval(li + 1, tid + 256 * m);
    float* w = (float*)P.vbuf + ((size_t)bl * Lm + li) * 32 * nk;
    v4f y[4][NI];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int it = 0; it < NI; ++it) y[j][it] = (v4f){0.f, 0.f, 0.f, 0.f};
    constexpr int NJ = TWO ? 8 : 4;
#pragma unroll
    for (int st = 0; st < NJ; ++st) {
      const float4 wv = cok ? *(const float4*)(w + (size_t)(4 * st + q) * nk + col) : make_float4(0.f, 0.f, 0.f, 0.f);
      const float bw[4] = {wv.x, wv.y, wv.z, wv.w};
      const float a0 = Gs[buf][r][4 * st + q];
      const float a1 = TWO ? Gs[buf][16 + r][4 * st + q] : 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        y[j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bw[j], y[j][0], 0, 0, 0);
        if constexpr (TWO) y[j][NI - 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bw[j], y[j][NI - 1], 0, 0, 0);
      }
    }
    // y[j][it][m] = Y[16 it + 4 q + m][col + j]
    if (cok) {
#pragma unroll
      for (int it = 0; it < NI; ++it)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          float4* a = (float4*)(w + (size_t)(16 * it + 4 * q + m) * nk + col);
          const float4 wo = *a;
          dp.x += wo.x * y[0][it][m];
          dp.y += wo.y * y[1][it][m];
          dp.z += wo.z * y[2][it][m];
          dp.w += wo.w * y[3][it][m];
          *a = make_float4(y[0][it][m], y[1][it][m], y[2][it][m], y[3][it][m]);
        }
    }
  }
  dp.x += __shfl_xor(dp.x, 16);
  dp.y += __shfl_xor(dp.y, 16);
  dp.z += __shfl_xor(dp.z, 16);
  dp.w += __shfl_xor(dp.w, 16);
  dp.x += __shfl_xor(dp.x, 32);
  dp.y += __shfl_xor(dp.y, 32);
  dp.z += __shfl_xor(dp.z, 32);
  dp.w += __shfl_xor(dp.w, 32);
  if (q == 0 && cok) *(float4*)((float*)P.dpk_part + ((size_t)b * nlc + c) * nk + col) = dp;
}

// (a6) Adjoint transforms for one (point, multipole chunk, group of 4 tracers): wave w takes
// tracer 4 g + w through the chunk's multipoles, dx = 2 s F k^{-1-b} Y from its workspace row,
// r2c, dc += h conj(X) conj(U_l) in registers, flushed to the (point, chunk, tracer, band)
// partial row when the band changes; rows of bands the chunk never reaches are zeroed.
template <int M, bool TW_LDS>
__global__ __launch_bounds__(256) void k_bwd_adj(plan_dev P, swiftcl_inputs in, int b0, int nbp, int nlc) {
  constexpr int RL = M / SWIFTCL_WAVE;
  constexpr int N = 2 * M;
  __shared__ C2<float> lds[4][fft_lds_size(M, sizeof(float))];
  __shared__ C2<float> stw_s[TW_LDS ? N : 1];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / SWIFTCL_WAVE), lane = tid % SWIFTCL_WAVE;
  const int T = P.max_tracers, Lm = P.max_ell, nk = P.n_k, nb = P.n_bands;
  const int ng = (T + 3) / 4;
  const int g = blockIdx.x % ng;
  const int rest = blockIdx.x / ng;
  const int c = rest % nlc;
  const int bl = rest / nlc;
  if (bl >= nbp) return;
  if constexpr (TW_LDS) {
    for (int i = tid; i < N; i += 256) stw_s[i] = ((const C2<float>*)P.tw)[i];
    __syncthreads();
  }
  const C2<float>* stw = TW_LDS ? (const C2<float>*)stw_s : (const C2<float>*)P.tw;
  const int b = b0 + bl;
  const int t = 4 * g + wave;
  const int Tb = clampb(in.n_tracers[b], 0, T);
  if (t >= Tb) return;  // k_bwd_coeffs writes zeros for these tracers and reads no partial row
  const int Lb = clampb(in.n_ell[b], 0, Lm);
  const int l0 = (int)(((long)c * Lb) / nlc), l1 = (int)(((long)(c + 1) * Lb) / nlc);
  const int kind = tracer_kind(in, T, b, t);
  C2<float>* part = (C2<float>*)P.dchat_part + (((size_t)b * nlc + c) * T + t) * nb * M;
  const float* sq = (const float*)P.sqrt_s + (size_t)b * nk;
  C2<float> acc[RL];
#pragma unroll
  for (int e = 0; e < RL; ++e) acc[e] = mk<float>(0.f, 0.f);
  int cur_band = -1;
  unsigned flushed = 0;
  auto flush = [&]() {
    C2<float>* dst = part + (size_t)cur_band * M;
    const bool again = (flushed >> cur_band) & 1u;
#pragma unroll
    for (int e = 0; e < RL; ++e) {
      const int n = lane + SWIFTCL_WAVE * e;
      dst[n] = again ? cadd(dst[n], acc[e]) : acc[e];
      acc[e] = mk<float>(0.f, 0.f);
    }
    flushed |= 1u << cur_band;
  };
  for (int li = l0; li < l1; ++li) {
    int ei = in.ell_idx[(size_t)b * Lm + li];
    if (ei < 0 || ei >= P.n_ell) {
      if (lane == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
      ei = 0;
    }
    const int band = P.ell_band[ei];
    if (band != cur_band) {
      if (cur_band >= 0) flush();
      cur_band = band;
    }
    const float* y = (const float*)P.vbuf + (((size_t)bl * Lm + li) * 32 + t) * nk;
    const float* ks = (const float*)P.kscale + ((size_t)kind * nb + band) * nk;
    C2<float> v[RL];
#pragma unroll
    for (int e = 0; e < RL; ++e) {
      const int k0 = 2 * (lane + SWIFTCL_WAVE * e);
      if (k0 < nk) {
        const C2<float> y2 = *(const C2<float>*)(y + k0);
        const C2<float> kk = *(const C2<float>*)(ks + k0);
        const C2<float> s2 = *(const C2<float>*)(sq + k0);
        v[e] = mk<float>(2.f * s2.x * s2.x * kk.x * y2.x, 2.f * s2.y * s2.y * kk.y * y2.y);
      } else {
        v[e] = mk<float>(0.f, 0.f);
      }
    }
    wave_sync();
    wave_r2c<float, M>(v, lds[wave], stw, lane);
    const C2<float>* Ur = (const C2<float>*)P.U + ((size_t)kind * P.n_ell + ei) * M;
#pragma unroll
    for (int e = 0; e < RL; ++e) {
      const int n = lane + SWIFTCL_WAVE * e;
      const float h = n == 0 ? 1.f : 2.f;
      acc[e] = cadd(acc[e], cscale(cmul(cconj(v[e]), cconj(Ur[n])), h));
    }
  }
  if (cur_band >= 0) flush();
  for (int bi = 0; bi < nb; ++bi) {
    if ((flushed >> bi) & 1u) continue;
#pragma unroll
    for (int e = 0; e < RL; ++e) part[(size_t)bi * M + lane + SWIFTCL_WAVE * e] = mk<float>(0.f, 0.f);
  }
}

// Reduce dc over chunks and take it back through the forward real transform: dg per
// (point, tracer, band), one wavefront per row.
template <typename R, int M>
__global__ __launch_bounds__(256) void k_bwd_coeffs(plan_dev P, swiftcl_inputs in, int nchunk) {
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
  if (row >= rows) return;
  const int bi = (int)(row % nb);
  const int t = (int)((row / nb) % T);
  const int b = (int)(row / ((long)nb * T));
  C2<R>* out = (C2<R>*)((R*)P.dg + row * N);
  const int Tb = clampb(in.n_tracers[b], 0, T);
  if (t >= Tb) {
#pragma unroll
    for (int e = 0; e < RL; ++e) out[lane + SWIFTCL_WAVE * e] = mk<R>(0, 0);
    return;
  }
  C2<R> v[RL];
#pragma unroll
  for (int e = 0; e < RL; ++e) v[e] = mk<R>(0, 0);
  for (int c = 0; c < nchunk; ++c) {
    const C2<R>* src = (const C2<R>*)P.dchat_part + ((((size_t)b * nchunk + c) * T + t) * nb + bi) * M;
#pragma unroll
    for (int e = 0; e < RL; ++e) v[e] = cadd(v[e], src[lane + SWIFTCL_WAVE * e]);
  }
  const double* pt = P.pt + (size_t)b * PT_STRIDE;
  const int kind = tracer_kind(in, T, b, t);
  const double scale = pt[PT_CHI0B + kind * SWIFTCL_MAX_BANDS + bi] / (double)N;
  const double2* ph = (const double2*)P.phase + (size_t)b * M;
#pragma unroll
  for (int e = 0; e < RL; ++e) {
    const int n = lane + SWIFTCL_WAVE * e;
    const double cs = ph[n].x, sn = ph[n].y;
    // e_n = dc_n conj(alpha_n); the c2r doubles n > 0, so pass e_n / 2 there
    C2<R> en = cmul(v[e], mk<R>((R)(cs * scale), (R)(-sn * scale)));
    v[e] = n == 0 ? en : cscale(en, (R)0.5);
  }
  wave_c2r<R, M>(v, lds[wave], twp, lane);
#pragma unroll
  for (int e = 0; e < RL; ++e) out[lane + SWIFTCL_WAVE * e] = v[e];
}

size_t bwd_geometry_lds_bytes(const plan_dev& p) {
  return sizeof(double) * ((size_t)2 * p.n_zg + (size_t)6 * p.n_zs + (size_t)2 * p.n_union + 64);
}

// (a7) Chain rule through the kernel assembly for one (point, tracer) per workgroup of 512
// threads (FP64): dL/db_t, dL/dn_t (through the n(z) spline and, for lensing, the suffix integrals)
// and this tracer's share of the cotangents of the D samples and of D'' (summed over tracers by
// k_bwd_point).  The chi nodes' geometry (z, chi, dchi/dz, D and their intervals) comes from the
// forward assembly; the chi spline (for the lensing quadrature) sits in LDS.
// MAXN: chi nodes per thread (n_chi <= 512 MAXN; 2 at n_chi <= 1024 keeps the per-node lensing
// registers to what that needs).  Latency-bound FP64 work: registers capped for six waves per SIMD
// (three workgroups per CU, which the ~47 KB of LDS allows; a few words spill), 23% faster on the
// benchmark batch than at the four waves the uncapped register count gives.
template <typename R, int MAXN>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6))) void k_bwd_tracer(plan_dev P,
                                                                                           swiftcl_inputs in,
                                                                                           double* dbias,
                                                                                           double* dnz) {
  extern __shared__ double sh[];
  const int T = P.max_tracers;
  const int b = blockIdx.x / T, t = blockIdx.x % T;
  if (b >= in.batch) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int wave = tid / SWIFTCL_WAVE, lane = tid % SWIFTCL_WAVE;
  const int nzg = P.n_zg, nzs = P.n_zs, nb = P.n_bands, N = P.N, nu = P.n_union;
  const int Tb = clampb(in.n_tracers[b], 0, T);
  if (t >= Tb) {
    if (tid == 0 && dbias) dbias[(size_t)b * T + t] = 0.0;
    if (dnz)
      for (int i = tid; i < nzs; i += nth) dnz[((size_t)b * T + t) * nzs + i] = 0.0;
    return;
  }
  // the read-only grids (z, 1/h, chi and its spline moments) are read through the cache: LDS
  // holds the accumulators and this tracer's rows only (~47 KB at n_zg = 1024: three workgroups
  // per CU)
  const double* zg = P.z_geom;                              // [nzg]
  const double* zgih = P.lu_geom + 3 * (size_t)nzg;         // [nzg] 1/h
  const double* chi = in.chi_z + (size_t)b * nzg;           // [nzg]
  const double* mchi = P.m_chi + (size_t)b * nzg;           // [nzg]
  double* dDy = sh;                      // [nzg] cotangent of D samples (value terms)
  double* dDM = dDy + nzg;               // [nzg] cotangent of D'' (spline terms)
  double* zs = dDM + nzg;                // [nzs]
  double* zsih = zs + nzs;               // [nzs]
  double* dny = zsih + nzs;              // [nzs] cotangent of this tracer's n samples
  double* dnM = dny + nzs;               // [nzs]
  double* nt = dnM + nzs;                // [nzs] this tracer's n samples
  double* mt = nt + nzs;                 // [nzs] and their spline second derivatives
  double* seg0 = mt + nzs;               // [nu]
  double* seg1 = seg0 + nu;              // [nu]
  double* tmp = seg1 + nu;               // [64]

  const int kd = in.kind[(size_t)b * T + t];
  const int kind = tracer_kind(in, T, b, t);  // a tracer of an unknown kind has no cotangent below
  for (int i = tid; i < nzg; i += nth) {
    dDy[i] = 0.0;
    dDM[i] = 0.0;
  }
  for (int i = tid; i < nzs; i += nth) {
    zs[i] = P.z_nz[i];
    zsih[i] = P.lu_nz[3 * nzs + i];
    dny[i] = 0.0;
    dnM[i] = 0.0;
    nt[i] = in.nz[((size_t)b * T + t) * nzs + i];
    mt[i] = P.m_n[((size_t)b * T + t) * nzs + i];
  }
  const double* pt = P.pt + (size_t)b * PT_STRIDE;
  const double theta = pt[PT_THETA];
  const int m0 = P.m0, m1 = (int)pt[PT_M1];
  __syncthreads();

  // dL/df at node m: sum over bands of dg w e^{-b m Delta}
  auto df_at = [&](int m, double w) {
    double s = 0.0;
    for (int bi = 0; bi < nb; ++bi)
      s += (double)((const R*)P.dg)[(((size_t)b * T + t) * nb + bi) * N + m] * P.ebm[((size_t)kind * nb + bi) * N + m];
    return s * w;
  };
  auto fill = [&](node_state& s, int m) {
    const double* nf = P.node_f + (size_t)b * 4 * N + m;
    const int* ni = P.node_i + (size_t)b * 3 * N + m;
    s.z = nf[0];
    s.chiz = nf[N];
    s.dchi = nf[2 * N];
    s.D = nf[3 * N];
    s.ig = ni[0];
    s.inz = ni[N];
    s.u = ni[2 * N];
    s.w = (m == m0) ? 0.5 : (m == m1 ? 0.5 + theta : 1.0);
    s.zc = P.z_union[s.u + 1];
    s.ugi = P.union_iv[s.u];
    s.uni = P.union_iv[nu + s.u];
  };
  const double pref = 1.5 * in.omega_m[b] * SWIFTCL_H0_OVER_C * SWIFTCL_H0_OVER_C;
  double dbl = 0.0;
  if (kd == SWIFTCL_CLUSTERING) {
    const double bias = in.bias[(size_t)b * T + t];
    for (int m = m0 + tid; m <= m1; m += nth) {
      node_state s;
      fill(s, m);
      const double df = df_at(m, s.w);
      const double n = s.inz < 0 ? 0.0 : spline_at(zs, zsih, nt, mt, s.inz, s.z, nullptr);
      dbl += df * n * s.D / s.dchi;
      if (s.inz >= 0) spline_value_adjoint(zs, zsih, s.inz, s.z, df * bias * s.D / s.dchi, dny, dnM);
      spline_value_adjoint(zg, zgih, s.ig, s.z, df * bias * n / s.dchi, dDy, dDM);
    }
  } else if (kd == SWIFTCL_CMB_LENSING) {
    // Sec. 2.4: f = pref (1+z) (chi_* - chi) / (chi chi_*) D is linear in D alone; its last node
    // carries the linear-end weight 1/2 + theta/2
    const double chis = chi[nzg - 1];
    for (int m = m0 + tid; m <= m1; m += nth) {
      node_state s;
      fill(s, m);
      const double w = (m == m1 && m1 > m0) ? 0.5 + 0.5 * theta : s.w;
      const double df = df_at(m, w);
      const double x = s.chiz;
      spline_value_adjoint(zg, zgih, s.ig, s.z, df * pref * (1.0 + s.z) * (chis - x) / (x * chis), dDy, dDM);
    }
  } else if (kd == SWIFTCL_LENSING) {
    double dI0[MAXN], dI1[MAXN];
    int uu[MAXN];
#pragma unroll
    for (int k = 0; k < MAXN; ++k) {
      dI0[k] = dI1[k] = 0.0;
      uu[k] = -1;
      const int m = m0 + tid + k * nth;
      if (m > m1) continue;
      node_state s;
      fill(s, m);
      uu[k] = s.u;
      const double df = df_at(m, s.w);
      const double x = s.chiz;
      const double q = P.lens_q[((size_t)b * T + t) * N + m];  // the forward's q at this node
      double fq = q;
      if (in.ia) {
        // intrinsic alignment: f = (q + A_IA n dz/dchi) D / chi^2 is also local in n
        const double a = spline_at(zg, zgih, in.ia + (size_t)b * nzg, P.m_ia + (size_t)b * nzg, s.ig, s.z, nullptr);
        const double n = s.inz < 0 ? 0.0 : spline_at(zs, zsih, nt, mt, s.inz, s.z, nullptr);
        fq += a * n / s.dchi;
        if (s.inz >= 0) spline_value_adjoint(zs, zsih, s.inz, s.z, df * a * s.D / (s.dchi * x * x), dny, dnM);
      }
      spline_value_adjoint(zg, zgih, s.ig, s.z, df * fq / (x * x), dDy, dDM);
      const double dq = df * s.D / (x * x);
      dI0[k] = dq * pref * x * (1.0 + s.z);
      dI1[k] = -dq * pref * x * x * (1.0 + s.z);
    }
    __syncthreads();
    // transpose of I(z_m) = partial(z_m) + suffix(u_m + 1): full intervals u get the sum of
    // dI over nodes with u_m < u (an exclusive prefix over intervals)
    for (int u = tid; u < nu; u += nth) { seg0[u] = 0.0; seg1[u] = 0.0; }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXN; ++k) {
      if (uu[k] < 0) continue;
      unsafeAtomicAdd(&seg0[uu[k]], dI0[k]);
      unsafeAtomicAdd(&seg1[uu[k]], dI1[k]);
    }
    __syncthreads();
    block_scan(seg0, nu, tmp, true);
    block_scan(seg1, nu, tmp, true);
    for (int u = tid; u < nu; u += nth) {
      const int iv = P.union_iv[nu + u];
      if (iv < 0) continue;
      const double a = P.z_union[u], c = P.z_union[u + 1];
      const int ig = P.union_iv[u];
      const double w0 = seg0[u], w1 = seg1[u];
      spline_adj_acc ac;
      for (int qn = 0; qn < SWIFTCL_NGL; ++qn) {
        const double z = 0.5 * (c - a) * c_gl_x[qn] + 0.5 * (a + c);
        const double w = 0.5 * (c - a) * c_gl_w[qn];
        const double x = spline_at(zg, zgih, chi, mchi, ig, z, nullptr);
        ac.add(zs, zsih, iv, z, w * (w0 + w1 / x));
      }
      ac.flush(zs, iv, dny, dnM);
    }
#pragma unroll
    for (int k = 0; k < MAXN; ++k) {
      if (uu[k] < 0) continue;
      const int m = m0 + tid + k * nth;
      node_state s;
      fill(s, m);
      if (s.uni < 0) continue;
      const double a = s.z, c = s.zc;
      spline_adj_acc ac;
      for (int qn = 0; qn < SWIFTCL_NGL; ++qn) {
        const double z = 0.5 * (c - a) * c_gl_x[qn] + 0.5 * (a + c);
        const double w = 0.5 * (c - a) * c_gl_w[qn];
        const double x = spline_at(zg, zgih, chi, mchi, s.ugi, z, nullptr);
        ac.add(zs, zsih, s.uni, z, w * (dI0[k] + dI1[k] / x));
      }
      ac.flush(zs, s.uni, dny, dnM);
    }
  }
  // bias: block reduction
  for (int off = 32; off >= 1; off >>= 1) dbl += __shfl_xor(dbl, off);
  if (lane == 0) tmp[wave] = dbl;
  __syncthreads();
  if (tid == 0 && dbias) {
    double s = 0.0;
    for (int w = 0; w < nth / SWIFTCL_WAVE; ++w) s += tmp[w];
    dbias[(size_t)b * T + t] = kd == SWIFTCL_CLUSTERING ? s : 0.0;
  }
  // n spline transpose
  if (wave == 0) wave_spline_adjoint(dny, dnM, P.lu_nz, nzs, lane);
  __syncthreads();
  if (dnz)
    for (int i = tid; i < nzs; i += nth) dnz[((size_t)b * T + t) * nzs + i] = dny[i];
  double* part = P.ddD_part + ((size_t)b * T + t) * 2 * nzg;
  for (int i = tid; i < nzg; i += nth) {
    part[i] = dDy[i];
    part[nzg + i] = dDM[i];
  }
}

template <typename R>
static hipError_t launch_bwd_tracer(const plan_dev& p, const swiftcl_inputs* in, double* dbias, double* dnz,
                                    hipStream_t s) {
  const dim3 grid((unsigned)((size_t)in->batch * p.max_tracers));
  const size_t lg = bwd_geometry_lds_bytes(p);
  if (p.N <= 1024) hipLaunchKernelGGL((k_bwd_tracer<R, 2>), grid, dim3(512), lg, s, p, *in, dbias, dnz);
  else hipLaunchKernelGGL((k_bwd_tracer<R, 4>), grid, dim3(512), lg, s, p, *in, dbias, dnz);
  return hipGetLastError();
}

// Per point: dL/dP (the chunk partials times (2/pi) w k^3) and dL/dD (the tracers' shares summed
// in tracer order, then the D spline transpose), one workgroup of 1024 threads (FP64): one
// geometry sample per thread, its tracer loads issued together.
template <typename R>
__global__ __launch_bounds__(1024) void k_bwd_point(plan_dev P, swiftcl_inputs in, int nchunk, double* dpk,
                                                     double* dD) {
  extern __shared__ double sh[];
  const int b = blockIdx.x;
  if (b >= in.batch) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int wave = tid / SWIFTCL_WAVE, lane = tid % SWIFTCL_WAVE;
  const int T = P.max_tracers, nzg = P.n_zg, nk = P.n_k;
  if (dpk) {
    for (int k = tid; k < nk; k += nth) {
      double s = 0.0;
      for (int c = 0; c < nchunk; ++c) s += (double)((const R*)P.dpk_part)[((size_t)b * nchunk + c) * nk + k];
      dpk[(size_t)b * nk + k] = P.kw[k] * s;
    }
  }
  if (!dD) return;
  const int Tb = clampb(in.n_tracers[b], 0, T);
  double* dDy = sh;        // [nzg]
  double* dDM = dDy + nzg; // [nzg]
  for (int i = tid; i < nzg; i += nth) {
    double sy = 0.0, sm = 0.0;
#pragma unroll 8
    for (int t = 0; t < Tb; ++t) {  // (unrolled: the loads of 8 tracers in flight; the sum stays in order)
      const double* part = P.ddD_part + ((size_t)b * T + t) * 2 * nzg;
      sy += part[i];
      sm += part[nzg + i];
    }
    dDy[i] = sy;
    dDM[i] = sm;
  }
  __syncthreads();
  if (wave == 0) wave_spline_adjoint(dDy, dDM, P.lu_geom, nzg, lane);
  __syncthreads();
  for (int i = tid; i < nzg; i += nth) dD[(size_t)b * nzg + i] = dDy[i];
}

size_t bwd_windows_lds(const plan_dev& p) {
  if (p.precision == SWIFTCL_FP64) return windows_cl_lds(p.M, 2, false, true, 8, p.n_k);
  const size_t tw = 2 * (size_t)p.M * 2 * sizeof(float);  // FP32 stages the twiddles (TW = !dp)
  return tw + ((size_t)16 * compact_vs(p.n_k, p.M) + (size_t)(2 + SWIFTCL_NKINDS * p.n_bands) * p.n_k) * sizeof(float);
}

template <typename R, int M>
static hipError_t launch_bwd_t(const plan_dev& p, const swiftcl_inputs* in, const void* dC, double* dpk,
                               double* dbias, double* dnz, double* dD, hipStream_t s, hipEvent_t* ev) {
  constexpr bool dp = sizeof(R) == 8;
  constexpr int NW = dp ? 2 : 16;
  constexpr bool TW = !dp;
  const int nchunk = backward_chunks(p, in->batch);
  const size_t lds = bwd_windows_lds(p);
  // the packed adjoint writes two sub-chunks of partial rows per chunk
  const bool pack = !dp && p.bwd_pack && p.bwd_chunk_mul <= 4;
  auto k1 = pack ? k_bwd_windows<R, M, NW, TW, !dp> : k_bwd_windows<R, M, NW, TW>;
  hipError_t e;
  const size_t groups = (size_t)(in->batch + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD;
  const long n = (long)groups * nchunk * SWIFTCL_NXCD;
  const int ordered = p.bwd_order && n <= p.bwd_order_n && n <= BWD_ORDER_MAX;
  if (ordered) {
    hipLaunchKernelGGL(k_bwd_order, dim3(1), dim3(1024), 0, s, p, *in, nchunk, (int)n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k1, dim3((unsigned)n), dim3(NW * 64), lds, s, p, *in, (const R*)dC, nchunk, ordered);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  const long rows = (long)in->batch * p.max_tracers * p.n_bands;
  hipLaunchKernelGGL((k_bwd_coeffs<R, M>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, p, *in,
                     pack ? 2 * nchunk : nchunk);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  if ((dbias || dnz || dD) && (e = launch_bwd_tracer<R>(p, in, dbias, dnz, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bwd_point<R>, dim3(in->batch), dim3(1024), 2 * (size_t)p.n_zg * sizeof(double), s, p, *in,
                     nchunk, dpk, dD);
  return hipGetLastError();
}

template <typename R>
static hipError_t launch_chain_t(const plan_dev& p, const swiftcl_inputs* in, double* dbias, double* dnz, double* dD,
                                 hipStream_t s) {
  if (dbias || dnz || dD) {
    hipError_t e = launch_bwd_tracer<R>(p, in, dbias, dnz, s);
    if (e != hipSuccess) return e;
  }
  if (dD)
    hipLaunchKernelGGL(k_bwd_point<R>, dim3(in->batch), dim3(1024), 2 * (size_t)p.n_zg * sizeof(double), s, p, *in,
                       0, nullptr, dD);
  return hipGetLastError();
}

hipError_t launch_bwd_chain(const plan_dev& p, const swiftcl_inputs* in, double* dbias, double* dnz, double* dD,
                            hipStream_t s) {
  return p.precision == SWIFTCL_FP64 ? launch_chain_t<double>(p, in, dbias, dnz, dD, s)
                                     : launch_chain_t<float>(p, in, dbias, dnz, dD, s);
}

// Y = G W over the workspace rows of points b0 .. b0 + nbp - 1 (FP32 W rows written by the caller)
// with the dP partials of nchunk = bwd_nlc multipole chunks per point
hipError_t launch_bwd_gv(const plan_dev& p, const swiftcl_inputs* in, const void* dC, int b0, int nbp, hipStream_t s) {
  const int nlc = p.bwd_nlc, T = p.max_tracers;
  if (p.n_k % 4 == 0) {  // 16-byte rows
    const dim3 g4((unsigned)((size_t)nbp * nlc * ((p.n_k + 255) / 256)));
    if (T > 16) hipLaunchKernelGGL(k_bwd_gv4<true>, g4, dim3(256), 0, s, p, *in, (const float*)dC, b0, nbp, nlc);
    else hipLaunchKernelGGL(k_bwd_gv4<false>, g4, dim3(256), 0, s, p, *in, (const float*)dC, b0, nbp, nlc);
  } else {
    const dim3 g1((unsigned)((size_t)nbp * nlc * ((p.n_k + 63) / 64)));
    if (T > 16) hipLaunchKernelGGL(k_bwd_gv<true>, g1, dim3(256), 0, s, p, *in, (const float*)dC, b0, nbp, nlc);
    else hipLaunchKernelGGL(k_bwd_gv<false>, g1, dim3(256), 0, s, p, *in, (const float*)dC, b0, nbp, nlc);
  }
  return hipGetLastError();
}

// dL/dP from the partials of launch_bwd_gv (every point of the batch)
hipError_t launch_bwd_dpk(const plan_dev& p, const swiftcl_inputs* in, double* dpk, hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_point<float>, dim3(in->batch), dim3(1024), 2 * (size_t)p.n_zg * sizeof(double), s, p, *in,
                     p.bwd_nlc, dpk, nullptr);
  return hipGetLastError();
}

// The adjoint through the workspace (FP32; plans with adjoint == 2)
template <int M>
static hipError_t launch_bwd_ws(const plan_dev& p, const swiftcl_inputs* in, const void* dC, double* dpk,
                                double* dbias, double* dnz, double* dD, hipStream_t s, hipEvent_t* ev) {
  const int nlc = p.bwd_nlc, T = p.max_tracers;
  const int ng = (T + 3) / 4;
  hipError_t e;
  for (int b0 = 0; b0 < in->batch; b0 += p.vchunk) {
    const int nbp = in->batch - b0 < p.vchunk ? in->batch - b0 : p.vchunk;
    if ((e = launch_windows_w(p, in, b0, nbp, s)) != hipSuccess) return e;
    if ((e = launch_bwd_gv(p, in, dC, b0, nbp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_bwd_adj<M, (M <= 1024)>), dim3((unsigned)((size_t)nbp * nlc * ng)), dim3(256), 0, s, p,
                       *in, b0, nbp, nlc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  const long rows = (long)in->batch * T * p.n_bands;
  hipLaunchKernelGGL((k_bwd_coeffs<float, M>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, p, *in, nlc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  if ((dbias || dnz || dD) && (e = launch_bwd_tracer<float>(p, in, dbias, dnz, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bwd_point<float>, dim3(in->batch), dim3(1024), 2 * (size_t)p.n_zg * sizeof(double), s, p, *in,
                     nlc, dpk, dD);
  return hipGetLastError();
}

hipError_t launch_backward(const plan_dev& p, const swiftcl_inputs* in, const void* dC, double* dpk, double* dbias,
                           double* dnz, double* dD, hipStream_t s, hipEvent_t* ev) {
  if (p.adjoint == 2) {
    switch (p.M) {
      case 128: return launch_bwd_ws<128>(p, in, dC, dpk, dbias, dnz, dD, s, ev);
      case 256: return launch_bwd_ws<256>(p, in, dC, dpk, dbias, dnz, dD, s, ev);
      case 512: return launch_bwd_ws<512>(p, in, dC, dpk, dbias, dnz, dD, s, ev);
      case 1024: return launch_bwd_ws<1024>(p, in, dC, dpk, dbias, dnz, dD, s, ev);
    }
    return hipErrorInvalidValue;
  }
  const bool dp = p.precision == SWIFTCL_FP64;
  switch (p.M) {
    case 128: return dp ? launch_bwd_t<double, 128>(p, in, dC, dpk, dbias, dnz, dD, s, ev)
                        : launch_bwd_t<float, 128>(p, in, dC, dpk, dbias, dnz, dD, s, ev);
    case 256: return dp ? launch_bwd_t<double, 256>(p, in, dC, dpk, dbias, dnz, dD, s, ev)
                        : launch_bwd_t<float, 256>(p, in, dC, dpk, dbias, dnz, dD, s, ev);
    case 512: return dp ? launch_bwd_t<double, 512>(p, in, dC, dpk, dbias, dnz, dD, s, ev)
                        : launch_bwd_t<float, 512>(p, in, dC, dpk, dbias, dnz, dD, s, ev);
    case 1024: return dp ? launch_bwd_t<double, 1024>(p, in, dC, dpk, dbias, dnz, dD, s, ev)
                         : launch_bwd_t<float, 1024>(p, in, dC, dpk, dbias, dnz, dD, s, ev);
  }
  return hipErrorInvalidValue;
}

