// Shared device helpers: complex arithmetic, small in-register DFTs and a wavefront-level
// Stockham FFT for gfx950 (64-lane wavefronts).  Everything is templated on the real type
// (float for the FP32 / split paths, double for the FP64 path).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SWIFTCL_WAVE 64

template <typename R> struct cplx_t;
template <> struct cplx_t<float> { typedef float2 type; };
template <> struct cplx_t<double> { typedef double2 type; };

template <typename R> using C2 = typename cplx_t<R>::type;

template <typename R> __device__ __forceinline__ C2<R> mk(R x, R y) { C2<R> c; c.x = x; c.y = y; return c; }
template <typename T> __device__ __forceinline__ T cadd(T a, T b) { a.x += b.x; a.y += b.y; return a; }
template <typename T> __device__ __forceinline__ T csub(T a, T b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
  T c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c;
}
template <typename T> __device__ __forceinline__ T cconj(T a) { a.y = -a.y; return a; }
template <typename T, typename R> __device__ __forceinline__ T cscale(T a, R s) { a.x *= s; a.y *= s; return a; }
// multiply by S*i (S = +1 or -1)
template <int S, typename T> __device__ __forceinline__ T mul_si(T a) {
  T c; if (S > 0) { c.x = -a.y; c.y = a.x; } else { c.x = a.y; c.y = -a.x; } return c;
}

// Ordering of LDS traffic inside one wavefront (no block barrier needed: a wavefront's LDS
// instructions execute in order; this stops the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// cos / sin of 2*pi*k/16 for k = 0..3 (exact constants of the 16-point circle)
#define SWIFTCL_C16_1 0.92387953251128675613
#define SWIFTCL_S16_1 0.38268343236508977173
#define SWIFTCL_R2_2 0.70710678118654752440

// e^{S 2 pi i k / r} for the constant twiddles of a radix-r butterfly, k < r/2
template <typename R, int r, int S> __device__ __forceinline__ C2<R> const_tw(int k) {
  // r in {4, 8, 16}; k/r reduced to sixteenths
  const int k16 = k * (16 / r);
  R c, s;
  switch (k16) {
    case 0: c = 1; s = 0; break;
    case 1: c = (R)SWIFTCL_C16_1; s = (R)SWIFTCL_S16_1; break;
    case 2: c = (R)SWIFTCL_R2_2; s = (R)SWIFTCL_R2_2; break;
    case 3: c = (R)SWIFTCL_S16_1; s = (R)SWIFTCL_C16_1; break;
    case 4: c = 0; s = 1; break;
    case 5: c = -(R)SWIFTCL_S16_1; s = (R)SWIFTCL_C16_1; break;
    case 6: c = -(R)SWIFTCL_R2_2; s = (R)SWIFTCL_R2_2; break;
    default: c = -(R)SWIFTCL_C16_1; s = (R)SWIFTCL_S16_1; break;
  }
  return mk<R>(c, S > 0 ? s : -s);
}

// In-register DFT of size r (power of two <= 16), sign S: Y_k = sum_i y_i e^{S 2 pi i i k / r}.
// Radix-2 decimation in time, unrolled at compile time.
template <typename R, int r, int S> __device__ __forceinline__ void dft(C2<R>* v) {
  if constexpr (r == 1) {
    return;
  } else if constexpr (r == 2) {
    C2<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else {
    C2<R> e[r / 2], o[r / 2];
#pragma unroll
    for (int i = 0; i < r / 2; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
    dft<R, r / 2, S>(e);
    dft<R, r / 2, S>(o);
#pragma unroll
    for (int k = 0; k < r / 2; ++k) {
      C2<R> t;
      if (k == 0) t = o[k];
      else if (4 * k == r) t = mul_si<S>(o[k]);
      else t = cmul(o[k], const_tw<R, r, S>(k));
      v[k] = cadd(e[k], t);
      v[k + r / 2] = csub(e[k], t);
    }
  }
}

// Radix schedule of an M-point wavefront FFT: each lane holds RL = M/64 elements and every
// pass uses a radix that divides RL, so a lane runs RL/r butterflies per pass.
template <int M> struct fft_plan;
template <> struct fft_plan<128> { static constexpr int RL = 2, NP = 7; static constexpr int rad[7] = {2, 2, 2, 2, 2, 2, 2}; };
template <> struct fft_plan<256> { static constexpr int RL = 4, NP = 4; static constexpr int rad[4] = {4, 4, 4, 4}; };
template <> struct fft_plan<512> { static constexpr int RL = 8, NP = 3; static constexpr int rad[3] = {8, 8, 8}; };
template <> struct fft_plan<1024> { static constexpr int RL = 16, NP = 3; static constexpr int rad[3] = {16, 8, 8}; };
template <> struct fft_plan<2048> { static constexpr int RL = 32, NP = 3; static constexpr int rad[3] = {16, 16, 8}; };

// The same schedule for host code: radix of pass p and number of passes of an M-point FFT.
__host__ __device__ constexpr int fft_npass(int M) { return M == 128 ? 7 : (M == 256 ? 4 : 3); }
__host__ __device__ constexpr int fft_radix(int M, int p) {
  return M == 128 ? 2 : M == 256 ? 4 : M == 512 ? 8 : M == 1024 ? (p == 0 ? 16 : 8) : (p < 2 ? 16 : 8);
}

// Twiddle table of an M-point wave FFT inside a real transform of length N = 2M (2M - 1 complex
// entries, built on the host):
//   [0, M)                                  e^{-2 pi i n / N}      (real-transform post-processing)
//   M + Ls - 1 + (i - 1) Ls + j, i = 1..r-1, j < Ls   e^{-2 pi i i j / (Ls r)}   for the pass of
//                                           radix r and stride Ls (Ls = product of the earlier radices)
// Each pass reads its twiddles at consecutive addresses (j = lane mod Ls), free of bank conflicts;
// the pass blocks tile [M, 2M - 1) since sum over passes of (r - 1) Ls = M - 1.
__host__ __device__ constexpr int fft_tw_index(int M, int Ls, int i, int j) { return M + Ls - 1 + (i - 1) * Ls + j; }

// LDS scratch layouts of the wave FFT.  Measured on gfx950 (rocprofv3 SQ_LDS_BANK_CONFLICT of
// single-pattern kernels): a 64-bit read serves 32 lanes per cycle from 32 slots of 8 bytes, a
// 64-bit write 16 lanes per cycle from 16 slots, so a read is conflict-free when each half
// wavefront hits 32 distinct slots mod 32 and a write when each quarter hits 16 distinct slots
// mod 16.  Every layout adds to the complex index c a function of its bits that is additive over
// disjoint bit sets, so every access of a pass is a per-lane base plus a compile-time offset (no
// per-access address arithmetic).  The buffer between two passes and the real transforms'
// exchange each take their own layout (BUF 0: written by pass 1, read by pass 2; BUF 1: written
// by pass 2, read by pass 3; BUF 2: the exchange, consecutive writes and mirrored reads):
//  * FP32, M = 512 (radix 8, 8, 8): BUF 0 c + (c >> 4) (the stride-8 writes of pass 1 land on 16
//    distinct slots; one 2-way slot per half-wave read), BUF 1 c XOR 8 bit6(c) (a bijection: the two
//    runs of 8 of each pass-2 write quarter land on the two halves of the 16 slots, the reads stay
//    runs of 32), BUF 2 c: at most 543 slots, small enough for two 1024-thread workgroups per CU.
//  * FP32, M = 1024 (radix 16, 8, 8): BUF 0 c + (c >> 4), BUF 1 c + (c >> 5), BUF 2 c (1087 slots).
//  * otherwise: c + (c >> 3) for every buffer.
// A wavefront's scratch holds fft_lds_size(M, sizeof(R)) complex values.
__host__ __device__ constexpr bool fft_compact_layout(int M, int rs) { return rs == 4 && (M == 512 || M == 1024); }
__host__ __device__ constexpr int fft_lds_size(int M, int rs) { return fft_compact_layout(M, rs) ? M + M / 16 : M + M / 8; }
// Row stride (floats) of a [16][n_k] LDS tile whose row t doubles as the FFT scratch of the
// wavefront that owns tracer t: room for both.  A 32-bit LDS read serves 32 lanes per cycle from
// 32 banks (measured like the 64-bit accesses above), so the stride is chosen per access pattern:
//  * the adjoint (compact_vs) reads MFMA operands of rows 4 (lane / 16) + s, 16 consecutive k:
//    stride == 4 (mod 32) puts the two row groups of a half-wave 16 banks apart;
//  * the forward projection (compact_vs_fwd) reads rows lane % 16 at k + lane / 16: stride == 2
//    (mod 32) gives the 32 lanes of a half-wave 32 distinct banks.
__host__ __device__ constexpr int compact_vs(int n_k, int M) {
  return (((n_k > 2 * fft_lds_size(M, 4) ? n_k : 2 * fft_lds_size(M, 4)) + 63) / 64) * 64 + 4;
}
__host__ __device__ constexpr int compact_vs_fwd(int n_k, int M) {
  return (((n_k > 2 * fft_lds_size(M, 4) ? n_k : 2 * fft_lds_size(M, 4)) + 31) / 32) * 32 + 2;
}
// fft_idx<R, M, BUF>(lp, K): the slot of complex index lp + K, lp a per-lane part and K a
// compile-time part with no bit in common (the unrolled loops make K a constant).  The additive
// layouts give fft_at(lp) + fft_at(K); BUF 2 (the identity, or c + (c >> 3)) is also linear on
// multiples of 64, which the mirrored read of the real transforms, M - n = (64 - lane) +
// 64 (RL - 1 - e), uses for lane 0.  The XOR layout flips bit 3 where bit 6 is set: with K's bits
// known, the slot is one of lp, lp ^ 8, lp - 8 bit6(lp), lp ^ (8 bit6(lp)) plus a constant, so the
// compiler keeps at most two bases per pass and folds the rest into the instruction offsets.
template <typename R, int M, int BUF> __device__ __forceinline__ int fft_at(int c) {
  if constexpr (fft_compact_layout(M, (int)sizeof(R))) {
    if constexpr (BUF == 0) return c + (c >> 4);
    else if constexpr (BUF == 1) return c + (c >> 5);  // (M = 1024; M = 512 takes the XOR layout)
    else return c;
  } else {
    return c + (c >> 3);
  }
}
template <typename R, int M, int BUF> __device__ __forceinline__ int fft_idx(int lp, int K) {
  if constexpr (fft_compact_layout(M, (int)sizeof(R)) && M == 512 && BUF == 1) {
    const int k6 = (K >> 6) & 1, k3 = (K >> 3) & 1;
    const int l6 = (lp >> 6) & 1;
    if (k6) return k3 ? lp + K - 8 : (lp ^ 8) + K;
    return k3 ? lp - 8 * l6 + K : (lp ^ (8 * l6)) + K;
  } else {
    return fft_at<R, M, BUF>(lp) + fft_at<R, M, BUF>(K);
  }
}

// One Stockham pass (self-sorting, natural-order output) of radix r on an M-point sequence.
// Butterfly q (q = lane + 64 u) reads x[q + i M/r], applies twiddles e^{S 2 pi i i j / (Ls r)}
// with j = q mod Ls, runs dft<r> and writes Y_i to (q / Ls) Ls r + j + i Ls.
// tw is the table described at fft_tw_index (global memory or LDS).
template <typename R, int M, int r, int Ls, int S, bool FIRST, bool LAST, int PASS>
__device__ __forceinline__ void stockham_pass(C2<R>* v, C2<R>* lds, const C2<R>* __restrict__ tw, int lane) {
  constexpr int BR = PASS - 1 < 1 ? PASS - 1 : 1;  // buffer this pass reads (passes beyond 3 share
  constexpr int BW = PASS < 1 ? PASS : 1;          // BUF 1: only the compact layouts differ)
  constexpr int RL = M / SWIFTCL_WAVE;
  constexpr int BPL = RL / r;
  constexpr int L = Ls * r;
  C2<R> b[RL];
  if constexpr (FIRST) {
    // registers hold x[lane + 64 e]; butterfly u input i is e = u + i * BPL
#pragma unroll
    for (int u = 0; u < BPL; ++u)
#pragma unroll
      for (int i = 0; i < r; ++i) b[u * r + i] = v[u + i * BPL];
  } else {
#pragma unroll
    for (int u = 0; u < BPL; ++u) {
#pragma unroll
      for (int i = 0; i < r; ++i) b[u * r + i] = lds[fft_idx<R, M, BR>(lane, SWIFTCL_WAVE * u + i * (M / r))];
    }
    wave_sync();
  }
#pragma unroll
  for (int u = 0; u < BPL; ++u) {
    if constexpr (Ls > 1) {
      const int q = lane + SWIFTCL_WAVE * u;
      const int j = q & (Ls - 1);
#pragma unroll
      for (int i = 1; i < r; ++i) {
        C2<R> w = tw[fft_tw_index(M, Ls, i, j)];
        if (S > 0) w = cconj(w);
        b[u * r + i] = cmul(b[u * r + i], w);
      }
    }
    dft<R, r, S>(&b[u * r]);
  }
  if constexpr (LAST) {
#pragma unroll
    for (int u = 0; u < BPL; ++u)
#pragma unroll
      for (int i = 0; i < r; ++i) v[u + i * BPL] = b[u * r + i];
  } else {
#pragma unroll
    for (int u = 0; u < BPL; ++u) {
      const int q = lane + SWIFTCL_WAVE * u;
      const int j = q & (Ls - 1);
      const int base = (q / Ls) * L + j;
#pragma unroll
      for (int i = 0; i < r; ++i) lds[fft_idx<R, M, BW>(base, i * Ls)] = b[u * r + i];
    }
    wave_sync();
  }
}

// M-point complex FFT by one wavefront.  In and out: v[e] holds element lane + 64 e (natural
// order).  lds: fft_lds_size(M, sizeof(R)) complex of scratch private to this wavefront.  S = -1 forward, +1 inverse
// (unnormalised).  tw: the table of fft_tw_index.
template <typename R, int M, int S>
__device__ __forceinline__ void wave_fft(C2<R>* v, C2<R>* lds, const C2<R>* __restrict__ tw, int lane) {
  using P = fft_plan<M>;
  if constexpr (P::NP == 3) {
    constexpr int r0 = P::rad[0], r1 = P::rad[1], r2 = P::rad[2];
    stockham_pass<R, M, r0, 1, S, true, false, 0>(v, lds, tw, lane);
    stockham_pass<R, M, r1, r0, S, false, false, 1>(v, lds, tw, lane);
    stockham_pass<R, M, r2, r0 * r1, S, false, true, 2>(v, lds, tw, lane);
  } else if constexpr (P::NP == 4) {
    stockham_pass<R, M, 4, 1, S, true, false, 0>(v, lds, tw, lane);
    stockham_pass<R, M, 4, 4, S, false, false, 1>(v, lds, tw, lane);
    stockham_pass<R, M, 4, 16, S, false, false, 2>(v, lds, tw, lane);
    stockham_pass<R, M, 4, 64, S, false, true, 3>(v, lds, tw, lane);
  } else {
    stockham_pass<R, M, 2, 1, S, true, false, 0>(v, lds, tw, lane);
    stockham_pass<R, M, 2, 2, S, false, false, 1>(v, lds, tw, lane);
    stockham_pass<R, M, 2, 4, S, false, false, 2>(v, lds, tw, lane);
    stockham_pass<R, M, 2, 8, S, false, false, 3>(v, lds, tw, lane);
    stockham_pass<R, M, 2, 16, S, false, false, 4>(v, lds, tw, lane);
    stockham_pass<R, M, 2, 32, S, false, false, 5>(v, lds, tw, lane);
    stockham_pass<R, M, 2, 64, S, false, true, 6>(v, lds, tw, lane);
  }
}

// Number of XCDs (each with its own L2) on MI355X; workgroups are dispatched round-robin over
// them, so blockIdx % 8 names the XCD.
#define SWIFTCL_NXCD 8

// Real forward transform of length N = 2M by one wavefront.
// In: v[e] = (x[2j], x[2j+1]), j = lane + 64 e.  Out: v[e] = X_n = sum_m x_m e^{-2 pi i n m / N},
// n = lane + 64 e < M (X_0 is real).
template <typename R, int M>
__device__ __forceinline__ void wave_r2c(C2<R>* v, C2<R>* lds, const C2<R>* __restrict__ tw, int lane) {
  constexpr int RL = M / SWIFTCL_WAVE;
  wave_fft<R, M, -1>(v, lds, tw, lane);
#pragma unroll
  for (int e = 0; e < RL; ++e) lds[fft_idx<R, M, 2>(lane, SWIFTCL_WAVE * e)] = v[e];
  wave_sync();
#pragma unroll
  for (int e = 0; e < RL; ++e) {
    const int n = lane + SWIFTCL_WAVE * e;
    const C2<R> Zn = v[e];
    if (n == 0) {
      v[e] = mk<R>(Zn.x + Zn.y, (R)0);
    } else {
      const C2<R> Zm = cconj(lds[fft_idx<R, M, 2>(SWIFTCL_WAVE - lane, SWIFTCL_WAVE * (RL - 1 - e))]);
      const C2<R> A = cscale(cadd(Zn, Zm), (R)0.5);
      const C2<R> Bd = cscale(csub(Zn, Zm), (R)0.5);
      const C2<R> t2 = cmul(tw[n], Bd);
      v[e] = mk<R>(A.x + t2.y, A.y - t2.x);  // A - i w^n Bd
    }
  }
  wave_sync();
}

// Real inverse transform of length N = 2M by one wavefront, from the half spectrum with the
// Nyquist term dropped: x_m = Re X_0 + 2 Re sum_{n=1}^{M-1} X_n e^{+2 pi i n m / N}.
// In: v[e] = X_n, n = lane + 64 e (only Re X_0 is used).  Out: v[e] = (x[2j], x[2j+1]).
template <typename R, int M>
__device__ __forceinline__ void wave_c2r(C2<R>* v, C2<R>* lds, const C2<R>* __restrict__ tw, int lane) {
  constexpr int RL = M / SWIFTCL_WAVE;
#pragma unroll
  for (int e = 0; e < RL; ++e) lds[fft_idx<R, M, 2>(lane, SWIFTCL_WAVE * e)] = v[e];
  wave_sync();
#pragma unroll
  for (int e = 0; e < RL; ++e) {
    const int n = lane + SWIFTCL_WAVE * e;
    if (n == 0) {
      v[e] = mk<R>(v[e].x, v[e].x);  // X_0 (1 + i)
    } else {
      const C2<R> Xm = cconj(lds[fft_idx<R, M, 2>(SWIFTCL_WAVE - lane, SWIFTCL_WAVE * (RL - 1 - e))]);  // X_{n+M} = conj(X_{M-n})
      const C2<R> A = cadd(v[e], Xm);
      const C2<R> Bd = csub(v[e], Xm);
      const C2<R> t2 = cmul(cconj(tw[n]), Bd);
      v[e] = mk<R>(A.x - t2.y, A.y + t2.x);  // A + i e^{2 pi i n / N} Bd
    }
  }
  wave_sync();
  wave_fft<R, M, +1>(v, lds, tw, lane);
}
