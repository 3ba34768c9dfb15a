// FP64 device helpers of the geometry stage, shared by the forward assembly and its adjoint:
// natural-spline evaluation, interval search, the per-node state (z, D, dchi/dz, weights) and
// the Gauss-Legendre integrals of n and n/chi over one sub-interval.
#pragma once

#include "common.h"

#define SWIFTCL_H0_OVER_C (1.0 / 2997.92458)

// 6-point Gauss-Legendre nodes and weights on [-1, 1]: the lensing quadrature per interval of the
// union of the geometry and n(z) grids, where n is one cubic and 1/chi smooth (with 1024 geometry
// samples over 0.01 <= z <= 3 and 200 n(z) samples, q agrees with a 12-point rule to 3e-15 relative)
#define SWIFTCL_NGL 6
__constant__ static const double c_gl_x[SWIFTCL_NGL] = {
    -0.93246951420315205, -0.66120938646626448, -0.23861918608319693,
    0.23861918608319693, 0.66120938646626448, 0.93246951420315205};
__constant__ static const double c_gl_w[SWIFTCL_NGL] = {
    0.17132449237916975, 0.36076157304813894, 0.46791393457269137,
    0.46791393457269137, 0.36076157304813894, 0.17132449237916975};

// value (and derivative) of the natural spline on interval i at z; ih = 1/h per interval
__device__ __forceinline__ double spline_at(const double* __restrict__ x, const double* __restrict__ ih,
                                            const double* __restrict__ y, const double* __restrict__ Mv, int i,
                                            double z, double* deriv) {
  const double h = x[i + 1] - x[i];
  const double A = (x[i + 1] - z) * ih[i];
  const double B = (z - x[i]) * ih[i];
  const double v = A * y[i] + B * y[i + 1] + ((A * A * A - A) * Mv[i] + (B * B * B - B) * Mv[i + 1]) * (h * h / 6.0);
  if (deriv)
    *deriv = (y[i + 1] - y[i]) * ih[i] + (-(3.0 * A * A - 1.0) * Mv[i] + (3.0 * B * B - 1.0) * Mv[i + 1]) * (h / 6.0);
  return v;
}

// Weights of the natural-spline value on interval i at z: value = wa y_i + wb y_{i+1} + wc M_i +
// wd M_{i+1} (shared by every spline on the same knots).
struct spline_w {
  double wa, wb, wc, wd;
  __device__ __forceinline__ spline_w(const double* __restrict__ x, const double* __restrict__ ih, int i, double z) {
    const double h = x[i + 1] - x[i];
    wa = (x[i + 1] - z) * ih[i];
    wb = (z - x[i]) * ih[i];
    const double h6 = h * h / 6.0;
    wc = (wa * wa * wa - wa) * h6;
    wd = (wb * wb * wb - wb) * h6;
  }
  __device__ __forceinline__ double at(const double* __restrict__ y, const double* __restrict__ Mv, int i) const {
    return wa * y[i] + wb * y[i + 1] + wc * Mv[i] + wd * Mv[i + 1];
  }
};

// largest i in [0, n-2] with x[i] <= v
__device__ __forceinline__ int find_interval(const double* __restrict__ x, int n, double v) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// Everything the assembly (and its adjoint) needs at one chi node inside the support.
struct node_state {
  bool active;
  double z, chiz, dchi, D, w;
  int ig, inz;        // geometry and n(z) intervals holding z (inz < 0: outside the n(z) grid)
  int u, ugi, uni;    // lensing union interval, its geometry and n(z) intervals
  double zc;          // right end of the union interval
};

// z at chi node m: the lower support edge for m == m0, else the root of chi(z) = chi_0 e^{m Delta}
// on the geometry spline (Newton from the linear estimate, kept inside the interval); ig returns
// the geometry interval.
__device__ __forceinline__ double node_z(int m, int m0, double chi0, double delta, const double* zg,
                                         const double* zgih, const double* chi, const double* mchi, int nzg, int* ig_out) {
  if (m == m0) {
    *ig_out = 0;
    return zg[0];
  }
  const double target = fmin(chi0 * exp((double)m * delta), chi[nzg - 1]);
  const int ig = find_interval(chi, nzg, target);
  const double za = zg[ig], zb = zg[ig + 1];
  double z = za + (target - chi[ig]) / (chi[ig + 1] - chi[ig]) * (zb - za);
  for (int it = 0; it < 6; ++it) {
    double d;
    const double v = spline_at(zg, zgih, chi, mchi, ig, z, &d);
    z -= (v - target) / d;
    z = fmin(fmax(z, za), zb);
  }
  *ig_out = ig;
  return z;
}

// Everything else at a node from its z and geometry interval.
__device__ __forceinline__ void node_fill(node_state& s, double z, int ig, int m, int m0, int m1, double theta,
                                          const double* zg, const double* zgih, const double* chi, const double* mchi,
                                          const double* Dz, const double* mD, const double* zs, int nzs,
                                          const double* __restrict__ z_union, int nu, const int* __restrict__ union_iv) {
  s.z = z;
  s.ig = ig;
  s.chiz = spline_at(zg, zgih, chi, mchi, ig, z, &s.dchi);
  s.D = spline_at(zg, zgih, Dz, mD, ig, z, nullptr);
  s.inz = (z >= zs[0] && z <= zs[nzs - 1]) ? find_interval(zs, nzs, z) : -1;
  s.w = (m == m0) ? 0.5 : (m == m1 ? 0.5 + theta : 1.0);
  int u = find_interval(z_union, nu + 1, z);
  u = u < nu - 1 ? u : nu - 1;
  s.u = u;
  s.zc = z_union[u + 1];
  s.ugi = union_iv[u];
  s.uni = union_iv[nu + u];
}

__device__ __forceinline__ void locate_node(node_state& s, int m, int m0, int m1, double theta, double chi0,
                                            double delta, const double* zg, const double* zgih, const double* chi,
                                            const double* mchi, const double* Dz, const double* mD, int nzg,
                                            const double* zs, int nzs, const double* __restrict__ z_union, int nu,
                                            const int* __restrict__ union_iv) {
  int ig;
  const double z = node_z(m, m0, chi0, delta, zg, zgih, chi, mchi, nzg, &ig);
  node_fill(s, z, ig, m, m0, m1, theta, zg, zgih, chi, mchi, Dz, mD, zs, nzs, z_union, nu, union_iv);
}

// int_a^c n dz and int_a^c n / chi dz on one union sub-interval (Gauss-Legendre);
// ig / iv: geometry and n(z) intervals of the sub-interval (iv < 0: n = 0 there).
__device__ __forceinline__ void lens_interval(double a, double c, int ig, int iv, const double* zg, const double* zgih,
                                              const double* chi, const double* mchi, const double* zs,
                                              const double* zsih, const double* nt, const double* mt, double* s0,
                                              double* s1) {
  double r0 = 0.0, r1 = 0.0;
  if (iv >= 0) {
    for (int q = 0; q < SWIFTCL_NGL; ++q) {
      const double z = 0.5 * (c - a) * c_gl_x[q] + 0.5 * (a + c);
      const double w = 0.5 * (c - a) * c_gl_w[q];
      const double n = spline_at(zs, zsih, nt, mt, iv, z, nullptr);
      const double x = spline_at(zg, zgih, chi, mchi, ig, z, nullptr);
      r0 += w * n;
      r1 += w * n / x;
    }
  }
  *s0 = r0;
  *s1 = r1;
}

// Wavefront-parallel solve of the natural-spline tridiagonal system A z = rhs on the interior
// rows 1..n-2 (A is symmetric; Thomas factors a, 1/pivot, c' of the grid in lu).  x holds rhs on
// entry and z on exit (LDS); x[0] and x[n-1] are set to 0.  The two Thomas recurrences are
// affine maps y_i = alpha_i y_{i-1} + beta_i: every lane composes the maps of a contiguous chunk
// of rows, a shuffle scan composes the chunks, and every lane replays its chunk.
__device__ inline void wave_tridiag_solve(double* __restrict__ x, const double* __restrict__ lu, int n, int lane) {
  const double* a = lu;
  const double* inv = lu + n;
  const double* cp = lu + 2 * n;
  const int rows = n - 2;
  const int C = (rows + SWIFTCL_WAVE - 1) / SWIFTCL_WAVE;
  const int lo = 1 + lane * C;
  const int hi = min(1 + (lane + 1) * C, n - 1);
  double A = 1.0, B = 0.0;
  for (int i = lo; i < hi; ++i) {
    const double al = -a[i] * inv[i], be = x[i] * inv[i];
    A = al * A;
    B = al * B + be;
  }
  for (int off = 1; off < SWIFTCL_WAVE; off <<= 1) {
    const double Ap = __shfl_up(A, off), Bp = __shfl_up(B, off);
    if (lane >= off) { B = A * Bp + B; A = A * Ap; }
  }
  double prev = __shfl_up(B, 1);
  if (lane == 0) prev = 0.0;
  for (int i = lo; i < hi; ++i) {
    prev = (x[i] - a[i] * prev) * inv[i];
    x[i] = prev;
  }
  A = 1.0;
  B = 0.0;
  for (int i = hi - 1; i >= lo; --i) {
    const double g = -cp[i];
    A = g * A;
    B = g * B + x[i];
  }
  for (int off = 1; off < SWIFTCL_WAVE; off <<= 1) {
    const double Ap = __shfl_down(A, off), Bp = __shfl_down(B, off);
    if (lane + off < SWIFTCL_WAVE) { B = A * Bp + B; A = A * Ap; }
  }
  double next = __shfl_down(B, 1);
  if (lane == SWIFTCL_WAVE - 1) next = 0.0;
  for (int i = hi - 1; i >= lo; --i) {
    next = x[i] - cp[i] * next;
    x[i] = next;
  }
  if (lane == 0) { x[0] = 0.0; x[n - 1] = 0.0; }
}

// Natural cubic spline second derivatives Mo of samples y on the grid of lu (1/h in lu[3n..]).
__device__ inline void wave_spline(const double* __restrict__ y, const double* __restrict__ lu, int n,
                                   double* __restrict__ Mo, int lane) {
  const double* ih = lu + 3 * n;
  for (int i = 1 + lane; i < n - 1; i += SWIFTCL_WAVE)
    Mo[i] = (y[i + 1] - y[i]) * ih[i] - (y[i] - y[i - 1]) * ih[i - 1];
  wave_sync();
  wave_tridiag_solve(Mo, lu, n, lane);
  wave_sync();
}

// Adjoint of wave_spline plus evaluation: given dy (cotangent of the samples through the
// value terms) and dM (cotangent of the second derivatives), adds the contribution of dM to dy:
// dy += R^T A^{-1} dM, R the second-difference operator of the right-hand side.  dM is
// overwritten.
__device__ inline void wave_spline_adjoint(double* __restrict__ dy, double* __restrict__ dM,
                                           const double* __restrict__ lu, int n, int lane) {
  const double* ih = lu + 3 * n;
  wave_tridiag_solve(dM, lu, n, lane);
  wave_sync();
  // dy_j += ih_{j-1} z_{j-1} - (ih_j + ih_{j-1}) z_j + ih_j z_{j+1}, z_0 = z_{n-1} = 0
  for (int j = lane; j < n; j += SWIFTCL_WAVE) {
    double acc = 0.0;
    if (j >= 2) acc += ih[j - 1] * dM[j - 1];
    if (j >= 1 && j <= n - 2) acc -= (ih[j] + ih[j - 1]) * dM[j];
    if (j + 1 <= n - 2) acc += ih[j] * dM[j + 1];
    dy[j] += acc;
  }
  wave_sync();
}

// Cotangent of one spline value v = A y_i + B y_{i+1} + cA M_i + cB M_{i+1} (interval i, point z)
// accumulated into dy / dM with native LDS FP64 atomic adds (their order, hence the last bit of
// the sums, may vary from run to run).
__device__ __forceinline__ void spline_value_adjoint(const double* __restrict__ x, const double* __restrict__ ih,
                                                     int i, double z, double dv, double* dy, double* dM) {
  const double h = x[i + 1] - x[i];
  const double A = (x[i + 1] - z) * ih[i];
  const double B = (z - x[i]) * ih[i];
  unsafeAtomicAdd(&dy[i], A * dv);
  unsafeAtomicAdd(&dy[i + 1], B * dv);
  unsafeAtomicAdd(&dM[i], (A * A * A - A) * (h * h / 6.0) * dv);
  unsafeAtomicAdd(&dM[i + 1], (B * B * B - B) * (h * h / 6.0) * dv);
}

// The same four cotangent weights summed in registers over points of one interval i (z, dv),
// then added to LDS once: flush() after the last point.
struct spline_adj_acc {
  double y0 = 0.0, y1 = 0.0, m0 = 0.0, m1 = 0.0;
  __device__ __forceinline__ void add(const double* __restrict__ x, const double* __restrict__ ih, int i, double z,
                                      double dv) {
    const double A = (x[i + 1] - z) * ih[i];
    const double B = (z - x[i]) * ih[i];
    y0 += A * dv;
    y1 += B * dv;
    m0 += (A * A * A - A) * dv;
    m1 += (B * B * B - B) * dv;
  }
  __device__ __forceinline__ void flush(const double* __restrict__ x, int i, double* dy, double* dM) const {
    const double h = x[i + 1] - x[i];
    unsafeAtomicAdd(&dy[i], y0);
    unsafeAtomicAdd(&dy[i + 1], y1);
    unsafeAtomicAdd(&dM[i], m0 * (h * h / 6.0));
    unsafeAtomicAdd(&dM[i + 1], m1 * (h * h / 6.0));
  }
};

// In-place suffix sums x[u] <- sum_{v >= u} x[v] (prefix = false) or exclusive prefix sums
// x[u] <- sum_{v < u} x[v] (prefix = true) over n values in LDS, by the whole block.
// tmp: 2 * (blockDim / 64) doubles of LDS.
__device__ inline void block_scan(double* x, int n, double* tmp, bool prefix) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int wave = tid / SWIFTCL_WAVE, lane = tid % SWIFTCL_WAVE, nw = nth / SWIFTCL_WAVE;
  const int C = (n + nth - 1) / nth;
  // element of rank r (scan order) sits at idx(r)
  auto idx = [&](int r) { return prefix ? r : n - 1 - r; };
  double loc = 0.0;
  for (int k = 0; k < C; ++k) {
    const int r = tid * C + k;
    if (r < n) loc += x[idx(r)];
  }
  double incl = loc;
  for (int off = 1; off < SWIFTCL_WAVE; off <<= 1) {
    const double p = __shfl_up(incl, off);
    if (lane >= off) incl += p;
  }
  if (lane == SWIFTCL_WAVE - 1) tmp[wave] = incl;
  __syncthreads();
  if (tid == 0) {
    double acc = 0.0;
    for (int w = 0; w < nw; ++w) { tmp[nw + w] = acc; acc += tmp[w]; }
  }
  __syncthreads();
  double run = incl - loc + tmp[nw + wave];
  for (int k = 0; k < C; ++k) {
    const int r = tid * C + k;
    if (r < n) {
      const double v = x[idx(r)];
      if (prefix) { x[idx(r)] = run; run += v; }
      else { run += v; x[idx(r)] = run; }
    }
  }
  __syncthreads();
}
