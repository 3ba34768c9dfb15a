// FP64 device helpers of the geometry stage, shared by the forward assembly and its adjoint:
// natural-spline evaluation, interval search, the per-node state (z, D, dchi/dz, weights) and
// the 12-point Gauss-Legendre integrals of n and n/chi over one sub-interval.
#pragma once

#include "common.h"

#define SWIFTCL_H0_OVER_C (1.0 / 2997.92458)

__constant__ static const double c_gl12_x[12] = {
    -0.9815606342467192, -0.9041172563704748, -0.7699026741943047, -0.5873179542866175,
    -0.3678314989981802, -0.1252334085114689, 0.1252334085114689,  0.3678314989981802,
    0.5873179542866175,  0.7699026741943047,  0.9041172563704748,  0.9815606342467192};
__constant__ static const double c_gl12_w[12] = {
    0.04717533638651202, 0.10693932599531888, 0.1600783285433461,  0.20316742672306565,
    0.23349253653835464, 0.2491470458134027,  0.2491470458134027,  0.23349253653835464,
    0.20316742672306565, 0.1600783285433461,  0.10693932599531888, 0.04717533638651202};

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

__device__ __forceinline__ void locate_node(node_state& s, int m, int m0, int m1, double theta, double chi0,
                                            double delta, const double* zg, const double* zgih, const double* chi,
                                            const double* mchi, const double* Dz, const double* mD, int nzg,
                                            const double* zs, int nzs, const double* __restrict__ z_union, int nu,
                                            const int* __restrict__ union_iv) {
  double z;
  int ig;
  if (m == m0) {
    z = zg[0];  // the lower support edge sits on node m0 by construction
    ig = 0;
  } else {
    const double target = fmin(chi0 * exp((double)m * delta), chi[nzg - 1]);
    ig = find_interval(chi, nzg, target);
    const double za = zg[ig], zb = zg[ig + 1];
    z = za + (target - chi[ig]) / (chi[ig + 1] - chi[ig]) * (zb - za);
    for (int it = 0; it < 6; ++it) {
      double d;
      const double v = spline_at(zg, zgih, chi, mchi, ig, z, &d);
      z -= (v - target) / d;
      z = fmin(fmax(z, za), zb);
    }
  }
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

// int_a^c n dz and int_a^c n / chi dz on one union sub-interval (12-point Gauss-Legendre);
// ig / iv: geometry and n(z) intervals of the sub-interval (iv < 0: n = 0 there).
__device__ __forceinline__ void lens_interval(double a, double c, int ig, int iv, const double* zg, const double* zgih,
                                              const double* chi, const double* mchi, const double* zs,
                                              const double* zsih, const double* nt, const double* mt, double* s0,
                                              double* s1) {
  double r0 = 0.0, r1 = 0.0;
  if (iv >= 0) {
    for (int q = 0; q < 12; ++q) {
      const double z = 0.5 * (c - a) * c_gl12_x[q] + 0.5 * (a + c);
      const double w = 0.5 * (c - a) * c_gl12_w[q];
      const double n = spline_at(zs, zsih, nt, mt, iv, z, nullptr);
      const double x = spline_at(zg, zgih, chi, mchi, ig, z, nullptr);
      r0 += w * n;
      r1 += w * n / x;
    }
  }
  *s0 = r0;
  *s1 = r1;
}
