// Radial-kernel assembly on the log-chi grid, in FP64 (the geometry and the lensing
// integral keep double precision; only the FFT input is rounded to the FFT type).
//
//   clustering (Sec. 2.2):  f = b n(z) (dz/dchi) D(z)
//   lensing    (Sec. 2.3, eq. tomographic lens efficiency written in z):
//              f = q D / chi^2,  q = 1.5 Om (H0/c)^2 chi (1+z) [I0(z) - chi I1(z)],
//              I0 = int_z^zmax n dz',  I1 = int_z^zmax n / chi(z') dz'
// Sampled inputs are continued by natural cubic splines; z(chi) inverts the chi(z) spline.
// Output g[b][t][band][m] = w_m f(chi_m) exp(-b_band m Delta) on chi_m = chi_0 e^{m Delta},
// with w = 1/2 on the lower support edge (node m0), 1/2 + theta on the last node m1 and zero
// outside [m0, m1]: the DFT of g is then the trapezoid rule of the cut kernel.
#include "common.h"
#include "internal.h"

#define H0_OVER_C (1.0 / 2997.92458)

__constant__ double c_gl12_x[12] = {-0.9815606342467192, -0.9041172563704748, -0.7699026741943047,
                                    -0.5873179542866175, -0.3678314989981802, -0.1252334085114689,
                                    0.1252334085114689,  0.3678314989981802,  0.5873179542866175,
                                    0.7699026741943047,  0.9041172563704748,  0.9815606342467192};
__constant__ double c_gl12_w[12] = {0.04717533638651202, 0.10693932599531888, 0.1600783285433461,
                                    0.20316742672306565, 0.23349253653835464, 0.2491470458134027,
                                    0.2491470458134027,  0.23349253653835464, 0.20316742672306565,
                                    0.1600783285433461,  0.10693932599531888, 0.04717533638651202};

// Natural cubic spline second derivatives with the grid's Thomas factors (a, inv, c').
__device__ void natural_spline(const double* __restrict__ x, const double* __restrict__ y, int n,
                               const double* __restrict__ lu, double* __restrict__ Mo) {
  const double* a = lu;
  const double* inv = lu + n;
  const double* cp = lu + 2 * n;
  Mo[0] = 0.0;
  Mo[n - 1] = 0.0;
  double prev = 0.0;
  for (int i = 1; i < n - 1; ++i) {
    const double r = (y[i + 1] - y[i]) / (x[i + 1] - x[i]) - (y[i] - y[i - 1]) / (x[i] - x[i - 1]);
    prev = (r - a[i] * prev) * inv[i];
    Mo[i] = prev;
  }
  for (int i = n - 3; i >= 1; --i) Mo[i] -= cp[i] * Mo[i + 1];
}

// value (and derivative) of the spline on interval i at z
__device__ __forceinline__ double spline_at(const double* __restrict__ x, const double* __restrict__ y,
                                            const double* __restrict__ Mv, int i, double z, double* deriv) {
  const double h = x[i + 1] - x[i];
  const double A = (x[i + 1] - z) / h;
  const double B = (z - x[i]) / h;
  const double v = A * y[i] + B * y[i + 1] + ((A * A * A - A) * Mv[i] + (B * B * B - B) * Mv[i + 1]) * h * h / 6.0;
  if (deriv)
    *deriv = (y[i + 1] - y[i]) / h + (-(3.0 * A * A - 1.0) * Mv[i] + (3.0 * B * B - 1.0) * Mv[i + 1]) * h / 6.0;
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

__global__ void k_spline_setup(plan_dev P, swiftcl_inputs in) {
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  if (b >= in.batch) return;
  const int nzg = P.n_zg, nzs = P.n_zs, T = P.max_tracers;
  int Tb = in.n_tracers[b];
  if (Tb < 1 || Tb > T) {
    if (t == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
    Tb = Tb < 1 ? 0 : T;
  }
  const double* chi = in.chi_z + (size_t)b * nzg;
  if (t == 0) {
    natural_spline(P.z_geom, chi, nzg, P.lu_geom, P.m_chi + (size_t)b * nzg);
    double* pt = P.pt + (size_t)b * PT_STRIDE;
    const double chi_min = chi[0], chi_max = chi[nzg - 1];
    const double chi0 = chi_min * exp(-(double)P.m0 * P.delta);
    const double lchi0 = log(chi0);
    const double u_hi = log(chi_max / chi0) / P.delta;
    double m1 = floor(u_hi);
    double theta = u_hi - m1;
    if (!(chi_min > 0.0) || !(chi_max > chi_min) || !isfinite(u_hi)) {
      atomicOr(P.flags, FLAG_NONFINITE);
      m1 = P.m0;
      theta = 0.0;
    } else if (m1 > P.N - 2) {
      atomicOr(P.flags, FLAG_SUPPORT_OVERFLOW);
      m1 = P.N - 2;
      theta = 0.0;
    }
    pt[PT_CHI0] = chi0;
    pt[PT_LNK0CHI0] = log(P.k0) + lchi0;
    pt[PT_M1] = m1;
    pt[PT_THETA] = theta;
    for (int kind = 0; kind < 2; ++kind)
      for (int bi = 0; bi < SWIFTCL_MAX_BANDS; ++bi)
        pt[PT_CHI0B + kind * SWIFTCL_MAX_BANDS + bi] = exp(-P.fftlog_b[kind][bi] * lchi0);
  } else if (t == 1) {
    natural_spline(P.z_geom, in.D_z + (size_t)b * nzg, nzg, P.lu_geom, P.m_D + (size_t)b * nzg);
  } else if (t >= 2 && t - 2 < Tb) {
    const int tt = t - 2;
    natural_spline(P.z_nz, in.nz + ((size_t)b * T + tt) * nzs, nzs, P.lu_nz, P.m_n + ((size_t)b * T + tt) * nzs);
  }
}

// n_t(z) on a known n(z) interval (iv < 0: outside the sampled range, n = 0)
__device__ __forceinline__ double nz_at(const plan_dev& P, const double* nzrow, const double* mrow,
                                        int iv, double z) {
  if (iv < 0) return 0.0;
  return spline_at(P.z_nz, nzrow, mrow, iv, z, nullptr);
}

// Per lensing tracer: suffix sums over the union knot intervals of int n and int n/chi.
__global__ void k_lens_prefix(plan_dev P, swiftcl_inputs in) {
  extern __shared__ double seg[];  // [2][n_union]
  const int b = blockIdx.x, t = blockIdx.y;
  if (b >= in.batch) return;
  const int T = P.max_tracers;
  const int Tb = min(max(in.n_tracers[b], 0), T);
  if (t >= Tb || in.kind[(size_t)b * T + t] != SWIFTCL_LENSING) return;
  const int nu = P.n_union;
  const double* chi = in.chi_z + (size_t)b * P.n_zg;
  const double* mchi = P.m_chi + (size_t)b * P.n_zg;
  const double* nzrow = in.nz + ((size_t)b * T + t) * P.n_zs;
  const double* mrow = P.m_n + ((size_t)b * T + t) * P.n_zs;
  for (int u = threadIdx.x; u < nu; u += blockDim.x) {
    const double a = P.z_union[u], c = P.z_union[u + 1];
    const int ig = P.union_iv[u], in_ = P.union_iv[nu + u];
    double s0 = 0.0, s1 = 0.0;
    for (int q = 0; q < 12; ++q) {
      const double z = 0.5 * (c - a) * c_gl12_x[q] + 0.5 * (a + c);
      const double w = 0.5 * (c - a) * c_gl12_w[q];
      const double n = nz_at(P, nzrow, mrow, in_, z);
      const double x = spline_at(P.z_geom, chi, mchi, ig, z, nullptr);
      s0 += w * n;
      s1 += w * n / x;
    }
    seg[u] = s0;
    seg[nu + u] = s1;
  }
  __syncthreads();
  double* suf = P.lens_suf + ((size_t)b * T + t) * 2 * (nu + 1);
  if (threadIdx.x < 2) {
    const int which = threadIdx.x;
    double acc = 0.0;
    suf[which * (nu + 1) + nu] = 0.0;
    for (int u = nu - 1; u >= 0; --u) {
      acc += seg[which * nu + u];
      suf[which * (nu + 1) + u] = acc;
    }
  }
}

template <typename R>
__global__ void k_assemble(plan_dev P, swiftcl_inputs in) {
  const int b = blockIdx.y;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= in.batch || m >= P.N) return;
  const int T = P.max_tracers, nb = P.n_bands, N = P.N, nzg = P.n_zg;
  const int Tb = min(max(in.n_tracers[b], 0), T);
  const double* pt = P.pt + (size_t)b * PT_STRIDE;
  const int m0 = P.m0;
  const int m1 = (int)pt[PT_M1];
  R* g = (R*)P.g;
  if (m < m0 || m > m1) {
    for (int t = 0; t < T; ++t)
      for (int bi = 0; bi < nb; ++bi) g[(((size_t)b * T + t) * nb + bi) * N + m] = (R)0;
    return;
  }
  const double* chi = in.chi_z + (size_t)b * nzg;
  const double* mchi = P.m_chi + (size_t)b * nzg;
  double z;
  int ig;
  if (m == m0) {
    z = P.z_geom[0];
    ig = 0;
  } else {
    const double target = fmin(pt[PT_CHI0] * exp((double)m * P.delta), chi[nzg - 1]);
    ig = find_interval(chi, nzg, target);
    const double za = P.z_geom[ig], zb = P.z_geom[ig + 1];
    z = za + (target - chi[ig]) / (chi[ig + 1] - chi[ig]) * (zb - za);
    for (int it = 0; it < 8; ++it) {
      double d;
      const double v = spline_at(P.z_geom, chi, mchi, ig, z, &d);
      z -= (v - target) / d;
      z = fmin(fmax(z, za), zb);
    }
  }
  double dchi;
  const double chiz = spline_at(P.z_geom, chi, mchi, ig, z, &dchi);
  const double D = spline_at(P.z_geom, in.D_z + (size_t)b * nzg, P.m_D + (size_t)b * nzg, ig, z, nullptr);
  const bool in_nz = z >= P.z_nz[0] && z <= P.z_nz[P.n_zs - 1];
  const int inz = in_nz ? find_interval(P.z_nz, P.n_zs, z) : -1;
  double w = 1.0;
  if (m == m0) w = 0.5;
  else if (m == m1) w = 0.5 + pt[PT_THETA];
  // lensing: union interval holding z
  const int nu = P.n_union;
  int u = find_interval(P.z_union, nu + 1, z);
  u = min(u, nu - 1);
  const double zc = P.z_union[u + 1];
  const int ugi = P.union_iv[u], uni = P.union_iv[nu + u];
  const double om = in.omega_m[b];
  for (int t = 0; t < T; ++t) {
    double f = 0.0;
    if (t < Tb) {
      const double* nzrow = in.nz + ((size_t)b * T + t) * P.n_zs;
      const double* mrow = P.m_n + ((size_t)b * T + t) * P.n_zs;
      if (in.kind[(size_t)b * T + t] == SWIFTCL_CLUSTERING) {
        f = in.bias[(size_t)b * T + t] * nz_at(P, nzrow, mrow, inz, z) * D / dchi;
      } else {
        const double* suf = P.lens_suf + ((size_t)b * T + t) * 2 * (nu + 1);
        double p0 = 0.0, p1 = 0.0;
        for (int q = 0; q < 12; ++q) {
          const double zz = 0.5 * (zc - z) * c_gl12_x[q] + 0.5 * (zc + z);
          const double ww = 0.5 * (zc - z) * c_gl12_w[q];
          const double n = nz_at(P, nzrow, mrow, uni, zz);
          const double x = spline_at(P.z_geom, chi, mchi, ugi, zz, nullptr);
          p0 += ww * n;
          p1 += ww * n / x;
        }
        const double I0 = p0 + suf[u + 1];
        const double I1 = p1 + suf[(nu + 1) + u + 1];
        const double q = 1.5 * om * H0_OVER_C * H0_OVER_C * chiz * (1.0 + z) * (I0 - chiz * I1);
        f = q * D / (chiz * chiz);
      }
    }
    const int kind = (t < Tb) ? in.kind[(size_t)b * T + t] : 0;
    for (int bi = 0; bi < nb; ++bi) {
      const double tilt = exp(-P.fftlog_b[kind & 1][bi] * (double)m * P.delta);
      g[(((size_t)b * T + t) * nb + bi) * N + m] = (R)(w * f * tilt);
    }
  }
}

hipError_t launch_assemble(const plan_dev& pd, const swiftcl_inputs* in, hipStream_t s) {
  const plan_dev* p = &pd;
  const int B = in->batch;
  hipLaunchKernelGGL(k_spline_setup, dim3(B), dim3(64 * ((p->max_tracers + 2 + 63) / 64)), 0, s, pd, *in);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = 2 * sizeof(double) * (size_t)p->n_union;
  hipLaunchKernelGGL(k_lens_prefix, dim3(B, p->max_tracers), dim3(256), lds, s, pd, *in);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((p->N + 127) / 128, B);
  if (p->precision == SWIFTCL_FP64) hipLaunchKernelGGL(k_assemble<double>, grid, dim3(128), 0, s, pd, *in);
  else hipLaunchKernelGGL(k_assemble<float>, grid, dim3(128), 0, s, pd, *in);
  return hipGetLastError();
}
