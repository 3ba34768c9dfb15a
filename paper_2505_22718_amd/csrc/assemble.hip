// Radial-kernel assembly on the log-chi grid, in FP64 (the geometry and the lensing
// integral keep double precision; only the FFT input is rounded to the FFT type).
//
//   clustering (Sec. 2.2):  f = b n(z) (dz/dchi) D(z)
//   lensing    (Sec. 2.3, eq. tomographic lens efficiency written in z):
//              f = q D / chi^2,  q = 1.5 Om (H0/c)^2 chi (1+z) [I0(z) - chi I1(z)],
//              I0 = int_z^zmax n dz',  I1 = int_z^zmax n / chi(z') dz'
//   CMB lensing (Sec. 2.4): f = 1.5 Om (H0/c)^2 (1+z) (chi_* - chi) / (chi chi_*) D, chi_* the top of
//              the geometry grid; its last node takes the linear-end weight 1/2 + theta/2
// Sampled inputs are continued by natural cubic splines; z(chi) inverts the chi(z) spline.
// Output g[b][t][band][m] = w_m f(chi_m) exp(-b_band m Delta) on chi_m = chi_0 e^{m Delta},
// with w = 1/2 on the lower support edge (node m0), 1/2 + theta on the last node m1 and zero
// outside [m0, m1]: the DFT of g is then the trapezoid rule of the cut kernel.
//
// One workgroup of GEOM_THREADS threads owns one parameter point and keeps all of its samples in LDS:
// every spline is solved by one wavefront (the Thomas recurrences as parallel affine-map scans),
// and the threads assemble g of the clustering tracers node by node; the lensing tracers follow
// in k_geom_lens (one workgroup each: interval integrals, suffix scans, q at every node).
#include "common.h"
#include "geometry.h"
#include "internal.h"

// tracers whose n(z) rows sit in LDS at once
#define GEOM_GROUP 16
// threads per point: two chi nodes of state per thread (n_chi <= 2048) fit 128 VGPRs without
// spilling, and the n(z) splines of up to 16 tracers run in one round of wavefronts
#define GEOM_THREADS 1024

size_t geometry_lds_bytes(const plan_dev& p) {
  const size_t tg = p.max_tracers < GEOM_GROUP ? p.max_tracers : GEOM_GROUP;
  return sizeof(double) * ((size_t)7 * p.n_zg + (size_t)3 * p.n_zs + (size_t)2 * tg * p.n_zs);
}

template <typename R>
__global__ __launch_bounds__(GEOM_THREADS) void k_geometry(plan_dev P, swiftcl_inputs in) {
  extern __shared__ double sh[];
  const int b = blockIdx.x;
  if (b >= in.batch) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int wave = tid / SWIFTCL_WAVE, lane = tid % SWIFTCL_WAVE, nw = nth / SWIFTCL_WAVE;
  const int T = P.max_tracers, nzg = P.n_zg, nzs = P.n_zs, nb = P.n_bands, N = P.N, nu = P.n_union;
  int Tb = in.n_tracers[b];
  if (Tb < 1 || Tb > T) {
    if (tid == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
    Tb = Tb < 1 ? 0 : T;
  }
  // LDS layout
  double* zg = sh;                      // [nzg] geometry grid
  double* zgih = zg + nzg;              // [nzg] 1/h
  double* chi = zgih + nzg;             // [nzg]
  double* mchi = chi + nzg;             // [nzg]
  double* Dz = mchi + nzg;              // [nzg]
  double* mD = Dz + nzg;                // [nzg]
  double* zs = mD + nzg;                // [nzs] n(z) grid
  double* zsih = zs + nzs;              // [nzs]
  const int TG = T < GEOM_GROUP ? T : GEOM_GROUP;
  double* nzr = zsih + 2 * (size_t)nzs; // [TG][nzs] n(z) rows of the current tracer group (one spare row of
                                        // nzs before it keeps the layout simple)
  double* mn = nzr + (size_t)TG * nzs;  // [TG][nzs]
  double* mia = mn + (size_t)TG * nzs;  // [nzg] spline moments of A_IA(z), if given

  const double* chig = in.chi_z + (size_t)b * nzg;
  const double* Dg = in.D_z + (size_t)b * nzg;
  for (int i = tid; i < nzg; i += nth) {
    zg[i] = P.z_geom[i];
    zgih[i] = P.lu_geom[3 * nzg + i];
    chi[i] = chig[i];
    Dz[i] = Dg[i];
  }
  for (int i = tid; i < nzs; i += nth) {
    zs[i] = P.z_nz[i];
    zsih[i] = P.lu_nz[3 * nzs + i];
  }
  __syncthreads();

  // splines of chi(z), D(z) and A_IA(z), one wavefront each
  const double* iag = in.ia ? in.ia + (size_t)b * nzg : nullptr;
  if (wave == 0) wave_spline(chi, P.lu_geom, nzg, mchi, lane);
  else if (wave == 1) wave_spline(Dz, P.lu_geom, nzg, mD, lane);
  else if (wave == 2 && iag) {
    bool bad = false;
    for (int i = lane; i < nzg; i += SWIFTCL_WAVE) bad |= !isfinite(iag[i]);
    if (bad) atomicOr(P.flags, FLAG_NONFINITE);
    wave_spline(iag, P.lu_geom, nzg, mia, lane);
  }
  __syncthreads();
  // keep the spline coefficients for the lensing kernels and the adjoint
  for (int i = tid; i < nzg; i += nth) {
    P.m_chi[(size_t)b * nzg + i] = mchi[i];
    P.m_D[(size_t)b * nzg + i] = mD[i];
    if (iag) P.m_ia[(size_t)b * nzg + i] = mia[i];
  }

  // per-point scalars
  const double chi_min = chi[0], chi_max = chi[nzg - 1];
  const double chi0 = chi_min * exp(-(double)P.m0 * P.delta);
  const double lchi0 = log(chi0);
  const double u_hi = log(chi_max / chi0) / P.delta;
  double m1d = floor(u_hi), theta = u_hi - m1d;
  int flag = 0;
  if (!(chi_min > 0.0) || !(chi_max > chi_min) || !isfinite(u_hi)) {
    flag = FLAG_NONFINITE;
    m1d = P.m0;
    theta = 0.0;
  } else if (m1d > N - 2) {
    flag = FLAG_SUPPORT_OVERFLOW;
    m1d = N - 2;
    theta = 0.0;
  }
  const int m0 = P.m0, m1 = (int)m1d;
  {
    // FFTLog phase of every coefficient, shared by all tracers and bands of the point
    const double dphi = -2.0 * M_PI * (log(P.k0) + lchi0) / ((double)N * P.delta);
    double2* ph = (double2*)P.phase + (size_t)b * (N / 2);
    for (int n = tid; n < N / 2; n += nth) {
      double sn, cs;
      sincos(dphi * (double)n, &sn, &cs);
      ph[n] = make_double2(cs, sn);
    }
  }
  if (tid == 0) {
    if (flag) atomicOr(P.flags, flag);
    double* pt = P.pt + (size_t)b * PT_STRIDE;
    pt[PT_CHI0] = chi0;
    pt[PT_LNK0CHI0] = log(P.k0) + lchi0;
    pt[PT_M1] = m1d;
    pt[PT_THETA] = theta;
    for (int kind = 0; kind < SWIFTCL_NKINDS; ++kind)
      for (int bi = 0; bi < SWIFTCL_MAX_BANDS; ++bi)
        pt[PT_CHI0B + kind * SWIFTCL_MAX_BANDS + bi] = exp(-P.fftlog_b[kind][bi] * lchi0);
  }

  // node state: each thread owns nodes m = tid + k * nth
  constexpr int MAXN = 2048 / GEOM_THREADS;  // n_chi <= 2048 (checked at plan time)
  node_state ns[MAXN];
  R* g = (R*)P.g;
#pragma unroll
  for (int k = 0; k < MAXN; ++k) {
    const int m = tid + k * nth;
    ns[k].active = false;
    if (m >= N) continue;
    if (m < m0 || m > m1) {
      for (int t = 0; t < T; ++t)
        for (int bi = 0; bi < nb; ++bi) {
          g[(((size_t)b * T + t) * nb + bi) * N + m] = (R)0;
          if (P.rsd) ((R*)P.g_r)[(((size_t)b * T + t) * nb + bi) * N + m] = (R)0;
          if (P.mag) ((R*)P.g_mu)[(((size_t)b * T + t) * nb + bi) * N + m] = (R)0;
        }
      continue;
    }
    ns[k].active = true;
    locate_node(ns[k], m, m0, m1, theta, chi0, P.delta, zg, zgih, chi, mchi, Dz, mD, nzg, zs, nzs, P.z_union, nu,
                P.union_iv);
    // the node geometry, for the adjoint
    double* nf = P.node_f + (size_t)b * 4 * N + m;
    int* ni = P.node_i + (size_t)b * 3 * N + m;
    nf[0] = ns[k].z;
    nf[N] = ns[k].chiz;
    nf[2 * N] = ns[k].dchi;
    nf[3 * N] = ns[k].D;
    ni[0] = ns[k].ig;
    ni[N] = ns[k].inz;
    ni[2 * N] = ns[k].u;
  }
  for (int g0 = 0; g0 < T; g0 += TG) {
  const int g1 = min(g0 + TG, T);
  // n(z) rows and their splines for tracers [g0, g1) of this point
  for (int i = tid; i < (g1 - g0) * nzs; i += nth) {
    const int tt = g0 + i / nzs;
    nzr[i] = tt < Tb ? in.nz[((size_t)b * T + g0) * nzs + i] : 0.0;
  }
  __syncthreads();
  for (int c = wave; c < min(g1, Tb) - g0; c += nw)
    wave_spline(nzr + (size_t)c * nzs, P.lu_nz, nzs, mn + (size_t)c * nzs, lane);
  __syncthreads();
  for (int i = tid; i < (min(g1, Tb) - g0) * nzs; i += nth) P.m_n[((size_t)b * T + g0) * nzs + i] = mn[i];
  // clustering and CMB-lensing tracers, tracers of an unknown kind and padded slots
  const double pref = 1.5 * in.omega_m[b] * SWIFTCL_H0_OVER_C * SWIFTCL_H0_OVER_C;
  const double chis = chi[nzg - 1];  // chi_* of the CMB-lensing kernel: the top of the geometry grid
#pragma unroll
  for (int k = 0; k < MAXN; ++k) {
    if (!ns[k].active) continue;
    const int m = tid + k * nth;
    // RSD (eq. RSD): -f(z) n dz/dchi D with f = dln D/dln a = -(1+z) D'/D, i.e. (1+z) D' n / (dchi/dz)
    double dD = 0.0;
    if (P.rsd) (void)spline_at(zg, zgih, Dz, mD, ns[k].ig, ns[k].z, &dD);
    for (int t = g0; t < g1; ++t) {
      const int kd = t < Tb ? in.kind[(size_t)b * T + t] : -1;  // -1: padded slot
      if (kd == SWIFTCL_LENSING) {
        for (int bi = 0; bi < nb; ++bi) {
          if (P.rsd) ((R*)P.g_r)[(((size_t)b * T + t) * nb + bi) * N + m] = (R)0;
          if (P.mag) ((R*)P.g_mu)[(((size_t)b * T + t) * nb + bi) * N + m] = (R)0;
        }
        continue;
      }
      const bool known = kd == SWIFTCL_CLUSTERING || kd == SWIFTCL_CMB_LENSING;
      if (t < Tb && !known && m == m0) atomicOr(P.flags, FLAG_BAD_INDEX);  // its samples stay zero
      // (the magnification samples of clustering tracers come from k_geom_lens)
      if (kd != SWIFTCL_CLUSTERING && P.mag)
        for (int bi = 0; bi < nb; ++bi) ((R*)P.g_mu)[(((size_t)b * T + t) * nb + bi) * N + m] = (R)0;
      double f = 0.0, fr = 0.0, w = ns[k].w;
      if (kd == SWIFTCL_CLUSTERING) {
        const double n = ns[k].inz < 0 ? 0.0
                         : spline_at(zs, zsih, nzr + (size_t)(t - g0) * nzs, mn + (size_t)(t - g0) * nzs, ns[k].inz,
                                     ns[k].z, nullptr);
        f = in.bias[(size_t)b * T + t] * n * ns[k].D / ns[k].dchi;
        fr = (1.0 + ns[k].z) * dD * n / ns[k].dchi;
      } else if (kd == SWIFTCL_CMB_LENSING) {
        // Sec. 2.4: one source plane at chi_*; the kernel falls linearly to zero there, so the last
        // node takes the trapezoid weight of a linear end, 1/2 + theta/2
        const double x = ns[k].chiz;
        f = pref * (1.0 + ns[k].z) * (chis - x) / (x * chis) * ns[k].D;
        if (m == m1 && m1 > m0) w = 0.5 + 0.5 * theta;
      }
      const int kc = known ? kd : SWIFTCL_CLUSTERING;
      for (int bi = 0; bi < nb; ++bi) {
        g[(((size_t)b * T + t) * nb + bi) * N + m] = (R)(w * f * P.ebm[((size_t)kc * nb + bi) * N + m]);
        if (P.rsd)
          ((R*)P.g_r)[(((size_t)b * T + t) * nb + bi) * N + m] = (R)(w * fr * P.ebm[(size_t)bi * N + m]);
      }
    }
  }
  // (lensing tracers: k_geom_lens, one workgroup per (point, tracer))
  __syncthreads();
  }  // tracer groups
}

size_t lens_lds_bytes(const plan_dev& p) {
  return sizeof(double) * ((size_t)4 * p.n_zs + (size_t)2 * p.n_union + 64);
}

// Lensing tracers (Sec. 2.3, eq. tomographic lens efficiency): one workgroup of 512 threads per
// (point, tracer), idle for clustering and padded slots.  The interval integrals of n and n/chi
// over the union of the z grids, their suffix sums (block scans), then q and g at every active
// node; the node geometry and the n(z) spline moments come from k_geometry.
template <typename R>
__global__ __launch_bounds__(512) void k_geom_lens(plan_dev P, swiftcl_inputs in) {
  extern __shared__ double sh[];
  const int T = P.max_tracers;
  const int b = blockIdx.x / T, t = blockIdx.x % T;
  if (b >= in.batch) return;
  const int Tb = in.n_tracers[b] < T ? in.n_tracers[b] : T;
  if (t >= Tb) return;
  // lensing tracers, and clustering tracers whose magnification needs their own lens efficiency
  const int kd = in.kind[(size_t)b * T + t];
  const bool lensing = kd == SWIFTCL_LENSING;
  if (!lensing && !(kd == SWIFTCL_CLUSTERING && P.mag && in.mag)) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nzg = P.n_zg, nzs = P.n_zs, nb = P.n_bands, N = P.N, nu = P.n_union;
  // the read-only grids (z, 1/h, chi and its spline moments) are read through the cache: LDS holds
  // this tracer's rows and the interval sums (~27 KB)
  const double* zg = P.z_geom;                          // [nzg]
  const double* zgih = P.lu_geom + 3 * (size_t)nzg;     // [nzg]
  const double* chi = in.chi_z + (size_t)b * nzg;       // [nzg]
  const double* mchi = P.m_chi + (size_t)b * nzg;       // [nzg]
  double* zs = sh;              // [nzs]
  double* zsih = zs + nzs;      // [nzs]
  double* nt = zsih + nzs;      // [nzs] this tracer's n samples
  double* mt = nt + nzs;        // [nzs] and their spline moments
  double* seg0 = mt + nzs;      // [nu]
  double* seg1 = seg0 + nu;     // [nu]
  double* tmp = seg1 + nu;      // [64]
  for (int i = tid; i < nzs; i += nth) {
    zs[i] = P.z_nz[i];
    zsih[i] = P.lu_nz[3 * nzs + i];
    nt[i] = in.nz[((size_t)b * T + t) * nzs + i];
    mt[i] = P.m_n[((size_t)b * T + t) * nzs + i];
  }
  __syncthreads();
  for (int u = tid; u < nu; u += nth) {
    double s0, s1;
    lens_interval(P.z_union[u], P.z_union[u + 1], P.union_iv[u], P.union_iv[nu + u], zg, zgih, chi, mchi, zs, zsih,
                  nt, mt, &s0, &s1);
    seg0[u] = s0;
    seg1[u] = s1;
  }
  __syncthreads();
  block_scan(seg0, nu, tmp, false);
  block_scan(seg1, nu, tmp, false);
  const double* pt = P.pt + (size_t)b * PT_STRIDE;
  const double theta = pt[PT_THETA];
  const int m0 = P.m0, m1 = (int)pt[PT_M1];
  const double pref = 1.5 * in.omega_m[b] * SWIFTCL_H0_OVER_C * SWIFTCL_H0_OVER_C;
  R* g = (R*)P.g;
  for (int m = m0 + tid; m <= m1; m += nth) {
    const double* nf = P.node_f + (size_t)b * 4 * N + m;
    const int* ni = P.node_i + (size_t)b * 3 * N + m;
    const double z = nf[0], x = nf[N], D = nf[3 * N];
    const int u = ni[2 * N];
    const double w = (m == m0) ? 0.5 : (m == m1 ? 0.5 + theta : 1.0);
    double p0, p1;
    lens_interval(z, P.z_union[u + 1], P.union_iv[u], P.union_iv[nu + u], zg, zgih, chi, mchi, zs, zsih, nt, mt, &p0,
                  &p1);
    const double I0 = p0 + (u + 1 < nu ? seg0[u + 1] : 0.0);
    const double I1 = p1 + (u + 1 < nu ? seg1[u + 1] : 0.0);
    const double q = pref * x * (1.0 + z) * (I0 - x * I1);
    if (!lensing) {
      // magnification (eq. magnification bias): C_g q D / chi^2, tilted with the bias b - 2
      const double fm = in.mag[(size_t)b * T + t] * q * D / (x * x);
      const double e2 = exp(2.0 * (double)m * P.delta);
      for (int bi = 0; bi < nb; ++bi)
        ((R*)P.g_mu)[(((size_t)b * T + t) * nb + bi) * N + m] = (R)(w * fm * P.ebm[(size_t)bi * N + m] * e2);
      continue;
    }
    P.lens_q[((size_t)b * T + t) * N + m] = q;  // for the adjoint
    double fq = q;
    if (in.ia) {
      // intrinsic alignment (NLA): n(chi) A_IA(z) joins the lens efficiency
      const int ig = ni[0], inz = ni[N];
      const double a = spline_at(zg, zgih, in.ia + (size_t)b * nzg, P.m_ia + (size_t)b * nzg, ig, z, nullptr);
      const double n = inz < 0 ? 0.0 : spline_at(zs, zsih, nt, mt, inz, z, nullptr);
      fq += a * n / nf[2 * N];
    }
    const double fv = fq * D / (x * x);
    for (int bi = 0; bi < nb; ++bi)
      g[(((size_t)b * T + t) * nb + bi) * N + m] = (R)(w * fv * P.ebm[((size_t)nb + bi) * N + m]);
  }
}

// Kernel samples given by the caller (inputs.kernel_chi): the per-point scalars from chi(z_min) alone
// (chi_0, the FFTLog phases and chi_0^{-b}), then g = f(chi_m) e^{-b m Delta} on every node, no support
// cut and no edge weights.  One workgroup per point.
template <typename R>
__global__ __launch_bounds__(256) void k_kernel_samples(plan_dev P, swiftcl_inputs in) {
  const int b = blockIdx.x;
  if (b >= in.batch) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int T = P.max_tracers, nb = P.n_bands, N = P.N;
  int Tb = in.n_tracers[b];
  if (Tb < 1 || Tb > T) {
    if (tid == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
    Tb = Tb < 1 ? 0 : T;
  }
  const double chi_min = in.chi_z[(size_t)b * P.n_zg];
  const bool okchi = chi_min > 0.0 && isfinite(chi_min);
  const double chi0 = okchi ? chi_min * exp(-(double)P.m0 * P.delta) : 1.0;
  const double lchi0 = log(chi0);
  const double dphi = -2.0 * M_PI * (log(P.k0) + lchi0) / ((double)N * P.delta);
  double2* ph = (double2*)P.phase + (size_t)b * (N / 2);
  for (int n = tid; n < N / 2; n += nth) {
    double sn, cs;
    sincos(dphi * (double)n, &sn, &cs);
    ph[n] = make_double2(cs, sn);
  }
  if (tid == 0) {
    if (!okchi) atomicOr(P.flags, FLAG_NONFINITE);
    double* pt = P.pt + (size_t)b * PT_STRIDE;
    pt[PT_CHI0] = chi0;
    pt[PT_LNK0CHI0] = log(P.k0) + lchi0;
    pt[PT_M1] = (double)(N - 1);
    pt[PT_THETA] = 0.0;
    for (int kind = 0; kind < SWIFTCL_NKINDS; ++kind)
      for (int bi = 0; bi < SWIFTCL_MAX_BANDS; ++bi)
        pt[PT_CHI0B + kind * SWIFTCL_MAX_BANDS + bi] = exp(-P.fftlog_b[kind][bi] * lchi0);
  }
  R* g = (R*)P.g;
  bool bad = false;
  for (int t = 0; t < T; ++t) {
    const int kd = t < Tb ? in.kind[(size_t)b * T + t] : -1;
    const bool known = kd >= 0 && kd < SWIFTCL_NKINDS;
    if (t < Tb && !known && tid == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
    const double* src = in.kernel_chi + ((size_t)b * T + t) * N;
    for (int m = tid; m < N; m += nth) {
      double f = 0.0;
      if (known) {
        f = src[m];
        if (!isfinite(f)) {
          bad = true;
          f = 0.0;
        }
      }
      for (int bi = 0; bi < nb; ++bi)
        g[(((size_t)b * T + t) * nb + bi) * N + m] = (R)(f * P.ebm[((size_t)(known ? kd : 0) * nb + bi) * N + m]);
    }
  }
  if (bad) atomicOr(P.flags, FLAG_NONFINITE);
}

hipError_t launch_assemble(const plan_dev& p, const swiftcl_inputs* in, hipStream_t s) {
  if (in->kernel_chi) {
    if (p.precision == SWIFTCL_FP64) hipLaunchKernelGGL(k_kernel_samples<double>, dim3(in->batch), dim3(256), 0, s, p, *in);
    else hipLaunchKernelGGL(k_kernel_samples<float>, dim3(in->batch), dim3(256), 0, s, p, *in);
    return hipGetLastError();
  }
  const size_t lds = geometry_lds_bytes(p), ll = lens_lds_bytes(p);
  const dim3 gl((unsigned)((size_t)in->batch * p.max_tracers));
  if (p.precision == SWIFTCL_FP64) {
    hipLaunchKernelGGL(k_geometry<double>, dim3(in->batch), dim3(GEOM_THREADS), lds, s, p, *in);
    hipLaunchKernelGGL(k_geom_lens<double>, gl, dim3(512), ll, s, p, *in);
  } else {
    hipLaunchKernelGGL(k_geometry<float>, dim3(in->batch), dim3(GEOM_THREADS), lds, s, p, *in);
    hipLaunchKernelGGL(k_geom_lens<float>, gl, dim3(512), ll, s, p, *in);
  }
  return hipGetLastError();
}
