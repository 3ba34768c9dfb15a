// The Limber limit (paper Sec. 2.6, eq. Limber): j_l(k chi) acts as a delta function at
// k = (l + 1/2) / chi, so for every multipole
//   C_l^{ij} = int dchi / chi^2 g_i(chi) g_j(chi) P((l + 1/2) / chi),   g = c(l, k) f,
// with c = 1 for clustering, F(l) / k^2 = F(l) chi^2 / (l + 1/2)^2 for lensing and l(l+1) chi^2 /
// (l + 1/2)^2 for CMB lensing (Sec. 2.4).  The integral
// runs on the log-chi nodes of the FFTLog path (dchi = chi dln chi), with the same edge weights:
//   C_l^{ij} = Delta sum_m w_m g_i(chi_m) g_j(chi_m) P((l + 1/2) / chi_m) / chi_m,
// P by the natural cubic spline of ln P in ln k (zero outside the k nodes).  The kernels come from
// the assembly (band 0 samples, untilted), so this is a cheap branch for high multipoles and a
// check of the FFTLog windows where the Limber error O(1/l) is small.
#include "common.h"
#include "geometry.h"
#include "internal.h"

namespace {

__device__ __forceinline__ int clamp_l(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

constexpr int LB_CH = 128;  // chi nodes per LDS chunk

// ln P and its natural-spline moments in ln k, one wavefront per point.
__global__ __launch_bounds__(64) void k_limber_pk(plan_dev P, swiftcl_inputs in) {
  extern __shared__ double sh[];
  const int b = blockIdx.x, lane = threadIdx.x, nk = P.n_k;
  double* y = sh;
  double* Mo = sh + nk;
  bool bad = false;
  for (int j = lane; j < nk; j += SWIFTCL_WAVE) {
    const double v = in.pk[(size_t)b * nk + j];
    bad |= !(v > 0.0) || !isfinite(v);
    y[j] = log(fmax(v, 1e-300));
  }
  if (bad) atomicOr(P.flags, FLAG_NONFINITE);
  wave_sync();
  wave_spline(y, P.lu_k, nk, Mo, lane);
  for (int j = lane; j < nk; j += SWIFTCL_WAVE) {
    P.lnp[((size_t)b * 2) * nk + j] = y[j];
    P.lnp[((size_t)b * 2 + 1) * nk + j] = Mo[j];
  }
}

// One block per (point, group of LB_LG multipole slots).  Per chunk of chi nodes: H_t(m) =
// w_m f_t(chi_m) [chi_m^2 for the lensing kinds] in LDS, once for the whole group (it does not
// depend on the multipole; w_m f_t is the band-0 kernel sample without its tilt; the CMB-lensing
// sample of the last node, which carries the linear-end weight, is brought to w_m), and the
// weights s_l(m) = Delta P(nu_l / chi_m) / (chi_m w_m) of every slot of the group, stored node by
// node so that a lane reads the group's weights of one node in one go; then every thread sums its
// tracer pairs for all slots of the group.  The factor c(l) / nu^2 (F(l) or l(l+1)) per
// lensing-kind tracer of the pair is applied at the end.
constexpr int LB_LG = 8;  // multipole slots per block

template <typename R>
__global__ __launch_bounds__(256) void k_limber(plan_dev P, swiftcl_inputs in, R* __restrict__ Cout) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = P.max_tracers, Lm = P.max_ell, N = P.N, nb = P.n_bands, nk = P.n_k;
  R* H = (R*)smem;                              // [T][LB_CH]
  R* s = H + (size_t)T * LB_CH;                 // [LB_CH][LB_LG]
  double* lnus = (double*)(s + LB_CH * LB_LG);  // [LB_LG] ln(l + 1/2) of the group's slots
  int* kinds = (int*)(lnus + LB_LG);            // [T] tracer kinds
  int* eis = kinds + T;                         // [LB_LG] multipole of each slot
  const int ngrp = (Lm + LB_LG - 1) / LB_LG;
  const int b = blockIdx.x / ngrp, l0 = (blockIdx.x % ngrp) * LB_LG;
  if (b >= in.batch) return;
  const int npair = T * (T + 1) / 2;
  const int Tb = clamp_l(in.n_tracers[b], 0, T);
  const int Lb = clamp_l(in.n_ell[b], 0, Lm);
  // slots of the group past the point's multipoles: zeros
  for (int e = threadIdx.x; e < LB_LG * npair; e += blockDim.x) {
    const int l = l0 + e / npair;
    if (l < Lm && l >= Lb) Cout[((size_t)b * Lm + l) * npair + e % npair] = (R)0;
  }
  const int nl = Lb - l0 < LB_LG ? Lb - l0 : LB_LG;  // slots of the group this point has
  if (nl <= 0) return;
  if (threadIdx.x < LB_LG) {
    int ei = 0;
    if ((int)threadIdx.x < nl) {
      ei = in.ell_idx[(size_t)b * Lm + l0 + threadIdx.x];
      if (ei < 0 || ei >= P.n_ell) {
        atomicOr(P.flags, FLAG_BAD_INDEX);
        ei = 0;
      }
    }
    eis[threadIdx.x] = ei;
    lnus[threadIdx.x] = log(P.ell_v[ei] + 0.5);
  }
  for (int t = threadIdx.x; t < T; t += blockDim.x) kinds[t] = t < Tb ? tracer_kind(in, T, b, t) : 0;
  // weights of the slots the point does not have stay zero
  for (int e = threadIdx.x; e < LB_CH * LB_LG; e += blockDim.x) s[e] = (R)0;
  __syncthreads();
  const double* pt = P.pt + (size_t)b * PT_STRIDE;
  const double chi0 = pt[PT_CHI0], lchi0 = log(chi0), theta = pt[PT_THETA];
  const int m0 = P.m0, m1 = (int)pt[PT_M1];
  const double* lnp = P.lnp + (size_t)b * 2 * nk;
  const double* lnk = P.lnk;
  const double* lkih = P.lu_k + 3 * (size_t)nk;
  // this thread's tracer pairs (row-major upper triangle)
  constexpr int MAXP = (32 * 33 / 2 + 255) / 256;
  int pi[MAXP], pj[MAXP];
  R acc[MAXP][LB_LG];
#pragma unroll
  for (int q = 0; q < MAXP; ++q) {
    const int p = threadIdx.x + 256 * q;
    int i = 0, rem = p;
    while (i < T && rem >= T - i) { rem -= T - i; ++i; }
    pi[q] = p < npair ? i : 0;
    pj[q] = p < npair ? i + rem : 0;
#pragma unroll
    for (int l = 0; l < LB_LG; ++l) acc[q][l] = (R)0;
  }
  for (int mc = m0; mc <= m1; mc += LB_CH) {
    __syncthreads();  // the previous chunk's readers are done
    for (int e = threadIdx.x; e < nl * LB_CH; e += blockDim.x) {
      const int l = e / LB_CH, idx = e % LB_CH;
      const int m = mc + idx;
      double sv = 0.0;
      if (m <= m1) {
        const double lchi = lchi0 + (double)m * P.delta;
        const double w = m == m0 ? 0.5 : (m == m1 ? 0.5 + theta : 1.0);
        const double x = lnus[l] - lchi;  // ln k of the Limber node
        if (x >= lnk[0] && x <= lnk[nk - 1]) {
          const int iv = clamp_l((int)floor((x - lnk[0]) / P.delta), 0, nk - 2);
          const double lv = spline_at(lnk, lkih, lnp, lnp + nk, iv, x, nullptr);
          sv = P.delta * exp(lv - lchi) / w;
        }
      }
      s[idx * LB_LG + l] = (R)sv;
    }
    for (int e = threadIdx.x; e < T * LB_CH; e += blockDim.x) {
      const int t = e / LB_CH, idx = e % LB_CH;
      const int m = mc + idx;
      double h = 0.0;
      if (t < Tb && m <= m1) {
        const int kind = kinds[t];
        const double gv = (double)((const R*)P.g)[(((size_t)b * T + t) * nb) * N + m];
        h = gv / P.ebm[((size_t)kind * nb) * N + m];
        if (kind != SWIFTCL_CLUSTERING) {
          const double chi = exp(lchi0 + (double)m * P.delta);
          h *= chi * chi;
        }
        if (kind == SWIFTCL_CMB_LENSING && m == m1 && m1 > m0) h *= (0.5 + theta) / (0.5 + 0.5 * theta);
      }
      H[(size_t)t * LB_CH + idx] = (R)h;
    }
    __syncthreads();
    const int cnt = m1 - mc + 1 < LB_CH ? m1 - mc + 1 : LB_CH;
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
      if (threadIdx.x + 256 * q >= npair) continue;
      const R* hi = H + (size_t)pi[q] * LB_CH;
      const R* hj = H + (size_t)pj[q] * LB_CH;
      R a[LB_LG];
#pragma unroll
      for (int l = 0; l < LB_LG; ++l) a[l] = acc[q][l];
      for (int idx = 0; idx < cnt; ++idx) {
        const R h = hi[idx] * hj[idx];
        const R* sw = s + idx * LB_LG;
#pragma unroll
        for (int l = 0; l < LB_LG; ++l) a[l] += h * sw[l];
      }
#pragma unroll
      for (int l = 0; l < LB_LG; ++l) acc[q][l] = a[l];
    }
  }
#pragma unroll
  for (int l = 0; l < LB_LG; ++l) {
    if (l >= nl) break;
    const int ei = eis[l];
    const double nu = P.ell_v[ei] + 0.5;
    const double inu2 = 1.0 / (nu * nu);
    R* c = Cout + ((size_t)b * Lm + l0 + l) * npair;
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
      const int p = threadIdx.x + 256 * q;
      if (p >= npair) continue;
      const int i = pi[q], j = pj[q];
      R v = (R)0;
      if (i < Tb && j < Tb) {
        double f = (double)acc[q][l];
        if (kinds[i]) f *= P.fell[(size_t)kinds[i] * P.n_ell + ei] * inu2;
        if (kinds[j]) f *= P.fell[(size_t)kinds[j] * P.n_ell + ei] * inu2;
        v = (R)f;
      }
      c[p] = v;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Adjoint of the Limber rule.  With H_t(m) and s_l(m) as above and a_t = c_t(l) / nu^2 (1 for
// clustering), C_l^{ij} = a_i a_j sum_m H_i H_j s_l, so for L = sum_l sum_{ij} G_ij C_l^{ij} (G the
// symmetrised cotangent) and Q_t = sum_j G_tj a_j H_j:
//   dL/dH_t(m)      = sum_l 2 a_t s_l(m) Q_t(m)
//   dL/dln P(k_lm)  = s_l(m) sum_t a_t H_t(m) Q_t(m)        (s is P at the node's Limber k)
// The second goes through the spline of ln P (value weights of each node, then the moments'
// adjoint), the first through H = g / e^{-b m Delta} [chi^2] back to the kernel-sample cotangents
// dg, from which the FFTLog adjoint's chain rule (k_bwd_tracer, k_bwd_point) gives db, dn(z), dD.
// ---------------------------------------------------------------------------------------------

__global__ void k_limber_zero(plan_dev P, swiftcl_inputs in) {
  const size_t n = (size_t)in.batch * 2 * P.n_k;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    P.lim_acc[i] = 0.0;
}

// One block per (point, chunk of LB_CH chi nodes), looping over the point's multipoles: dH of the
// chunk's nodes accumulates per thread (node idx = tid / 2, tracer half tid % 2: no atomics), the
// ln P cotangents in LDS (FP64 atomics) and then once per block in the point's global rows.
// Writes the dg rows of the chunk (band 0; the other bands 0).
template <typename R>
__global__ __launch_bounds__(256) void k_limber_bwd(plan_dev P, swiftcl_inputs in, const R* __restrict__ dC) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = P.max_tracers, Lm = P.max_ell, N = P.N, nb = P.n_bands, nk = P.n_k;
  double* H = (double*)smem;                  // [T][LB_CH]
  double* dH = H + (size_t)T * LB_CH;          // [T][LB_CH]
  double* Gs = dH + (size_t)T * LB_CH;         // [T][T]
  double* a = Gs + (size_t)T * T;              // [T]
  double* s = a + T;                           // [LB_CH]
  double* sw = s + LB_CH;                      // [LB_CH][4] spline value weights
  double* dy = sw + 4 * LB_CH;                 // [nk]
  double* dM = dy + nk;                        // [nk]
  int* iv = (int*)(dM + nk);                   // [LB_CH]
  int* kinds = iv + LB_CH;                     // [T]
  const int nch = (N + LB_CH - 1) / LB_CH;
  const int b = blockIdx.x / nch, mc = (blockIdx.x % nch) * LB_CH;
  if (b >= in.batch) return;
  const int tid = threadIdx.x;
  const int Tb = clamp_l(in.n_tracers[b], 0, T);
  const int Lb = clamp_l(in.n_ell[b], 0, Lm);
  const int npair = T * (T + 1) / 2;
  const double* pt = P.pt + (size_t)b * PT_STRIDE;
  const double lchi0 = log(pt[PT_CHI0]), theta = pt[PT_THETA];
  const int m0 = P.m0, m1 = (int)pt[PT_M1];
  for (int t = tid; t < T; t += blockDim.x) kinds[t] = t < Tb ? tracer_kind(in, T, b, t) : 0;
  __syncthreads();
  // H of the chunk (as the forward) and zeroed accumulators
  for (int e = tid; e < T * LB_CH; e += blockDim.x) {
    const int t = e / LB_CH, idx = e % LB_CH, m = mc + idx;
    double h = 0.0;
    if (t < Tb && m >= m0 && m <= m1) {
      const int kind = kinds[t];
      h = (double)((const R*)P.g)[(((size_t)b * T + t) * nb) * N + m] / P.ebm[((size_t)kind * nb) * N + m];
      if (kind != SWIFTCL_CLUSTERING) {
        const double chi = exp(lchi0 + (double)m * P.delta);
        h *= chi * chi;
      }
      if (kind == SWIFTCL_CMB_LENSING && m == m1 && m1 > m0) h *= (0.5 + theta) / (0.5 + 0.5 * theta);
    }
    H[e] = h;
    dH[e] = 0.0;
  }
  for (int j = tid; j < nk; j += blockDim.x) dy[j] = dM[j] = 0.0;
  const bool live = mc <= m1 && mc + LB_CH - 1 >= m0;  // the chunk holds support nodes
  const double* lnp = P.lnp + (size_t)b * 2 * nk;
  const double* lnk = P.lnk;
  const double* lkih = P.lu_k + 3 * (size_t)nk;
  const int idx = tid >> 1, half = tid & 1;
  const int th = (T + 1) / 2, t_lo = half * th, t_hi = half ? T : th;
  for (int li = 0; live && li < Lb; ++li) {
    __syncthreads();  // the previous multipole's readers are done
    int ei = in.ell_idx[(size_t)b * Lm + li];
    if (ei < 0 || ei >= P.n_ell) {
      if (tid == 0) atomicOr(P.flags, FLAG_BAD_INDEX);
      ei = 0;
    }
    const double nu = P.ell_v[ei] + 0.5;
    const double lnu = log(nu);
    for (int t = tid; t < T; t += blockDim.x)
      a[t] = (t < Tb && kinds[t]) ? P.fell[(size_t)kinds[t] * P.n_ell + ei] / (nu * nu) : 1.0;
    for (int e = tid; e < T * T; e += blockDim.x) {
      const int i = e / T, j = e % T;
      double gv = 0.0;
      if (i < Tb && j < Tb) {
        const int lo = i < j ? i : j, hi = i < j ? j : i;
        gv = (double)dC[((size_t)b * Lm + li) * npair + (lo * T - lo * (lo - 1) / 2 + (hi - lo))];
        if (i != j) gv *= 0.5;
      }
      Gs[e] = gv;
    }
    for (int q = tid; q < LB_CH; q += blockDim.x) {
      const int m = mc + q;
      double sv = 0.0;
      int ivq = -1;
      if (m >= m0 && m <= m1) {
        const double lchi = lchi0 + (double)m * P.delta;
        const double w = m == m0 ? 0.5 : (m == m1 ? 0.5 + theta : 1.0);
        const double x = lnu - lchi;
        if (x >= lnk[0] && x <= lnk[nk - 1]) {
          ivq = clamp_l((int)floor((x - lnk[0]) / P.delta), 0, nk - 2);
          const spline_w wt(lnk, lkih, ivq, x);
          const double lv = wt.wa * lnp[ivq] + wt.wb * lnp[ivq + 1] + wt.wc * lnp[nk + ivq] + wt.wd * lnp[nk + ivq + 1];
          sv = P.delta * exp(lv - lchi) / w;
          sw[4 * q] = wt.wa;
          sw[4 * q + 1] = wt.wb;
          sw[4 * q + 2] = wt.wc;
          sw[4 * q + 3] = wt.wd;
        }
      }
      s[q] = sv;
      iv[q] = ivq;
    }
    __syncthreads();
    const double sq = s[idx];
    double ap = 0.0;
    if (sq != 0.0) {
      for (int t = t_lo; t < t_hi; ++t) {
        double Q = 0.0;
        for (int j = 0; j < Tb; ++j) Q += Gs[t * T + j] * a[j] * H[(size_t)j * LB_CH + idx];
        dH[(size_t)t * LB_CH + idx] += 2.0 * sq * a[t] * Q;
        ap += a[t] * H[(size_t)t * LB_CH + idx] * Q;
      }
    }
    ap += __shfl_xor(ap, 1);
    if (half == 0 && sq != 0.0) {
      const double d = ap * sq;
      const int i0 = iv[idx];
      atomicAdd(&dy[i0], sw[4 * idx] * d);
      atomicAdd(&dy[i0 + 1], sw[4 * idx + 1] * d);
      atomicAdd(&dM[i0], sw[4 * idx + 2] * d);
      atomicAdd(&dM[i0 + 1], sw[4 * idx + 3] * d);
    }
  }
  __syncthreads();
  // dg of the chunk's nodes: band 0 from dH, the other bands 0
  R* dg = (R*)P.dg;
  for (int e = tid; e < T * LB_CH; e += blockDim.x) {
    const int t = e / LB_CH, q = e % LB_CH, m = mc + q;
    if (m >= N) continue;
    double v = 0.0;
    if (t < Tb && m >= m0 && m <= m1) {
      const int kind = kinds[t];
      v = dH[e] / P.ebm[((size_t)kind * nb) * N + m];
      if (kind != SWIFTCL_CLUSTERING) {
        const double chi = exp(lchi0 + (double)m * P.delta);
        v *= chi * chi;
      }
      if (kind == SWIFTCL_CMB_LENSING && m == m1 && m1 > m0) v *= (0.5 + theta) / (0.5 + 0.5 * theta);
    }
    for (int bi = 0; bi < nb; ++bi) dg[(((size_t)b * T + t) * nb + bi) * N + m] = (R)(bi == 0 ? v : 0.0);
  }
  if (live)
    for (int j = tid; j < nk; j += blockDim.x) {
      if (dy[j] != 0.0) atomicAdd(&P.lim_acc[((size_t)b * 2) * nk + j], dy[j]);
      if (dM[j] != 0.0) atomicAdd(&P.lim_acc[((size_t)b * 2 + 1) * nk + j], dM[j]);
    }
}

// dL/dP per point: the moments' cotangents through the spline solve, then ln P -> P.  One
// wavefront per point.
__global__ __launch_bounds__(64) void k_limber_bwd_pk(plan_dev P, swiftcl_inputs in, double* dpk) {
  extern __shared__ double sh[];
  const int b = blockIdx.x, lane = threadIdx.x, nk = P.n_k;
  double* dy = sh;
  double* dM = sh + nk;
  for (int j = lane; j < nk; j += SWIFTCL_WAVE) {
    dy[j] = P.lim_acc[((size_t)b * 2) * nk + j];
    dM[j] = P.lim_acc[((size_t)b * 2 + 1) * nk + j];
  }
  wave_sync();
  wave_spline_adjoint(dy, dM, P.lu_k, nk, lane);
  for (int j = lane; j < nk; j += SWIFTCL_WAVE) {
    const double v = in.pk[(size_t)b * nk + j];
    // ln P is taken of max(P, 1e-300): no gradient below that floor
    dpk[(size_t)b * nk + j] = v > 1e-300 ? dy[j] / v : 0.0;
  }
}

}  // namespace

size_t limber_bwd_lds_bytes(const plan_dev& p) {
  const size_t T = p.max_tracers;
  return sizeof(double) * (2 * T * LB_CH + T * T + T + 5 * LB_CH + 2 * (size_t)p.n_k) + sizeof(int) * (LB_CH + T);
}

size_t limber_lds_bytes(const plan_dev& p) {
  const size_t rs = p.precision == SWIFTCL_FP64 ? 8 : 4;
  return rs * ((size_t)p.max_tracers * LB_CH + (size_t)LB_CH * LB_LG) + sizeof(double) * LB_LG +
         sizeof(int) * ((size_t)p.max_tracers + LB_LG);
}

hipError_t launch_limber(const plan_dev& p, const swiftcl_inputs* in, void* C, hipStream_t s) {
  hipLaunchKernelGGL(k_limber_pk, dim3(in->batch), dim3(64), sizeof(double) * 2 * (size_t)p.n_k, s, p, *in);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((size_t)in->batch * ((p.max_ell + LB_LG - 1) / LB_LG)));
  if (p.precision == SWIFTCL_FP64)
    hipLaunchKernelGGL(k_limber<double>, grid, dim3(256), limber_lds_bytes(p), s, p, *in, (double*)C);
  else
    hipLaunchKernelGGL(k_limber<float>, grid, dim3(256), limber_lds_bytes(p), s, p, *in, (float*)C);
  return hipGetLastError();
}

hipError_t launch_limber_backward(const plan_dev& p, const swiftcl_inputs* in, const void* dC, double* dpk,
                                  double* dbias, double* dnz, double* dD, hipStream_t s) {
  hipLaunchKernelGGL(k_limber_pk, dim3(in->batch), dim3(64), sizeof(double) * 2 * (size_t)p.n_k, s, p, *in);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_limber_zero, dim3(256), dim3(256), 0, s, p, *in);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nch = (p.N + LB_CH - 1) / LB_CH;
  const dim3 grid((unsigned)((size_t)in->batch * nch));
  if (p.precision == SWIFTCL_FP64)
    hipLaunchKernelGGL(k_limber_bwd<double>, grid, dim3(256), limber_bwd_lds_bytes(p), s, p, *in, (const double*)dC);
  else
    hipLaunchKernelGGL(k_limber_bwd<float>, grid, dim3(256), limber_bwd_lds_bytes(p), s, p, *in, (const float*)dC);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (dpk) {
    hipLaunchKernelGGL(k_limber_bwd_pk, dim3(in->batch), dim3(64), sizeof(double) * 2 * (size_t)p.n_k, s, p, *in,
                       dpk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return launch_bwd_chain(p, in, dbias, dnz, dD, s);
}
