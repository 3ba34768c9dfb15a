// Host plan, argument checks, plan-time tables and the C entry points of libswiftcl.
//
// The plan fixes everything that depends only on the descriptor: the log-chi grid step
// (equal to the k grid's log step, so the FFTLog output lands on the caller's k nodes), the
// per-(kind, l) table of power-law Bessel integrals U_l(n) of eq. int_jl (computed on the GPU
// in FP64 from a complex log-gamma), the k scale tables, FFT twiddles, spline factorisations
// and the workspace for max_batch points.  Calls after swiftcl_plan allocate nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

swiftcl_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return SWIFTCL_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return SWIFTCL_E_DEVICE;
}

extern "C" const char* swiftcl_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------------------------
// Complex log-gamma in FP64 (Stirling's series with Bernoulli-number coefficients after an
// upward recurrence shift; valid for Re z > 0).  Only exp() of differences is used, so the
// branch of the imaginary part is irrelevant.
// ---------------------------------------------------------------------------------------------
struct zd { double x, y; };
__device__ inline zd zadd(zd a, zd b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline zd zsub(zd a, zd b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline zd zmul(zd a, zd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline zd zdiv(zd a, zd b) {
  double d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__device__ inline zd zlog(zd a) { return {log(hypot(a.x, a.y)), atan2(a.y, a.x)}; }

__device__ zd zlgamma(zd z) {
  // shift so that Re z >= 12, accumulating log of the product z (z+1) ... in chunks
  zd acc = {0.0, 0.0};
  zd prod = {1.0, 0.0};
  int cnt = 0;
  while (z.x < 12.0) {
    prod = zmul(prod, z);
    z.x += 1.0;
    if (++cnt == 8) { acc = zadd(acc, zlog(prod)); prod = {1.0, 0.0}; cnt = 0; }
  }
  acc = zadd(acc, zlog(prod));
  // Stirling: (z - 1/2) ln z - z + ln(2 pi)/2 + sum_k B_2k / (2k (2k-1) z^{2k-1})
  const double c[10] = {1.0 / 12.0, -1.0 / 360.0, 1.0 / 1260.0, -1.0 / 1680.0, 1.0 / 1188.0,
                        -691.0 / 360360.0, 1.0 / 156.0, -3617.0 / 122400.0, 43867.0 / 244188.0,
                        -174611.0 / 125400.0};
  zd lz = zlog(z);
  zd r = zsub(zmul({z.x - 0.5, z.y}, lz), z);
  r.x += 0.91893853320467274178;  // ln(2 pi)/2
  zd iz = zdiv({1.0, 0.0}, z);
  zd iz2 = zmul(iz, iz);
  zd term = iz;
  for (int k = 0; k < 10; ++k) {
    r = zadd(r, {c[k] * term.x, c[k] * term.y});
    term = zmul(term, iz2);
  }
  return zsub(r, acc);
}

// FFTLog biases of every kind and band, passed by value to the table kernels.
struct bias_table {
  double b[SWIFTCL_NKINDS][SWIFTCL_MAX_BANDS];
};

// U_l(n) = sqrt(pi) 2^{p-1} Gamma((1+l+p)/2) / Gamma((2+l-p)/2) at p = b + i eta (eq. int_jl with the
// corrected denominator; the k^{-1-p} factor is applied on the k side).
__device__ inline zd u_value(double l, double b, double eta) {
  zd pa = {0.5 * (1.0 + l + b), 0.5 * eta};
  zd pb = {0.5 * (2.0 + l - b), -0.5 * eta};
  zd lg = zsub(zlgamma(pa), zlgamma(pb));
  // 2^{p-1} = exp((p-1) ln 2)
  lg.x += (b - 1.0) * 0.69314718055994530942;
  lg.y += eta * 0.69314718055994530942;
  const double mag = 1.7724538509055160273 * exp(lg.x);  // sqrt(pi)
  double sn, cs;
  sincos(lg.y, &sn, &cs);
  return {mag * cs, mag * sn};
}

// the cosine taper of the top fraction of |n| ("smoothing at the tails", Sec. 3.1)
__device__ inline double taper_of(int n, int M, double taper_frac) {
  if (!(taper_frac > 0.0)) return 1.0;
  const double x = (double)n / (double)M, x0 = 1.0 - taper_frac;
  return x > x0 ? 0.5 * (1.0 + cos(M_PI * fmin((x - x0) / taper_frac, 1.0))) : 1.0;
}

// F(l) U_l(n) * taper(n) for every kind at eta_n = 2 pi n / (N Delta), n = 0..M-1, with the bias of
// the kind's row in l's band.  The kind's multipole prefactor F(l) (fell: 1, the shear factor, or
// l(l+1)) is real and multiplies the whole window, so it is folded into the table once here rather
// than into every window element (forward, adjoint and k-dependent-growth paths alike).
template <typename R>
__global__ void k_u_table(C2<R>* __restrict__ U, const double* __restrict__ ell, const int* __restrict__ band,
                          const double* __restrict__ fell, bias_table bt, int n_ell, int M, double delta,
                          double taper_frac) {
  const int li = blockIdx.x;
  const int n = blockIdx.y * blockDim.x + threadIdx.x;
  if (li >= n_ell || n >= M) return;
  const double l = ell[li];
  const int bi = band[li];
  const double eta = 2.0 * M_PI * (double)n / (2.0 * M * delta);
  const double tap = taper_of(n, M, taper_frac);
  for (int kind = 0; kind < SWIFTCL_NKINDS; ++kind) {
    const zd u = u_value(l, bt.b[kind][bi], eta);
    const double f = fell[(size_t)kind * n_ell + li] * tap;
    C2<R> v;
    v.x = (R)(u.x * f);
    v.y = (R)(n == 0 ? 0.0 : u.y * f);
    U[((size_t)kind * n_ell + li) * M + n] = v;
  }
}

// The RSD table (eq. RSD): the integral of chi^p j_l'' is that of chi^p times
// a j_{l-2} + b j_l + c j_{l+2} (j_l' = (l j_{l-1} - (l+1) j_{l+1}) / (2l+1) applied twice), i.e. the
// same combination of three U values of eq. int_jl at the clustering bias of l's band.
template <typename R>
__global__ void k_u_rsd(C2<R>* __restrict__ UR, const double* __restrict__ ell, const int* __restrict__ band,
                        bias_table bt, int n_ell, int M, double delta, double taper_frac) {
  const int li = blockIdx.x;
  const int n = blockIdx.y * blockDim.x + threadIdx.x;
  if (li >= n_ell || n >= M) return;
  const double l = ell[li];
  const double b = bt.b[SWIFTCL_CLUSTERING][band[li]];
  const double eta = 2.0 * M_PI * (double)n / (2.0 * M * delta);
  const double tap = taper_of(n, M, taper_frac);
  const double am = l * (l - 1.0) / ((2.0 * l - 1.0) * (2.0 * l + 1.0));
  const double a0 = -(2.0 * l * l + 2.0 * l - 1.0) / ((2.0 * l - 1.0) * (2.0 * l + 3.0));
  const double ap = (l + 1.0) * (l + 2.0) / ((2.0 * l + 1.0) * (2.0 * l + 3.0));
  const zd um = u_value(l - 2.0, b, eta), u0 = u_value(l, b, eta), up = u_value(l + 2.0, b, eta);
  double vx = (am * um.x + a0 * u0.x + ap * up.x) * tap;
  double vy = (am * um.y + a0 * u0.y + ap * up.y) * tap;
  if (n == 0) vy = 0.0;
  C2<R> v;
  v.x = (R)vx;
  v.y = (R)vy;
  UR[(size_t)li * M + n] = v;
}

// Magnification (eq. magnification bias): l(l+1) U_l(n) at the bias b - 2 of the clustering band, so
// that with the clustering k scale k^{-1-b} the window carries l(l+1) k^{-2} k^{-1-(b-2)-i eta}.
template <typename R>
__global__ void k_u_mag(C2<R>* __restrict__ Um, const double* __restrict__ ell, const int* __restrict__ band,
                        bias_table bt, int n_ell, int M, double delta, double taper_frac) {
  const int li = blockIdx.x;
  const int n = blockIdx.y * blockDim.x + threadIdx.x;
  if (li >= n_ell || n >= M) return;
  const double l = ell[li];
  const double b = bt.b[SWIFTCL_CLUSTERING][band[li]] - 2.0;
  const double eta = 2.0 * M_PI * (double)n / (2.0 * M * delta);
  const zd u = u_value(l, b, eta);
  const double f = l * (l + 1.0) * taper_of(n, M, taper_frac);
  C2<R> v;
  v.x = (R)(f * u.x);
  v.y = (R)(n == 0 ? 0.0 : f * u.y);
  Um[(size_t)li * M + n] = v;
}

hipError_t launch_u_table(const plan_dev& pd, const double* d_ell, hipStream_t s) {
  const plan_dev* p = &pd;
  dim3 grid(p->n_ell, (p->M + 127) / 128);
  bias_table bt;
  for (int k = 0; k < SWIFTCL_NKINDS; ++k)
    for (int j = 0; j < SWIFTCL_MAX_BANDS; ++j) bt.b[k][j] = p->fftlog_b[k][j];
  if (p->precision == SWIFTCL_FP64)
    hipLaunchKernelGGL(k_u_table<double>, grid, dim3(128), 0, s, (double2*)p->U, d_ell, p->ell_band, p->fell, bt,
                       p->n_ell, p->M, p->delta, p->taper_frac);
  else
    hipLaunchKernelGGL(k_u_table<float>, grid, dim3(128), 0, s, (float2*)p->U, d_ell, p->ell_band, p->fell, bt,
                       p->n_ell, p->M, p->delta, p->taper_frac);
  if (p->rsd)  // RSD and magnification plans are FP32 / split
    hipLaunchKernelGGL(k_u_rsd<float>, grid, dim3(128), 0, s, (float2*)p->UR, d_ell, p->ell_band, bt, p->n_ell, p->M,
                       p->delta, p->taper_frac);
  if (p->mag)
    hipLaunchKernelGGL(k_u_mag<float>, grid, dim3(128), 0, s, (float2*)p->Umu, d_ell, p->ell_band, bt, p->n_ell,
                       p->M, p->delta, p->taper_frac);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Descriptor checks (host only, no device work)
// ---------------------------------------------------------------------------------------------
static bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

static swiftcl_status check_increasing(const double* x, int n, const char* name) {
  if (!x) { set_error(std::string(name) + " is NULL"); return SWIFTCL_E_INVALID; }
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(x[i])) { set_error(std::string(name) + " has a non-finite entry"); return SWIFTCL_E_INVALID; }
    if (i && !(x[i] > x[i - 1])) { set_error(std::string(name) + " is not strictly increasing"); return SWIFTCL_E_INVALID; }
  }
  return SWIFTCL_OK;
}

static int default_edge_node(int n_chi, double delta) {
  // centre a support of 5 e-folds (z in [0.01, 3] for LCDM) in the chi box
  return (int)std::lround(0.5 * (n_chi - 5.0 / delta));
}

static swiftcl_status validate_desc(const swiftcl_plan_desc* d) {
  if (!d) { set_error("descriptor is NULL"); return SWIFTCL_E_INVALID; }
  if (!is_pow2(d->n_chi) || d->n_chi < 256 || d->n_chi > 4096) {
    set_error("n_chi must be a power of two in [256, 4096]");
    return is_pow2(d->n_chi) ? SWIFTCL_E_UNSUPPORTED : SWIFTCL_E_INVALID;
  }
  if (d->n_chi > 2048) { set_error("n_chi = 4096 is not built"); return SWIFTCL_E_UNSUPPORTED; }
  if (d->n_k < 2 || d->n_k > d->n_chi) { set_error("need 2 <= n_k <= n_chi"); return SWIFTCL_E_INVALID; }
  if (d->n_k % 2) { set_error("n_k must be even"); return SWIFTCL_E_UNSUPPORTED; }
  swiftcl_status st;
  if ((st = check_increasing(d->k, d->n_k, "k")) != SWIFTCL_OK) return st;
  if (d->k[0] <= 0) { set_error("k must be positive"); return SWIFTCL_E_DOMAIN; }
  const double delta = std::log(d->k[d->n_k - 1] / d->k[0]) / (d->n_k - 1);
  for (int j = 0; j + 1 < d->n_k; ++j) {
    const double dj = std::log(d->k[j + 1] / d->k[j]);
    if (std::fabs(dj - delta) > 1e-9 * std::max(1.0, delta) + 1e-9 * delta) {
      set_error("k is not log-spaced");
      return SWIFTCL_E_DOMAIN;
    }
  }
  if (d->n_ell < 1) { set_error("n_ell must be >= 1"); return SWIFTCL_E_INVALID; }
  if ((st = check_increasing(d->ell, d->n_ell, "ell")) != SWIFTCL_OK) return st;
  if (d->ell[0] < 2.0) { set_error("multipoles must be >= 2"); return SWIFTCL_E_DOMAIN; }
  if (d->n_bands < 1 || d->n_bands > SWIFTCL_MAX_BANDS) { set_error("n_bands must be in 1..4"); return SWIFTCL_E_INVALID; }
  for (int j = 1; j < d->n_bands; ++j)
    if (!(d->band_ell_lo[j] > d->band_ell_lo[j - 1])) { set_error("band_ell_lo must increase"); return SWIFTCL_E_INVALID; }
  if (d->band_ell_lo[0] > d->ell[0]) { set_error("band_ell_lo[0] exceeds the smallest multipole"); return SWIFTCL_E_INVALID; }
  for (int i = 0; i < d->n_ell; ++i) {
    int bi = 0;
    while (bi + 1 < d->n_bands && d->ell[i] >= d->band_ell_lo[bi + 1]) ++bi;
    for (int kind = 0; kind < SWIFTCL_NKINDS; ++kind) {
      const double b = d->fftlog_b[kind][bi];
      if (!(b > -d->ell[i] - 1.0 && b < 1.0) || !std::isfinite(b)) {
        set_error("FFTLog bias b outside (-l-1, 1) for some multipole");
        return SWIFTCL_E_DOMAIN;
      }
    }
    // RSD evaluates eq. int_jl at l - 2 and magnification at the bias b - 2 (both with the
    // clustering row): each converges only for b > 1 - l
    if ((d->rsd || d->magnification) && !(d->fftlog_b[SWIFTCL_CLUSTERING][bi] > 1.0 - d->ell[i])) {
      set_error("with rsd or magnification the clustering FFTLog bias must exceed 1 - l for every multipole");
      return SWIFTCL_E_DOMAIN;
    }
  }
  if (!(d->taper_frac >= 0.0 && d->taper_frac < 1.0)) { set_error("taper_frac must be in [0, 1)"); return SWIFTCL_E_INVALID; }
  if (d->n_zg < 4 || d->n_zs < 4) { set_error("need at least 4 geometry and n(z) samples"); return SWIFTCL_E_INVALID; }
  if ((st = check_increasing(d->z_geom, d->n_zg, "z_geom")) != SWIFTCL_OK) return st;
  if ((st = check_increasing(d->z_nz, d->n_zs, "z_nz")) != SWIFTCL_OK) return st;
  if (d->z_geom[0] < 0.0) { set_error("z_geom must be >= 0"); return SWIFTCL_E_DOMAIN; }
  if (d->n_zg > 1536 || d->n_zs > 1536) { set_error("at most 1536 geometry and n(z) samples"); return SWIFTCL_E_UNSUPPORTED; }
  if (d->z_nz[0] < d->z_geom[0] || d->z_nz[d->n_zs - 1] > d->z_geom[d->n_zg - 1]) {
    set_error("z_nz must lie inside the geometry range");
    return SWIFTCL_E_INVALID;
  }
  const int m0 = d->edge_node > 0 ? d->edge_node : default_edge_node(d->n_chi, delta);
  if (m0 < 1 || m0 > d->n_chi - 2) { set_error("edge_node outside 1..n_chi-2"); return SWIFTCL_E_INVALID; }
  if (d->max_batch < 1 || d->max_tracers < 1 || d->max_ell < 1) { set_error("capacities must be >= 1"); return SWIFTCL_E_INVALID; }
  if (d->max_tracers > 32) { set_error("max_tracers > 32 is not built"); return SWIFTCL_E_UNSUPPORTED; }
  if (d->precision < 0 || d->precision > 2) { set_error("unknown precision"); return SWIFTCL_E_INVALID; }
  if (d->rsd != 0 && d->rsd != 1) { set_error("rsd must be 0 or 1"); return SWIFTCL_E_INVALID; }
  if (d->magnification != 0 && d->magnification != 1) { set_error("magnification must be 0 or 1"); return SWIFTCL_E_INVALID; }
  if (d->magnification && d->precision == SWIFTCL_FP64) {
    set_error("magnification bias is built for FP32 and split precision");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if (d->rsd && d->precision == SWIFTCL_FP64) {
    set_error("redshift-space distortions are built for FP32 and split precision");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if (d->n_interp != 0) {
    if (d->n_interp < 2 || d->n_interp > d->n_k) { set_error("n_interp must be 0 or in 2..n_k"); return SWIFTCL_E_INVALID; }
    if (d->precision == SWIFTCL_FP64) {
      set_error("scale-dependent growth (n_interp > 0) is built for FP32 and split precision");
      return SWIFTCL_E_UNSUPPORTED;
    }
  }
  return SWIFTCL_OK;
}

// Thomas factors of the natural cubic spline system on grid x (interior rows 1..n-2), and 1/h.
static void spline_lu(const double* x, int n, std::vector<double>& out) {
  out.assign(4 * (size_t)n, 0.0);
  double* a = out.data();
  double* inv = a + n;
  double* cp = a + 2 * n;
  double* ih = a + 3 * n;
  for (int i = 0; i + 1 < n; ++i) ih[i] = 1.0 / (x[i + 1] - x[i]);
  for (int i = 1; i < n - 1; ++i) {
    const double h0 = x[i] - x[i - 1], h1 = x[i + 1] - x[i];
    const double ai = h0 / 6.0, bi = (h0 + h1) / 3.0, ci = h1 / 6.0;
    const double den = (i == 1) ? bi : bi - ai * cp[i - 1];
    a[i] = ai;
    inv[i] = 1.0 / den;
    cp[i] = ci / den;
  }
}

template <typename T> static swiftcl_status dalloc(T** ptr, size_t count, const char* what) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    set_error(std::string("hipMalloc failed for ") + what);
    return SWIFTCL_E_NOMEM;
  }
  return SWIFTCL_OK;
}

static void free_plan(swiftcl_plan_s* p) {
  if (!p) return;
  void* ptrs[] = {p->d.U, p->d.kscale, p->d.tw, p->d.fell, p->d.ell_band, p->d.kw, p->d.ell_v, p->d.lnk, p->d.lu_k,
                  p->d.lnp, p->d.lim_acc, p->d.ebm, p->d.z_geom, p->d.z_nz, p->d.lu_geom,
                  p->d.lu_nz, p->d.z_union, p->d.union_iv, p->d.pt, p->d.m_chi, p->d.m_D, p->d.m_ia, p->d.m_n, p->d.lens_q, p->d.phase, p->d.node_f, p->d.node_i, p->d.ddD_part, p->d.g,
                  p->d.chat, p->d.sqrt_s, p->d.kss, p->d.flags, p->d.dchat_part, p->d.dpk_part, p->d.dg, p->d.sched, p->d.bwd_order, p->d.vbuf,
                  p->d.kg_ones, p->d.kg_ia, p->d.kg_w, p->d.kg_ip, p->d.kg_uh, p->d.kg_c, p->d.kg_m, p->d.kg_perm,
                  p->d.kg_tile, p->d.UR, p->d.g_r, p->d.chat_r, p->d.Umu, p->d.g_mu, p->d.chat_mu};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
}

extern "C" swiftcl_status swiftcl_plan(const swiftcl_plan_desc* d, void* stream, swiftcl_plan_t* out) {
  if (!out) { set_error("out is NULL"); return SWIFTCL_E_INVALID; }
  *out = nullptr;
  swiftcl_status st = validate_desc(d);
  if (st != SWIFTCL_OK) return st;
  if ((st = hip_check(hipSetDevice(d->device), "hipSetDevice")) != SWIFTCL_OK) return st;
  (void)hipGetLastError();  // drop a stale error of an earlier, unrelated call
  // the device address of the static workspace of swiftcl_cl_noalloc, once per device
  if ((st = noalloc_setup(d->device)) != SWIFTCL_OK) return st;
  int lds_max = 0;
  if ((st = hip_check(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, d->device),
                      "device attribute")) != SWIFTCL_OK)
    return st;
  bool fused = false;
  {
    const bool dp = d->precision == SWIFTCL_FP64;
    const int M = d->n_chi / 2;
    const size_t need = windows_cl_lds(M, windows_nw(d->precision), windows_tw_lds(d->precision, M), true,
                                       dp ? 8 : 4, d->n_k);
    fused = d->max_tracers <= 16 && need <= (size_t)lds_max && !d->rsd && !d->magnification;
    if (!fused && dp) {
      set_error("the FP64 path keeps the windows of <= 16 tracers in LDS; this n_chi / n_k / max_tracers needs " +
                std::to_string(need) + " bytes per workgroup, the device has " + std::to_string(lds_max));
      return SWIFTCL_E_UNSUPPORTED;
    }
    if (!fused && windows_cl_lds(M, 16, unfused_tw_lds(M), false, 4, d->n_k) > (size_t)lds_max) {
      set_error("n_chi too large for the LDS of one workgroup");
      return SWIFTCL_E_UNSUPPORTED;
    }
  }
  {
    // the geometry kernel keeps one point's samples in LDS
    std::set<double> us(d->z_geom, d->z_geom + d->n_zg);
    for (int i = 0; i < d->n_zs; ++i) us.insert(d->z_nz[i]);
    plan_dev probe{};
    probe.n_zg = d->n_zg;
    probe.n_zs = d->n_zs;
    probe.max_tracers = d->max_tracers;
    probe.n_union = (int)us.size() - 1;
    if (geometry_lds_bytes(probe) > (size_t)lds_max || bwd_geometry_lds_bytes(probe) > (size_t)lds_max ||
        (d->n_interp > 0 && kgrowth_fft_lds(d->n_chi / 2, d->n_zg) > (size_t)lds_max)) {
      set_error("geometry samples exceed the LDS of one workgroup (n_zg, n_zs, max_tracers too large)");
      return SWIFTCL_E_UNSUPPORTED;
    }
  }
  hipStream_t s = (hipStream_t)stream;

  swiftcl_plan_s* p = new (std::nothrow) swiftcl_plan_s();
  if (!p) { set_error("host allocation failed"); return SWIFTCL_E_NOMEM; }
  p->d.device = d->device;
  p->d.precision = d->precision;
  p->d.N = d->n_chi;
  p->d.M = d->n_chi / 2;
  p->d.n_k = d->n_k;
  p->d.n_ell = d->n_ell;
  p->d.n_zg = d->n_zg;
  p->d.n_zs = d->n_zs;
  p->d.n_bands = d->n_bands;
  p->d.max_batch = d->max_batch;
  p->d.max_tracers = d->max_tracers;
  p->d.max_ell = d->max_ell;
  p->d.delta = std::log(d->k[d->n_k - 1] / d->k[0]) / (d->n_k - 1);
  p->d.k0 = d->k[0];
  p->d.taper_frac = d->taper_frac;
  p->d.m0 = d->edge_node > 0 ? d->edge_node : default_edge_node(d->n_chi, p->d.delta);
  p->d.fused = fused ? 1 : 0;
  p->d.rsd = d->rsd;
  p->d.mag = d->magnification;
  // the adjoint: the fused kernel when its LDS fits (+ the kernel's static LDS), else (FP32 and
  // split plans) through the workspace.  RSD and magnification plans (FP32 / split, never fused)
  // take the workspace adjoint, whose recomputed W carries their terms: dL/dP and dL/db only
  // (dL/dn and dL/dD would need the adjoints of their kernel assemblies)
  if (fused && bwd_windows_lds(p->d) + 4096 <= (size_t)lds_max) p->d.adjoint = 1;
  else p->d.adjoint = d->precision == SWIFTCL_FP64 ? 0 : 2;
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d->device) != hipSuccess || ncu < 8)
      ncu = 256;
    p->d.persist_blocks = (ncu / SWIFTCL_NXCD) * SWIFTCL_NXCD;
    p->d.fwd_mode = 0;
    p->d.bwd_chunk_mul = 1;
    p->d.bwd_pack = 0;
  }
  for (int j = 0; j < SWIFTCL_MAX_BANDS; ++j) {
    p->d.band_ell_lo[j] = j < d->n_bands ? d->band_ell_lo[j] : 1e300;
    for (int kind = 0; kind < SWIFTCL_NKINDS; ++kind) p->d.fftlog_b[kind][j] = j < d->n_bands ? d->fftlog_b[kind][j] : 0.0;
  }
  p->ell_host.assign(d->ell, d->ell + d->n_ell);
  p->real_size = d->precision == SWIFTCL_FP64 ? 8 : 4;
  const size_t rs = p->real_size;
  const int N = p->d.N, M = p->d.M, nk = p->d.n_k, T = p->d.max_tracers, B = p->d.max_batch, nb = p->d.n_bands;

  // --- host tables ---
  const int nl = p->d.n_ell;
  std::vector<int> band(nl);
  std::vector<double> fell((size_t)SWIFTCL_NKINDS * nl);
  for (int i = 0; i < nl; ++i) {
    int bi = 0;
    while (bi + 1 < nb && d->ell[i] >= d->band_ell_lo[bi + 1]) ++bi;
    band[i] = bi;
    const double l = d->ell[i];
    fell[i] = 1.0;                                                                   // clustering
    fell[(size_t)SWIFTCL_LENSING * nl + i] = std::sqrt((l + 2.0) * (l + 1.0) * l * (l - 1.0));  // shear
    fell[(size_t)SWIFTCL_CMB_LENSING * nl + i] = l * (l + 1.0);                      // convergence
  }
  std::vector<double> kscale((size_t)SWIFTCL_NKINDS * nb * nk), kw(nk);
  for (int kind = 0; kind < SWIFTCL_NKINDS; ++kind)
    for (int bi = 0; bi < nb; ++bi)
      for (int j = 0; j < nk; ++j) {
        const double lk = std::log(d->k[0]) + j * p->d.delta;  // the grid node k_0 e^{j Delta}
        double v = std::exp((-1.0 - p->d.fftlog_b[kind][bi]) * lk);
        if (kind != SWIFTCL_CLUSTERING) v *= std::exp(-2.0 * lk);  // the 1/k^2 of both lensing kinds
        kscale[((size_t)kind * nb + bi) * nk + j] = v;
      }
  for (int j = 0; j < nk; ++j) {
    const double w = (j == 0 || j == nk - 1) ? 0.5 * p->d.delta : p->d.delta;
    kw[j] = (2.0 / M_PI) * w * d->k[j] * d->k[j] * d->k[j];
  }
  // FFTLog bias factors e^{-b m Delta} per kind, band and chi node
  std::vector<double> ebm((size_t)SWIFTCL_NKINDS * nb * N);
  for (int kind = 0; kind < SWIFTCL_NKINDS; ++kind)
    for (int bi = 0; bi < nb; ++bi)
      for (int m = 0; m < N; ++m)
        ebm[((size_t)kind * nb + bi) * N + m] = std::exp(-d->fftlog_b[kind][bi] * (double)m * p->d.delta);
  // FFT twiddles in the layout of fft_tw_index (the last of the N slots is unused)
  std::vector<double> twd(2 * (size_t)N, 0.0);
  {
    const int M = N / 2;
    auto put = [&](int idx, double num, double den) {
      twd[2 * (size_t)idx] = std::cos(2.0 * M_PI * num / den);
      twd[2 * (size_t)idx + 1] = -std::sin(2.0 * M_PI * num / den);
    };
    for (int n = 0; n < M; ++n) put(n, n, N);
    int Ls = 1;
    for (int pass = 0; pass < fft_npass(M); ++pass) {
      const int r = fft_radix(M, pass);
      for (int i = 1; i < r; ++i)
        for (int j = 0; j < Ls; ++j) put(fft_tw_index(M, Ls, i, j), (double)i * j, (double)Ls * r);
      Ls *= r;
    }
  }
  std::vector<double> lug, lun, luk, lnk(nk);
  spline_lu(d->z_geom, d->n_zg, lug);
  spline_lu(d->z_nz, d->n_zs, lun);
  for (int j = 0; j < nk; ++j) lnk[j] = std::log(d->k[j]);
  spline_lu(lnk.data(), nk, luk);
  // knots of the lensing quadrature: union of both grids inside the geometry range
  std::set<double> us(d->z_geom, d->z_geom + d->n_zg);
  for (int i = 0; i < d->n_zs; ++i) us.insert(d->z_nz[i]);
  std::vector<double> zu(us.begin(), us.end());
  p->d.n_union = (int)zu.size() - 1;
  std::vector<int> uiv(2 * (size_t)p->d.n_union);
  for (int u = 0; u < p->d.n_union; ++u) {
    const double mid = 0.5 * (zu[u] + zu[u + 1]);
    int ig = (int)(std::upper_bound(d->z_geom, d->z_geom + d->n_zg, mid) - d->z_geom) - 1;
    ig = std::min(std::max(ig, 0), d->n_zg - 2);
    int in = (int)(std::upper_bound(d->z_nz, d->z_nz + d->n_zs, mid) - d->z_nz) - 1;
    if (mid < d->z_nz[0] || mid > d->z_nz[d->n_zs - 1]) in = -1;
    else in = std::min(std::max(in, 0), d->n_zs - 2);
    uiv[u] = ig;
    uiv[p->d.n_union + u] = in;
  }

  // --- device allocations ---
#define ALLOC(ptr, type, count)                                             \
  do {                                                                      \
    type* tmp_ = nullptr;                                                   \
    if ((st = dalloc<type>(&tmp_, (count), #ptr)) != SWIFTCL_OK) {          \
      free_plan(p);                                                         \
      return st;                                                            \
    }                                                                       \
    p->d.ptr = (decltype(p->d.ptr))tmp_;                                        \
  } while (0)
  ALLOC(U, char, (size_t)SWIFTCL_NKINDS * p->d.n_ell * M * 2 * rs);
  ALLOC(kscale, char, kscale.size() * rs);
  ALLOC(tw, char, (size_t)N * 2 * rs);
  ALLOC(fell, double, fell.size());
  ALLOC(ell_band, int, p->d.n_ell);
  ALLOC(kw, double, nk);
  ALLOC(ell_v, double, p->d.n_ell);
  ALLOC(lnk, double, nk);
  ALLOC(lu_k, double, luk.size());
  ALLOC(lnp, double, (size_t)B * 2 * nk);
  ALLOC(ebm, double, ebm.size());
  ALLOC(z_geom, double, p->d.n_zg);
  ALLOC(z_nz, double, p->d.n_zs);
  ALLOC(lu_geom, double, lug.size());
  ALLOC(lu_nz, double, lun.size());
  ALLOC(z_union, double, zu.size());
  ALLOC(union_iv, int, uiv.size());
  ALLOC(pt, double, (size_t)B * PT_STRIDE);
  ALLOC(m_chi, double, (size_t)B * p->d.n_zg);
  ALLOC(m_D, double, (size_t)B * p->d.n_zg);
  ALLOC(m_ia, double, (size_t)B * p->d.n_zg);
  ALLOC(m_n, double, (size_t)B * T * p->d.n_zs);
  ALLOC(lens_q, double, (size_t)B * T * N);
  ALLOC(phase, double, (size_t)B * N);
  ALLOC(node_f, double, (size_t)B * 4 * N);
  ALLOC(node_i, int, (size_t)B * 3 * N);
  ALLOC(ddD_part, double, (size_t)B * T * 2 * p->d.n_zg);  // the FFTLog and Limber adjoints
  ALLOC(lim_acc, double, (size_t)B * 2 * nk);
  ALLOC(g, char, (size_t)B * T * nb * N * rs);
  ALLOC(chat, char, (size_t)B * T * nb * M * 2 * rs);
  if (p->d.mag) {
    ALLOC(Umu, char, (size_t)p->d.n_ell * M * 2 * rs);
    ALLOC(g_mu, char, (size_t)B * T * nb * N * rs);
    ALLOC(chat_mu, char, (size_t)B * T * nb * M * 2 * rs);
  }
  if (p->d.rsd) {
    ALLOC(UR, char, (size_t)p->d.n_ell * M * 2 * rs);
    ALLOC(g_r, char, (size_t)B * T * nb * N * rs);
    ALLOC(chat_r, char, (size_t)B * T * nb * M * 2 * rs);
  }
  ALLOC(sqrt_s, char, (size_t)B * nk * rs);
  ALLOC(kss, char, (size_t)B * SWIFTCL_NKINDS * nb * nk * rs);
  ALLOC(flags, int, 1);
  {
    // (point, chunk) slots of the backward partials: the most any batch size and chunk
    // multiplier ask for (the packed adjoint, bwd_chunk_mul <= 4, writes two per chunk)
    long slots = 0;
    plan_dev probe = p->d, probe4 = p->d;
    probe.bwd_chunk_mul = 8;
    probe4.bwd_chunk_mul = 4;
    long grid = 0;
    for (int bb = 1; bb <= B; ++bb) {
      slots = std::max(slots, (long)bb * backward_chunks(probe, bb));
      slots = std::max(slots, (long)bb * 2 * backward_chunks(probe4, bb));
      grid = std::max(grid, (long)((bb + SWIFTCL_NXCD - 1) / SWIFTCL_NXCD) * SWIFTCL_NXCD * backward_chunks(probe, bb));
    }
    p->d.bwd_slots = (int)slots;
    p->d.bwd_order_n = (int)grid;
  }
  p->d.n_interp = d->n_interp;
  if (!p->d.fused || p->d.n_interp > 0 || p->d.adjoint == 2) {
    // workspace of the unfused projection (V of up to 32 tracer slots) and of scale-dependent
    // growth (node coefficients and their spline moments), a chunk of points at a time
    const size_t per_point = (size_t)p->d.max_ell * 32 * nk * 4;
    size_t chunk = ((size_t)512 << 20) / per_point;
    if (p->d.n_interp > 0) {
      const size_t per_kg = per_point + (size_t)2 * T * nb * p->d.n_interp * M * 8;
      chunk = ((size_t)4 << 30) / per_kg;
    }
    if (chunk < 1) chunk = 1;
    if (chunk > (size_t)B) chunk = B;
    p->d.vchunk = (int)chunk;
    ALLOC(vbuf, char, chunk * per_point);
  }
  std::vector<int> kg_ia;
  std::vector<float> kg_w, kg_ip;
  std::vector<double> kg_ones;
  if (p->d.n_interp > 0) {
    const int A = p->d.n_interp;
    const size_t chunk = p->d.vchunk;
    p->d.kg_ntile = (p->d.max_ell + 63) / 64 + nb;
    ALLOC(kg_ones, double, (size_t)B * p->d.n_zg);
    ALLOC(kg_ia, int, nk);
    ALLOC(kg_w, float, (size_t)4 * nk);
    ALLOC(kg_ip, float, A);
    ALLOC(kg_uh, float, (size_t)SWIFTCL_NKINDS * p->d.n_ell * 2 * M);
    ALLOC(kg_c, char, chunk * T * nb * A * M * 8);
    ALLOC(kg_m, char, chunk * T * nb * A * M * 8);
    ALLOC(kg_perm, int, chunk * p->d.max_ell);
    ALLOC(kg_tile, int, chunk * p->d.kg_ntile * 4);
    // natural spline through the nodes, uniform in ln k: interval, offset and weights of every k node
    const double lk0 = std::log(d->k[0]);
    const double h = (std::log(d->k[nk - 1]) - lk0) / (A - 1);
    kg_ia.resize(nk);
    kg_w.resize((size_t)4 * nk);
    for (int j = 0; j < nk; ++j) {
      const double u = (std::log(d->k[j]) - lk0) / h;
      const int a = std::min(std::max((int)std::floor(u), 0), A - 2);
      const double tt = u - a, ut = 1.0 - tt;
      kg_ia[j] = a;
      kg_w[4 * (size_t)j] = (float)ut;
      kg_w[4 * (size_t)j + 1] = (float)tt;
      kg_w[4 * (size_t)j + 2] = (float)(h * h / 6.0 * (ut * ut * ut - ut));
      kg_w[4 * (size_t)j + 3] = (float)(h * h / 6.0 * (tt * tt * tt - tt));
    }
    // node rows a 64-node k tile of the windows GEMM reads (its intervals and the one after the last)
    int rows = 0;
    for (int j0 = 0; j0 < nk; j0 += 64) rows = std::max(rows, kg_ia[std::min(j0 + 63, nk - 1)] - kg_ia[j0] + 2);
    p->d.kg_stage = rows <= 16 ? 1 : 0;
    kg_ip.assign(A, 0.f);
    double ip = 0.0;
    for (int a = 1; a + 1 < A; ++a) {
      ip = 1.0 / (4.0 - ip);
      kg_ip[a] = (float)ip;
    }
    kg_ones.assign((size_t)B * p->d.n_zg, 1.0);
  }
  p->d.sched_stride = sched_stride_for(B);
  ALLOC(sched, int, sched_ints(p->d.sched_stride));
  if (p->d.adjoint == 1) ALLOC(bwd_order, int, p->d.bwd_order_n);
  if (p->d.adjoint == 2 || p->d.n_interp > 0) {
    // multipole chunks per point of the workspace adjoint (and of the scale-dependent growth
    // adjoint): about 4096 wavefronts of adjoint transforms per chunk of points (one per point,
    // chunk and tracer)
    const long pts = std::min(p->d.vchunk, B);
    long nlc = (4096 + pts * T - 1) / (pts * T);
    nlc = std::max(1L, std::min(nlc, (long)p->d.max_ell));
    p->d.bwd_nlc = (int)nlc;
    p->d.bwd_slots = std::max(p->d.bwd_slots, (int)(nlc * B));
  }
  ALLOC(dchat_part, char, (size_t)p->d.bwd_slots * T * nb * M * 2 * rs);
  ALLOC(dpk_part, char, (size_t)p->d.bwd_slots * nk * rs);
  ALLOC(dg, char, (size_t)B * T * nb * N * rs);
#undef ALLOC

  // --- uploads (host tables converted to the FFT precision) ---
  auto to_real = [&](const std::vector<double>& v) {
    std::vector<char> buf(v.size() * rs);
    if (rs == 8) std::memcpy(buf.data(), v.data(), buf.size());
    else for (size_t i = 0; i < v.size(); ++i) ((float*)buf.data())[i] = (float)v[i];
    return buf;
  };
  std::vector<char> kscale_r = to_real(kscale), tw_r = to_real(twd);
  double* d_ell = nullptr;
  hipError_t e = hipMalloc((void**)&d_ell, sizeof(double) * p->d.n_ell);
  if (e != hipSuccess) { free_plan(p); set_error("hipMalloc failed for ell"); return SWIFTCL_E_NOMEM; }
  struct Up { void* dst; const void* src; size_t n; } ups[] = {
      {p->d.kscale, kscale_r.data(), kscale_r.size()},
      {p->d.tw, tw_r.data(), tw_r.size()},
      {p->d.fell, fell.data(), fell.size() * sizeof(double)},
      {p->d.ell_band, band.data(), band.size() * sizeof(int)},
      {p->d.kw, kw.data(), kw.size() * sizeof(double)},
      {p->d.ell_v, d->ell, (size_t)p->d.n_ell * sizeof(double)},
      {p->d.lnk, lnk.data(), lnk.size() * sizeof(double)},
      {p->d.lu_k, luk.data(), luk.size() * sizeof(double)},
      {p->d.ebm, ebm.data(), ebm.size() * sizeof(double)},
      {p->d.z_geom, d->z_geom, (size_t)p->d.n_zg * sizeof(double)},
      {p->d.z_nz, d->z_nz, (size_t)p->d.n_zs * sizeof(double)},
      {p->d.lu_geom, lug.data(), lug.size() * sizeof(double)},
      {p->d.lu_nz, lun.data(), lun.size() * sizeof(double)},
      {p->d.z_union, zu.data(), zu.size() * sizeof(double)},
      {p->d.union_iv, uiv.data(), uiv.size() * sizeof(int)},
      {d_ell, d->ell, (size_t)p->d.n_ell * sizeof(double)},
  };
  for (auto& u : ups) {
    e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) break;
  }
  if (e == hipSuccess && p->d.n_interp > 0) {
    const Up kg[] = {{p->d.kg_ones, kg_ones.data(), kg_ones.size() * sizeof(double)},
                     {p->d.kg_ia, kg_ia.data(), kg_ia.size() * sizeof(int)},
                     {p->d.kg_w, kg_w.data(), kg_w.size() * sizeof(float)},
                     {p->d.kg_ip, kg_ip.data(), kg_ip.size() * sizeof(float)}};
    for (auto& u : kg) {
      e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, s);
      if (e != hipSuccess) break;
    }
  }
  if (e == hipSuccess) e = hipMemsetAsync(p->d.flags, 0, sizeof(int), s);
  if (e == hipSuccess) e = launch_u_table(p->d, d_ell, s);
  if (e == hipSuccess && p->d.n_interp > 0) e = launch_kgrowth_tables(p->d, s);
  // the host vectors above die at return: finish the copies before handing the plan out
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_ell);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_check(e, "plan set-up");
  }
  *out = p;
  return SWIFTCL_OK;
}

extern "C" swiftcl_status swiftcl_plan_destroy(swiftcl_plan_t p) {
  if (!p) { set_error("plan is NULL"); return SWIFTCL_E_INVALID; }
  free_plan(p);
  return SWIFTCL_OK;
}

extern "C" swiftcl_status swiftcl_device_flags(swiftcl_plan_t p, void* stream, int32_t* flags) {
  if (!p || !flags) { set_error("NULL argument"); return SWIFTCL_E_INVALID; }
  hipStream_t s = (hipStream_t)stream;
  int v = 0;
  hipError_t e = hipMemcpyAsync(&v, p->d.flags, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemsetAsync(p->d.flags, 0, sizeof(int), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_check(e, "device flags");
  *flags = v;
  return SWIFTCL_OK;
}

swiftcl_status check_inputs(swiftcl_plan_t p, const swiftcl_inputs* in) {
  if (!p) { set_error("plan is NULL"); return SWIFTCL_E_INVALID; }
  if (!in) { set_error("inputs is NULL"); return SWIFTCL_E_INVALID; }
  if (in->mag && !p->d.mag) { set_error("inputs carry magnification; build the plan with magnification = 1"); return SWIFTCL_E_INVALID; }
  if (in->batch < 1 || in->batch > p->d.max_batch) { set_error("batch outside 1..max_batch"); return SWIFTCL_E_INVALID; }
  const void* req[] = {in->n_tracers, in->kind, in->n_ell, in->ell_idx, in->chi_z, in->pk};
  for (const void* q : req)
    if (!q) { set_error("a required input pointer is NULL"); return SWIFTCL_E_INVALID; }
  if (in->kernel_chi) {
    // kernel samples replace the assembly: n(z), bias, D(z), Omega_m, A_IA and C_g are not read
    if (p->d.rsd || p->d.mag) {
      set_error("kernel samples (kernel_chi) are not built with redshift-space distortions or magnification");
      return SWIFTCL_E_UNSUPPORTED;
    }
    return SWIFTCL_OK;
  }
  const void* req_asm[] = {in->D_z, in->omega_m, in->nz, in->bias};
  for (const void* q : req_asm)
    if (!q) { set_error("a required input pointer is NULL (nz, bias, D_z and omega_m unless kernel_chi is given)"); return SWIFTCL_E_INVALID; }
  return SWIFTCL_OK;
}

// The workspace state (kernel samples, spline moments, lensing integrals, FFTLog coefficients)
// now belongs to `in`; a backward call may skip recomputing it (SWIFTCL_BWD_REUSE_FORWARD).
static void note_forward(swiftcl_plan_t p, const swiftcl_inputs* in) {
  p->fwd_valid = true;
  p->fwd_in = *in;
}

static bool same_inputs(const swiftcl_inputs& a, const swiftcl_inputs& b) {
  return a.batch == b.batch && a.n_tracers == b.n_tracers && a.kind == b.kind && a.n_ell == b.n_ell &&
         a.ell_idx == b.ell_idx && a.chi_z == b.chi_z && a.D_z == b.D_z && a.omega_m == b.omega_m && a.nz == b.nz &&
         a.bias == b.bias && a.pk == b.pk && a.ia == b.ia && a.mag == b.mag && a.kernel_chi == b.kernel_chi;
}

static swiftcl_status run_forward(swiftcl_plan_t p, const swiftcl_inputs* in, void* W, void* C, void* stream) {
  swiftcl_status st = check_inputs(p, in);
  if (st != SWIFTCL_OK) return st;
  if (!W && !C) { set_error("output is NULL"); return SWIFTCL_E_INVALID; }
  if ((st = hip_check(hipSetDevice(p->d.device), "hipSetDevice")) != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  p->fwd_valid = false;
  hipError_t e = launch_assemble(p->d, in, s);
  if (e == hipSuccess) e = launch_forward_fft(p->d, in, s);
  if (e == hipSuccess) note_forward(p, in);
  if (e == hipSuccess) e = launch_windows_cl(p->d, in, W, C, s);
  return hip_check(e, "forward launch");
}

extern "C" swiftcl_status swiftcl_windows(swiftcl_plan_t p, const swiftcl_inputs* in, void* W, void* stream) {
  if (!W) { set_error("W is NULL"); return SWIFTCL_E_INVALID; }
  if (p && (p->d.rsd || p->d.mag)) {
    set_error("windows output is not built with redshift-space distortions or magnification (C_l is)");
    return SWIFTCL_E_UNSUPPORTED;
  }
  return run_forward(p, in, W, nullptr, stream);
}

extern "C" swiftcl_status swiftcl_cl(swiftcl_plan_t p, const swiftcl_inputs* in, void* C, void* stream) {
  if (!C) { set_error("C is NULL"); return SWIFTCL_E_INVALID; }
  return run_forward(p, in, nullptr, C, stream);
}

extern "C" swiftcl_status swiftcl_cl_timed(swiftcl_plan_t p, const swiftcl_inputs* in, void* C, void* stream,
                                           float* stage_ms) {
  swiftcl_status st = check_inputs(p, in);
  if (st != SWIFTCL_OK) return st;
  if (!C || !stage_ms) { set_error("C or stage_ms is NULL"); return SWIFTCL_E_INVALID; }
  if ((st = hip_check(hipSetDevice(p->d.device), "hipSetDevice")) != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  p->fwd_valid = false;
  if (e == hipSuccess) e = hipEventRecord(ev[0], s);
  if (e == hipSuccess) e = launch_assemble(p->d, in, s);
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess) e = launch_forward_fft(p->d, in, s);
  if (e == hipSuccess) note_forward(p, in);
  if (e == hipSuccess) e = hipEventRecord(ev[2], s);
  if (e == hipSuccess) e = launch_windows_cl(p->d, in, nullptr, C, s);
  if (e == hipSuccess) e = hipEventRecord(ev[3], s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
  for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventElapsedTime(&stage_ms[i], ev[i], ev[i + 1]);
  for (int i = 0; i < 4; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  return hip_check(e, "timed forward");
}

extern "C" swiftcl_status swiftcl_cl_kgrowth(swiftcl_plan_t p, const swiftcl_inputs* in, const double* D_kz, void* C,
                                             void* stream) {
  if (!p) { set_error("plan is NULL"); return SWIFTCL_E_INVALID; }
  if (!in) { set_error("inputs is NULL"); return SWIFTCL_E_INVALID; }
  if (!D_kz || !C) { set_error("D_kz or C is NULL"); return SWIFTCL_E_INVALID; }
  if (p->d.n_interp < 2) {
    set_error("the plan has no interpolation nodes in k (n_interp = 0)");
    return SWIFTCL_E_INVALID;
  }
  if (p->d.rsd || p->d.mag) {
    set_error("scale-dependent growth is not built with redshift-space distortions or magnification");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if (in->kernel_chi) {
    set_error("scale-dependent growth assembles its kernels per k node; kernel samples (kernel_chi) are refused");
    return SWIFTCL_E_UNSUPPORTED;
  }
  // the kernels are assembled without growth (D = 1); growth enters per node
  swiftcl_inputs in1 = *in;
  in1.D_z = p->d.kg_ones;
  swiftcl_status st = check_inputs(p, &in1);
  if (st != SWIFTCL_OK) return st;
  if ((st = hip_check(hipSetDevice(p->d.device), "hipSetDevice")) != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  p->fwd_valid = false;
  hipError_t e = launch_assemble(p->d, &in1, s);
  if (e == hipSuccess) e = launch_sqrt_s(p->d, &in1, s);
  if (e == hipSuccess) e = launch_kgrowth(p->d, &in1, D_kz, C, s);
  return hip_check(e, "scale-dependent growth launch");
}

extern "C" swiftcl_status swiftcl_cl_kgrowth_backward(swiftcl_plan_t p, const swiftcl_inputs* in, const double* D_kz,
                                                      const void* C, const void* dC, double* dpk, double* dbias,
                                                      void* stream) {
  if (!p) { set_error("plan is NULL"); return SWIFTCL_E_INVALID; }
  if (!in) { set_error("inputs is NULL"); return SWIFTCL_E_INVALID; }
  if (!D_kz || !dC) { set_error("D_kz or dC is NULL"); return SWIFTCL_E_INVALID; }
  if (dbias && !C) { set_error("dbias needs C, the forward output"); return SWIFTCL_E_INVALID; }
  if (p->d.n_interp < 2) {
    set_error("the plan has no interpolation nodes in k (n_interp = 0)");
    return SWIFTCL_E_INVALID;
  }
  if (p->d.rsd || p->d.mag) {
    set_error("scale-dependent growth is not built with redshift-space distortions or magnification");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if (in->kernel_chi) {
    set_error("scale-dependent growth assembles its kernels per k node; kernel samples (kernel_chi) are refused");
    return SWIFTCL_E_UNSUPPORTED;
  }
  swiftcl_inputs in1 = *in;
  in1.D_z = p->d.kg_ones;
  swiftcl_status st = check_inputs(p, &in1);
  if (st != SWIFTCL_OK) return st;
  if ((st = hip_check(hipSetDevice(p->d.device), "hipSetDevice")) != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  p->fwd_valid = false;
  hipError_t e = hipSuccess;
  if (dpk) {
    e = launch_assemble(p->d, &in1, s);
    if (e == hipSuccess) e = launch_sqrt_s(p->d, &in1, s);
  }
  if (e == hipSuccess) e = launch_kgrowth_backward(p->d, &in1, D_kz, C, dC, dpk, dbias, s);
  return hip_check(e, "scale-dependent growth backward launch");
}

extern "C" swiftcl_status swiftcl_cl_limber(swiftcl_plan_t p, const swiftcl_inputs* in, void* C, void* stream) {
  swiftcl_status st = check_inputs(p, in);
  if (st != SWIFTCL_OK) return st;
  if (!C) { set_error("C is NULL"); return SWIFTCL_E_INVALID; }
  if (p->d.rsd || p->d.mag) {
    set_error("the Limber path does not include redshift-space distortions or magnification");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if (in->kernel_chi) {
    set_error("the Limber path takes its kernels from the assembly; kernel samples (kernel_chi) are refused");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if ((st = hip_check(hipSetDevice(p->d.device), "hipSetDevice")) != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  p->fwd_valid = false;  // the FFTLog coefficients are not computed
  hipError_t e = launch_assemble(p->d, in, s);
  if (e == hipSuccess) e = launch_limber(p->d, in, C, s);
  return hip_check(e, "Limber launch");
}

size_t limber_bwd_lds_bytes(const plan_dev& p);

extern "C" swiftcl_status swiftcl_cl_limber_backward(swiftcl_plan_t p, const swiftcl_inputs* in, const void* dC,
                                                     double* dpk, double* dbias, double* dnz, double* dD,
                                                     void* stream) {
  swiftcl_status st = check_inputs(p, in);
  if (st != SWIFTCL_OK) return st;
  if (!dC) { set_error("dC is NULL"); return SWIFTCL_E_INVALID; }
  if (p->d.rsd || p->d.mag) {
    set_error("the Limber path does not include redshift-space distortions or magnification");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if (in->kernel_chi) {
    set_error("the Limber path takes its kernels from the assembly; kernel samples (kernel_chi) are refused");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if ((st = hip_check(hipSetDevice(p->d.device), "hipSetDevice")) != SWIFTCL_OK) return st;
  int lds_max = 0;
  if ((st = hip_check(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->d.device),
                      "device attribute")) != SWIFTCL_OK)
    return st;
  if (limber_bwd_lds_bytes(p->d) > (size_t)lds_max) {
    set_error("the Limber adjoint needs " + std::to_string(limber_bwd_lds_bytes(p->d)) +
              " bytes of LDS per workgroup (max_tracers, n_k); the device has " + std::to_string(lds_max));
    return SWIFTCL_E_UNSUPPORTED;
  }
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  p->fwd_valid = false;
  hipError_t e = launch_assemble(p->d, in, s);
  if (e == hipSuccess) e = launch_limber_backward(p->d, in, dC, dpk, dbias, dnz, dD, s);
  return hip_check(e, "Limber backward launch");
}

// Checks shared by the two backward entry points; `reuse` is set when the forward state is kept.
static swiftcl_status backward_checks(swiftcl_plan_t p, const swiftcl_inputs* in, const void* dC, uint32_t flags,
                                      bool* reuse, const double* dbias, const double* dnz, const double* dD) {
  swiftcl_status st = check_inputs(p, in);
  if (st != SWIFTCL_OK) return st;
  if (!dC) { set_error("dC is NULL"); return SWIFTCL_E_INVALID; }
  if (in->kernel_chi && (dbias || dnz || dD)) {
    set_error("with kernel samples (kernel_chi) the backward gives dpk only: dbias, dnz and dD must be NULL");
    return SWIFTCL_E_INVALID;
  }
  if (flags & ~(uint32_t)SWIFTCL_BWD_REUSE_FORWARD) { set_error("unknown backward flag"); return SWIFTCL_E_INVALID; }
  if (!p->d.adjoint) {
    set_error("the FP64 adjoint keeps the windows of <= 16 tracers in LDS; this n_chi / n_k does not fit");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if ((p->d.rsd || p->d.mag) && (dnz || dD)) {
    set_error("with redshift-space distortions or magnification the backward gives dpk and dbias only: dnz and dD "
              "must be NULL");
    return SWIFTCL_E_UNSUPPORTED;
  }
  *reuse = (flags & SWIFTCL_BWD_REUSE_FORWARD) != 0;
  if (*reuse && !(p->fwd_valid && same_inputs(p->fwd_in, *in))) {
    set_error("SWIFTCL_BWD_REUSE_FORWARD: the plan's last forward call was made with other inputs");
    return SWIFTCL_E_INVALID;
  }
  return hip_check(hipSetDevice(p->d.device), "hipSetDevice");
}

extern "C" swiftcl_status swiftcl_cl_backward(swiftcl_plan_t p, const swiftcl_inputs* in, const void* dC,
                                              double* dpk, double* dbias, double* dnz, double* dD, uint32_t flags,
                                              void* stream) {
  bool reuse = false;
  swiftcl_status st = backward_checks(p, in, dC, flags, &reuse, dbias, dnz, dD);
  if (st != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (!reuse) {
    p->fwd_valid = false;
    e = launch_assemble(p->d, in, s);
    if (e == hipSuccess) e = launch_forward_fft(p->d, in, s);
    if (e == hipSuccess) note_forward(p, in);
  }
  if (e == hipSuccess) e = launch_backward(p->d, in, dC, dpk, dbias, dnz, dD, s);
  return hip_check(e, "backward launch");
}

extern "C" swiftcl_status swiftcl_cl_backward_timed(swiftcl_plan_t p, const swiftcl_inputs* in, const void* dC,
                                                    double* dpk, double* dbias, double* dnz, double* dD,
                                                    uint32_t flags, void* stream, float* stage_ms) {
  if (!stage_ms) { set_error("stage_ms is NULL"); return SWIFTCL_E_INVALID; }
  bool reuse = false;
  swiftcl_status st = backward_checks(p, in, dC, flags, &reuse, dbias, dnz, dD);
  if (st != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 6 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  if (e == hipSuccess) e = hipEventRecord(ev[0], s);
  if (e == hipSuccess && !reuse) {
    p->fwd_valid = false;
    e = launch_assemble(p->d, in, s);
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess && !reuse) {
    e = launch_forward_fft(p->d, in, s);
    if (e == hipSuccess) note_forward(p, in);
  }
  if (e == hipSuccess) e = hipEventRecord(ev[2], s);
  if (e == hipSuccess) e = launch_backward(p->d, in, dC, dpk, dbias, dnz, dD, s, &ev[3]);
  if (e == hipSuccess) e = hipEventRecord(ev[5], s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
  for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipEventElapsedTime(&stage_ms[i], ev[i], ev[i + 1]);
  for (int i = 0; i < 6; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  return hip_check(e, "timed backward");
}

// ---------------------------------------------------------------------------------------------
// Autotuner: times the launch variants on the caller's inputs and keeps the fastest in the plan.
// Choices: fwd_mode (one workgroup per slot / persistent per-XCD lists / persistent packed lists)
// and bwd_chunk_mul (1, 2, 4, 8 x the base multipole-chunk count of the adjoint).  Results are cached, one JSON object per
// line, keyed by device architecture and shape.
// ---------------------------------------------------------------------------------------------
static std::string tune_key(const swiftcl_plan_s* p, int batch) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->d.device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|N%d|nk%d|T%d|L%d|B%d|p%d|bands%d", arch.c_str(), p->d.N, p->d.n_k,
           p->d.max_tracers, p->d.max_ell, batch, p->d.precision, p->d.n_bands);
  return buf;
}

static bool cache_lookup(const char* path, const std::string& key, int* fwd_mode, int* chunk_mul, int* pack) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  const std::string needle = "\"key\": \"" + key + "\"";
  while (fgets(line, sizeof(line), f)) {
    if (!strstr(line, needle.c_str())) continue;
    const char* a = strstr(line, "\"fwd_mode\": ");
    const char* b = strstr(line, "\"bwd_chunk_mul\": ");
    const char* c = strstr(line, "\"bwd_pack\": ");
    if (a && b) {
      *fwd_mode = atoi(a + 12);
      *chunk_mul = atoi(b + 17);
      *pack = c ? atoi(c + 12) : 0;
      found = (*fwd_mode >= 0 && *fwd_mode <= 2) &&
              (*chunk_mul == 1 || *chunk_mul == 2 || *chunk_mul == 4 || *chunk_mul == 8) &&
              (*pack == 0 || (*pack == 1 && *chunk_mul <= 4));
    }
  }
  fclose(f);
  return found;
}

static float time_ms(hipStream_t s, const std::function<hipError_t()>& fn, hipError_t* err) {
  hipEvent_t a = nullptr, b = nullptr;
  float best = 1e30f;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = fn();  // warm-up
  for (int r = 0; r < 3 && e == hipSuccess; ++r) {
    e = hipEventRecord(a, s);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess && ms < best) best = ms;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  *err = e;
  return best;
}

extern "C" swiftcl_status swiftcl_autotune(swiftcl_plan_t p, const swiftcl_inputs* in, void* C, const void* dC,
                                           void* stream, const char* cache_path, char* report, int32_t report_len) {
  swiftcl_status st = check_inputs(p, in);
  if (st != SWIFTCL_OK) return st;
  if (!C) { set_error("C is NULL"); return SWIFTCL_E_INVALID; }
  if ((st = hip_check(hipSetDevice(p->d.device), "hipSetDevice")) != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = (hipStream_t)stream;
  const std::string key = tune_key(p, in->batch);
  std::string rep;
  int fm = 0, cm = 1, pk = 0;
  if (cache_lookup(cache_path, key, &fm, &cm, &pk)) {
    p->d.fwd_mode = fm;
    p->d.bwd_chunk_mul = cm;
    p->d.bwd_pack = pk;
    rep = "cached " + key + ": fwd_mode=" + std::to_string(fm) + " bwd_chunk_mul=" + std::to_string(cm) +
          " bwd_pack=" + std::to_string(pk);
  } else {
    p->fwd_valid = false;
    hipError_t e = launch_assemble(p->d, in, s);
    if (e == hipSuccess) e = launch_forward_fft(p->d, in, s);
    if (e == hipSuccess) note_forward(p, in);
    const bool tune_bwd = dC && p->d.fused && p->d.precision != SWIFTCL_SPLIT_BF16;
    // warm-up in the default shapes: the clock ramps up over the first milliseconds of work, which
    // would favour the variants timed last; then two rounds over the variants, keeping each one's best
    p->d.fwd_mode = 0;
    p->d.bwd_chunk_mul = 1;
    p->d.bwd_pack = 0;
    for (int r = 0; r < 10 && e == hipSuccess; ++r) {
      e = launch_windows_cl(p->d, in, nullptr, C, s);
      if (e == hipSuccess && tune_bwd) e = launch_backward(p->d, in, dC, nullptr, nullptr, nullptr, nullptr, s);
    }
    float tf[3] = {1e30f, 1e30f, 1e30f};
    for (int round = 0; round < 2; ++round)
      for (int m = 0; m < (p->d.fused ? 3 : 1) && e == hipSuccess; ++m) {
        p->d.fwd_mode = m;
        tf[m] = std::min(tf[m], time_ms(s, [&]() { return launch_windows_cl(p->d, in, nullptr, C, s); }, &e));
      }
    if (e != hipSuccess) { p->d.fwd_mode = 0; return hip_check(e, "autotune forward"); }
    // a variant other than the default must win by 2% (run-to-run noise is ~1%)
    int fb = 0;
    for (int m = 1; m < 3; ++m)
      if (tf[m] < tf[fb]) fb = m;
    p->d.fwd_mode = tf[fb] < 0.98f * tf[0] ? fb : 0;
    // the adjoint: chunk multipliers 1, 2, 4, 8 unpacked, then 1, 2, 4 packed (FP32 plans)
    float tb[7] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
    const int muls[7] = {1, 2, 4, 8, 1, 2, 4};
    const int packs[7] = {0, 0, 0, 0, 1, 1, 1};
    if (tune_bwd) {
      const int nv = p->d.precision == SWIFTCL_FP32 ? 7 : 4;
      for (int round = 0; round < 2; ++round)
        for (int i = 0; i < nv && e == hipSuccess; ++i) {
          p->d.bwd_chunk_mul = muls[i];
          p->d.bwd_pack = packs[i];
          tb[i] = std::min(tb[i], time_ms(s, [&]() {
            return launch_backward(p->d, in, dC, nullptr, nullptr, nullptr, nullptr, s);
          }, &e));
        }
      if (e != hipSuccess) {
        p->d.bwd_chunk_mul = 1;
        p->d.bwd_pack = 0;
        return hip_check(e, "autotune backward");
      }
      int bi = 0;
      for (int i = 1; i < nv; ++i)
        if (tb[i] < tb[bi]) bi = i;
      if (tb[bi] >= 0.98f * tb[0]) bi = 0;
      p->d.bwd_chunk_mul = muls[bi];
      p->d.bwd_pack = packs[bi];
    }
    auto tv = [&](int i) { return dC && tb[i] < 1e29f ? tb[i] : 0.f; };
    char buf[640];
    snprintf(buf, sizeof(buf),
             "{\"key\": \"%s\", \"fwd_mode\": %d, \"bwd_chunk_mul\": %d, \"bwd_pack\": %d, "
             "\"fwd_ms\": [%.4f, %.4f, %.4f], \"bwd_ms\": [%.4f, %.4f, %.4f, %.4f], \"bwd_pack_ms\": [%.4f, %.4f, %.4f]}",
             key.c_str(), p->d.fwd_mode, p->d.bwd_chunk_mul, p->d.bwd_pack, tf[0], tf[1], tf[2], tv(0), tv(1), tv(2),
             tv(3), tv(4), tv(5), tv(6));
    rep = buf;
    if (cache_path) {
      FILE* f = fopen(cache_path, "a");
      if (f) {
        fprintf(f, "%s\n", buf);
        fclose(f);
      }
    }
  }
  if (report && report_len > 0) {
    strncpy(report, rep.c_str(), (size_t)report_len - 1);
    report[report_len - 1] = '\0';
  }
  return SWIFTCL_OK;
}

extern "C" swiftcl_status swiftcl_set_launch(swiftcl_plan_t p, int32_t fwd_mode, int32_t bwd_chunk_mul,
                                             int32_t bwd_pack) {
  if (!p) { set_error("plan is NULL"); return SWIFTCL_E_INVALID; }
  if (fwd_mode > 2) { set_error("fwd_mode must be 0, 1 or 2"); return SWIFTCL_E_INVALID; }
  if (bwd_chunk_mul >= 0 && bwd_chunk_mul != 1 && bwd_chunk_mul != 2 && bwd_chunk_mul != 4 && bwd_chunk_mul != 8) {
    set_error("bwd_chunk_mul must be 1, 2, 4 or 8");
    return SWIFTCL_E_INVALID;
  }
  if (bwd_pack > 1) { set_error("bwd_pack must be 0 or 1"); return SWIFTCL_E_INVALID; }
  const int cm = bwd_chunk_mul >= 0 ? bwd_chunk_mul : p->d.bwd_chunk_mul;
  const int pk = bwd_pack >= 0 ? bwd_pack : p->d.bwd_pack;
  if (pk && cm > 4) { set_error("the packed adjoint takes bwd_chunk_mul 1, 2 or 4"); return SWIFTCL_E_INVALID; }
  if (fwd_mode >= 0) p->d.fwd_mode = fwd_mode;
  p->d.bwd_chunk_mul = cm;
  p->d.bwd_pack = pk;
  return SWIFTCL_OK;
}

extern "C" swiftcl_status swiftcl_plan_info(swiftcl_plan_t p, int32_t* fused, int32_t* adjoint, int32_t* point_chunk) {
  if (!p) { set_error("plan is NULL"); return SWIFTCL_E_INVALID; }
  if (fused) *fused = p->d.fused;
  if (adjoint) *adjoint = p->d.adjoint;
  if (point_chunk) *point_chunk = p->d.vbuf ? p->d.vchunk : 0;
  return SWIFTCL_OK;
}

extern "C" swiftcl_status swiftcl_get_launch(swiftcl_plan_t p, int32_t* fwd_mode, int32_t* bwd_chunk_mul,
                                             int32_t* bwd_pack) {
  if (!p || !fwd_mode || !bwd_chunk_mul || !bwd_pack) { set_error("NULL argument"); return SWIFTCL_E_INVALID; }
  *fwd_mode = p->d.fwd_mode;
  *bwd_chunk_mul = p->d.bwd_chunk_mul;
  *bwd_pack = p->d.bwd_pack;
  return SWIFTCL_OK;
}
