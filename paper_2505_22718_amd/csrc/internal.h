// Internal plan layout and kernel launchers shared by the translation units of libswiftcl.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/swiftcl.h"
#include "sched_layout.h"

// Per-point scalars written by the spline set-up kernel (FP64), PT_STRIDE doubles per point.
enum {
  PT_CHI0 = 0,        // chi_0 = chi(z_min) exp(-edge_node Delta)
  PT_LNK0CHI0 = 1,    // ln(k_0 chi_0)
  PT_M1 = 2,          // last node inside the support (as a double)
  PT_THETA = 3,       // fractional position of chi(z_max) above node m1
  PT_CHI0B = 4,       // chi_0^{-b} for [kind][band]: SWIFTCL_NKINDS * SWIFTCL_MAX_BANDS entries
  PT_STRIDE = 16
};
static_assert(PT_CHI0B + SWIFTCL_NKINDS * SWIFTCL_MAX_BANDS <= PT_STRIDE, "per-point scalars overflow");

// Device flag bits (swiftcl_device_flags)
enum { FLAG_SUPPORT_OVERFLOW = 1, FLAG_NONFINITE = 2, FLAG_BAD_INDEX = 4 };

// Everything the kernels need: scalars and device pointers only (trivially copyable, passed
// by value to every kernel).
struct plan_dev {
  int device;
  int precision;
  int N, M, n_k, n_ell, n_zg, n_zs, n_bands, m0;
  int max_batch, max_tracers, max_ell;
  int n_union;
  double delta, k0, taper_frac;
  double band_ell_lo[SWIFTCL_MAX_BANDS];
  double fftlog_b[SWIFTCL_NKINDS][SWIFTCL_MAX_BANDS];

  // --- plan-time device tables ---
  void* U;          // [kind][n_ell][M] complex real: Bessel power-law integral U_l(n) (taper folded in)
  void* kscale;     // [kind][n_bands][n_k] real: k^{-1-b} (times k^-2 for the lensing kinds)
  void* tw;         // [N] complex real: e^{-2 pi i m / N}
  double* fell;     // [kind][n_ell] the multipole prefactor: 1, F(l) (lensing), l(l+1) (CMB lensing)
  int* ell_band;    // [n_ell]
  double* kw;       // [n_k] (2/pi) w_j k_j^3
  double* ell_v;    // [n_ell] the multipoles
  double* lnk;      // [n_k] ln k_j
  double* lu_k;     // [4][n_k] natural-spline Thomas factors of the ln k grid and 1/h (Limber P)
  double* ebm;      // [kind][n_bands][N] e^{-b m Delta}: the FFTLog bias factor of chi node m
  double* z_geom;   // [n_zg]
  double* z_nz;     // [n_zs]
  double* lu_geom;  // [4][n_zg] natural-spline Thomas factors (a, 1/pivot, c') and 1/h
  double* lu_nz;    // [4][n_zs]
  double* z_union;  // [n_union + 1] knots of the lensing quadrature
  int* union_iv;    // [2][n_union] geometry interval, n(z) interval (-1 = outside)

  // --- workspace sized for max_batch ---
  double* pt;       // [B][PT_STRIDE]
  double* m_chi;    // [B][n_zg] spline second derivatives
  double* m_D;      // [B][n_zg]
  double* m_ia;     // [B][n_zg] spline moments of A_IA(z) (intrinsic alignment inputs only)
  double* m_n;      // [B][T][n_zs]
  double* lens_q;   // [B][T][N] lensing efficiency q at the active chi nodes (forward assembly)
  double* lnp;      // [B][2][n_k] ln P and its spline moments in ln k (Limber)
  double* lim_acc;  // [B][2][n_k] Limber adjoint: cotangents of the ln P samples and of their moments
  double* phase;    // [B][N/2] complex e^{-2 pi i n ln(k_0 chi_0) / (N Delta)}: the FFTLog phase
                    // of coefficient n (forward assembly)
  double* node_f;   // [B][4][N] z, chi, dchi/dz, D at the active chi nodes (forward assembly)
  int* node_i;      // [B][3][N] their geometry, n(z) and union intervals
  double* ddD_part; // [B][T][2][n_zg] per-tracer cotangents of the D samples and of D'' (adjoint)
  void* g;          // [B][T][n_bands][N] real: tilted, edge-weighted kernel samples
  void* chat;       // [B][T][n_bands][M] complex real: FFTLog coefficients (phased)
  void* sqrt_s;     // [B][n_k] real: sqrt((2/pi) w k^3 P)
  void* kss;        // [B][kind][n_bands][n_k] real: kscale * sqrt_s, the window-to-V factor
  int* flags;       // [1]
  // backward workspace
  void* dchat_part; // [bwd_slots][T][n_bands][M] complex real: dc partials per (point, chunk)
  void* dpk_part;   // [bwd_slots][n_k] real: sum_t W Y partials per (point, chunk)
  void* dg;         // [B][T][n_bands][N] real
  int bwd_slots;    // capacity of (point, chunk) slots
  int* bwd_order;   // [bwd_order_n] workgroup -> (point, chunk) item of the fused adjoint, heaviest first
  int bwd_order_n;  // its capacity (the largest fused-adjoint grid)
  // launch configuration (autotuned; see swiftcl_autotune)
  int fwd_mode;       // 0: one workgroup per (point, multipole slot); 1: persistent, per-XCD lists;
                      // 2: persistent, packed per-XCD lists (two items of few tracers per task)
  int persist_blocks; // grid of the persistent launch (a multiple of 8)
  int bwd_chunk_mul;  // multiplier of the backward multipole-chunk count (1, 2, 4 or 8)
  int bwd_pack;       // FP32 fused adjoint: two sub-chunks per chunk, side by side for points of <= 8
                      // tracers (0 or 1; with bwd_chunk_mul <= 4)
  int* sched;         // sched_ints(sched_stride): per-XCD work lists of the persistent launch
  int sched_stride;
  // projection path: fused (windows in LDS, <= 16 tracers) or through the workspace below
  int fused;
  int adjoint;        // swiftcl_cl_backward: 0 not built, 1 fused (windows in LDS), 2 through the workspace
  int bwd_nlc;        // multipole chunks per point of the workspace adjoint
  int vchunk;         // points per chunk of the unfused path
  void* vbuf;         // [vchunk][max_ell][32][n_k] FP32, or bf16 hi then lo (unfused and kgrowth paths)
  // scale-dependent growth (swiftcl_cl_kgrowth); points run in chunks of vchunk
  int n_interp;       // k nodes (0 = not built)
  // redshift-space distortions (eq. RSD) of the clustering tracers: a second coefficient set per
  // (tracer, band) times the table of the integral of chi^p j_l''
  int rsd;
  void* UR;           // [n_ell][M] complex: sum_s a_s(l) U_s(n) over s = l-2, l, l+2 (clustering bias)
  void* g_r;          // [B][T][n_bands][N] real: tilted, edge-weighted RSD kernel samples
  void* chat_r;       // [B][T][n_bands][M] complex: their FFTLog coefficients
  // magnification bias of the clustering tracers: a lensing-type kernel decomposed with the bias
  // b - 2, so that its l(l+1)/k^2 window shares the density window's k scale
  int mag;
  void* Umu;          // [n_ell][M] complex: l(l+1) U_l(n) at the bias b - 2 of the clustering band
  void* g_mu;         // [B][T][n_bands][N] real: tilted, edge-weighted C_g q D / chi^2 samples
  void* chat_mu;      // [B][T][n_bands][M] complex: their FFTLog coefficients
  int kg_ntile;       // slot tiles per (point, tracer): ceil(max_ell / 64) + n_bands
  int kg_stage;       // 1: every 64-node k tile spans <= KG_NA node rows, which the GEMM stages in LDS
  double* kg_ones;    // [max_batch][n_zg] ones: the assembly's D(z) while growth sits at the nodes
  int* kg_ia;         // [n_k] node interval a_j of k_j
  float* kg_w;        // [n_k][4] spline weights of c_a, c_{a+1}, M_a, M_{a+1} at k_j
  float* kg_ip;       // [n_interp] 1 / pivot of the node spline's tridiagonal system
  float* kg_uh;       // [kind][n_ell][M / 16][4][8] U in the GEMM's A-operand order (h_n and signs folded)
  void* kg_c;         // [vchunk][T][n_bands][n_interp][M] complex float: node coefficients
  void* kg_m;         // same layout: their second derivatives along ln k
  int* kg_perm;       // [vchunk][max_ell] multipole slots grouped by band
  int* kg_tile;       // [vchunk][kg_ntile][4] band, first entry of kg_perm, count, 0
};

// Tracer kind of slot t of point b as the kernels use it: a value outside the three kinds reads as
// clustering (the assembly flags it, FLAG_BAD_INDEX, and writes zero kernel samples for it).
__device__ __forceinline__ int tracer_kind(const swiftcl_inputs& in, int T, int b, int t) {
  const int k = in.kind[(size_t)b * T + t];
  return (unsigned)k < (unsigned)SWIFTCL_NKINDS ? k : SWIFTCL_CLUSTERING;
}

struct swiftcl_plan_s {
  plan_dev d{};
  std::vector<double> ell_host;
  size_t real_size = 4;  // sizeof(real) on the FFT path
  // inputs whose assembly and FFTLog coefficients the last forward launch left in the workspace
  bool fwd_valid = false;
  swiftcl_inputs fwd_in{};
};

void set_error(const std::string& msg);
// host checks of a call's inputs against the plan (no device work)
swiftcl_status check_inputs(swiftcl_plan_t p, const swiftcl_inputs* in);
// takes the device address of swiftcl_cl_noalloc's static workspace on `device` (current), once
swiftcl_status noalloc_setup(int device);
size_t bwd_windows_lds(const plan_dev& p);  // dynamic LDS of the adjoint windows kernel
size_t windows_cl_lds(int M, int NW, bool tw_lds, bool do_cl, size_t rs, int n_k);
bool unfused_tw_lds(int M);
size_t geometry_lds_bytes(const plan_dev& p);
int windows_nw(int precision);
bool windows_tw_lds(int precision, int M);
size_t bwd_geometry_lds_bytes(const plan_dev& p);
int backward_chunks(const plan_dev& p, int batch);
swiftcl_status hip_check(hipError_t e, const char* what);

// Launchers (each returns the first HIP error of its launches)
hipError_t launch_u_table(const plan_dev& p, const double* d_ell, hipStream_t s);
hipError_t launch_assemble(const plan_dev& p, const swiftcl_inputs* in, hipStream_t s);
hipError_t launch_forward_fft(const plan_dev& p, const swiftcl_inputs* in, hipStream_t s);
hipError_t launch_windows_cl(const plan_dev& p, const swiftcl_inputs* in, void* W, void* C, hipStream_t s);
hipError_t launch_sqrt_s(const plan_dev& p, const swiftcl_inputs* in, hipStream_t s);
// FP32 rows W (not sqrt(s) W) of points [b0, b0 + nbp) into the workspace (vbuf), for the adjoint
hipError_t launch_windows_w(const plan_dev& p, const swiftcl_inputs* in, int b0, int nbp, hipStream_t s);
// C of points [b0, b0 + nbp) from the V rows in the workspace (vbuf)
hipError_t launch_contract(const plan_dev& p, const swiftcl_inputs* in, void* C, int b0, int nbp, hipStream_t s);
hipError_t launch_kgrowth(const plan_dev& p, const swiftcl_inputs* in, const double* D_kz, void* C, hipStream_t s);
hipError_t launch_kgrowth_backward(const plan_dev& p, const swiftcl_inputs* in, const double* D_kz, const void* C,
                                   const void* dC, double* dpk, double* dbias, hipStream_t s);
hipError_t launch_bwd_gv(const plan_dev& p, const swiftcl_inputs* in, const void* dC, int b0, int nbp, hipStream_t s);
hipError_t launch_bwd_dpk(const plan_dev& p, const swiftcl_inputs* in, double* dpk, hipStream_t s);
size_t kgrowth_fft_lds(int M, int n_zg);  // dynamic LDS of the node-coefficient kernel
hipError_t launch_limber(const plan_dev& p, const swiftcl_inputs* in, void* C, hipStream_t s);
// adjoint of launch_limber (after launch_assemble): dpk, dbias, dnz, dD each optional (NULL)
hipError_t launch_limber_backward(const plan_dev& p, const swiftcl_inputs* in, const void* dC, double* dpk,
                                  double* dbias, double* dnz, double* dD, hipStream_t s);
// chain rule from the kernel-sample cotangents dg (P.dg) to dbias, dnz (k_bwd_tracer) and dD
// (k_bwd_point), as the FFTLog adjoint ends; dP is left to the caller
hipError_t launch_bwd_chain(const plan_dev& p, const swiftcl_inputs* in, double* dbias, double* dnz, double* dD,
                            hipStream_t s);
hipError_t launch_kgrowth_tables(const plan_dev& p, hipStream_t s);  // plan time, after the U table
// ev (optional): two events recorded after the first and second backward kernels
hipError_t launch_backward(const plan_dev& p, const swiftcl_inputs* in, const void* dC, double* dpk,
                           double* dbias, double* dnz, double* dD, hipStream_t s, hipEvent_t* ev = nullptr);
