/*
 * swiftcl.h -- C ABI of the MI355X (gfx950) beyond-Limber angular power spectrum path.
 *
 * Method (Reymond, Reeves, Zhang & Refregier, "SwiftC_l: fast differentiable angular
 * power spectra beyond Limber"):
 *   C_l^{ij} = (2/pi) int dk k^2 Delta_l^i(k) Delta_l^j(k) P(k)             (Sec. 2.1)
 *   Delta_l^i(k) = c_i(l, k) int dchi f_i(chi) j_l(k chi)                   (Sec. 2.1-2.3)
 * with f_i the radial kernel of tracer i times growth (and bias):
 *   clustering  f = b n(z) (dz/dchi) D(z),          c = 1                     (Sec. 2.2)
 *   lensing     f = q(chi) D(z) / chi^2,             c = sqrt((l+2)!/(l-2)!) / k^2   (Sec. 2.3,
 *               q = eq. "tomographic lens efficiency")
 *   CMB lensing f = 1.5 Om (H0/c)^2 (1+z) (chi_* - chi) / (chi chi_*) D(z),  c = l(l+1) / k^2
 *               (Sec. 2.4: one source plane at the last-scattering distance chi_*)
 * The chi integral uses an FFTLog decomposition of f in ln chi (Sec. 3.1, eq. FFTLog) and the
 * analytic integral of chi^p j_l(k chi) (eq. int_jl, with the denominator Gamma((2+l-p)/2));
 * the k integral runs over the caller's k nodes (Sec. 3.2).
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - k must be log-spaced; the chi grid has the same log step Delta, so the windows land on the
 *     caller's k nodes; the lower support edge chi(z_min) sits on node `edge_node`.
 *   - The kernel is zero outside [chi(z_min), chi(z_max)]; edge nodes carry trapezoid weights
 *     (1/2 on the lower edge, 1/2 + theta on the upper one).
 *   - The Nyquist coefficient is dropped; the FFTLog bias b is chosen per tracer kind and per
 *     multipole band.
 *   - Samples (chi(z), D(z) on z_geom; n(z) on z_nz) are continued by natural cubic splines.
 *   - The k integral is the trapezoid rule in ln k.
 *
 * Every function returns a swiftcl_status and never throws, exits or synchronises implicitly.
 * Argument checks that need no device data run before any device work.  The message of the last
 * error on the calling thread is returned by swiftcl_last_error().
 */
#ifndef SWIFTCL_H
#define SWIFTCL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SWIFTCL_OK = 0,
  SWIFTCL_E_INVALID = -1,     /* a bad argument (null pointer, size, layout) */
  SWIFTCL_E_DOMAIN = -2,      /* a value outside the method's domain (b range, k spacing) */
  SWIFTCL_E_NOMEM = -3,       /* device or host allocation failed (swiftcl_plan only) */
  SWIFTCL_E_DEVICE = -4,      /* a HIP runtime error */
  SWIFTCL_E_UNSUPPORTED = -5  /* a size the library does not handle (e.g. n_chi) */
} swiftcl_status;

/* Tracer kinds.  The CMB-lensing kernel ends at chi_* = chi(z_geom[n_zg-1]): the top of the geometry
 * grid is the last-scattering surface (z_*), so a plan that carries CMB lensing continues its
 * geometry grid to z_*; the kernel falls linearly to zero there, so its last node takes the
 * trapezoid weight of a linear end, 1/2 + theta/2, in place of a jump's 1/2 + theta. */
enum { SWIFTCL_CLUSTERING = 0, SWIFTCL_LENSING = 1, SWIFTCL_CMB_LENSING = 2 };
#define SWIFTCL_NKINDS 3

typedef enum {
  SWIFTCL_FP64 = 0,       /* FFTs and contraction in double; outputs double */
  SWIFTCL_FP32 = 1,       /* FFTs and contraction in float; outputs float */
  SWIFTCL_SPLIT_BF16 = 2  /* FFTs in float; contraction as bf16 hi+lo MFMA, FP32 accumulate */
} swiftcl_precision;

#define SWIFTCL_MAX_BANDS 4

typedef struct swiftcl_plan_s* swiftcl_plan_t; /* opaque, owned by the library */

/* Plan descriptor.  Host memory; everything is copied by swiftcl_plan. */
typedef struct {
  int32_t n_chi;        /* FFTLog length N_FFT (Sec. 3.1): power of two in [64, 4096], >= n_k   */
  int32_t edge_node;    /* chi-grid node of chi(z_min), 1..n_chi-2; <= 0 picks a centred default */
  int32_t n_bands;      /* number of multipole bands, 1..SWIFTCL_MAX_BANDS                      */
  double band_ell_lo[SWIFTCL_MAX_BANDS]; /* band j holds band_ell_lo[j] <= l < band_ell_lo[j+1];
                                            band_ell_lo[0] <= min(ell), strictly increasing     */
  double fftlog_b[SWIFTCL_NKINDS][SWIFTCL_MAX_BANDS]; /* FFTLog bias b per tracer kind and band
                                            (Sec. 3.1); every l of the band needs -l-1 < b < 1
                                            (eq. int_jl); plans with rsd or magnification also need
                                            1-l < b for the clustering row (they evaluate eq.
                                            int_jl at l-2, and at b-2)                           */
  double taper_frac;    /* cosine taper of c_n over the top fraction of |n| ("smoothing at the
                           tails", Sec. 3.1); 0 = none; in [0, 1)                              */
  int32_t n_k;          /* number of k nodes (Sec. 3.2: the k integral runs over all of them)   */
  const double* k;      /* [n_k] h/Mpc, increasing, log-spaced to 1e-9 relative                 */
  int32_t n_ell;        /* size of the multipole union                                           */
  const double* ell;    /* [n_ell] real multipoles >= 2, increasing                              */
  int32_t n_zg;         /* geometry samples: chi(z), D(z)                                        */
  const double* z_geom; /* [n_zg] increasing; kernel support is [z_geom[0], z_geom[n_zg-1]]     */
  int32_t n_zs;         /* n(z) samples per tracer                                               */
  const double* z_nz;   /* [n_zs] increasing, inside the geometry range; n is 0 outside it      */
  int32_t max_batch;    /* capacity: parameter points per call                                   */
  int32_t max_tracers;  /* capacity: tracers per point (row stride of per-tracer inputs)        */
  int32_t max_ell;      /* capacity: multipoles per point (row stride of ell_idx and outputs)   */
  int32_t precision;    /* swiftcl_precision                                                     */
  int32_t device;       /* HIP device ordinal the plan lives on                                  */
  int32_t n_interp;     /* scale-dependent growth (Sec. 3.2, swiftcl_cl_kgrowth): number of k nodes
                           N_interp, 0 = none, else 2..n_k; FP32 and split-precision plans only   */
  int32_t rsd;          /* 1: redshift-space distortions of the clustering tracers (eq. RSD),
                           -int dchi f(z) n dz/dchi D j_l''(k chi) added to their windows, with
                           f = dln D/dln a from the D(z) spline; 0: none.  FP32 and split plans;
                           the projection runs through the workspace; swiftcl_windows,
                           swiftcl_cl_backward, swiftcl_cl_kgrowth and swiftcl_cl_limber refuse
                           such plans                                                              */
  int32_t magnification; /* 1: the plan can carry magnification bias of the clustering tracers
                           (eq. magnification bias; inputs `mag`), with the same restrictions as
                           rsd; 0: none                                                            */
} swiftcl_plan_desc;

/* Per-call inputs.  Device pointers owned by the caller, row-major, never written. */
typedef struct {
  int32_t batch;             /* B, 1..max_batch (0 is refused with SWIFTCL_E_INVALID)            */
  const int32_t* n_tracers;  /* [B] tracers of each point, 1..max_tracers                       */
  const int32_t* kind;       /* [B][max_tracers] SWIFTCL_CLUSTERING, SWIFTCL_LENSING or
                                SWIFTCL_CMB_LENSING; any other value raises FLAG_BAD_INDEX of
                                swiftcl_device_flags and that tracer's windows and C_l are 0     */
  const int32_t* n_ell;      /* [B] multipoles of each point, 1..max_ell                         */
  const int32_t* ell_idx;    /* [B][max_ell] indices into the plan's ell union                   */
  const double* chi_z;       /* [B][n_zg] comoving distance chi(z_geom) in Mpc/h, increasing     */
  const double* D_z;         /* [B][n_zg] growth D(z_geom), D(0) = 1 (z_fid = 0)                 */
  const double* omega_m;     /* [B] Omega_m of the lensing prefactors (eq. lens efficiency, Sec. 2.4) */
  const double* nz;          /* [B][max_tracers][n_zs] n(z) samples per unit z (ignored for
                                CMB-lensing tracers)                                             */
  const double* bias;        /* [B][max_tracers] linear bias b_1 (clustering only)              */
  const double* pk;          /* [B][n_k] P(k, z_fid) on the plan's k nodes, (Mpc/h)^3, > 0      */
  const double* ia;          /* [B][n_zg] NLA amplitude A_IA(z_geom) of the lensing tracers, or NULL
                                (no intrinsic alignment; Sec. 2.3: their kernel becomes
                                (q + A_IA n dz/dchi) D / chi^2); the backward calls carry it into
                                dL/dn and dL/dD but do not differentiate A_IA itself                 */
  const double* mag;         /* [B][max_tracers] lensing-bias coefficients C_g of the clustering
                                tracers (eq. magnification bias: l(l+1)/k^2 C_g int dchi / chi^2
                                q_g D j_l joins their window, q_g the lens efficiency of their own
                                n(z)), or NULL; needs a plan built with magnification = 1            */
  const double* kernel_chi;  /* [B][max_tracers][n_chi] or NULL: kernel samples in place of the
                                assembly from n(z), D(z), bias and the lensing integrals.  Entry m
                                is f_t(chi_m) of Sec. 2.1 (the radial kernel per unit chi, growth
                                and bias included) at chi_m = chi(z_geom[0]) e^{(m - edge_node)
                                Delta}, m = 0..n_chi-1 (chi(z_geom[0]) = chi_z[b][0]); the library
                                applies the FFTLog tilt (chi_m / chi_0)^{-b} and nothing else (no
                                support cut, no edge weights: the samples are used as the FFT takes
                                them).  kind still selects c(l, k).  In this mode nz, bias, D_z, ia
                                and mag are not read (may be NULL; omega_m too); swiftcl_cl_backward
                                gives dpk only, and swiftcl_cl_kgrowth, swiftcl_cl_limber and plans
                                with rsd or magnification refuse it with SWIFTCL_E_UNSUPPORTED    */
} swiftcl_inputs;

/* Build a plan: validates the descriptor, builds the log-chi grid, the FP64 table of Bessel
 * power-law integrals U_l(n) (eq. int_jl), the k scale tables and the workspace for max_batch
 * points.  Allocates device memory; the only call that does.  `stream` is a hipStream_t (may be
 * NULL); the plan is ready when the stream reaches the end of the call. */
swiftcl_status swiftcl_plan(const swiftcl_plan_desc* desc, void* stream, swiftcl_plan_t* out);

/* Free a plan.  The caller must ensure no call using it is still in flight. */
swiftcl_status swiftcl_plan_destroy(swiftcl_plan_t plan);

/* Thread-local message of the last failure on this thread ("" if none). */
const char* swiftcl_last_error(void);

/* Data checks made on the device during the last calls (support outside the chi box, non-finite
 * inputs): returns the accumulated flag word (0 = clean) and clears it.  Synchronises `stream`. */
swiftcl_status swiftcl_device_flags(swiftcl_plan_t plan, void* stream, int32_t* flags);

/* k-windows W[b][l][t][j] = Delta_l^t(k_j) (Sec. 2.1) for every point, multipole slot and tracer
 * slot; padded slots (t >= n_tracers[b], l >= n_ell[b]) are written as 0.  `W` is device memory
 * of B*max_ell*max_tracers*n_k elements: double for SWIFTCL_FP64, float otherwise. */
swiftcl_status swiftcl_windows(swiftcl_plan_t plan, const swiftcl_inputs* in, void* W, void* stream);

/* Angular power spectra C[b][l][p] (Sec. 2.1 / 3.2) with p running over the packed upper
 * triangle (i <= j, row-major) of max_tracers x max_tracers; padded slots are 0.  `C` is device
 * memory of B*max_ell*max_tracers*(max_tracers+1)/2 elements (double for FP64, float otherwise).
 * No allocation and no synchronisation: safe inside hipGraph capture. */
swiftcl_status swiftcl_cl(swiftcl_plan_t plan, const swiftcl_inputs* in, void* C, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation) and would rather not keep a workspace per plan: swiftcl_cl with
 * the call's workspace (kernel samples, FFTLog coefficients, node geometry, phases, work lists) in a
 * static device array of the library, 64 MiB per device, held until the process ends, instead of
 * the plan's.  Same arguments, kernels and results (bit for bit) as swiftcl_cl; calls no allocating
 * routine and synchronises nothing.  Only for plans with the fused projection (<= 16 tracers, no
 * rsd or magnification; else SWIFTCL_E_UNSUPPORTED).  A batch whose workspace exceeds the array
 * (about 0.6 MiB per point at 15 tracers, N_chi = N_k = 1024, FP32: some 100 points) is refused
 * with SWIFTCL_E_INVALID before any launch.  Every call on a device shares that device's array:
 * calls that overlap on one device (other streams, other threads, other plans) race and must be
 * ordered by the caller.  The array's address on a device is taken when the first plan there is
 * built. */
swiftcl_status swiftcl_cl_noalloc(swiftcl_plan_t plan, const swiftcl_inputs* in, void* C, void* stream);

/* Measurement variant of swiftcl_cl: the same launches, with HIP events recorded on `stream`
 * between its stages; writes the device time in ms of [0] kernel assembly (FP64 splines, lensing
 * integrals, sampling on the chi grid), [1] forward FFTLog coefficients, [2] windows + projection.
 * Creates events and synchronises `stream`: not for use under graph capture. */
swiftcl_status swiftcl_cl_timed(swiftcl_plan_t plan, const swiftcl_inputs* in, void* C, void* stream,
                                float* stage_ms);

/* Flags of the backward calls. */
enum {
  /* Keep the kernel samples, spline moments, lensing integrals and FFTLog coefficients that the
   * plan's last forward call (swiftcl_cl, swiftcl_windows, or a backward call) left in its
   * workspace instead of recomputing them (as autograd keeps saved activations).  The caller
   * asserts that this call's inputs are that call's inputs, unmodified, and that the calls are
   * ordered on the device (same stream, or synchronised).  Fails with SWIFTCL_E_INVALID if the
   * plan holds no forward state or the last forward call had another input descriptor. */
  SWIFTCL_BWD_REUSE_FORWARD = 1
};

/* Reverse-mode derivative of L = sum_b sum_l sum_{i<=j} dC[b][l][p(i,j)] C[b][l][p(i,j)] (the
 * paper differentiates its pipeline end to end, Sec. 1 and 4.3).  Windows are recomputed, not
 * stored.  Outputs (device, double; any may be NULL = not requested; padded slots written 0):
 *   dpk   [B][n_k]                  dL/dP(k_j)
 *   dbias [B][max_tracers]          dL/db_t (0 for lensing tracers)
 *   dnz   [B][max_tracers][n_zs]    dL/dn_t(z_s) through the n(z) spline (and the lensing q)
 *   dD    [B][n_zg]                 dL/dD(z_s) through the D(z) spline
 * `dC` has the layout and type of swiftcl_cl's output; `flags` is 0 or SWIFTCL_BWD_REUSE_FORWARD.
 * Plans with rsd or magnification: the recomputed windows carry the RSD and magnification terms
 * (eq. RSD, eq. magnification bias), so dpk is complete, and dbias (which scales the density term
 * alone) too; dnz and dD must be NULL (else SWIFTCL_E_UNSUPPORTED): the adjoints of those kernels'
 * assemblies are not built.
 * No allocation and no synchronisation: safe inside hipGraph capture. */
swiftcl_status swiftcl_cl_backward(swiftcl_plan_t plan, const swiftcl_inputs* in, const void* dC,
                                   double* dpk, double* dbias, double* dnz, double* dD, uint32_t flags,
                                   void* stream);

/* Launch-shape autotuner (used by batched callers, e.g. many parameter points of uneven tracer and
 * multipole counts).  Times, on the caller's inputs, the forward projection launched as one
 * workgroup per (point, multipole slot), as a persistent grid walking per-XCD compact work lists,
 * or as a persistent grid walking per-XCD packed lists (two (point, multipole) items whose tracer
 * counts sum to at most 16 share a workgroup), and (if dC is not NULL) the adjoint with 1, 2, 4 or
 * 8 times its base number of multipole chunks (base: about 256 workgroups, one round on the chip,
 * which suits uniform batches; ragged batches run better with more) and, on FP32 plans, the packed
 * adjoint at 1, 2 and 4; keeps the fastest in the plan (a variant other than the default, fwd_mode
 * 0, bwd_chunk_mul 1 and bwd_pack 0, must be at least 2% faster).  With cache_path (may
 * be NULL) the choice is read from, or appended to, a file with one JSON object per line keyed by
 * architecture and shape.  `C` (output-shaped scratch, overwritten) and `dC` are device buffers
 * laid out as for swiftcl_cl / swiftcl_cl_backward.  `report` (may be NULL) receives a one-line
 * summary.  Synchronises `stream`; call it outside graph capture, then capture or call swiftcl_cl /
 * swiftcl_cl_backward as usual. */
swiftcl_status swiftcl_autotune(swiftcl_plan_t plan, const swiftcl_inputs* in, void* C, const void* dC,
                                void* stream, const char* cache_path, char* report, int32_t report_len);

/* Set (values < 0 leave a field unchanged) or read the launch configuration the autotuner chooses:
 * fwd_mode 0 = one workgroup per (point, multipole slot), 1 = persistent grid over per-XCD compact
 * work lists, 2 = persistent grid over per-XCD packed lists (plans whose projection is fused; the
 * others run mode 0 whatever is set); bwd_chunk_mul in {1, 2, 4, 8} scales the adjoint's number of
 * multipole chunks; bwd_pack 1 (FP32 plans with a fused adjoint; FP64 plans run unpacked whatever
 * is set) splits each chunk into two halves with partial rows of their own, which a point of at
 * most 8 tracers runs side by side on the two halves of the workgroup's 16 wavefronts (needs
 * bwd_chunk_mul <= 4).  A combination outside these sets returns SWIFTCL_E_INVALID and changes
 * nothing.  Every configuration computes the same C_l bit for bit; the gradients differ only in
 * the order of their FP32 partial sums.  get: every pointer must be non-NULL. */
swiftcl_status swiftcl_set_launch(swiftcl_plan_t plan, int32_t fwd_mode, int32_t bwd_chunk_mul, int32_t bwd_pack);
swiftcl_status swiftcl_get_launch(swiftcl_plan_t plan, int32_t* fwd_mode, int32_t* bwd_chunk_mul, int32_t* bwd_pack);

/* What a built plan runs (host only, no device work): *fused = 1 when the C_l projection keeps the
 * windows of a (point, multipole) in one workgroup's LDS, 0 when it goes through the device
 * workspace in chunks of *point_chunk points (0 when the plan has no workspace); *adjoint = which
 * swiftcl_cl_backward the plan runs: 0 none (FP64 windows that do not fit LDS), 1 the fused adjoint
 * (windows recomputed in LDS), 2 the adjoint through the workspace (FP32 and split: more than 16
 * tracers, windows too large for LDS, RSD or magnification).  Any pointer may be NULL. */
swiftcl_status swiftcl_plan_info(swiftcl_plan_t plan, int32_t* fused, int32_t* adjoint, int32_t* point_chunk);

/* Measurement variant of swiftcl_cl_backward: the same launches with HIP events between its
 * stages; writes the device time in ms of [0] kernel assembly, [1] forward FFTLog coefficients
 * (both 0 with SWIFTCL_BWD_REUSE_FORWARD), [2] backward windows (recomputed W, G W on MFMA,
 * adjoint FFTs), [3] reduction of the coefficient cotangents and their inverse transform,
 * [4] chain rule through the kernels.  Creates events and synchronises `stream`: not for use
 * under graph capture. */
swiftcl_status swiftcl_cl_backward_timed(swiftcl_plan_t plan, const swiftcl_inputs* in, const void* dC,
                                         double* dpk, double* dbias, double* dnz, double* dD, uint32_t flags,
                                         void* stream, float* stage_ms);

/* Angular power spectra with scale-dependent growth D(k, z) (Sec. 3.2: P(k, chi, chi') =
 * P(k, z_fid) D(k, z(chi)) D(k, z(chi')), FFTLog coefficients c_n(k) of f(chi) D(k, chi)).  The
 * coefficients are computed at the plan's n_interp nodes kappa_a = k_0 (k_max / k_0)^{a / (n_interp-1)}
 * (uniform in ln k, both ends included) and continued to every k node by the natural cubic spline in
 * ln k through the node values (its second derivatives within 2e-10 of the exact solve, relative to
 * the moments 17 nodes on, in FP32 arithmetic); the window at k_j uses c_n(k_j), so the inverse transform becomes a
 * dense sum over n per k (run as a GEMM on MFMA).  Growth at a node is continued in z by the natural
 * cubic spline, like D(z).
 *   D_kz  device, double, [B][n_interp][n_zg]: D(kappa_a, z_geom) of every point; it replaces
 *         in->D_z, which is not read.
 *   C     as for swiftcl_cl (float).
 * Needs a plan with n_interp >= 2 (else SWIFTCL_E_INVALID); FP32 or split precision.  Non-finite
 * D_kz samples raise the device flag of non-finite inputs.  Overwrites the plan's forward state (a
 * backward call after it cannot use SWIFTCL_BWD_REUSE_FORWARD).  No allocation and no
 * synchronisation: safe inside hipGraph capture. */
swiftcl_status swiftcl_cl_kgrowth(swiftcl_plan_t plan, const swiftcl_inputs* in, const double* D_kz, void* C,
                                  void* stream);

/* Reverse-mode derivative of L = sum dC C for the scale-dependent growth path (the paper
 * differentiates its pipeline end to end, Sec. 1): the windows of swiftcl_cl_kgrowth are
 * recomputed (as W, FP32), Y = G W on MFMA gives dL/dP(k_j) = (2/pi) w_j k_j^3 sum_l sum_t W Y, and
 * dL/db_t follows from the forward output, since every node's kernel is linear in the bias:
 * dC^{ij}/db_t = C^{ij} (delta_it + delta_jt) / b_t.
 *   D_kz  as for swiftcl_cl_kgrowth (the same inputs as the forward call).
 *   C     device, float: swiftcl_cl_kgrowth's output for these inputs (read for dbias; may be NULL
 *         if dbias is NULL).
 *   dC    device, float, laid out as C.
 *   dpk   device, double, [B][n_k], or NULL.    dbias  device, double, [B][max_tracers], or NULL
 *         (0 for lensing tracers and padded slots).
 * The gradients with respect to n(z) and D(k, z) are not built.  Same plans and refusals as
 * swiftcl_cl_kgrowth.  No allocation and no synchronisation: safe inside hipGraph capture. */
swiftcl_status swiftcl_cl_kgrowth_backward(swiftcl_plan_t plan, const swiftcl_inputs* in, const double* D_kz,
                                           const void* C, const void* dC, double* dpk, double* dbias,
                                           void* stream);

/* The Limber limit (Sec. 2.6, eq. Limber): j_l(k chi) taken as a delta function at k = (l + 1/2)/chi,
 *   C_l^{ij} = int dchi / chi^2 g_i g_j P((l + 1/2)/chi),  g = f (clustering), F(l) f / k^2 (lensing),
 * integrated on the plan's log-chi nodes with the FFTLog path's edge weights (dchi = chi dln chi),
 * P continued by the natural cubic spline of ln P in ln k and zero outside the k nodes.  Its error
 * is O(1/l): a cheap path for high multipoles and a check of the windows there.  Same inputs and
 * output layout as swiftcl_cl, every precision.  Overwrites the plan's forward state.  No allocation
 * and no synchronisation: safe inside hipGraph capture. */
swiftcl_status swiftcl_cl_limber(swiftcl_plan_t plan, const swiftcl_inputs* in, void* C, void* stream);

/* Adjoint of swiftcl_cl_limber (Sec. 2.6, eq. Limber, on the same nodes; the paper differentiates
 * every step, Sec. 1): for L = sum over points, multipoles and pairs of dC * C_limber, with dC laid
 * out like C (device, the plan's real type), writes dL/dP (dpk [batch][n_k]), dL/db (dbias
 * [batch][max_tracers], 0 for lensing-kind tracers and empty slots), dL/dn(z) (dnz
 * [batch][max_tracers][n_zs]) and dL/dD(z) (dD [batch][n_zg]); device FP64 arrays, each optional
 * (NULL skips it).  The ln P spline is differentiated exactly (k nodes whose Limber k no node
 * reaches get 0; samples at or below 1e-300, where ln P is clamped, get 0).  Recomputes the kernel
 * assembly.  Same plan and input restrictions as swiftcl_cl_limber (no RSD or magnification, no
 * kernel samples); SWIFTCL_E_UNSUPPORTED if its LDS (about 8 (2 T 128 + T^2 + 2 n_k) bytes) exceeds
 * the device's.  No allocation and no synchronisation: safe inside hipGraph capture. */
swiftcl_status swiftcl_cl_limber_backward(swiftcl_plan_t plan, const swiftcl_inputs* in, const void* dC,
                                          double* dpk, double* dbias, double* dnz, double* dD, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SWIFTCL_H */
