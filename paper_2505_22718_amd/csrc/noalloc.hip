// swiftcl_cl_noalloc: the C_l of swiftcl_cl with the call's workspace (per-point scalars, spline
// moments, node geometry, lensing efficiencies, FFTLog phases, kernel samples, coefficients, the
// sqrt(s) and k-scale rows and the persistent launch's work lists) carved from a static device array
// instead of the plan's workspace.  The plan's constant tables (U table, twiddles, k scales, spline
// factors) are read as by swiftcl_cl; the kernels are the same, so the C_l are the same bit for bit.
//
// The array exists once per device for the life of the process; its address on each device is
// taken once, with that device current, when a plan is built there (noalloc_setup).  Every call on
// a device shares that device's array: calls that overlap on one device race.  Nothing in the
// workspace needs to start at zero (every entry a call reads is written earlier in the same call).
#include <mutex>
#include <string>

#include "common.h"
#include "internal.h"

// 64 MiB: at the 15-tracer shape (N_chi = N_k = 1024, three bias bands, FP32) one point needs
// about 0.6 MiB, so up to ~100 points per call.
#define SWIFTCL_SCRATCH_BYTES ((size_t)64 << 20)

static __device__ __align__(256) unsigned char scratch[SWIFTCL_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];  // the device address of `scratch` on each device (null: not taken yet)

// Sub-buffers of the workspace of a call of `batch` points, in order, each 256-byte aligned.
struct carve {
  char* base;  // null: only count
  size_t off = 0;
  template <typename T> T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* ptr = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return ptr;
  }
};

// Points q's workspace pointers into `base` (or, with base null, only counts); returns the bytes.
size_t layout(plan_dev& q, int batch, char* base, size_t rs) {
  carve c{base};
  const size_t B = (size_t)batch, T = q.max_tracers, nb = q.n_bands, N = q.N, nk = q.n_k;
  q.pt = c.take<double>(B * PT_STRIDE);
  q.m_chi = c.take<double>(B * q.n_zg);
  q.m_D = c.take<double>(B * q.n_zg);
  q.m_ia = c.take<double>(B * q.n_zg);
  q.m_n = c.take<double>(B * T * q.n_zs);
  q.lens_q = c.take<double>(B * T * N);
  q.phase = c.take<double>(B * N);
  q.node_f = c.take<double>(B * 4 * N);
  q.node_i = c.take<int>(B * 3 * N);
  q.g = c.take<char>(B * T * nb * N * rs);
  q.chat = c.take<char>(B * T * nb * N * rs);  // [B][T][nb][N/2] complex
  q.sqrt_s = c.take<char>(B * nk * rs);
  q.kss = c.take<char>(B * SWIFTCL_NKINDS * nb * nk * rs);
  q.sched_stride = sched_stride_for(batch);
  q.sched = c.take<int>(sched_ints(q.sched_stride));
  return c.off;
}

}  // namespace

// Takes the address of `scratch` on `device` (the current device) once per process.
swiftcl_status noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return SWIFTCL_OK;  // swiftcl_cl_noalloc refuses such a device
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return SWIFTCL_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "address of the static workspace");
  g_scratch[device] = ptr;
  return SWIFTCL_OK;
}

size_t noalloc_bytes(const plan_dev& p, int batch, size_t rs) {
  plan_dev q = p;
  return layout(q, batch, nullptr, rs);
}

extern "C" swiftcl_status swiftcl_cl_noalloc(swiftcl_plan_t p, const swiftcl_inputs* in, void* C, void* stream) {
  if (!p) { set_error("plan is NULL"); return SWIFTCL_E_INVALID; }
  if (!in) { set_error("inputs is NULL"); return SWIFTCL_E_INVALID; }
  if (!C) { set_error("C is NULL"); return SWIFTCL_E_INVALID; }
  if (!p->d.fused) {
    set_error("swiftcl_cl_noalloc runs the fused projection only (<= 16 tracers, no rsd or magnification); "
              "this plan projects through its workspace");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if (in->batch >= 1 && in->batch <= p->d.max_batch) {
    const size_t need = noalloc_bytes(p->d, in->batch, p->real_size);
    if (need > SWIFTCL_SCRATCH_BYTES) {
      set_error("swiftcl_cl_noalloc: a batch of " + std::to_string(in->batch) + " points needs " +
                std::to_string(need) + " bytes of workspace; the static workspace holds " +
                std::to_string((size_t)SWIFTCL_SCRATCH_BYTES) + " (about " +
                std::to_string(need / (size_t)in->batch) + " bytes per point)");
      return SWIFTCL_E_INVALID;
    }
  }
  swiftcl_status st = check_inputs(p, in);
  if (st != SWIFTCL_OK) return st;
  const int dev = p->d.device;
  void* base = (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
  if (!base) {
    set_error("swiftcl_cl_noalloc: the static workspace of device " + std::to_string(dev) + " was not set up");
    return SWIFTCL_E_UNSUPPORTED;
  }
  if ((st = hip_check(hipSetDevice(dev), "hipSetDevice")) != SWIFTCL_OK) return st;
  (void)hipGetLastError();
  plan_dev q = p->d;  // the plan's tables and launch configuration, this call's workspace
  layout(q, in->batch, (char*)base, p->real_size);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_assemble(q, in, s);
  if (e == hipSuccess) e = launch_forward_fft(q, in, s);
  if (e == hipSuccess) e = launch_windows_cl(q, in, nullptr, C, s);
  return hip_check(e, "forward launch (static workspace)");
}
