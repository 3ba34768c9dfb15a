"""ctypes binding of libswiftcl (include/swiftcl.h): argument marshalling only.

The functions below carry the C names and forward to the shared library; every step of
the computation runs in the HIP kernels.  There is no CPU fallback: if the library is
missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswiftcl.so")

SWIFTCL_OK = 0
SWIFTCL_E_INVALID = -1
SWIFTCL_E_DOMAIN = -2
SWIFTCL_E_NOMEM = -3
SWIFTCL_E_DEVICE = -4
SWIFTCL_E_UNSUPPORTED = -5
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_DOMAIN", -3: "E_NOMEM", -4: "E_DEVICE", -5: "E_UNSUPPORTED"}

SWIFTCL_CLUSTERING = 0
SWIFTCL_LENSING = 1
SWIFTCL_CMB_LENSING = 2
NKINDS = 3
SWIFTCL_BWD_REUSE_FORWARD = 1
SWIFTCL_FP64 = 0
SWIFTCL_FP32 = 1
SWIFTCL_SPLIT_BF16 = 2
MAX_BANDS = 4

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class swiftcl_plan_desc(ctypes.Structure):
    _fields_ = [
        ("n_chi", ctypes.c_int32),
        ("edge_node", ctypes.c_int32),
        ("n_bands", ctypes.c_int32),
        ("band_ell_lo", ctypes.c_double * MAX_BANDS),
        ("fftlog_b", (ctypes.c_double * MAX_BANDS) * NKINDS),
        ("taper_frac", ctypes.c_double),
        ("n_k", ctypes.c_int32),
        ("k", _dp),
        ("n_ell", ctypes.c_int32),
        ("ell", _dp),
        ("n_zg", ctypes.c_int32),
        ("z_geom", _dp),
        ("n_zs", ctypes.c_int32),
        ("z_nz", _dp),
        ("max_batch", ctypes.c_int32),
        ("max_tracers", ctypes.c_int32),
        ("max_ell", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("n_interp", ctypes.c_int32),
        ("rsd", ctypes.c_int32),
        ("magnification", ctypes.c_int32),
    ]


class swiftcl_inputs(ctypes.Structure):
    _fields_ = [
        ("batch", ctypes.c_int32),
        ("n_tracers", ctypes.c_void_p),
        ("kind", ctypes.c_void_p),
        ("n_ell", ctypes.c_void_p),
        ("ell_idx", ctypes.c_void_p),
        ("chi_z", ctypes.c_void_p),
        ("D_z", ctypes.c_void_p),
        ("omega_m", ctypes.c_void_p),
        ("nz", ctypes.c_void_p),
        ("bias", ctypes.c_void_p),
        ("pk", ctypes.c_void_p),
        ("ia", ctypes.c_void_p),
        ("mag", ctypes.c_void_p),
        ("kernel_chi", ctypes.c_void_p),
    ]


EXPORTED = ["swiftcl_plan", "swiftcl_plan_destroy", "swiftcl_last_error", "swiftcl_device_flags",
            "swiftcl_windows", "swiftcl_cl", "swiftcl_cl_timed", "swiftcl_cl_backward",
            "swiftcl_cl_backward_timed", "swiftcl_autotune", "swiftcl_set_launch", "swiftcl_get_launch",
            "swiftcl_cl_kgrowth", "swiftcl_cl_limber", "swiftcl_cl_noalloc", "swiftcl_plan_info",
            "swiftcl_cl_limber_backward", "swiftcl_cl_kgrowth_backward"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libswiftcl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libswiftcl.so not found at {path}: build it with "
                           "`python -m paper_2505_22718_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.swiftcl_plan.argtypes = [ctypes.POINTER(swiftcl_plan_desc), vp, ctypes.POINTER(vp)]
    lib.swiftcl_plan_destroy.argtypes = [vp]
    lib.swiftcl_last_error.restype = ctypes.c_char_p
    lib.swiftcl_device_flags.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32)]
    lib.swiftcl_windows.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp]
    lib.swiftcl_cl.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp]
    lib.swiftcl_cl_noalloc.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp]
    lib.swiftcl_cl_timed.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp, ctypes.POINTER(ctypes.c_float)]
    lib.swiftcl_cl_kgrowth.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp, vp]
    lib.swiftcl_cl_limber.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp]
    lib.swiftcl_cl_backward.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp, vp, vp, vp, ctypes.c_uint32, vp]
    lib.swiftcl_cl_limber_backward.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp, vp, vp, vp, vp]
    lib.swiftcl_cl_kgrowth_backward.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp, vp, vp, vp, vp]
    lib.swiftcl_autotune.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp, vp, ctypes.c_char_p,
                                     ctypes.c_char_p, ctypes.c_int32]
    lib.swiftcl_set_launch.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.swiftcl_get_launch.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.swiftcl_plan_info.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int32)] * 3
    lib.swiftcl_cl_backward_timed.argtypes = [vp, ctypes.POINTER(swiftcl_inputs), vp, vp, vp, vp, vp,
                                              ctypes.c_uint32, vp, ctypes.POINTER(ctypes.c_float)]
    for name in EXPORTED:
        f = getattr(lib, name)
        if name != "swiftcl_last_error":
            f.restype = ctypes.c_int
    _lib = lib
    return lib


class SwiftclError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"swiftcl {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(status):
    if status != SWIFTCL_OK:
        raise SwiftclError(status, load().swiftcl_last_error().decode())
    return status


def swiftcl_last_error() -> str:
    return load().swiftcl_last_error().decode()


def swiftcl_plan(desc: swiftcl_plan_desc, stream: int = 0):
    handle = ctypes.c_void_p()
    _check(load().swiftcl_plan(ctypes.byref(desc), ctypes.c_void_p(stream), ctypes.byref(handle)))
    return handle


def swiftcl_plan_destroy(plan):
    _check(load().swiftcl_plan_destroy(plan))


def swiftcl_device_flags(plan, stream: int = 0) -> int:
    v = ctypes.c_int32()
    _check(load().swiftcl_device_flags(plan, ctypes.c_void_p(stream), ctypes.byref(v)))
    return v.value


def swiftcl_windows(plan, inputs: swiftcl_inputs, W: int, stream: int = 0):
    _check(load().swiftcl_windows(plan, ctypes.byref(inputs), ctypes.c_void_p(W), ctypes.c_void_p(stream)))


def swiftcl_cl(plan, inputs: swiftcl_inputs, C: int, stream: int = 0):
    _check(load().swiftcl_cl(plan, ctypes.byref(inputs), ctypes.c_void_p(C), ctypes.c_void_p(stream)))


def swiftcl_cl_noalloc(plan, inputs: swiftcl_inputs, C: int, stream: int = 0):
    _check(load().swiftcl_cl_noalloc(plan, ctypes.byref(inputs), ctypes.c_void_p(C), ctypes.c_void_p(stream)))


def swiftcl_cl_kgrowth(plan, inputs: swiftcl_inputs, D_kz: int, C: int, stream: int = 0):
    _check(load().swiftcl_cl_kgrowth(plan, ctypes.byref(inputs), ctypes.c_void_p(D_kz), ctypes.c_void_p(C),
                                     ctypes.c_void_p(stream)))


def swiftcl_cl_limber(plan, inputs: swiftcl_inputs, C: int, stream: int = 0):
    _check(load().swiftcl_cl_limber(plan, ctypes.byref(inputs), ctypes.c_void_p(C), ctypes.c_void_p(stream)))


def swiftcl_cl_limber_backward(plan, inputs: swiftcl_inputs, dC: int, dpk: int = 0, dbias: int = 0, dnz: int = 0,
                               dD: int = 0, stream: int = 0):
    vp = ctypes.c_void_p
    _check(load().swiftcl_cl_limber_backward(plan, ctypes.byref(inputs), vp(dC), vp(dpk or None), vp(dbias or None),
                                             vp(dnz or None), vp(dD or None), vp(stream)))


def swiftcl_cl_kgrowth_backward(plan, inputs: swiftcl_inputs, D_kz: int, C: int, dC: int, dpk: int = 0,
                                dbias: int = 0, stream: int = 0):
    vp = ctypes.c_void_p
    _check(load().swiftcl_cl_kgrowth_backward(plan, ctypes.byref(inputs), vp(D_kz), vp(C or None), vp(dC),
                                              vp(dpk or None), vp(dbias or None), vp(stream)))


def swiftcl_cl_timed(plan, inputs: swiftcl_inputs, C: int, stream: int = 0):
    """Returns the device time (ms) of the three forward stages."""
    ms = (ctypes.c_float * 3)()
    _check(load().swiftcl_cl_timed(plan, ctypes.byref(inputs), ctypes.c_void_p(C), ctypes.c_void_p(stream), ms))
    return [ms[0], ms[1], ms[2]]


def swiftcl_cl_backward(plan, inputs: swiftcl_inputs, dC: int, dpk: int = 0, dbias: int = 0, dnz: int = 0,
                        dD: int = 0, flags: int = 0, stream: int = 0):
    vp = ctypes.c_void_p
    _check(load().swiftcl_cl_backward(plan, ctypes.byref(inputs), vp(dC), vp(dpk or None), vp(dbias or None),
                                      vp(dnz or None), vp(dD or None), ctypes.c_uint32(flags), vp(stream)))


def swiftcl_cl_backward_timed(plan, inputs: swiftcl_inputs, dC: int, dpk: int = 0, dbias: int = 0, dnz: int = 0,
                              dD: int = 0, flags: int = 0, stream: int = 0):
    """Returns the device time (ms) of the five stages of a backward call."""
    vp = ctypes.c_void_p
    ms = (ctypes.c_float * 5)()
    _check(load().swiftcl_cl_backward_timed(plan, ctypes.byref(inputs), vp(dC), vp(dpk or None), vp(dbias or None),
                                            vp(dnz or None), vp(dD or None), ctypes.c_uint32(flags), vp(stream), ms))
    return [ms[i] for i in range(5)]


def swiftcl_autotune(plan, inputs: swiftcl_inputs, C: int, dC: int = 0, stream: int = 0, cache_path=None) -> str:
    """Picks the fastest launch shapes for these inputs; returns the one-line report."""
    buf = ctypes.create_string_buffer(512)
    path = cache_path.encode() if cache_path else None
    _check(load().swiftcl_autotune(plan, ctypes.byref(inputs), ctypes.c_void_p(C), ctypes.c_void_p(dC or None),
                                   ctypes.c_void_p(stream), path, buf, 512))
    return buf.value.decode()


def swiftcl_set_launch(plan, fwd_mode: int = -1, bwd_chunk_mul: int = -1, bwd_pack: int = -1):
    _check(load().swiftcl_set_launch(plan, fwd_mode, bwd_chunk_mul, bwd_pack))


def swiftcl_plan_info(plan):
    f, a, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().swiftcl_plan_info(plan, ctypes.byref(f), ctypes.byref(a), ctypes.byref(c)))
    return {"fused": f.value, "adjoint": a.value, "point_chunk": c.value}


def swiftcl_get_launch(plan):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().swiftcl_get_launch(plan, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return {"fwd_mode": a.value, "bwd_chunk_mul": b.value, "bwd_pack": c.value}


def raw_status(fn_name: str, *args) -> int:
    """Call an entry point and return its status without raising (for error-path tests)."""
    return getattr(load(), fn_name)(*args)
