"""Torch-facing plan: device buffers and streams around the C entry points.

Every computation happens in libswiftcl.so; this module only builds the descriptor, checks that
every tensor it hands over has the layout the library reads (shape in the plan's sizes, type,
contiguity, the plan's device: a kernel would index any other tensor out of bounds), hands over
device pointers and the current HIP stream, and allocates outputs.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import binding as bd

# Default FFTLog bias bands of the library: bands start at l = 0, 3 and 6; per band the bias b
# (paper Sec. 3.1) of clustering, lensing and CMB-lensing tracers.
DEFAULT_BAND_ELL_LO = (0.0, 3.0, 6.0)
DEFAULT_FFTLOG_B = ((0.1, -0.2, -0.5), (-1.5, -2.0, -2.5), (-1.0, -1.0, -2.0))

PRECISIONS = {"fp64": bd.SWIFTCL_FP64, "fp32": bd.SWIFTCL_FP32, "split_bf16": bd.SWIFTCL_SPLIT_BF16}


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# The per-call input tensors in the layout the library reads (swiftcl_inputs in include/swiftcl.h),
# each dimension named after a plan size; B is the batch.
INPUT_LAYOUT = (
    ("n_tracers", torch.int32, ("B",)),
    ("kind", torch.int32, ("B", "max_tracers")),
    ("n_ell", torch.int32, ("B",)),
    ("ell_idx", torch.int32, ("B", "max_ell")),
    ("chi_z", torch.float64, ("B", "n_zg")),
    ("D_z", torch.float64, ("B", "n_zg")),
    ("omega_m", torch.float64, ("B",)),
    ("nz", torch.float64, ("B", "max_tracers", "n_zs")),
    ("bias", torch.float64, ("B", "max_tracers")),
    ("pk", torch.float64, ("B", "n_k")),
)
OPTIONAL_INPUT_LAYOUT = (
    ("ia", torch.float64, ("B", "n_zg")),
    ("mag", torch.float64, ("B", "max_tracers")),
    ("kernel_chi", torch.float64, ("B", "max_tracers", "n_chi")),
)
# inputs the kernel-samples mode (kernel_chi given) does not read: optional there
KERNEL_MODE_OPTIONAL = ("D_z", "omega_m", "nz", "bias")
# gradient outputs of the backward calls
GRAD_LAYOUT = (
    ("pk", ("B", "n_k")),
    ("bias", ("B", "max_tracers")),
    ("nz", ("B", "max_tracers", "n_zs")),
    ("D", ("B", "n_zg")),
)


def check_tensor(name, x, shape, dtype, device):
    """Raise ValueError unless x is a contiguous `dtype` tensor of exactly `shape` on `device`.  The
    kernels index every buffer with the plan's sizes, so any other tensor would be read or written
    out of bounds; the check reads metadata only (no synchronisation, fine under graph capture)."""
    shape = tuple(int(v) for v in shape)
    if (isinstance(x, torch.Tensor) and tuple(x.shape) == shape and x.dtype == dtype and x.device == device
            and x.is_contiguous()):
        return
    if isinstance(x, torch.Tensor):
        got = f"{tuple(x.shape)} {x.dtype} on {x.device}" + ("" if x.is_contiguous() else ", not contiguous")
    else:
        got = type(x).__name__
    raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {shape} on {device}; got {got}")


def check_inputs(t, dims, device):
    """Check a dict of per-call input tensors against INPUT_LAYOUT before its pointers are handed
    over.  dims: the plan's max_tracers, max_ell, n_zg, n_zs, n_k and n_chi.  Returns the batch B."""
    n = t.get("n_tracers")
    if not isinstance(n, torch.Tensor) or n.dim() != 1:
        raise ValueError("inputs need n_tracers, a 1-d tensor of the batch's tracer counts")
    size = dict(dims, B=int(n.shape[0]))
    kernel_mode = t.get("kernel_chi") is not None
    for name, dtype, layout in INPUT_LAYOUT:
        if t.get(name) is None and kernel_mode and name in KERNEL_MODE_OPTIONAL:
            continue
        if name not in t:
            raise ValueError(f"inputs lack {name!r}")
        check_tensor(name, t[name], [size[d] for d in layout], dtype, device)
    for name, dtype, layout in OPTIONAL_INPUT_LAYOUT:
        if t.get(name) is not None:
            check_tensor(name, t[name], [size[d] for d in layout], dtype, device)
    return size["B"]


def check_grads(outs, B, dims, device):
    """Check preallocated gradient tensors (any subset of pk, bias, nz, D; float64)."""
    size = dict(dims, B=B)
    for name, layout in GRAD_LAYOUT:
        if outs.get(name) is not None:
            check_tensor(f"gradient {name}", outs[name], [size[d] for d in layout], torch.float64, device)


# Plans dropped while a stream is being captured into a graph: freeing device memory then would
# invalidate the capture, so their release waits for the next close() outside capture.
_deferred_handles = []


def _capturing():
    try:
        return torch.cuda.is_current_stream_capturing()
    except Exception:
        return False


class Plan:
    """Owns one swiftcl plan on one device."""

    def __init__(self, k, ell, z_geom, z_nz, n_chi, max_batch, max_tracers, max_ell, precision="fp32",
                 band_ell_lo=DEFAULT_BAND_ELL_LO, fftlog_b=DEFAULT_FFTLOG_B, taper_frac=0.0, edge_node=0,
                 device=0, n_interp=0, rsd=False, magnification=False):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}, got {precision!r}")
        nb = len(band_ell_lo)
        if not 1 <= nb <= bd.MAX_BANDS:
            raise ValueError(f"band_ell_lo must have 1..{bd.MAX_BANDS} entries, got {nb}")
        if len(fftlog_b) != bd.NKINDS or any(len(fftlog_b[kind]) != nb for kind in range(bd.NKINDS)):
            # entries left unset would reach the library as b = 0
            raise ValueError(f"fftlog_b needs a row of {nb} biases (one per band) for each of the {bd.NKINDS} "
                             "tracer kinds (clustering, lensing, CMB lensing)")
        self.k = _f64(k)
        self.ell = _f64(ell)
        self.z_geom = _f64(z_geom)
        self.z_nz = _f64(z_nz)
        self.n_chi = int(n_chi)
        self.max_batch, self.max_tracers, self.max_ell = int(max_batch), int(max_tracers), int(max_ell)
        self.precision = precision
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, 0)
        d = bd.swiftcl_plan_desc()
        d.n_chi = self.n_chi
        d.edge_node = int(edge_node)
        d.n_bands = len(band_ell_lo)
        for j, v in enumerate(band_ell_lo):
            d.band_ell_lo[j] = float(v)
        for kind in range(bd.NKINDS):
            for j, v in enumerate(fftlog_b[kind]):
                d.fftlog_b[kind][j] = float(v)
        d.taper_frac = float(taper_frac)
        dp = ctypes.POINTER(ctypes.c_double)
        d.n_k, d.k = len(self.k), self.k.ctypes.data_as(dp)
        d.n_ell, d.ell = len(self.ell), self.ell.ctypes.data_as(dp)
        d.n_zg, d.z_geom = len(self.z_geom), self.z_geom.ctypes.data_as(dp)
        d.n_zs, d.z_nz = len(self.z_nz), self.z_nz.ctypes.data_as(dp)
        d.max_batch, d.max_tracers, d.max_ell = self.max_batch, self.max_tracers, self.max_ell
        d.precision = PRECISIONS[precision]
        d.device = self.device.index
        d.n_interp = int(n_interp)
        self.n_interp = int(n_interp)
        d.rsd = 1 if rsd else 0
        self.rsd = bool(rsd)
        d.magnification = 1 if magnification else 0
        self.magnification = bool(magnification)
        self.desc = d
        self.out_dtype = torch.float64 if precision == "fp64" else torch.float32
        with torch.cuda.device(self.device):
            self.handle = bd.swiftcl_plan(d, torch.cuda.current_stream(self.device).cuda_stream)
        self.state_token = None

    @classmethod
    def for_workload(cls, wl, max_batch=None, precision=None, **kw):
        return cls(wl["k"], wl["ell"], wl["z_geom"], wl["z_nz"], wl["n_chi"],
                   max_batch or wl["batch"], wl["nz"].shape[1], wl["ell_idx"].shape[1],
                   precision=precision or ("fp32" if wl["precision"] == "split_bf16" else wl["precision"]), **kw)

    def close(self):
        h = getattr(self, "handle", None)
        self.handle = None
        if _capturing():
            if h:
                _deferred_handles.append(h)
            return
        while _deferred_handles:
            bd.swiftcl_plan_destroy(_deferred_handles.pop())
        if h:
            bd.swiftcl_plan_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_pairs(self):
        return self.max_tracers * (self.max_tracers + 1) // 2

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    @property
    def dims(self):
        """The plan sizes that the input, output and gradient layouts are written in."""
        return dict(max_tracers=self.max_tracers, max_ell=self.max_ell, n_zg=len(self.z_geom),
                    n_zs=len(self.z_nz), n_k=len(self.k), n_chi=self.n_chi)

    def _cl_buffer(self, name, x, B):
        """A [B][max_ell][n_pairs] buffer of the output type: checked if given, else allocated."""
        shape = (B, self.max_ell, self.n_pairs)
        if x is None:
            return torch.empty(shape, dtype=self.out_dtype, device=self.device)
        check_tensor(name, x, shape, self.out_dtype, self.device)
        return x

    def inputs_struct(self, t):
        """The swiftcl_inputs of a dict of device tensors, after check_inputs."""
        s = bd.swiftcl_inputs()
        s.batch = check_inputs(t, self.dims, self.device)
        for name in ("n_tracers", "kind", "n_ell", "ell_idx", "chi_z", "D_z", "omega_m", "nz", "bias", "pk"):
            x = t.get(name)  # (the kernel-samples mode leaves D_z, omega_m, nz and bias optional)
            setattr(s, name, x.data_ptr() if x is not None else None)
        ia = t.get("ia")  # NLA amplitude A_IA(z) of the lensing tracers, optional
        s.ia = ia.data_ptr() if ia is not None else None
        mag = t.get("mag")  # lensing-bias coefficients C_g of the clustering tracers, optional
        s.mag = mag.data_ptr() if mag is not None else None
        kc = t.get("kernel_chi")  # kernel samples on the chi nodes in place of the assembly, optional
        s.kernel_chi = kc.data_ptr() if kc is not None else None
        return s

    # Every call that (re)computes the workspace's forward state sets a fresh token; autograd keeps
    # the token of its forward call and reuses the state in backward if no other call came between.
    def _new_state(self):
        self.state_token = object()
        return self.state_token

    def cl(self, t, out=None):
        s = self.inputs_struct(t)
        out = self._cl_buffer("out", out, s.batch)
        self._new_state()
        bd.swiftcl_cl(self.handle, s, out.data_ptr(), self._stream())
        return out

    def cl_kgrowth(self, t, D_kz, out=None):
        """C_l with scale-dependent growth: D_kz [B][n_interp][n_zg] float64 on the plan's device."""
        s = self.inputs_struct(t)
        check_tensor("D_kz", D_kz, (s.batch, self.n_interp, len(self.z_geom)), torch.float64, self.device)
        out = self._cl_buffer("out", out, s.batch)
        self._new_state()
        bd.swiftcl_cl_kgrowth(self.handle, s, D_kz.data_ptr(), out.data_ptr(), self._stream())
        return out

    def kgrowth_backward(self, t, D_kz, C, dC, want=("pk", "bias")):
        """Gradients of sum(dC * C_kgrowth) with respect to pk and bias (swiftcl_cl_kgrowth_backward);
        C is cl_kgrowth's output for the same inputs."""
        s = self.inputs_struct(t)
        B = s.batch
        check_tensor("D_kz", D_kz, (B, self.n_interp, len(self.z_geom)), torch.float64, self.device)
        C = self._cl_buffer("C", C.contiguous(), B)
        dC = self._cl_buffer("dC", dC.contiguous(), B)
        bad = set(want) - {"pk", "bias"}
        if bad:
            raise ValueError(f"the scale-dependent growth adjoint gives pk and bias gradients, not {sorted(bad)}")
        outs = self._grad_outputs(B, want)
        self._new_state()
        bd.swiftcl_cl_kgrowth_backward(self.handle, s, D_kz.data_ptr(), C.data_ptr(), dC.data_ptr(),
                                       outs["pk"].data_ptr() if outs["pk"] is not None else 0,
                                       outs["bias"].data_ptr() if outs["bias"] is not None else 0, self._stream())
        return {k: v for k, v in outs.items() if v is not None}

    def cl_limber(self, t, out=None):
        """C_l in the Limber limit on the plan's chi nodes (same layout as cl)."""
        s = self.inputs_struct(t)
        out = self._cl_buffer("out", out, s.batch)
        self._new_state()
        bd.swiftcl_cl_limber(self.handle, s, out.data_ptr(), self._stream())
        return out

    def cl_timed(self, t, out):
        """Forward C_l with per-stage device times (ms): assembly, FFTLog coefficients, windows + C."""
        s = self.inputs_struct(t)
        out = self._cl_buffer("out", out, s.batch)
        self._new_state()
        return bd.swiftcl_cl_timed(self.handle, s, out.data_ptr(), self._stream())

    def windows(self, t, out=None):
        s = self.inputs_struct(t)
        shape = (s.batch, self.max_ell, self.max_tracers, len(self.k))
        if out is None:
            out = torch.empty(shape, dtype=self.out_dtype, device=self.device)
        else:
            check_tensor("out", out, shape, self.out_dtype, self.device)
        self._new_state()
        bd.swiftcl_windows(self.handle, s, out.data_ptr(), self._stream())
        return out

    def backward(self, t, dC, want=("pk", "bias", "nz", "D"), reuse_forward=False):
        """Gradients of sum(dC * C).  reuse_forward: `t` is the input of the last forward call on
        this plan (same tensors, unmodified), whose assembly and FFTLog state are kept."""
        s = self.inputs_struct(t)
        B = s.batch
        dC = self._cl_buffer("dC", dC.contiguous(), B)
        outs = self._grad_outputs(B, want)
        ptr = {k: (v.data_ptr() if v is not None else 0) for k, v in outs.items()}
        if not reuse_forward:
            self._new_state()
        bd.swiftcl_cl_backward(self.handle, s, dC.data_ptr(), ptr["pk"], ptr["bias"], ptr["nz"], ptr["D"],
                               _flags(reuse_forward), self._stream())
        return {k: v for k, v in outs.items() if v is not None}

    def limber_backward(self, t, dC, want=("pk", "bias", "nz", "D")):
        """Gradients of sum(dC * C_limber) (swiftcl_cl_limber_backward)."""
        s = self.inputs_struct(t)
        B = s.batch
        dC = self._cl_buffer("dC", dC.contiguous(), B)
        outs = self._grad_outputs(B, want)
        ptr = {k: (v.data_ptr() if v is not None else 0) for k, v in outs.items()}
        self._new_state()
        bd.swiftcl_cl_limber_backward(self.handle, s, dC.data_ptr(), ptr["pk"], ptr["bias"], ptr["nz"], ptr["D"],
                                      self._stream())
        return {k: v for k, v in outs.items() if v is not None}

    def _grad_outputs(self, B, want):
        f64 = dict(dtype=torch.float64, device=self.device)
        return {
            "pk": torch.empty((B, len(self.k)), **f64) if "pk" in want else None,
            "bias": torch.empty((B, self.max_tracers), **f64) if "bias" in want else None,
            "nz": torch.empty((B, self.max_tracers, len(self.z_nz)), **f64) if "nz" in want else None,
            "D": torch.empty((B, len(self.z_geom)), **f64) if "D" in want else None,
        }

    def backward_timed(self, t, dC, outs, reuse_forward=False):
        """Backward with per-stage device times (ms); outs: dict of preallocated gradient tensors."""
        s, ptr = self._backward_args(t, dC, outs)
        if not reuse_forward:
            self._new_state()
        return bd.swiftcl_cl_backward_timed(self.handle, s, dC.data_ptr(), ptr["pk"], ptr["bias"], ptr["nz"],
                                            ptr["D"], _flags(reuse_forward), self._stream())

    def backward_into(self, t, dC, outs, reuse_forward=False):
        """Backward into preallocated gradient tensors (no allocation)."""
        s, ptr = self._backward_args(t, dC, outs)
        if not reuse_forward:
            self._new_state()
        bd.swiftcl_cl_backward(self.handle, s, dC.data_ptr(), ptr["pk"], ptr["bias"], ptr["nz"], ptr["D"],
                               _flags(reuse_forward), self._stream())

    def _backward_args(self, t, dC, outs):
        """Checked inputs struct and gradient pointers of the preallocating backward calls."""
        s = self.inputs_struct(t)
        self._cl_buffer("dC", dC, s.batch)
        check_grads(outs, s.batch, self.dims, self.device)
        ptr = {k: (outs[k].data_ptr() if outs.get(k) is not None else 0) for k in ("pk", "bias", "nz", "D")}
        return s, ptr

    def autotune(self, t, dC=None, cache_path=None):
        """Choose the launch shapes for inputs like `t` (see swiftcl_autotune); returns the report."""
        s = self.inputs_struct(t)
        if dC is not None:
            self._cl_buffer("dC", dC, s.batch)
        self._new_state()
        C = self._cl_buffer("out", None, s.batch)
        return bd.swiftcl_autotune(self.handle, s, C.data_ptr(), dC.data_ptr() if dC is not None else 0,
                                   self._stream(), cache_path)

    def set_launch(self, fwd_mode=None, bwd_chunk_mul=None, bwd_pack=None):
        """Force a launch configuration (what swiftcl_autotune would choose)."""
        bd.swiftcl_set_launch(self.handle, -1 if fwd_mode is None else fwd_mode,
                              -1 if bwd_chunk_mul is None else bwd_chunk_mul,
                              -1 if bwd_pack is None else int(bwd_pack))

    def launch_config(self):
        return bd.swiftcl_get_launch(self.handle)

    @property
    def adjoint_mode(self):
        """0: no adjoint, 1: fused (windows recomputed in LDS), 2: through the workspace."""
        return bd.swiftcl_plan_info(self.handle)["adjoint"]

    @property
    def vchunk(self):
        """Points per chunk of the workspace paths (0 without a workspace)."""
        return bd.swiftcl_plan_info(self.handle)["point_chunk"]

    def device_flags(self):
        return bd.swiftcl_device_flags(self.handle, self._stream())


def _flags(reuse_forward):
    return bd.SWIFTCL_BWD_REUSE_FORWARD if reuse_forward else 0


def device_inputs(wl, device="cuda:0", points=None):
    """Device tensors of a synthetic workload (optionally a subset of its points)."""
    sel = slice(None) if points is None else np.asarray(points)
    dev = torch.device(device)

    def f(x, dt):
        return torch.as_tensor(np.ascontiguousarray(np.asarray(x)[sel]), dtype=dt).to(dev)

    out = {
        "n_tracers": f(wl["n_tracers"], torch.int32),
        "kind": f(wl["kind"], torch.int32),
        "n_ell": f(wl["n_ell"], torch.int32),
        "ell_idx": f(wl["ell_idx"], torch.int32),
        "chi_z": f(wl["chi_z"], torch.float64),
        "D_z": f(wl["D_z"], torch.float64),
        "omega_m": f(wl["omega_m"], torch.float64),
        "nz": f(wl["nz"], torch.float64),
        "bias": f(wl["bias"], torch.float64),
        "pk": f(wl["pk"], torch.float64),
    }
    if wl.get("ia") is not None:
        out["ia"] = f(wl["ia"], torch.float64)
    if wl.get("mag") is not None:
        out["mag"] = f(wl["mag"], torch.float64)
    if wl.get("kernel_chi") is not None:
        out["kernel_chi"] = f(wl["kernel_chi"], torch.float64)
    return out
