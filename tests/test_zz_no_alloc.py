"""The allocation-free entry point swiftcl_cl_noalloc (C ABI): the same C_l as swiftcl_cl, bit for
bit, from the workspace in the library's static device array; two calls in a row (the second with
a smaller batch, so the array keeps the first call's larger contents), both launch modes, FP32 and
FP64, and kernel samples in place of the assembly.  A batch whose workspace exceeds the array is
refused with SWIFTCL_E_INVALID before any launch, leaving the output untouched."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _noalloc(plan, t, out):
    """swiftcl_cl_noalloc through the C ABI (ctypes), on the current stream; returns the status."""
    from paper_2505_22718_amd import binding as bd
    s = plan.inputs_struct(t)
    lib = bd.load()
    return lib.swiftcl_cl_noalloc(plan.handle, ctypes.byref(s), ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream(plan.device).cuda_stream))


@pytest.mark.parametrize("name,precision,fwd_mode", [("cfg1_batch", "fp32", 0), ("cfg1_batch", "fp32", 1),
                                                     ("cfg3", "fp32", 2), ("cfg0", "fp64", 0)])
def test_noalloc_matches_swiftcl_cl(dev, name, precision, fwd_mode):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload(name, batch=24) if name in ("cfg1_batch", "cfg3") else synth.make_workload(name)
    B = int(wl["batch"])
    plan = Plan.for_workload(wl, precision=precision)
    plan.set_launch(fwd_mode=fwd_mode)
    for n in (B, max(1, B // 3)):  # the second call is smaller
        t = device_inputs(wl, dev, points=list(range(n)))
        ref = plan.cl(t).clone()
        out = torch.full_like(ref, float("nan"))
        assert _noalloc(plan, t, out) == 0
        torch.cuda.synchronize()
        assert plan.device_flags() == 0
        _say(f"  {name} {precision} fwd_mode={fwd_mode} batch {n}: equal = {torch.equal(out, ref)}")
        assert torch.equal(out, ref)


def test_noalloc_kernel_samples(dev):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    from oracle import fftlog
    from oracle.geometry import point_geometry
    wl = synth.make_workload("cfg1")
    m = fftlog.method_for(wl)
    wl["kernel_chi"] = fftlog.sampled_kernels(point_geometry(wl, 0), m)[2][None]
    plan = Plan.for_workload(wl)
    t = device_inputs(wl, dev)
    ref = plan.cl(t).clone()
    out = torch.zeros_like(ref)
    assert _noalloc(plan, t, out) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_refuses_a_batch_beyond_the_array(dev):
    from paper_2505_22718_amd import binding as bd
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg1_batch", batch=256)
    plan = Plan.for_workload(wl)
    t = device_inputs(wl, dev)
    out = torch.zeros((256, plan.max_ell, plan.n_pairs), dtype=torch.float32, device=dev)
    st = _noalloc(plan, t, out)
    msg = bd.swiftcl_last_error()
    _say(f"  256 points: status {st}: {msg}")
    assert st == bd.SWIFTCL_E_INVALID and "static workspace" in msg
    torch.cuda.synchronize()
    assert bool(torch.all(out == 0))
    # a plan that projects through its workspace (more than 16 tracers) is refused too
    w4 = synth.make_workload("cfg4", batch=1)
    p4 = Plan.for_workload(w4)
    o4 = torch.zeros((1, p4.max_ell, p4.n_pairs), dtype=torch.float32, device=dev)
    assert _noalloc(p4, device_inputs(w4, dev), o4) == bd.SWIFTCL_E_UNSUPPORTED
