"""Redshift-space distortions of the clustering tracers (eq. RSD) on the GPU: plans with rsd = 1
add -int dchi f(z) n dz/dchi D j_l''(k chi) to every clustering window (through the workspace
projection path), compared element by element with the FFTLog oracle on the Q12 metric (1e-4 FP32,
1e-3 BF16 hi+lo).  The paths that do not carry RSD (Limber, windows output, the n(z) and D(z)
gradients) refuse such plans."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fftlog
from tests.helpers import eps_metric, full_from_packed

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _wl(name="cfg1", step=6, batch=None):
    """The workload with RSD on, at every step-th multipole slot of each point."""
    wl = synth.make_workload(name, batch=batch)
    wl["rsd"] = True
    wl["ell_idx"] = wl["ell_idx"][:, ::step].copy()
    wl["n_ell"] = ((wl["n_ell"] + step - 1) // step).astype(np.int32)
    return wl


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("split_bf16", 1e-3)])
def test_rsd_parity(dev, precision, tol):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _wl()
    _say(f"RSD cfg1 {precision}")
    p = Plan.for_workload(wl, precision=precision, rsd=True)
    C = p.cl(device_inputs(wl, dev)).cpu().numpy()[0].astype(np.float64)
    assert p.device_flags() == 0
    Cref = fftlog.cl(wl, 0)
    e = eps_metric(full_from_packed(C, 15), full_from_packed(Cref, 15))
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < tol
    # RSD is switched on: the clustering autos at low l move away from the RSD-free oracle
    C0 = fftlog.cl(dict(wl, rsd=False), 0)
    iu = np.triu_indices(15)
    autos = [q for q, (i, j) in enumerate(zip(*iu)) if i == j and i < 10]
    assert np.max(np.abs(C[0, autos] / C0[0, autos] - 1)) > 0.1


def test_rsd_ragged_batch(dev):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _wl("cfg3", step=9, batch=12)
    _say("RSD cfg3 ragged, 12 points")
    p = Plan.for_workload(wl, rsd=True)
    C = p.cl(device_inputs(wl, dev)).cpu().numpy().astype(np.float64)
    assert p.device_flags() == 0
    for b in (0, 5, 11):
        T, L = int(wl["n_tracers"][b]), int(wl["n_ell"][b])
        full = full_from_packed(C[b, :L], 15)
        e = eps_metric(full[:, :T, :T], full_from_packed(fftlog.cl(wl, b), T))
        _say(f"  point {b} (T={T}, L={L}) max eps {e.max():.3e}")
        assert e.max() < 1e-4
        assert np.all(C[b, L:] == 0)


def test_rsd_refused_where_not_built(dev):
    from paper_2505_22718_amd import binding as bd
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _wl()
    p = Plan.for_workload(wl, rsd=True)
    t = device_inputs(wl, dev)
    p.cl(t)
    dC = torch.ones((1, p.max_ell, p.n_pairs), dtype=p.out_dtype, device=dev)
    # (the adjoint gives dL/dP and dL/db on such plans, tests/test_gpu_backward_rsd.py; not dL/dn)
    for call in (lambda: p.backward(t, dC, want=("nz",)), lambda: p.cl_limber(t), lambda: p.windows(t)):
        with pytest.raises(bd.SwiftclError) as ei:
            call()
        assert ei.value.status == bd.SWIFTCL_E_UNSUPPORTED


# --- magnification bias (eq. magnification bias) -----------------------------------------------------

@pytest.mark.parametrize("precision,tol,rsd", [("fp32", 1e-4, False), ("split_bf16", 1e-3, False),
                                               ("fp32", 1e-4, True)])
def test_magnification_parity(dev, precision, tol, rsd):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.magnification_bias(_wl())
    wl["rsd"] = rsd
    _say(f"magnification cfg1 {precision}, rsd={rsd}")
    p = Plan.for_workload(wl, precision=precision, rsd=rsd, magnification=True)
    C = p.cl(device_inputs(wl, dev)).cpu().numpy()[0].astype(np.float64)
    assert p.device_flags() == 0
    e = eps_metric(full_from_packed(C, 15), full_from_packed(fftlog.cl(wl, 0), 15))
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < tol
    # the term is on: clustering x lensing spectra move away from the magnification-free oracle
    C0 = fftlog.cl(dict(wl, mag=None), 0)
    assert np.max(np.abs(C[0] - C0[0]) / np.max(np.abs(C0[0]))) > 1e-3


def test_magnification_plan_without_inputs_and_inputs_without_plan(dev):
    from paper_2505_22718_amd import binding as bd
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.magnification_bias(_wl())
    wl["rsd"] = False
    t = device_inputs(wl, dev)
    # a magnification plan called without C_g: no magnification term
    p = Plan.for_workload(wl, magnification=True)
    t0 = {k: v for k, v in t.items() if k != "mag"}
    C = p.cl(t0).cpu().numpy()[0].astype(np.float64)
    e = eps_metric(full_from_packed(C, 15), full_from_packed(fftlog.cl(dict(wl, mag=None), 0), 15))
    assert e.max() < 1e-4
    # C_g given to a plan built without magnification
    q = Plan.for_workload(wl)
    with pytest.raises(bd.SwiftclError) as ei:
        q.cl(t)
    assert ei.value.status == bd.SWIFTCL_E_INVALID
