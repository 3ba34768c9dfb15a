"""CMB lensing (paper Sec. 2.4) on the GPU: a tracer of kind 2 whose kernel is the lens efficiency of
one source plane at chi_* (the top of the geometry grid) with the convergence prefactor l(l+1)/k^2,
against the FFTLog oracle (pinned to direct quadrature, an Einstein-de Sitter closed form and the
Limber limit in tests/test_oracle_cmb.py).

Tolerances: FP64 1e-10 and FP32 1e-4 on |dC^{ij}| / sqrt(C^{ii} C^{jj}) and per window row (as
for the other kinds); Limber 1e-10 / 1e-5 against the chi-node rule; gradients 1e-9 (FP64) of the
largest entry.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fftlog, gradients, limber
from oracle.geometry import point_geometry
from tests.helpers import eps_metric, full_from_packed, row_rel

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _subset_ells(wl, step):
    wl["ell_idx"] = np.ascontiguousarray(wl["ell_idx"][:, ::step])
    wl["n_ell"] = np.full(wl["batch"], wl["ell_idx"].shape[1], np.int32)
    return wl


def test_cmb_fp64_small(dev):
    """Two clustering bins and the CMB-lensing tracer, N_chi = 512, every multipole."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.cmb_lensing(synth.make_workload("cfg0"))
    _say("cmb fp64 cfg0 + CMB lensing: windows and C_l")
    p = Plan.for_workload(wl)
    inp = device_inputs(wl, dev)
    W = p.windows(inp).cpu().numpy()[0]
    C = p.cl(inp).cpu().numpy()[0]
    assert p.device_flags() == 0
    Cref, Wref = fftlog.cl(wl, 0, return_windows=True)
    r = row_rel(W, Wref)
    e = eps_metric(full_from_packed(C, 3), full_from_packed(Cref, 3))
    _say(f"  windows max row rel {r.max():.3e} (CMB row {r[:, 2].max():.3e}), C_l eps {e.max():.3e}")
    assert r.max() < 1e-10
    assert e.max() < 1e-10


def test_cmb_fp32_15_tracers(dev):
    """The 15-tracer set plus the CMB-lensing tracer (16 tracers, the fused projection), sampled
    multipoles."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _subset_ells(synth.cmb_lensing(synth.make_workload("cfg1")), 9)
    _say(f"cmb fp32 cfg1 + CMB lensing: {wl['ell_idx'].shape[1]} multipoles")
    p = Plan.for_workload(wl)
    C = p.cl(device_inputs(wl, dev)).cpu().numpy()[0].astype(np.float64)
    assert p.device_flags() == 0
    Cref = fftlog.cl(wl, 0)
    e = eps_metric(full_from_packed(C, 16), full_from_packed(Cref, 16))
    _say(f"  eps {e.max():.3e}; CMB auto {e[:, 15, 15].max():.3e}")
    assert e.max() < 1e-4


def test_cmb_limber(dev):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    for name, prec, tol in (("cfg0", "fp64", 1e-10), ("cfg1", "fp32", 1e-5)):
        wl = synth.cmb_lensing(synth.make_workload(name))
        if name == "cfg1":
            wl = _subset_ells(wl, 9)
        T = int(wl["n_tracers"][0])
        p = Plan.for_workload(wl, precision=prec)
        C = p.cl_limber(device_inputs(wl, dev)).cpu().numpy()[0].astype(np.float64)
        assert p.device_flags() == 0
        ref = limber.cl_limber_grid(point_geometry(wl, 0), fftlog.point_ells(wl, 0), fftlog.method_for(wl),
                                    wl["pk"][0])
        e = eps_metric(full_from_packed(C, T), ref)
        _say(f"cmb limber {name} {prec}: eps {e.max():.3e}")
        assert e.max() < tol


def test_cmb_backward_fp64(dev):
    """dL/dP, and dL/dD entry by entry (the CMB kernel is linear in D), with the oracle's full gradient;
    the CMB tracer's dL/dn row and dL/db entry are 0."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.cmb_lensing(synth.make_workload("cfg0"))
    p = Plan.for_workload(wl)
    inp = device_inputs(wl, dev)
    T, L = 3, wl["ell_idx"].shape[1]
    G = np.random.default_rng(21).standard_normal((1, L, 6))
    g = {k: v.cpu().numpy()[0] for k, v in p.backward(inp, torch.as_tensor(G, device=dev)).items()}
    assert p.device_flags() == 0
    m = fftlog.method_for(wl)
    C, W = fftlog.cl(wl, 0, m, return_windows=True)
    gp = gradients.grad_pk(G[0], W, m)
    gD = gradients.grad_D_full(wl, 0, G[0], m)
    gn = gradients.grad_nz_full(wl, 0, G[0], m)
    ep = np.max(np.abs(g["pk"] - gp)) / np.max(np.abs(gp))
    eD = np.max(np.abs(g["D"] - gD)) / np.max(np.abs(gD))
    en = np.max(np.abs(g["nz"][:T] - gn)) / np.max(np.abs(gn))
    _say(f"cmb backward fp64: dP {ep:.3e}, dD {eD:.3e}, dn {en:.3e}")
    assert ep < 1e-9 and eD < 1e-9 and en < 1e-9
    assert np.all(g["nz"][2] == 0) and g["bias"][2] == 0


def test_cmb_split_bf16(dev):
    """The 16-tracer set with the CMB tracer through the fused split-precision projection (1e-3)."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _subset_ells(synth.cmb_lensing(synth.make_workload("cfg1")), 17)
    p = Plan.for_workload(wl, precision="split_bf16")
    C = p.cl(device_inputs(wl, dev)).cpu().numpy()[0].astype(np.float64)
    assert p.device_flags() == 0
    e = eps_metric(full_from_packed(C, 16), full_from_packed(fftlog.cl(wl, 0), 16))
    _say(f"cmb split bf16: eps {e.max():.3e}")
    assert e.max() < 1e-3


def test_cmb_scale_dependent_growth(dev):
    """Growth at 8 k nodes on the 2-bin set with the CMB tracer, against oracle/kgrowth.py (FP32 1e-4)."""
    from oracle import kgrowth
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.scale_dependent_growth(synth.cmb_lensing(synth.make_workload("cfg0")), 8, f_nu=0.3)
    p = Plan.for_workload(wl, precision="fp32", n_interp=8)
    D = torch.as_tensor(wl["D_kz"], dtype=torch.float64, device=dev)
    C = p.cl_kgrowth(device_inputs(wl, dev), D).cpu().numpy()[0].astype(np.float64)
    assert p.device_flags() == 0
    e = eps_metric(full_from_packed(C, 3), full_from_packed(kgrowth.cl(wl, 0), 3))
    _say(f"cmb scale-dependent growth: eps {e.max():.3e}")
    assert e.max() < 1e-4
