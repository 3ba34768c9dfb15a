"""The adjoint of plans with redshift-space distortions (eq. RSD) and magnification bias (eq.
magnification bias), through the workspace: the recomputed windows carry both terms, so dL/dP is
complete, and so is dL/db (the bias scales the density term alone).  Entry by entry against the
oracle: gradients.grad_pk on the oracle's windows with both terms, and gradients.grad_bias_windows
(pinned in tests/test_oracle_grad_rsd.py), 1e-4 relative to each vector's largest entry (the
adjoint computes in FP32 on FP32 and split plans alike).  Ragged batches with padded tracer and
multipole slots; dL/dn and dL/dD are refused before any launch."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fftlog, gradients

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _wl(mag):
    """Three points of the ragged batch (6, 10 or 15 tracers), every 9th multipole slot kept."""
    wl = synth.make_workload("cfg3", batch=3)
    wl["rsd"] = True
    wl["ell_idx"] = np.ascontiguousarray(wl["ell_idx"][:, ::9])
    wl["n_ell"] = ((wl["n_ell"] + 8) // 9).astype(np.int32)
    if mag:
        synth.magnification_bias(wl)
    return wl


@pytest.mark.parametrize("precision,mag", [("fp32", False), ("fp32", True), ("split_bf16", True)])
def test_rsd_adjoint_pk_and_bias(dev, precision, mag):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _wl(mag)
    _say(f"RSD adjoint {precision}, magnification={mag}, T={wl['n_tracers'].tolist()}, L={wl['n_ell'].tolist()}")
    p = Plan.for_workload(wl, precision=precision, rsd=True, magnification=mag)
    assert p.adjoint_mode == 2
    inp = device_inputs(wl, dev)
    B = int(wl["batch"])
    G = np.random.default_rng(41).standard_normal((B, wl["ell_idx"].shape[1], p.n_pairs))
    dC = torch.as_tensor(G, dtype=torch.float32, device=dev)
    out = p.backward(inp, dC, want=("pk", "bias"))
    assert p.device_flags() == 0
    out = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    m = fftlog.method_for(wl)
    Tm = p.max_tracers
    at = {(i, j): q for q, (i, j) in enumerate(zip(*np.triu_indices(Tm)))}  # pairs packed for max_tracers
    for b in range(B):
        T, L = int(wl["n_tracers"][b]), int(wl["n_ell"][b])
        Gb = G[b, :L][:, [at[(i, j)] for i, j in zip(*np.triu_indices(T))]]
        _, W = fftlog.cl(wl, b, m, return_windows=True)
        e_pk = _rel(out["pk"][b], gradients.grad_pk(Gb, W, m))
        e_b = _rel(out["bias"][b, :T], gradients.grad_bias_windows(wl, b, Gb, m))
        _say(f"  point {b} (T={T}, L={L}): dP {e_pk:.2e}, db {e_b:.2e}")
        assert e_pk < 1e-4 and e_b < 1e-4
        assert np.all(out["bias"][b, T:] == 0)


def test_rsd_adjoint_refuses_nz_and_D(dev):
    from paper_2505_22718_amd.binding import SwiftclError, SWIFTCL_E_UNSUPPORTED
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _wl(True)
    p = Plan.for_workload(wl, rsd=True, magnification=True)
    inp = device_inputs(wl, dev)
    dC = torch.zeros((int(wl["batch"]), wl["ell_idx"].shape[1], p.n_pairs), dtype=torch.float32, device=dev)
    for want in (("pk", "nz"), ("D",)):
        with pytest.raises(SwiftclError) as ei:
            p.backward(inp, dC, want=want)
        assert ei.value.status == SWIFTCL_E_UNSUPPORTED
        _say(f"  {want}: {ei.value}")
