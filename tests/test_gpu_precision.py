"""Split-precision projection and the unfused path for more than 16 tracers.

* split BF16 (hi + lo, 16x16x32 bf16 MFMA, FP32 accumulation) against the FP64 oracle: every C_l
  within 1e-3 on the Q12 metric (the split target of the method); the per-l maximum is printed.
* 30 tracers (20 clustering + 10 lensing), N_k = N_chi = 2048, 200 l in [2, 3000]: the unfused
  projection (windows through the workspace, 32 x 32 Gram on MFMA tiles) in FP32 (1e-4) and split
  BF16 (1e-3); the oracle runs on every tenth multipole.
"""
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


def _per_ell(Cg, Cref, T):
    e = eps_metric(full_from_packed(Cg, T), full_from_packed(Cref, T))
    return e.reshape(e.shape[0], -1).max(axis=1)


def test_split_bf16_fused_15_tracers(dev):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg1")
    plan = Plan.for_workload(wl, precision="split_bf16")
    Cg = plan.cl(device_inputs(wl, dev)).cpu().numpy()[0].astype(np.float64)
    C = fftlog.cl(wl, 0)
    e = _per_ell(Cg, C, 15)
    _say("split bf16, 15 tracers: max eps per l: " + " ".join(f"{x:.1e}" for x in e))
    assert e.max() < 1e-3


def _cfg4_subset(batch):
    wl = synth.make_workload("cfg4", batch=batch)
    w = dict(wl)
    w["ell_idx"] = wl["ell_idx"][:, ::10].copy()
    w["n_ell"] = np.full(batch, w["ell_idx"].shape[1], np.int32)
    return w


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("split_bf16", 1e-3)])
def test_unfused_30_tracers(dev, precision, tol):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _cfg4_subset(2)
    plan = Plan.for_workload(wl, precision=precision)
    Cg = plan.cl(device_inputs(wl, dev)).cpu().numpy().astype(np.float64)
    assert plan.device_flags() == 0
    for b in range(2):
        C = fftlog.cl(wl, b)
        e = _per_ell(Cg[b], C, 30)
        _say(f"{precision}, 30 tracers, point {b}: max eps per l: " + " ".join(f"{x:.1e}" for x in e))
        assert e.max() < tol


def test_unfused_ragged_tracers(dev):
    """Points with 30 and with 12 tracers in one unfused batch: padded pairs are 0."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = _cfg4_subset(2)
    wl["n_tracers"] = np.array([30, 12], np.int32)
    plan = Plan.for_workload(wl, precision="fp32")
    Cg = plan.cl(device_inputs(wl, dev)).cpu().numpy().astype(np.float64)
    C = fftlog.cl(wl, 1)
    full = full_from_packed(Cg[1], 30)
    e = eps_metric(full[:, :12, :12], full_from_packed(C, 12))
    _say(f"ragged unfused: max eps {e.max():.2e}")
    assert e.max() < 1e-4
    full[:, :12, :12] = 0
    assert np.all(full == 0)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("split_bf16", 1e-3)])
def test_unfused_30_tracers_across_workspace_chunks(dev, precision, tol):
    """The 30-tracer shape with all 200 multipoles at 12 points: the workspace holds 10 points, so the
    call runs two chunks (the second from point 10 on), as the benchmark's 64-point batch runs seven.
    Points at both ends of each chunk against the oracle on every twentieth multipole."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    B = 12
    wl = synth.make_workload("cfg4", batch=B)
    plan = Plan.for_workload(wl, precision=precision)
    Cg = plan.cl(device_inputs(wl, dev)).cpu().numpy().astype(np.float64)
    assert plan.device_flags() == 0
    sub = dict(wl)
    sub["ell_idx"] = wl["ell_idx"][:, ::20].copy()
    sub["n_ell"] = np.full(B, sub["ell_idx"].shape[1], np.int32)
    for b in (0, 9, 10, 11):
        C = fftlog.cl(sub, b)
        e = _per_ell(Cg[b, ::20], C, 30)
        _say(f"{precision}, 30 tracers x 200 l, point {b}: max eps per sampled l: " + " ".join(f"{x:.1e}" for x in e))
        assert e.max() < tol
