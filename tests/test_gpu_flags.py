"""Data checks that need device data (swiftcl_device_flags): a non-finite P(k) sample, a multipole
index outside the plan's union, a point with no tracers and a chi(z) reaching past the chi box
raise their flag bits; the kernels clamp what they read, so the other points of the batch are
computed as if alone, and the adjoint runs on the same batch.
"""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

FLAG_SUPPORT_OVERFLOW, FLAG_NONFINITE, FLAG_BAD_INDEX = 1, 2, 4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_device_flags_and_isolation(dev):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg3", batch=5)
    plan = Plan.for_workload(wl)
    clean = device_inputs(wl, dev)
    C_clean = plan.cl(clean).clone()
    assert plan.device_flags() == 0

    bad = {k: v.clone() for k, v in clean.items()}
    bad["pk"][0, 5] = float("nan")                      # point 0: non-finite P(k)
    bad["ell_idx"][1, 0] = len(wl["ell"]) + 5           # point 1: index outside the union
    bad["n_tracers"][2] = 0                             # point 2: no tracers
    c3 = bad["chi_z"][3]
    bad["chi_z"][3] = c3[0] * (c3 / c3[0]) ** 3          # point 3: chi(z_max)/chi(z_min) past the chi box
    C_bad = plan.cl(bad)
    flags = plan.device_flags()
    _say(f"  flags after the bad batch: {flags}")
    assert flags == FLAG_SUPPORT_OVERFLOW | FLAG_NONFINITE | FLAG_BAD_INDEX
    assert torch.equal(C_bad[4], C_clean[4])            # point 4 untouched
    assert torch.all(C_bad[2] == 0)                     # no tracers: every spectrum 0
    assert bool(torch.isfinite(C_bad[1]).all()) and bool(torch.isfinite(C_bad[3]).all())
    # the flag word is cleared by the read
    assert plan.device_flags() == 0

    dC = torch.ones_like(C_bad)
    g = plan.backward(bad, dC)
    _say(f"  flags after the adjoint: {plan.device_flags()}")
    g_clean = plan.backward(clean, dC)
    for k in g:
        assert torch.equal(g[k][4], g_clean[k][4]) or \
            float((g[k][4] - g_clean[k][4]).abs().max()) <= 1e-12 * float(g_clean[k][4].abs().max()), k
        assert torch.all(g[k][2] == 0), k


def test_unknown_tracer_kind_is_flagged_and_zeroed(dev):
    """A tracer whose kind is none of the three raises FLAG_BAD_INDEX; its windows are zero, so every
    pair holding it is 0, the point's other pairs and the other points are as in a clean call, and the
    adjoint gives it no gradient."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    from tests.helpers import full_from_packed
    wl = synth.make_workload("cfg3", batch=3)
    plan = Plan.for_workload(wl)
    clean = device_inputs(wl, dev)
    C_clean = plan.cl(clean).clone()
    assert plan.device_flags() == 0
    bad = {k: v.clone() for k, v in clean.items()}
    bad["kind"][1, 0] = 3
    C_bad = plan.cl(bad)
    flags = plan.device_flags()
    _say(f"  flags with a tracer of kind 3: {flags}")
    assert flags == FLAG_BAD_INDEX
    assert torch.equal(C_bad[0], C_clean[0]) and torch.equal(C_bad[2], C_clean[2])
    T = plan.max_tracers
    fb = full_from_packed(C_bad[1].cpu().numpy(), T)
    fc = full_from_packed(C_clean[1].cpu().numpy(), T)
    assert np.all(fb[:, 0, :] == 0)
    assert np.array_equal(fb[:, 1:, 1:], fc[:, 1:, 1:])
    g = plan.backward(bad, torch.ones_like(C_bad))
    assert plan.device_flags() == FLAG_BAD_INDEX
    assert float(g["bias"][1, 0]) == 0.0 and bool(torch.all(g["nz"][1, 0] == 0))
