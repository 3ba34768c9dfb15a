"""The Limber path on the GPU (swiftcl_cl_limber through the C ABI) against the oracle's Limber rule
on the same chi nodes (oracle/limber.cl_limber_grid), element by element on the Q12 metric, and
against the GPU's own FFTLog C_l at high l (the Limber error is O(1/l)).

Tolerances: 1e-10 for FP64 (FP64 roundoff over ~500 node terms and the spline of ln P), 1e-5 for
FP32 and split-precision plans (kernel samples rounded to FP32, FP32 sums of ~500 positive-weight
terms).
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fftlog, geometry, limber
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


def _oracle(wl, b):
    m = fftlog.method_for(wl)
    return limber.cl_limber_grid(geometry.point_geometry(wl, b), fftlog.point_ells(wl, b), m, wl["pk"][b])


@pytest.mark.parametrize("name,precision,tol", [("cfg0", "fp64", 1e-10), ("cfg1", "fp32", 1e-5),
                                                ("cfg1", "split_bf16", 1e-5)])
def test_limber_parity(dev, name, precision, tol):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload(name)
    _say(f"limber {name} {precision}")
    p = Plan.for_workload(wl, precision=precision)
    C = p.cl_limber(device_inputs(wl, dev)).cpu().numpy()[0].astype(np.float64)
    assert p.device_flags() == 0
    T = int(wl["n_tracers"][0])
    e = eps_metric(full_from_packed(C, T), _oracle(wl, 0))
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < tol


def test_limber_ragged_batch(dev):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg3", batch=24)
    _say("limber cfg3 ragged, 24 points")
    p = Plan.for_workload(wl)
    C = p.cl_limber(device_inputs(wl, dev)).cpu().numpy().astype(np.float64)
    assert p.device_flags() == 0
    for b in (0, 7, 23):
        T, L = int(wl["n_tracers"][b]), int(wl["n_ell"][b])
        full = full_from_packed(C[b, :L], 15)
        e = eps_metric(full[:, :T, :T], _oracle(wl, b))
        _say(f"  point {b} (T={T}, L={L}) max eps {e.max():.3e}")
        assert e.max() < 1e-5
        assert np.all(C[b, L:] == 0)
        assert np.all(full[:, T:, :] == 0)


def test_limber_agrees_with_fftlog_at_high_ell(dev):
    """The built-in consistency check: clustering autos within 1e-2 of the FFTLog C_l for l >= 500,
    lensing autos within 2e-2 for l >= 1000, the clustering error shrinking with l."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg1")
    p = Plan.for_workload(wl)
    t = device_inputs(wl, dev)
    CL = full_from_packed(p.cl_limber(t).cpu().numpy()[0].astype(np.float64), 15)
    CF = full_from_packed(p.cl(t).cpu().numpy()[0].astype(np.float64), 15)
    ells = wl["ell"][wl["ell_idx"][0]]
    rel = np.abs(np.einsum("ltt->lt", CF) / np.einsum("ltt->lt", CL) - 1)
    _say(f"limber vs fftlog: clustering {rel[ells >= 500, :10].max():.3e}, lensing {rel[ells >= 1000, 10:].max():.3e}")
    assert rel[ells >= 500, :10].max() < 1e-2
    assert rel[-1, :10].mean() < rel[np.argmax(ells >= 300), :10].mean()
    assert rel[ells >= 1000, 10:].max() < 2e-2


def test_limber_invalidates_forward_state(dev):
    from paper_2505_22718_amd import binding as bd
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg0")
    p = Plan.for_workload(wl, precision="fp32")
    t = device_inputs(wl, dev)
    p.cl(t)
    p.cl_limber(t)
    dC = torch.ones((1, p.max_ell, p.n_pairs), dtype=p.out_dtype, device=dev)
    with pytest.raises(bd.SwiftclError):
        p.backward(t, dC, want=("pk",), reuse_forward=True)
