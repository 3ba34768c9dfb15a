"""Parity of the HIP path (through the C ABI) with the FFTLog oracle, element by element.

Tolerances:
  FP64 path   1e-10 on the Q12 metric |dC^{ij}| / sqrt(C^{ii} C^{jj}) and per window row:
              FP64 roundoff (1e-16) grown by the FFT depth, the U-table log-gamma
              cancellation (|ln Gamma| <= 1e4 -> 1e-12) and the spline solves.
  FP32 path   1e-4 on the same metric and on every window row relative to its maximum
              (the FP32 target of the method against an FP64 reference).  Windows sit
              closer to it than C_l: the tilted FFT output spans decades over k, so its
              FP32 roundoff, relative to the row maximum, is amplified where k^{-1-b} is
              large; C_l weights those nodes little.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fftlog
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


def _plan(wl, **kw):
    from paper_2505_22718_amd.plan import Plan
    return Plan.for_workload(wl, **kw)


def _oracle_point(wl, b, method=None):
    m = method or fftlog.method_for(wl)
    return fftlog.cl(wl, b, m, return_windows=True)


@pytest.fixture(scope="module")
def cfg0():
    wl = synth.make_workload("cfg0")
    C, W = _oracle_point(wl, 0)
    return wl, C, W


@pytest.fixture(scope="module")
def cfg1():
    wl = synth.make_workload("cfg1")
    C, W = _oracle_point(wl, 0)
    return wl, C, W


def test_windows_cfg0_fp64(dev, cfg0):
    from paper_2505_22718_amd.plan import device_inputs
    wl, C, W = cfg0
    _say("windows cfg0 fp64")
    p = _plan(wl)
    Wg = p.windows(device_inputs(wl, dev)).cpu().numpy()[0]
    assert p.device_flags() == 0
    r = row_rel(Wg[:, :2], W)
    _say(f"  max row rel {r.max():.3e}")
    assert r.max() < 1e-10


def test_cl_cfg0_fp64(dev, cfg0):
    from paper_2505_22718_amd.plan import device_inputs
    wl, C, W = cfg0
    _say("cl cfg0 fp64")
    p = _plan(wl)
    Cg = p.cl(device_inputs(wl, dev)).cpu().numpy()[0]
    e = eps_metric(full_from_packed(Cg, 2), full_from_packed(C, 2))
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < 1e-10


def test_windows_cfg1_fp32(dev, cfg1):
    from paper_2505_22718_amd.plan import device_inputs
    wl, C, W = cfg1
    _say("windows cfg1 fp32")
    p = _plan(wl)
    Wg = p.windows(device_inputs(wl, dev)).cpu().numpy()[0]
    r = row_rel(Wg.astype(np.float64), W)
    _say(f"  max row rel {r.max():.3e} median {np.median(r):.3e}")
    assert r.max() < 1e-4


def test_cl_cfg1_fp32(dev, cfg1):
    from paper_2505_22718_amd.plan import device_inputs
    wl, C, W = cfg1
    _say("cl cfg1 fp32")
    p = _plan(wl)
    Cg = p.cl(device_inputs(wl, dev)).cpu().numpy()[0].astype(np.float64)
    e = eps_metric(full_from_packed(Cg, 15), full_from_packed(C, 15))
    _say(f"  max eps {e.max():.3e} median {np.median(e):.3e}")
    assert e.max() < 1e-4
    assert p.device_flags() == 0


def test_cl_fp64_instantiation_on_cfg1(dev, cfg1):
    """The same 15-tracer workload through the FP64 template: roundoff-level agreement."""
    from paper_2505_22718_amd.plan import device_inputs
    wl, C, W = cfg1
    _say("cl cfg1 fp64")
    p = _plan(wl, precision="fp64")
    Cg = p.cl(device_inputs(wl, dev)).cpu().numpy()[0]
    e = eps_metric(full_from_packed(Cg, 15), full_from_packed(C, 15))
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < 1e-10


def test_batch_bench_config_sampled(dev):
    """The benchmark's configuration (256 points of the 15-tracer workload, FP32): sampled points."""
    from paper_2505_22718_amd.plan import device_inputs
    wl = synth.make_workload("cfg1_batch", batch=256)
    _say("cl cfg1_batch B=256 fp32")
    p = _plan(wl)
    Cg = p.cl(device_inputs(wl, dev)).cpu().numpy().astype(np.float64)
    assert p.device_flags() == 0
    for b in (0, 101, 255):
        C = fftlog.cl(wl, b)
        e = eps_metric(full_from_packed(Cg[b], 15), full_from_packed(C, 15))
        _say(f"  point {b}: max eps {e.max():.3e}")
        assert e.max() < 1e-4


def test_ragged_batch(dev):
    """Uneven tracer and multipole counts: every real slot matches, every padded slot is 0."""
    from paper_2505_22718_amd.plan import device_inputs
    wl = synth.make_workload("cfg3", batch=6)
    _say(f"cl cfg3 ragged B=6 T={wl['n_tracers'].tolist()} L={wl['n_ell'].tolist()}")
    p = _plan(wl)
    Cg = p.cl(device_inputs(wl, dev)).cpu().numpy().astype(np.float64)
    T = wl["nz"].shape[1]
    for b in range(6):
        Tb, Lb = int(wl["n_tracers"][b]), int(wl["n_ell"][b])
        C = fftlog.cl(wl, b)
        full = full_from_packed(Cg[b], T)
        e = eps_metric(full[:Lb, :Tb, :Tb], full_from_packed(C, Tb))
        _say(f"  point {b}: max eps {e.max():.3e}")
        assert e.max() < 1e-4
        pad = full.copy()
        pad[:Lb, :Tb, :Tb] = 0
        assert np.all(pad == 0)


def test_single_tracer_single_ell(dev):
    from paper_2505_22718_amd.plan import device_inputs
    wl = synth.make_workload("cfg1")
    w = dict(wl)
    sel = [12]  # one lensing tracer
    w["nz"] = wl["nz"][:, sel]
    w["kind"] = wl["kind"][:, sel]
    w["bias"] = wl["bias"][:, sel]
    w["n_tracers"] = np.array([1], np.int32)
    w["ell"] = np.array([57.0])
    w["ell_idx"] = np.zeros((1, 1), np.int32)
    w["n_ell"] = np.array([1], np.int32)
    _say("cl single tracer, single l")
    p = _plan(w)
    Cg = p.cl(device_inputs(w, dev)).cpu().numpy().astype(np.float64)
    C = fftlog.cl(w, 0)
    assert abs(Cg[0, 0, 0] / C[0, 0] - 1) < 1e-4
