"""Scale-dependent growth D(k, z) on the GPU (swiftcl_cl_kgrowth through the C ABI) against the
FP64 oracle of Sec. 3.2 (oracle/kgrowth.py), element by element on the Q12 metric
|dC^{ij}| / sqrt(C^{ii} C^{jj}).

Tolerances: 1e-4 for FP32 (the FP32 target of the method against an FP64 reference; the dense
n-sum of the GEMM rounds like the FFT of the scale-free path), 1e-3 for the BF16 hi+lo projection.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fftlog, kgrowth
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


def _run(wl, dev, precision="fp32"):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    p = Plan.for_workload(wl, precision=precision, n_interp=wl["n_interp"])
    D = torch.as_tensor(wl["D_kz"], dtype=torch.float64, device=dev)
    C = p.cl_kgrowth(device_inputs(wl, dev), D).cpu().numpy()
    return p, C


def _oracle(wl, b, slots):
    """Oracle C at multipole slots `slots` of point b: [len(slots), T_b(T_b+1)/2]."""
    m = fftlog.method_for(wl)
    ells = fftlog.point_ells(wl, b)[slots]
    W = kgrowth.windows_point(kgrowth.node_geometries(wl, b), ells, m)
    return fftlog.cl_from_windows(W, wl["pk"][b], m)


def _eps(Cg_point, Cref, slots, T):
    Tmax = int(round((np.sqrt(8 * Cg_point.shape[-1] + 1) - 1) / 2))
    full = full_from_packed(Cg_point[slots], Tmax)[:, :T, :T]
    return eps_metric(full, full_from_packed(Cref, T))


def test_kgrowth_cfg0_fp32(dev):
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 16, f_nu=0.3)
    _say("kgrowth cfg0 fp32, 16 nodes")
    p, C = _run(wl, dev)
    assert p.device_flags() == 0
    slots = np.arange(wl["n_ell"][0])
    e = _eps(C[0], _oracle(wl, 0, slots), slots, 2)
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < 1e-4


@pytest.mark.parametrize("n_nodes", [2, 3, 17, 18, 19, 34])
def test_kgrowth_node_count_edges(dev, n_nodes):
    """Node counts at the edges of the node spline's 16-node segments (no interior node, one, a
    segment filled exactly, one node past it, two segments and a remainder): parity with the
    oracle's natural spline at the FP32 bar."""
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, n_nodes, f_nu=0.3)
    _say(f"kgrowth cfg0 fp32, {n_nodes} nodes")
    p, C = _run(wl, dev)
    assert p.device_flags() == 0
    slots = np.arange(wl["n_ell"][0])
    e = _eps(C[0], _oracle(wl, 0, slots), slots, 2)
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < 1e-4


def test_kgrowth_dense_nodes(dev):
    """200 nodes over 256 k nodes: a 64-node k tile spans more node rows than the windows GEMM
    stages in LDS, so the plan runs the GEMM that gathers them per lane."""
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 200, f_nu=0.3)
    _say("kgrowth cfg0 fp32, 200 nodes over 256 k")
    p, C = _run(wl, dev)
    assert p.device_flags() == 0
    slots = np.arange(wl["n_ell"][0])
    e = _eps(C[0], _oracle(wl, 0, slots), slots, 2)
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < 1e-4


def test_kgrowth_cfg1_200_nodes(dev):
    """15 tracers (10 clustering, 5 lensing), 103 l, N_k = N_chi = 1024, the paper's N_interp = 200."""
    wl = synth.make_workload("cfg1")
    synth.scale_dependent_growth(wl, 200)
    _say("kgrowth cfg1 fp32, 200 nodes")
    p, C = _run(wl, dev)
    assert p.device_flags() == 0
    slots = np.arange(0, 103, 6)
    e = _eps(C[0], _oracle(wl, 0, slots), slots, 15)
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < 1e-4


def test_kgrowth_scale_free_matches_fftlog_path(dev):
    """Growth equal at every node: the GEMM path and the scale-free FFT path give the same C_l."""
    from paper_2505_22718_amd.plan import device_inputs
    wl = synth.make_workload("cfg1")
    wl["n_interp"] = 8
    wl["D_kz"] = np.repeat(wl["D_z"][:, None, :], 8, 1)
    _say("kgrowth scale-free vs swiftcl_cl, cfg1")
    p, Ck = _run(wl, dev)
    Cf = p.cl(device_inputs(wl, dev)).cpu().numpy()
    e = eps_metric(full_from_packed(Ck[0], 15), full_from_packed(Cf[0].astype(np.float64), 15))
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < 1e-4


def test_kgrowth_ragged_batch_two_chunks(dev):
    """256 points of 6/10/15 tracers and 50..103 l; the workspace holds fewer points than the batch,
    so the launch runs in chunks.  Points from both chunks are checked; padded slots are zero."""
    wl = synth.make_workload("cfg3")
    synth.scale_dependent_growth(wl, 24)
    _say("kgrowth cfg3 ragged, 24 nodes, 256 points")
    p, C = _run(wl, dev)
    assert p.device_flags() == 0
    assert p.desc.n_interp == 24
    for b in (0, 1, 200, 255):
        T, L = int(wl["n_tracers"][b]), int(wl["n_ell"][b])
        slots = np.arange(0, L, 9)
        e = _eps(C[b], _oracle(wl, b, slots), slots, T)
        _say(f"  point {b} (T={T}, L={L}) max eps {e.max():.3e}")
        assert e.max() < 1e-4
        assert np.all(C[b, L:] == 0)
        full = full_from_packed(C[b, :L], 15)
        assert np.all(full[:, T:, :] == 0)


def test_kgrowth_split_bf16(dev):
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 16, f_nu=0.3)
    _say("kgrowth cfg0 split bf16")
    p, C = _run(wl, dev, precision="split_bf16")
    slots = np.arange(wl["n_ell"][0])
    e = _eps(C[0], _oracle(wl, 0, slots), slots, 2)
    _say(f"  max eps {e.max():.3e}")
    assert e.max() < 1e-3


def test_kgrowth_flags_nonfinite_growth(dev):
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 8)
    wl["D_kz"][0, 3, 100] = np.nan
    _say("kgrowth non-finite growth sample")
    p, C = _run(wl, dev)
    assert p.device_flags() & 2


def test_kgrowth_leaves_no_forward_state(dev):
    """A backward call after swiftcl_cl_kgrowth cannot reuse the workspace state."""
    from paper_2505_22718_amd import binding as bd
    from paper_2505_22718_amd.plan import device_inputs
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 8)
    p, C = _run(wl, dev)
    t = device_inputs(wl, dev)
    p.cl(t)
    D = torch.as_tensor(wl["D_kz"], dtype=torch.float64, device=dev)
    p.cl_kgrowth(t, D)
    dC = torch.ones((1, p.max_ell, p.n_pairs), dtype=p.out_dtype, device=dev)
    with pytest.raises(bd.SwiftclError):
        p.backward(t, dC, want=("pk",), reuse_forward=True)
