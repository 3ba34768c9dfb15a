"""Parity of the hand-written adjoint (swiftcl_cl_backward) with the oracle's gradients.

The oracle gives dL/dP exactly (w k^3 W_i W_j), dL/db_t exactly (C^{ij}/b_t), and
directional derivatives along seeded directions v for n(z) and D(z) (every window is
linear in them, so one more oracle window pass is exact).  L = sum dC^{ij} C^{ij} with a
seeded cotangent dC.

Tolerances: FP32 path 1e-4 relative to the largest gradient entry (or to the directional
derivative); FP64 path 1e-9.
"""
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


def _run(wl, dev, precision, seed=11):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    p = Plan.for_workload(wl, precision=precision)
    inp = device_inputs(wl, dev)
    rng = np.random.default_rng(seed)
    B, L, npair = wl["batch"], wl["ell_idx"].shape[1], p.n_pairs
    G = rng.standard_normal((B, L, npair))
    dC = torch.as_tensor(G, dtype=p.out_dtype, device=dev)
    out = p.backward(inp, dC)
    assert p.device_flags() == 0
    return G, {k: v.cpu().numpy() for k, v in out.items()}


def _check(wl, G, out, tol, b=0, ndir=2):
    m = fftlog.method_for(wl)
    T = int(wl["n_tracers"][b])
    Lb = int(wl["n_ell"][b])
    npair = T * (T + 1) // 2
    full_T = wl["nz"].shape[1]
    # the GPU packs pairs of max_tracers; map the point's pairs
    iu_full = {(i, j): p for p, (i, j) in enumerate(zip(*np.triu_indices(full_T)))}
    Gb = np.array([[G[b, l, iu_full[(i, j)]] for (i, j) in zip(*np.triu_indices(T))] for l in range(Lb)])
    C, W = fftlog.cl(wl, b, m, return_windows=True)
    gp = gradients.grad_pk(Gb, W, m)
    e = np.max(np.abs(out["pk"][b] - gp)) / np.max(np.abs(gp))
    _say(f"  dP: rel err {e:.3e}")
    assert e < tol
    gb = gradients.grad_bias(Gb, C, wl["kind"][b, :T], wl["bias"][b, :T])
    e = np.max(np.abs(out["bias"][b, :T] - gb)) / np.max(np.abs(gb))
    _say(f"  db: rel err {e:.3e}")
    assert e < tol
    assert np.all(out["bias"][b, T:] == 0)
    rng = np.random.default_rng(5)
    kinds = wl["kind"][b, :T]
    picks = [int(np.nonzero(kinds == 0)[0][0])]
    if np.any(kinds == 1):
        picks.append(int(np.nonzero(kinds == 1)[0][-1]))
    for t in picks[:ndir]:
        v = rng.standard_normal(wl["nz"].shape[-1]) * wl["nz"][b, t].max()
        ref = gradients.directional_nz(wl, b, Gb, t, v, m)
        got = float(out["nz"][b, t] @ v)
        _say(f"  dn(z) tracer {t}: {got:.6e} vs {ref:.6e}")
        assert abs(got - ref) <= tol * abs(ref)
    v = rng.standard_normal(wl["D_z"].shape[-1])
    ref = gradients.directional_D(wl, b, Gb, v, m)
    got = float(out["D"][b] @ v)
    _say(f"  dD: {got:.6e} vs {ref:.6e}")
    assert abs(got - ref) <= tol * abs(ref)


def test_backward_cfg0_fp64(dev):
    wl = synth.make_workload("cfg0")
    _say("backward cfg0 fp64")
    G, out = _run(wl, dev, "fp64")
    _check(wl, G, out, 1e-9)


def test_backward_cfg2_fp32(dev):
    wl = synth.make_workload("cfg2")
    _say("backward cfg2 fp32")
    G, out = _run(wl, dev, "fp32")
    _check(wl, G, out, 1e-4)


def test_backward_intrinsic_alignment(dev):
    """NLA intrinsic alignment in the lensing kernels: the adjoint's dL/dn of a lensing tracer
    picks up the local n term, dL/dD the IA share of the kernel (directions checked for one
    clustering and one lensing tracer)."""
    wl = synth.intrinsic_alignment(synth.make_workload("cfg2"))
    _say("backward cfg2 fp64 with intrinsic alignment")
    G, out = _run(wl, dev, "fp64")
    _check(wl, G, out, 1e-9, ndir=2)


def test_backward_cfg2_fp64(dev):
    wl = synth.make_workload("cfg2")
    _say("backward cfg2 fp64")
    G, out = _run(wl, dev, "fp64")
    _check(wl, G, out, 1e-9, ndir=1)


def test_backward_ragged(dev):
    wl = synth.make_workload("cfg3", batch=4)
    _say(f"backward cfg3 ragged T={wl['n_tracers'].tolist()} L={wl['n_ell'].tolist()}")
    G, out = _run(wl, dev, "fp32")
    for b in range(4):
        _say(f" point {b}")
        _check(wl, G, out, 1e-4, b=b, ndir=1)
        T = int(wl["n_tracers"][b])
        assert np.all(out["nz"][b, T:] == 0)


def test_backward_reuse_forward(dev):
    """SWIFTCL_BWD_REUSE_FORWARD keeps the forward's assembly and FFTLog state: the gradients equal
    those of a recomputing call (to the FP64 atomics' summation order), and the call is refused
    when the plan's last forward had other inputs or there was none."""
    from paper_2505_22718_amd.binding import SwiftclError, SWIFTCL_E_INVALID
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg3", batch=4)
    p = Plan.for_workload(wl, precision="fp32")
    inp = device_inputs(wl, dev)
    rng = np.random.default_rng(3)
    dC = torch.as_tensor(rng.standard_normal((4, wl["ell_idx"].shape[1], p.n_pairs)), dtype=torch.float32,
                         device=dev)
    with pytest.raises(SwiftclError) as ei:
        p.backward(inp, dC, reuse_forward=True)
    assert ei.value.status == SWIFTCL_E_INVALID
    ref = p.backward(inp, dC)
    p.cl(inp)
    got = p.backward(inp, dC, reuse_forward=True)
    for k in ref:
        scale = max(ref[k].abs().max().item(), 1e-300)
        err = (got[k] - ref[k]).abs().max().item() / scale
        _say(f"  {k}: reuse vs recompute {err:.2e}")
        assert err < 1e-10
    other = dict(inp)
    other["pk"] = inp["pk"] * 1.01  # same shapes, another buffer
    p.cl(other)
    with pytest.raises(SwiftclError) as ei:
        p.backward(inp, dC, reuse_forward=True)
    assert ei.value.status == SWIFTCL_E_INVALID


def test_backward_unsupported_plans(dev):
    """Plans with redshift-space distortions or magnification run the workspace adjoint, which gives
    dL/dP and dL/db only (tests/test_gpu_backward_rsd.py): asking them for dL/dn or dL/dD is refused
    with SWIFTCL_E_UNSUPPORTED before launching anything."""
    from paper_2505_22718_amd.binding import SwiftclError, SWIFTCL_E_UNSUPPORTED
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg3", batch=2)
    inp = device_inputs(wl, dev)
    for opt in ({"rsd": True}, {"magnification": True}):
        p = Plan(wl["k"], wl["ell"], wl["z_geom"], wl["z_nz"], wl["n_chi"], 2, wl["nz"].shape[1],
                 wl["ell_idx"].shape[1], precision="fp32", **opt)
        assert p.adjoint_mode == 2
        dC = torch.zeros((2, wl["ell_idx"].shape[1], p.n_pairs), dtype=torch.float32, device=dev)
        with pytest.raises(SwiftclError) as ei:
            p.backward(inp, dC)
        assert ei.value.status == SWIFTCL_E_UNSUPPORTED
        _say(f"  {opt}: {ei.value}")


def test_backward_bench_config(dev):
    """The benchmark batch (256 points of the 15-tracer set) in the launch shapes the bench times:
    autotuned, forward then the adjoint reusing the forward state.  dP and db of two sampled
    points against the oracle; every point's gradients finite."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    B = 256
    wl = synth.make_workload("cfg1_batch", batch=B)
    p = Plan.for_workload(wl)
    inp = device_inputs(wl, dev)
    rng = np.random.default_rng(21)
    G = rng.standard_normal((B, wl["ell_idx"].shape[1], p.n_pairs))
    dC = torch.as_tensor(G, dtype=torch.float32, device=dev)
    _say("  " + p.autotune(inp, dC))
    p.cl(inp)
    out = p.backward(inp, dC, reuse_forward=True)
    assert p.device_flags() == 0
    out = {k: v.cpu().numpy() for k, v in out.items()}
    for k, v in out.items():
        assert np.all(np.isfinite(v)), k
    m = fftlog.method_for(wl)
    for b in (0, B - 1):
        T = int(wl["n_tracers"][b])
        Gb = G[b][:, :T * (T + 1) // 2]
        C, W = fftlog.cl(wl, b, m, return_windows=True)
        gp = gradients.grad_pk(Gb, W, m)
        e = np.max(np.abs(out["pk"][b] - gp)) / np.max(np.abs(gp))
        gb = gradients.grad_bias(Gb, C, wl["kind"][b, :T], wl["bias"][b, :T])
        eb = np.max(np.abs(out["bias"][b, :T] - gb)) / np.max(np.abs(gb))
        _say(f"  point {b}: dP rel err {e:.2e}, db rel err {eb:.2e}")
        assert e < 1e-4 and eb < 1e-4


def _with_padded_slot(wl):
    """The workload with one more tracer slot, left empty (n_tracers unchanged)."""
    B, T, ns = wl["nz"].shape
    nz = np.zeros((B, T + 1, ns))
    nz[:, :T] = wl["nz"]
    kind = np.zeros((B, T + 1), np.int32)
    kind[:, :T] = wl["kind"]
    bias = np.ones((B, T + 1))
    bias[:, :T] = wl["bias"]
    wl.update(nz=nz, kind=kind, bias=bias)
    return wl


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_backward_nz_and_D_entry_by_entry(dev, precision, tol):
    """dL/dn(z) of every tracer at every one of its 200 samples and dL/dD at every geometry sample,
    against the oracle's full gradient vectors (the chain rule through its own linear steps, pinned in
    tests/test_oracle_gradients_full.py): the 15-tracer set with perturbed biases, intrinsic
    alignment on, ten multipoles, and one empty tracer slot whose rows must be 0.  Tolerance
    relative to each vector's largest entry."""
    wl = _with_padded_slot(synth.intrinsic_alignment(synth.make_workload("cfg2")))
    wl["ell_idx"] = np.ascontiguousarray(wl["ell_idx"][:, ::11])
    wl["n_ell"] = np.array([wl["ell_idx"].shape[1]], np.int32)
    _say(f"backward {precision}: dn(z) and dD entry by entry, {wl['ell_idx'].shape[1]} multipoles, IA on")
    G, out = _run(wl, dev, precision, seed=17)
    T = 15
    iu_full = {(i, j): p for p, (i, j) in enumerate(zip(*np.triu_indices(T + 1)))}
    Gb = np.array([[G[0, l, iu_full[(i, j)]] for (i, j) in zip(*np.triu_indices(T))]
                   for l in range(wl["ell_idx"].shape[1])])
    m = fftlog.method_for(wl)
    kern = gradients.grad_kernels(wl, 0, Gb, m)
    gn = gradients.grad_nz_full(wl, 0, Gb, m, kern=kern)
    gD = gradients.grad_D_full(wl, 0, Gb, m, kern=kern)
    worst = 0.0
    for t in range(T):
        e = np.max(np.abs(out["nz"][0, t] - gn[t])) / np.max(np.abs(gn[t]))
        worst = max(worst, e)
        assert e < tol, (t, e)
    eD = np.max(np.abs(out["D"][0] - gD)) / np.max(np.abs(gD))
    _say(f"  dn(z): worst tracer {worst:.3e}; dD {eD:.3e}")
    assert eD < tol
    assert np.all(out["nz"][0, T] == 0) and out["bias"][0, T] == 0
