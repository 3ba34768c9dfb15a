"""Parity of the adjoint through the workspace (swiftcl_cl_backward on plans whose windows do not
fit one workgroup's LDS: more than 16 tracers, n_chi = 2048) and of the fused adjoint on a
split-precision plan, against the oracle's gradients (oracle/gradients.py, pinned in
tests/test_oracle_gradients_full.py).  L = sum dC^{ij} C^{ij} with a seeded cotangent.

The adjoint computes in FP32 on every FP32 and split plan (the split precision is that of the
forward projection only): tolerance 1e-4 relative to each gradient vector's largest entry, the FP32
bar of the fused adjoint.
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


def _thin_ells(wl, step):
    wl["ell_idx"] = np.ascontiguousarray(wl["ell_idx"][:, ::step])
    wl["n_ell"] = np.full(wl["batch"], wl["ell_idx"].shape[1], np.int32)
    return wl


def _thin_ells_keep_slots(wl, step):
    """Every step-th multipole in the first slots, the point's other slots left padded: the plan
    keeps the full multipole capacity (and so the full-size workspace chunking)."""
    sub = wl["ell_idx"][:, ::step]
    wl["ell_idx"] = np.zeros_like(wl["ell_idx"])
    wl["ell_idx"][:, :sub.shape[1]] = sub
    wl["n_ell"] = np.full(wl["batch"], sub.shape[1], np.int32)
    return wl


def _thirty_tracers_nchi1024():
    """The 15-tracer geometry and grids (n_chi = n_k = 1024) with the 30-tracer set (20 clustering
    + 10 lensing bins, biases perturbed by +-10%)."""
    wl = synth.make_workload("cfg2")
    nz1, kinds1, bias1 = synth.tracer_set(20, 10, wl["z_nz"])
    bias1 = bias1 * np.r_[np.random.default_rng(8).uniform(0.9, 1.1, 20), np.ones(10)]
    wl.update(nz=nz1[None].copy(), kind=kinds1[None].astype(np.int32), bias=bias1[None].copy(),
              n_tracers=np.array([30], np.int32))
    return wl


def _run(wl, dev, precision, seed):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    p = Plan.for_workload(wl, precision=precision)
    inp = device_inputs(wl, dev)
    G = np.random.default_rng(seed).standard_normal((wl["batch"], wl["ell_idx"].shape[1], p.n_pairs))
    dC = torch.as_tensor(G, dtype=torch.float32, device=dev)
    out = p.backward(inp, dC)
    assert p.device_flags() == 0
    return p, G, {k: v.cpu().numpy() for k, v in out.items()}


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _check_point(wl, G, out, b, tol, full):
    m = fftlog.method_for(wl)
    T = int(wl["n_tracers"][b])
    L = int(wl["n_ell"][b])
    Gb = G[b, :L, :T * (T + 1) // 2]
    C, W = fftlog.cl(wl, b, m, return_windows=True)
    e_pk = _rel(out["pk"][b], gradients.grad_pk(Gb, W, m))
    e_b = _rel(out["bias"][b, :T], gradients.grad_bias(Gb, C, wl["kind"][b, :T], wl["bias"][b, :T]))
    _say(f"  point {b}: dP {e_pk:.2e}, db {e_b:.2e}")
    assert e_pk < tol and e_b < tol
    if full:
        kern = gradients.grad_kernels(wl, b, Gb, m)
        gn = gradients.grad_nz_full(wl, b, Gb, m, kern=kern)
        gD = gradients.grad_D_full(wl, b, Gb, m, kern=kern)
        worst = max(_rel(out["nz"][b, t], gn[t]) for t in range(T))
        eD = _rel(out["D"][b], gD)
        _say(f"  point {b}: dn(z) worst tracer {worst:.2e}, dD {eD:.2e}")
        assert worst < tol and eD < tol


def test_ws_adjoint_30_tracers_fp32(dev):
    """30 tracers at n_chi = n_k = 1024 in FP32 (two 16-row tracer tiles of G W, 8 tracer groups
    of adjoint transforms): dP, db, dn(z) of every tracer and dD entry by entry."""
    wl = _thin_ells(_thirty_tracers_nchi1024(), 11)
    _say(f"workspace adjoint fp32, 30 tracers, n_chi 1024, {wl['ell_idx'].shape[1]} multipoles")
    p, G, out = _run(wl, dev, "fp32", seed=31)
    assert p.adjoint_mode == 2
    _check_point(wl, G, out, 0, 1e-4, full=True)


def test_ws_adjoint_split_nchi2048(dev):
    """The 30-tracer split-precision set (465 spectra, n_chi = n_k = 2048), two points, every 20th
    of the 200 multipoles: point 0 entry by entry (dP, db, dn(z), dD), point 1 dP and db."""
    wl = _thin_ells(synth.make_workload("cfg4", batch=2), 20)
    _say(f"workspace adjoint, split plan, 30 tracers, n_chi 2048, {wl['ell_idx'].shape[1]} multipoles")
    p, G, out = _run(wl, dev, "split_bf16", seed=32)
    assert p.adjoint_mode == 2
    _check_point(wl, G, out, 0, 1e-4, full=True)
    _check_point(wl, G, out, 1, 1e-4, full=False)


def test_ws_adjoint_across_point_chunks(dev):
    """12 points of the 30-tracer n_chi = 2048 set run as two chunks of the workspace (10 + 2
    points): dP and db of the points on both sides of the boundary against the oracle, and every
    point's gradients finite."""
    wl = _thin_ells_keep_slots(synth.make_workload("cfg4", batch=12), 40)
    _say(f"workspace adjoint across chunks: 12 points, {wl['n_ell'][0]} of {wl['ell_idx'].shape[1]} multipole slots")
    p, G, out = _run(wl, dev, "split_bf16", seed=33)
    assert p.vchunk < 12
    for k, v in out.items():
        assert np.all(np.isfinite(v)), k
    for b in (0, p.vchunk - 1, p.vchunk, 11):
        _check_point(wl, G, out, b, 1e-4, full=False)


def test_fused_adjoint_on_split_plan(dev):
    """A split-precision plan of 15 tracers keeps the fused adjoint (FP32 windows in LDS)."""
    wl = _thin_ells(synth.make_workload("cfg2"), 6)
    _say(f"fused adjoint, split plan, 15 tracers, {wl['ell_idx'].shape[1]} multipoles")
    p, G, out = _run(wl, dev, "split_bf16", seed=34)
    assert p.adjoint_mode == 1
    _check_point(wl, G, out, 0, 1e-4, full=True)
