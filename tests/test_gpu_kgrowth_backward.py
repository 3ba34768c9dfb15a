"""The adjoint of the scale-dependent growth path (swiftcl_cl_kgrowth_backward through the C ABI):
dL/dP and dL/db for L = sum dC C against the FP64 oracle of Sec. 3.2, entry by entry
(gradients.grad_pk on the kgrowth oracle's windows, and the closed form C/b of gradients.grad_bias;
both pinned in tests/test_oracle_grad_kgrowth.py), 1e-4 relative to each vector's largest entry
(the adjoint computes in FP32).  Covers 2 and 15 tracers, a ragged batch that spans two workspace
chunks, and the autograd function against central differences of the GPU forward."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fftlog, gradients, kgrowth

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


def _run(wl, dev, seed):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    p = Plan.for_workload(wl, precision="fp32", n_interp=wl["n_interp"])
    t = device_inputs(wl, dev)
    D = torch.as_tensor(wl["D_kz"], dtype=torch.float64, device=dev)
    C = p.cl_kgrowth(t, D)
    G = np.random.default_rng(seed).standard_normal(tuple(C.shape))
    dC = torch.as_tensor(G, dtype=torch.float32, device=dev)
    out = p.kgrowth_backward(t, D, C, dC)
    assert p.device_flags() == 0
    return p, G, {k: v.cpu().numpy() for k, v in out.items()}


def _check(wl, p, G, out, b, slots=None):
    m = fftlog.method_for(wl)
    T, L = int(wl["n_tracers"][b]), int(wl["n_ell"][b])
    at = {(i, j): q for q, (i, j) in enumerate(zip(*np.triu_indices(p.max_tracers)))}
    Gb = G[b, :L][:, [at[(i, j)] for i, j in zip(*np.triu_indices(T))]]
    C, W = kgrowth.cl(wl, b, m, return_windows=True)
    e_pk = _rel(out["pk"][b], gradients.grad_pk(Gb, W, m))
    e_b = _rel(out["bias"][b, :T], gradients.grad_bias(Gb, C, wl["kind"][b, :T], wl["bias"][b, :T]))
    _say(f"  point {b} (T={T}, L={L}): dP {e_pk:.2e}, db {e_b:.2e}")
    assert e_pk < 1e-4 and e_b < 1e-4
    assert np.all(out["bias"][b, T:] == 0)
    assert np.all(out["bias"][b, :T][np.asarray(wl["kind"][b, :T]) != 0] == 0)


def test_kgrowth_backward_cfg0(dev):
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 16, f_nu=0.3)
    _say("kgrowth adjoint cfg0, 16 nodes")
    p, G, out = _run(wl, dev, 51)
    _check(wl, p, G, out, 0)


def test_kgrowth_backward_cfg1_thinned(dev):
    """15 tracers (10 clustering, 5 lensing), N_k = N_chi = 1024, 40 nodes, every 8th multipole."""
    wl = synth.make_workload("cfg1")
    synth.scale_dependent_growth(wl, 40)
    wl["ell_idx"] = np.ascontiguousarray(wl["ell_idx"][:, ::8])
    wl["n_ell"] = np.array([wl["ell_idx"].shape[1]], np.int32)
    _say("kgrowth adjoint cfg1, 40 nodes, 13 multipoles")
    p, G, out = _run(wl, dev, 52)
    _check(wl, p, G, out, 0)


def test_kgrowth_backward_ragged_two_chunks(dev):
    """The ragged batch (256 points of 6/10/15 tracers, the full multipole slots, every 20th
    multipole filled) runs in workspace chunks: points at both ends of the first chunk and in the
    last one against the oracle."""
    wl = synth.make_workload("cfg3")
    synth.scale_dependent_growth(wl, 24)
    sub = wl["ell_idx"][:, ::20]
    wl["ell_idx"] = np.zeros_like(wl["ell_idx"])
    wl["ell_idx"][:, :sub.shape[1]] = sub
    wl["n_ell"] = np.full(wl["batch"], sub.shape[1], np.int32)
    p, G, out = _run(wl, dev, 53)
    chunk = p.vchunk
    _say(f"kgrowth adjoint cfg3 ragged, 256 points, chunks of {chunk}")
    assert 0 < chunk < 256
    for b in (0, chunk - 1, chunk, 255):
        _check(wl, p, G, out, b)


def test_kgrowth_autograd_central_differences(dev):
    """cl_kgrowth's gradients against central differences of the GPU forward along random
    directions (exact up to FP32 rounding: L is linear in P and quadratic in b)."""
    from paper_2505_22718_amd import autograd
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 16, f_nu=0.3)
    p = Plan.for_workload(wl, precision="fp32", n_interp=16)
    t = device_inputs(wl, dev)
    D = torch.as_tensor(wl["D_kz"], dtype=torch.float64, device=dev)
    pk = t["pk"].clone().requires_grad_(True)
    bias = t["bias"].clone().requires_grad_(True)
    C = autograd.cl_kgrowth(p, t, D, pk, bias)
    dC = torch.as_tensor(np.random.default_rng(54).standard_normal(tuple(C.shape)), dtype=torch.float32, device=dev)
    (C.double() * dC.double()).sum().backward()
    rng = np.random.default_rng(55)

    def loss(pk_, b_):
        with torch.no_grad():
            return float((autograd.cl_kgrowth(p, t, D, pk_, b_).double() * dC.double()).sum())

    v = torch.as_tensor(rng.standard_normal(tuple(pk.shape)), device=dev) * t["pk"]
    h = 0.1
    fd = (loss(t["pk"] + h * v, t["bias"]) - loss(t["pk"] - h * v, t["bias"])) / (2 * h)
    an = float((pk.grad * v).sum())
    _say(f"  dP along a direction: {an:.6e} vs central difference {fd:.6e}")
    assert abs(an - fd) <= 1e-4 * abs(fd)
    u = torch.as_tensor(rng.standard_normal(tuple(bias.shape)), device=dev)
    fd = (loss(t["pk"], t["bias"] + h * u) - loss(t["pk"], t["bias"] - h * u)) / (2 * h)
    an = float((bias.grad * u).sum())
    _say(f"  db along a direction: {an:.6e} vs central difference {fd:.6e}")
    assert abs(an - fd) <= 1e-4 * abs(fd)
