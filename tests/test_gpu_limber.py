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


# --- the adjoint (swiftcl_cl_limber_backward) -------------------------------------------------

def _limber_grads_oracle(wl, b, Gp):
    """The oracle's gradients of L = sum dC * C_limber for point b: dP (limber.grad_pk_grid), db
    (quadratic in the biases), dn(z) and dD (limber.grad_kernels_grid through the kernels of the
    unit samples)."""
    from oracle import gradients
    m = fftlog.method_for(wl)
    geo = geometry.point_geometry(wl, b)
    ells = fftlog.point_ells(wl, b)
    T = int(wl["n_tracers"][b])
    Gf = gradients.symmetric_cotangent(Gp, T)
    C = limber.cl_limber_grid(geo, ells, m, wl["pk"][b])
    iu = np.triu_indices(T)
    out = {"pk": limber.grad_pk_grid(Gf, geo, ells, m, wl["pk"][b]),
           "bias": gradients.grad_bias(Gp, C[:, iu[0], iu[1]], wl["kind"][b, :T], wl["bias"][b, :T])}
    kern = limber.grad_kernels_grid(Gf, geo, ells, m, wl["pk"][b])
    out["nz"] = gradients.grad_nz_full(wl, b, None, m, kern=kern)
    out["D"] = gradients.grad_D_full(wl, b, None, m, kern=kern)
    return out


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_limber_backward_entry_by_entry(dev, precision, tol):
    """The 15-tracer set plus a CMB-lensing tracer with intrinsic alignment on, perturbed biases,
    every 9th multipole: dP at every k node, db, dn(z) of every tracer at every sample and dD at
    every geometry sample against the oracle, relative to each vector's largest entry (the FP64
    and FP32 bars of the FFTLog adjoint)."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.intrinsic_alignment(synth.cmb_lensing(synth.make_workload("cfg2")))
    wl["ell_idx"] = np.ascontiguousarray(wl["ell_idx"][:, ::9])
    wl["n_ell"] = np.array([wl["ell_idx"].shape[1]], np.int32)
    _say(f"limber backward {precision}: 16 tracers (CMB, IA), {wl['ell_idx'].shape[1]} multipoles")
    p = Plan.for_workload(wl, precision=precision)
    T = int(wl["n_tracers"][0])
    Gp = np.random.default_rng(41).standard_normal((1, wl["ell_idx"].shape[1], p.n_pairs))
    out = p.limber_backward(device_inputs(wl, dev), torch.as_tensor(Gp, dtype=p.out_dtype, device=dev))
    assert p.device_flags() == 0
    out = {k: v.cpu().numpy()[0] for k, v in out.items()}
    ref = _limber_grads_oracle(wl, 0, Gp[0])
    e = {k: _rel(out[k][:T] if k in ("bias", "nz") else out[k], ref[k]) for k in ("pk", "bias", "D")}
    e["nz"] = max(_rel(out["nz"][t], ref["nz"][t]) for t in range(T - 1))  # the CMB tracer's row is 0
    _say("  " + ", ".join(f"d{k} {v:.2e}" for k, v in e.items()))
    assert max(e.values()) < tol
    assert np.all(out["nz"][T - 1] == 0)


def test_limber_backward_ragged(dev):
    """Six points of the ragged batch (6, 10 or 15 tracers, uneven multipole counts), FP32: dP and db
    of every point against the oracle, empty tracer slots 0."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg3", batch=6)
    _say(f"limber backward cfg3 ragged T={wl['n_tracers'].tolist()} L={wl['n_ell'].tolist()}")
    p = Plan.for_workload(wl)
    Gp = np.random.default_rng(42).standard_normal((6, wl["ell_idx"].shape[1], p.n_pairs))
    out = p.limber_backward(device_inputs(wl, dev), torch.as_tensor(Gp, dtype=torch.float32, device=dev),
                            want=("pk", "bias"))
    assert p.device_flags() == 0
    out = {k: v.cpu().numpy() for k, v in out.items()}
    from oracle import gradients
    m = fftlog.method_for(wl)
    full_T = wl["nz"].shape[1]
    iu_full = {(i, j): q for q, (i, j) in enumerate(zip(*np.triu_indices(full_T)))}
    for b in range(6):
        T, L = int(wl["n_tracers"][b]), int(wl["n_ell"][b])
        # the GPU packs the pairs of max_tracers: this point's pairs, in its own packed order
        Gb = Gp[b, :L][:, [iu_full[(i, j)] for (i, j) in zip(*np.triu_indices(T))]]
        Gf = gradients.symmetric_cotangent(Gb, T)
        geo = geometry.point_geometry(wl, b)
        ells = fftlog.point_ells(wl, b)
        gp = limber.grad_pk_grid(Gf, geo, ells, m, wl["pk"][b])
        C = limber.cl_limber_grid(geo, ells, m, wl["pk"][b])
        iu = np.triu_indices(T)
        gb = gradients.grad_bias(Gb, C[:, iu[0], iu[1]], wl["kind"][b, :T], wl["bias"][b, :T])
        ep, eb = _rel(out["pk"][b], gp), _rel(out["bias"][b, :T], gb)
        _say(f"  point {b} (T={T}, L={L}): dP {ep:.2e}, db {eb:.2e}")
        assert ep < 1e-4 and eb < 1e-4
        assert np.all(out["bias"][b, T:] == 0)
