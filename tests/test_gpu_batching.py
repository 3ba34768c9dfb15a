"""Batched, ragged launches: the persistent launch, the autotuner and hipGraph capture.

* The persistent projection (per-XCD compact work lists) gives bit-identical C_l to the
  one-workgroup-per-slot launch on a ragged batch, padded slots included; so does the packed
  persistent launch (two items of few tracers per workgroup) in every precision, on counts that
  include points with no multipoles, one tracer, and pairs that fill all 16 rows (a point
  without tracers is an input error, flagged; the host test of the list builder covers it).
* The autotuner picks a configuration, reports it, and reads it back from its cache; the adjoint's
  multipole chunkings agree, and so does the packed adjoint (two half-chunks side by side for
  points of at most 8 tracers).
* forward + backward captured in a hipGraph (torch.cuda.CUDAGraph) and replayed several times,
  with eager work between the replays: every replay reproduces the eager forward bit for bit and
  the eager gradients to roundoff (the geometry adjoint sums with FP64 atomics).
"""
import gc
import os
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _grads(plan, B, wl, dev):
    f64 = dict(dtype=torch.float64, device=dev)
    return {"pk": torch.zeros((B, len(wl["k"])), **f64), "bias": torch.zeros((B, plan.max_tracers), **f64),
            "nz": torch.zeros((B, plan.max_tracers, len(wl["z_nz"])), **f64),
            "D": torch.zeros((B, len(wl["z_geom"])), **f64)}


def test_persistent_matches_per_slot(dev):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg3", batch=40)
    _say(f"persistent vs per-slot, cfg3 B=40, L={wl['n_ell'].tolist()[:8]}...")
    plan = Plan.for_workload(wl)
    t = device_inputs(wl, dev)
    C0 = plan.cl(t).clone()
    plan.set_launch(fwd_mode=1)
    C1 = plan.cl(t)
    torch.cuda.synchronize()
    assert torch.equal(C0, C1)
    assert plan.device_flags() == 0


@pytest.mark.parametrize("precision", ["fp32", "split_bf16", "fp64"])
def test_packed_matches_per_slot(dev, precision):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg3", batch=40)
    plan = Plan.for_workload(wl, precision=precision)
    t = device_inputs(wl, dev)
    nt, nl = t["n_tracers"], t["n_ell"]
    nt[torch.tensor([0, 9])] = 2
    nt[torch.tensor([1, 17])] = 1
    nt[torch.tensor([2, 10, 18, 26])] = 8
    nt[torch.tensor([3, 11])] = 13
    nt[torch.tensor([19, 27])] = 3
    nl[4] = 0
    nl[12] = 1
    _say(f"packed vs per-slot, cfg3 B=40 {precision}: T={nt.tolist()[:20]}..., L={nl.tolist()[:14]}...")
    C0 = plan.cl(t).clone()
    plan.set_launch(fwd_mode=1)
    C1 = plan.cl(t).clone()
    plan.set_launch(fwd_mode=2)
    C2 = plan.cl(t).clone()
    C2b = plan.cl(t)  # a second call over the same lists
    torch.cuda.synchronize()
    assert plan.device_flags() == 0
    assert torch.equal(C0, C1)
    assert torch.equal(C0, C2)
    assert torch.equal(C0, C2b)
    assert C0.abs().sum().item() > 0


def test_adjoint_chunkings_agree(dev):
    """The adjoint's multipole chunking (bwd_chunk_mul 1, 2, 4, 8) changes only the order of the
    FP32 partial sums: the gradients of a ragged batch agree to the FP32 bar; other values are
    refused."""
    from paper_2505_22718_amd.binding import SwiftclError, SWIFTCL_E_INVALID
    from paper_2505_22718_amd.plan import Plan, device_inputs
    B = 24
    wl = synth.make_workload("cfg3", batch=B)
    plan = Plan.for_workload(wl)
    t = device_inputs(wl, dev)
    dC = torch.as_tensor(np.random.default_rng(17).standard_normal((B, plan.max_ell, plan.n_pairs)),
                         dtype=torch.float32, device=dev)
    ref = None
    for m in (1, 2, 4, 8):
        plan.set_launch(bwd_chunk_mul=m)
        g = {k: v.cpu().numpy() for k, v in plan.backward(t, dC).items()}
        assert plan.device_flags() == 0
        if ref is None:
            ref = g
            continue
        for k in g:
            e = float(np.max(np.abs(g[k] - ref[k])) / np.max(np.abs(ref[k])))
            _say(f"  bwd_chunk_mul {m}: {k} differs from 1 by {e:.2e}")
            assert e < 1e-4
    with pytest.raises(SwiftclError) as ei:
        plan.set_launch(bwd_chunk_mul=3)
    assert ei.value.status == SWIFTCL_E_INVALID


def test_packed_adjoint_agrees(dev):
    """The packed adjoint (each multipole chunk split into two halves with partial rows of their
    own, run side by side by the two halves of the workgroup for points of at most 8 tracers, one
    after the other otherwise) changes only the order of the FP32 partial sums: on a ragged batch
    with points of 1, 2, 7, 8 and 9 tracers and of 0, 1 and 2 multipoles, its gradients agree with
    the unpacked adjoint's to the FP32 bar at chunk multipliers 1, 2 and 4.  Packing with chunk
    multiplier 8 is refused."""
    from paper_2505_22718_amd.binding import SwiftclError, SWIFTCL_E_INVALID
    from paper_2505_22718_amd.plan import Plan, device_inputs
    B = 24
    wl = synth.make_workload("cfg3", batch=B)
    plan = Plan.for_workload(wl)
    t = device_inputs(wl, dev)
    nt, nl = t["n_tracers"], t["n_ell"]
    # lower the tracer count of points that have at least 10 (a slot past a point's own tracers
    # holds no n(z)); the others keep 6, 10 or 15
    big = [i for i in range(B) if int(nt[i]) >= 10]
    for i, want in zip(big, [1, 2, 7, 8, 9, 8, 7, 9]):
        nt[i] = want
    nl[big[0]] = 0
    nl[big[1]] = 1
    nl[big[2]] = 2
    _say(f"packed adjoint, cfg3 B={B}: T={nt.tolist()}, L={nl.tolist()}")
    dC = torch.as_tensor(np.random.default_rng(23).standard_normal((B, plan.max_ell, plan.n_pairs)),
                         dtype=torch.float32, device=dev)
    plan.set_launch(bwd_chunk_mul=1, bwd_pack=0)
    ref = {k: v.cpu().numpy() for k, v in plan.backward(t, dC).items()}
    assert plan.device_flags() == 0
    for m in (1, 2, 4):
        plan.set_launch(bwd_chunk_mul=m, bwd_pack=1)
        assert plan.launch_config()["bwd_pack"] == 1
        g = {k: v.cpu().numpy() for k, v in plan.backward(t, dC).items()}
        assert plan.device_flags() == 0
        for k in g:
            assert np.all(np.isfinite(g[k]))
            e = float(np.max(np.abs(g[k] - ref[k])) / np.max(np.abs(ref[k])))
            _say(f"  packed, bwd_chunk_mul {m}: {k} differs from the unpacked adjoint by {e:.2e}")
            assert e < 1e-4
    with pytest.raises(SwiftclError) as ei:
        plan.set_launch(bwd_chunk_mul=8)
    assert ei.value.status == SWIFTCL_E_INVALID
    assert plan.launch_config()["bwd_chunk_mul"] == 4
    plan.set_launch(bwd_pack=0)
    plan.set_launch(bwd_chunk_mul=8)
    with pytest.raises(SwiftclError) as ei:
        plan.set_launch(bwd_pack=1)
    assert ei.value.status == SWIFTCL_E_INVALID


def test_autotune_and_cache(dev, tmp_path):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg3", batch=32)
    plan = Plan.for_workload(wl)
    t = device_inputs(wl, dev)
    dC = torch.ones((32, plan.max_ell, plan.n_pairs), dtype=torch.float32, device=dev)
    cache = str(tmp_path / "tune.jsonl")
    rep = plan.autotune(t, dC, cache_path=cache)
    _say("  " + rep)
    assert '"fwd_mode"' in rep and os.path.exists(cache)
    cfg = plan.launch_config()
    plan2 = Plan.for_workload(wl)
    rep2 = plan2.autotune(t, dC, cache_path=cache)
    _say("  " + rep2)
    assert rep2.startswith("cached") and plan2.launch_config() == cfg
    # tuned plan still matches the default launch
    C_tuned = plan.cl(t)
    plan3 = Plan.for_workload(wl)
    assert torch.equal(plan3.cl(t), C_tuned)


@pytest.mark.parametrize("fwd_mode,reuse", [(0, False), (1, False), (1, True), (2, True)])
def test_graph_capture_replay(dev, fwd_mode, reuse):
    from paper_2505_22718_amd.plan import Plan, device_inputs
    B = 16
    wl = synth.make_workload("cfg3", batch=B)
    plan = Plan.for_workload(wl)
    plan.set_launch(fwd_mode=fwd_mode)
    t = device_inputs(wl, dev)
    rng = np.random.default_rng(9)
    dC = torch.as_tensor(rng.standard_normal((B, plan.max_ell, plan.n_pairs)), dtype=torch.float32, device=dev)
    C_ref = plan.cl(t).clone()
    g_ref = _grads(plan, B, wl, dev)
    plan.backward_into(t, dC, g_ref)
    torch.cuda.synchronize()

    C = torch.zeros_like(C_ref)
    g = _grads(plan, B, wl, dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            plan.cl(t, C)
            plan.backward_into(t, dC, g, reuse_forward=reuse)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    gc.collect()  # no plan of an earlier test may be released (freed) during the capture
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.cl(t, C)
        plan.backward_into(t, dC, g, reuse_forward=reuse)
    for r in range(3):
        C.zero_()
        for v in g.values():
            v.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, C_ref), f"replay {r}"
        for k in g:
            err = (g[k] - g_ref[k]).abs().max().item() / max(g_ref[k].abs().max().item(), 1e-300)
            assert err < 1e-10, (k, r, err)
        # eager work between replays
        other = plan.cl(t)
        torch.cuda.synchronize()
        assert torch.equal(other, C_ref)
    _say(f"  fwd_mode={fwd_mode} reuse={reuse}: 3 replays match")


def test_graph_capture_kgrowth_and_limber(dev):
    """swiftcl_cl_kgrowth (chunked launches) and swiftcl_cl_limber captured in one hipGraph: every
    replay, with eager work between them, reproduces the eager C_l bit for bit."""
    from paper_2505_22718_amd.plan import Plan, device_inputs
    B = 16
    wl = synth.scale_dependent_growth(synth.make_workload("cfg3", batch=B), 10)
    plan = Plan.for_workload(wl, n_interp=10)
    t = device_inputs(wl, dev)
    D = torch.as_tensor(wl["D_kz"], dtype=torch.float64, device=dev)
    Ck_ref = plan.cl_kgrowth(t, D).clone()
    Cl_ref = plan.cl_limber(t).clone()
    torch.cuda.synchronize()
    Ck, Cl = torch.zeros_like(Ck_ref), torch.zeros_like(Cl_ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            plan.cl_kgrowth(t, D, Ck)
            plan.cl_limber(t, Cl)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    gc.collect()  # no plan of an earlier test may be released (freed) during the capture
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.cl_kgrowth(t, D, Ck)
        plan.cl_limber(t, Cl)
    for r in range(3):
        Ck.zero_()
        Cl.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Ck, Ck_ref), f"kgrowth replay {r}"
        assert torch.equal(Cl, Cl_ref), f"limber replay {r}"
        other = plan.cl_kgrowth(t, D)
        torch.cuda.synchronize()
        assert torch.equal(other, Ck_ref)
    _say("  kgrowth + limber: 3 replays match")
