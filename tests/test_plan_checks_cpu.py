"""Host-side checks of the torch binding (no GPU): every tensor handed to the library must have the
layout of include/swiftcl.h (shape in the plan's sizes, type, contiguity, the plan's device), since
the kernels index it with those sizes.  The inputs of every workload the GPU tests use pass; each
kind of mismatch is refused before any pointer is handed over."""
import numpy as np
import pytest
import torch

import synth
from paper_2505_22718_amd import plan as pl

CPU = torch.device("cpu")


def _dims(wl):
    """The sizes Plan.for_workload gives a plan of this workload."""
    return dict(max_tracers=wl["nz"].shape[1], max_ell=wl["ell_idx"].shape[1], n_zg=len(wl["z_geom"]),
                n_zs=len(wl["z_nz"]), n_k=len(wl["k"]), n_chi=int(wl["n_chi"]))


def _workloads():
    yield "cfg0", synth.make_workload("cfg0")
    yield "cfg1", synth.make_workload("cfg1")
    yield "cfg3 ragged", synth.make_workload("cfg3", batch=12)
    yield "cfg1_batch", synth.make_workload("cfg1_batch", batch=4)
    yield "cfg4", synth.make_workload("cfg4", batch=2)
    yield "cfg1 + IA", synth.intrinsic_alignment(synth.make_workload("cfg1"))
    yield "cfg1 + magnification", synth.magnification_bias(synth.make_workload("cfg1"))


@pytest.fixture(scope="module")
def cfg1():
    wl = synth.intrinsic_alignment(synth.make_workload("cfg1_batch", batch=3))
    return wl, pl.device_inputs(wl, CPU)


def _plan_without_device(wl, precision="fp32", n_interp=0):
    """A Plan object with the sizes of this workload and no library handle, on the CPU device."""
    p = pl.Plan.__new__(pl.Plan)
    p.handle = None
    p.k, p.ell, p.z_geom, p.z_nz = wl["k"], wl["ell"], wl["z_geom"], wl["z_nz"]
    p.max_batch, p.max_tracers, p.max_ell = int(wl["batch"]), wl["nz"].shape[1], wl["ell_idx"].shape[1]
    p.n_chi = int(wl["n_chi"])
    p.n_interp = n_interp
    p.device = CPU
    p.out_dtype = torch.float64 if precision == "fp64" else torch.float32
    return p


def test_every_workload_passes():
    for label, wl in _workloads():
        t = pl.device_inputs(wl, CPU)
        assert pl.check_inputs(t, _dims(wl), CPU) == int(wl["batch"]), label
        # a subset of the points
        if int(wl["batch"]) > 2:
            t2 = pl.device_inputs(wl, CPU, points=[0, 2])
            assert pl.check_inputs(t2, _dims(wl), CPU) == 2, label


@pytest.mark.parametrize("name", [n for n, _, _ in pl.INPUT_LAYOUT] + ["ia"])
def test_each_input_mismatch_is_refused(cfg1, name):
    wl, t = cfg1
    dims = _dims(wl)
    x = t[name]
    other = torch.float32 if x.dtype == torch.float64 else torch.int64
    bad = [x.to(other)]                                             # type
    bad.append(torch.cat([x, x[:1]]))                               # batch size
    if x.dim() > 1:
        bad.append(x[..., :-1].contiguous())                        # inner size
        bad.append(x.transpose(0, 1).contiguous().transpose(0, 1))  # same shape, not contiguous
    for i, b in enumerate(bad):
        # n_tracers defines the batch: another length is refused at the next tensor
        with pytest.raises(ValueError, match=None if (name, i) == ("n_tracers", 1) else name):
            pl.check_inputs(dict(t, **{name: b}), dims, CPU)
    # a missing required tensor
    if name != "ia":
        with pytest.raises(ValueError):
            pl.check_inputs({k: v for k, v in t.items() if k != name}, dims, CPU)


def test_tensors_off_the_plans_device_are_refused(cfg1):
    wl, t = cfg1
    with pytest.raises(ValueError, match="on cuda:0; got .* on cpu"):
        pl.check_inputs(t, _dims(wl), torch.device("cuda", 0))
    with pytest.raises(ValueError, match="gradient pk .* on cuda:0"):
        pl.check_grads({"pk": torch.zeros((3, len(wl["k"])), dtype=torch.float64)}, 3, _dims(wl),
                       torch.device("cuda", 0))


def test_non_tensor_and_optional_inputs(cfg1):
    wl, t = cfg1
    dims = _dims(wl)
    with pytest.raises(ValueError, match="pk.*ndarray"):
        pl.check_inputs(dict(t, pk=wl["pk"]), dims, CPU)
    # optional inputs may be absent or None
    pl.check_inputs({k: v for k, v in t.items() if k != "ia"}, dims, CPU)
    pl.check_inputs(dict(t, ia=None, mag=None), dims, CPU)
    mag = torch.zeros((3, dims["max_tracers"]), dtype=torch.float64)
    pl.check_inputs(dict(t, mag=mag), dims, CPU)
    with pytest.raises(ValueError, match="mag"):
        pl.check_inputs(dict(t, mag=mag[:, :-1].contiguous()), dims, CPU)


def test_plan_methods_check_before_handing_over(cfg1):
    """inputs_struct, the C-shaped buffers and the gradient buffers of a Plan (without a library
    handle: every refusal comes before the first library call)."""
    wl, t = cfg1
    p = _plan_without_device(wl)
    s = p.inputs_struct(t)
    assert s.batch == 3 and s.pk == t["pk"].data_ptr() and s.ia == t["ia"].data_ptr() and not s.mag
    shape = (3, p.max_ell, p.n_pairs)
    good = torch.zeros(shape, dtype=torch.float32)
    assert p._cl_buffer("out", good, 3) is good
    assert p._cl_buffer("out", None, 3).shape == shape
    for bad in (torch.zeros(shape, dtype=torch.float64), torch.zeros((3, p.max_ell, p.n_pairs - 1))):
        with pytest.raises(ValueError, match="out"):
            p.cl(t, out=bad)
        with pytest.raises(ValueError, match="dC"):
            p.backward_into(t, bad, {})
    f64 = dict(dtype=torch.float64)
    grads = {"pk": torch.zeros((3, len(wl["k"])), **f64), "bias": torch.zeros((3, p.max_tracers), **f64),
             "nz": torch.zeros((3, p.max_tracers, len(wl["z_nz"])), **f64), "D": torch.zeros((3, len(wl["z_geom"])), **f64)}
    s2, ptr = p._backward_args(t, good, grads)
    assert ptr["nz"] == grads["nz"].data_ptr() and s2.batch == 3
    _, ptr = p._backward_args(t, good, {"pk": grads["pk"]})
    assert ptr["bias"] == 0 and ptr["D"] == 0
    with pytest.raises(ValueError, match="gradient D"):
        p._backward_args(t, good, dict(grads, D=grads["D"].float()))
    with pytest.raises(ValueError, match="gradient nz"):
        p._backward_args(t, good, dict(grads, nz=grads["nz"][:, :-1].contiguous()))
    # windows output: [B][max_ell][max_tracers][n_k]
    with pytest.raises(ValueError, match="out"):
        p.windows(t, out=torch.zeros((3, p.max_ell, p.max_tracers, len(wl["k"]) - 1), dtype=torch.float32))


def test_kgrowth_samples_are_checked():
    wl = synth.scale_dependent_growth(synth.make_workload("cfg0"), 8)
    t = pl.device_inputs(wl, CPU)
    p = _plan_without_device(wl, precision="fp64", n_interp=8)
    D = torch.as_tensor(wl["D_kz"], dtype=torch.float64)
    for bad in (D.float(), D[:, :-1].contiguous(), torch.cat([D, D])):
        with pytest.raises(ValueError, match="D_kz"):
            p.cl_kgrowth(t, bad)
    assert np.asarray(wl["D_kz"]).shape == tuple(D.shape)


def test_every_plan_method_reaches_the_library_with_checked_buffers(cfg1, monkeypatch):
    """Each Plan method runs to its library call (entry points stubbed: no device work) with the
    pointers of conforming tensors, as the GPU tests and the benchmark call them."""
    from paper_2505_22718_amd import binding as bd
    calls = {}

    def stub(name, ret=None):
        def f(*args):
            calls[name] = args
            return ret
        return f

    for name in ("swiftcl_cl", "swiftcl_cl_kgrowth", "swiftcl_cl_limber", "swiftcl_windows", "swiftcl_cl_backward"):
        monkeypatch.setattr(bd, name, stub(name))
    monkeypatch.setattr(bd, "swiftcl_cl_timed", stub("swiftcl_cl_timed", [0.0, 0.0, 0.0]))
    monkeypatch.setattr(bd, "swiftcl_cl_backward_timed", stub("swiftcl_cl_backward_timed", [0.0] * 4))
    monkeypatch.setattr(bd, "swiftcl_autotune", stub("swiftcl_autotune", "report"))
    wl, t = cfg1
    p = _plan_without_device(wl)
    p._stream = lambda: 0
    B = 3
    C = p.cl(t)
    assert C.shape == (B, p.max_ell, p.n_pairs) and C.dtype == torch.float32
    assert calls["swiftcl_cl"][2] == C.data_ptr()
    assert p.cl(t, C) is C
    assert p.cl_limber(t, C) is C and calls["swiftcl_cl_limber"][2] == C.data_ptr()
    assert p.cl_timed(t, C) == [0.0, 0.0, 0.0]
    W = p.windows(t)
    assert W.shape == (B, p.max_ell, p.max_tracers, len(wl["k"]))
    dC = torch.ones_like(C)
    g = p.backward(t, dC)
    assert set(g) == {"pk", "bias", "nz", "D"} and g["nz"].shape == (B, p.max_tracers, len(wl["z_nz"]))
    args = calls["swiftcl_cl_backward"]
    assert args[2] == dC.data_ptr() and args[3] == g["pk"].data_ptr() and args[7] == 0
    g1 = p.backward(t, dC, want=("pk",), reuse_forward=True)
    assert set(g1) == {"pk"} and calls["swiftcl_cl_backward"][4] == 0
    assert calls["swiftcl_cl_backward"][7] == bd.SWIFTCL_BWD_REUSE_FORWARD
    p.backward_into(t, dC, g)
    assert p.backward_timed(t, dC, g, reuse_forward=True) == [0.0] * 4
    assert p.autotune(t, dC) == "report" and p.autotune(t) == "report"
    # a non-contiguous dC is made contiguous by backward() (the other calls take it as it is)
    g2 = p.backward(t, dC.transpose(1, 2).contiguous().transpose(1, 2))
    assert g2["pk"].shape == (B, len(wl["k"]))
    # the autograd Function (smoke() and the gradient tests go through it)
    from paper_2505_22718_amd.autograd import cl as cl_ad
    leaves = {k: t[k].clone().requires_grad_(True) for k in ("pk", "bias", "nz", "D_z")}
    Ca = cl_ad(p, t, leaves["pk"], leaves["bias"], leaves["nz"], leaves["D_z"])
    (Ca * 1.0).sum().backward()
    assert calls["swiftcl_cl_backward"][7] == bd.SWIFTCL_BWD_REUSE_FORWARD
    assert leaves["nz"].grad.shape == leaves["nz"].shape and leaves["D_z"].grad.shape == leaves["D_z"].shape
    wk = synth.scale_dependent_growth(synth.make_workload("cfg0"), 8)
    pk = _plan_without_device(wk, precision="fp64", n_interp=8)
    pk._stream = lambda: 0
    Ck = pk.cl_kgrowth(pl.device_inputs(wk, CPU), torch.as_tensor(wk["D_kz"], dtype=torch.float64))
    assert Ck.dtype == torch.float64 and calls["swiftcl_cl_kgrowth"][3] == Ck.data_ptr()


def test_unknown_precision_is_refused_before_the_library():
    wl = synth.make_workload("cfg0")
    with pytest.raises(ValueError, match="precision"):
        pl.Plan.for_workload(wl, precision="fp16")


def test_band_table_shapes_are_refused_before_the_library():
    """Every band needs a bias for each of the three kinds (an unset entry would reach the library as
    b = 0)."""
    wl = synth.make_workload("cfg0")
    with pytest.raises(ValueError, match="fftlog_b"):
        pl.Plan.for_workload(wl, band_ell_lo=(0.0, 3.0, 6.0, 50.0))
    with pytest.raises(ValueError, match="fftlog_b"):
        pl.Plan.for_workload(wl, fftlog_b=((0.1, -0.2, -0.5),))
    with pytest.raises(ValueError, match="fftlog_b"):  # no CMB-lensing row
        pl.Plan.for_workload(wl, fftlog_b=((0.1, -0.2, -0.5), (-1.5, -2.0, -2.5)))
    with pytest.raises(ValueError, match="band_ell_lo"):
        pl.Plan.for_workload(wl, band_ell_lo=(0.0, 3.0, 6.0, 9.0, 12.0), fftlog_b=((0.1,) * 5, (-1.5,) * 5))
