"""The adjoint behind torch.autograd against central finite differences of the HIP forward.

FP64: torch.autograd.gradcheck with the full Jacobian (fast_mode=False: every input entry by
central differences, eps 1e-6 relative to the input scale) over P(k), biases, n(z) samples and
D(z) samples, on the 2-bin workload and on one clustering plus one lensing bin of the 15-tracer
set (N_chi = N_k = 1024, five multipoles), for the FFTLog C_l and for the Limber limit.
FP32 (15 tracers, biases scaled by U(0.9, 1.1)): central differences with a 1e-4 relative step
along seeded directions that move every entry of P(k) (random signs), of one tracer's n(z) or
of D(z) (by (0.5 + U(0, 1)) times the entry, so C moves by ~1e-4 relative; a single k node or
a random-sign n(z) direction moves C by 1e-7..1e-5, too close to FP32 resolution), and on single
biases.  The
FP32 forward's roundoff (~6e-8 of C) over a 1e-4 relative change gives the difference quotient
~1e-3 accuracy, so the tolerance is 1e-2.
The geometry adjoint sums with FP64 LDS atomics, so repeated backward calls agree to roundoff,
not bit for bit (gradcheck's reentrancy tolerance is set accordingly).
"""
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


def _one_clustering_one_lensing():
    wl = synth.make_workload("cfg1")
    for key in ("nz", "kind", "bias"):
        wl[key] = np.ascontiguousarray(wl[key][:, [4, 12]])
    wl["n_tracers"] = np.array([2], np.int32)
    wl["ell_idx"] = np.ascontiguousarray(wl["ell_idx"][:, [0, 10, 40, 70, 100]])
    wl["n_ell"] = np.array([5], np.int32)
    return wl


@pytest.mark.parametrize("path", ["fftlog", "limber"])
@pytest.mark.parametrize("name", ["cfg0", "clustering+lensing"])
def test_gradcheck_fp64(dev, name, path):
    from paper_2505_22718_amd import autograd
    from paper_2505_22718_amd.plan import Plan, device_inputs
    cl = autograd.cl if path == "fftlog" else autograd.cl_limber
    wl = synth.make_workload("cfg0") if name == "cfg0" else _one_clustering_one_lensing()
    plan = Plan.for_workload(wl, precision="fp64")
    t = device_inputs(wl, dev)
    rng = np.random.default_rng(3)
    G = torch.as_tensor(rng.standard_normal((1, plan.max_ell, plan.n_pairs)), dtype=torch.float64, device=dev)
    scale = {"pk": t["pk"].abs().max(), "bias": 1.0, "nz": t["nz"].abs().max(), "D": 1.0}

    def make(name):
        base = {"pk": t["pk"], "bias": t["bias"], "nz": t["nz"], "D": t["D_z"]}

        def f(x):
            args = dict(base)
            args[name] = x * scale[name]
            return (cl(plan, t, args["pk"], args["bias"], args["nz"], args["D"]) * G).sum()
        return f, (base[name] / scale[name]).clone().requires_grad_(True)

    for arg in ("pk", "bias", "nz", "D"):
        _say(f"gradcheck {path} {name} {arg}")
        f, x = make(arg)
        # the tolerance follows the gradient's own scale: a central difference of step eps carries
        # ~1e-16 sum|G C| / eps of rounding, ~1e-7 of the largest entry here, while L itself may be
        # small by cancellation between the random cotangent's terms
        xg = x.detach().clone().requires_grad_(True)
        f(xg).backward()
        gmax = float(xg.grad.abs().max()) + 1e-300
        assert torch.autograd.gradcheck(f, (x,), eps=1e-6, atol=1e-6 * gmax, rtol=1e-6, fast_mode=False,
                                        nondet_tol=1e-10 * gmax)


def test_central_differences_fp32(dev):
    from paper_2505_22718_amd.autograd import cl
    from paper_2505_22718_amd.plan import Plan, device_inputs
    wl = synth.make_workload("cfg2")
    plan = Plan.for_workload(wl)
    t = device_inputs(wl, dev)
    rng = np.random.default_rng(4)
    G = torch.as_tensor(rng.standard_normal((1, plan.max_ell, plan.n_pairs)), dtype=torch.float32, device=dev)
    x = {k: t[k].clone().requires_grad_(True) for k in ("pk", "bias", "nz", "D_z")}
    L = (cl(plan, t, x["pk"], x["bias"], x["nz"], x["D_z"]) * G).sum()
    L.backward()

    def loss(over):
        args = {k: v.detach() for k, v in x.items()}
        args.update(over)
        with torch.no_grad():
            return float((cl(plan, t, args["pk"], args["bias"], args["nz"], args["D_z"]).double() * G.double()).sum())

    dirs = rng.standard_normal
    cases = []
    vp = torch.as_tensor(dirs(x["pk"].shape), device=dev) * x["pk"].detach()
    cases.append(("pk", vp))
    for tr in (2, 12):
        vn = torch.zeros_like(x["nz"])
        vn[0, tr] = torch.as_tensor(0.5 + rng.uniform(size=x["nz"].shape[-1]), device=dev) * x["nz"].detach()[0, tr]
        cases.append(("nz", vn))
    cases.append(("D_z", torch.as_tensor(0.5 + rng.uniform(size=x["D_z"].shape), device=dev) * x["D_z"].detach()))
    for tr in (3, 8):
        vb = torch.zeros_like(x["bias"])
        vb[0, tr] = x["bias"].detach()[0, tr]
        cases.append(("bias", vb))
    for name, v in cases:
        h = 1e-4
        base = x[name].detach()
        fd = (loss({name: base + h * v}) - loss({name: base - h * v})) / (2 * h)
        ad = float((x[name].grad * v).sum())
        _say(f"  {name}: adjoint {ad:.6e} central difference {fd:.6e}")
        assert abs(ad - fd) <= 1e-2 * abs(fd)
