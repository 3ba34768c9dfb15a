"""Pins of the gradients the scale-dependent growth adjoint is compared with (CPU only, oracle of
Sec. 3.2): with D(k, z) every k node's kernel is still linear in the bias, so dL/db has the closed
form C/b of gradients.grad_bias, and dL/dP is gradients.grad_pk on the oracle's k-dependent
windows.  Both against central differences of L = sum G C of the kgrowth oracle, exact up to
rounding (C is quadratic in each bias and linear in P)."""
import numpy as np

import synth
from oracle import fftlog, gradients, kgrowth


def _wl():
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 16, f_nu=0.3)
    wl["ell_idx"] = wl["ell_idx"][:, ::3].copy()
    wl["n_ell"] = np.array([wl["ell_idx"].shape[1]], np.int32)
    return wl


def _loss(wl, G, m):
    return float(np.sum(G * kgrowth.cl(wl, 0, m)))


def test_kgrowth_bias_gradient_is_the_closed_form():
    wl = _wl()
    m = fftlog.method_for(wl)
    T = int(wl["n_tracers"][0])
    G = np.random.default_rng(5).standard_normal((int(wl["n_ell"][0]), T * (T + 1) // 2))
    C = kgrowth.cl(wl, 0, m)
    got = gradients.grad_bias(G, C, np.asarray(wl["kind"])[0, :T], np.asarray(wl["bias"])[0, :T])
    for t in range(T):
        h = 1e-2 * float(wl["bias"][0, t])
        up, dn = dict(wl), dict(wl)
        up["bias"] = np.array(wl["bias"], float)
        dn["bias"] = np.array(wl["bias"], float)
        up["bias"][0, t] += h
        dn["bias"][0, t] -= h
        fd = (_loss(up, G, m) - _loss(dn, G, m)) / (2 * h)
        assert abs(got[t] - fd) <= 1e-8 * np.max(np.abs(got))


def test_kgrowth_pk_gradient_matches_central_differences():
    wl = _wl()
    m = fftlog.method_for(wl)
    T = int(wl["n_tracers"][0])
    G = np.random.default_rng(6).standard_normal((int(wl["n_ell"][0]), T * (T + 1) // 2))
    _, W = kgrowth.cl(wl, 0, m, return_windows=True)
    got = gradients.grad_pk(G, W, m)
    for j in (5, 100, 230):
        h = 1e-3 * float(wl["pk"][0, j])
        up, dn = dict(wl), dict(wl)
        up["pk"] = np.array(wl["pk"], float)
        dn["pk"] = np.array(wl["pk"], float)
        up["pk"][0, j] += h
        dn["pk"][0, j] -= h
        fd = (_loss(up, G, m) - _loss(dn, G, m)) / (2 * h)
        assert abs(got[j] - fd) <= 1e-8 * np.max(np.abs(got))
