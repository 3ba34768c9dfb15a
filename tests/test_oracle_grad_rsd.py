"""Pins of the oracle's gradients for windows with terms the bias does not scale (CPU only):
the redshift-space-distortion term (eq. RSD) and the magnification term (eq. magnification bias).

* dL/db through the density window at unit bias (gradients.grad_bias_windows) equals the closed
  form C/b of gradients.grad_bias when neither term is on.
* With RSD, and with RSD plus magnification, it equals the central difference of
  L(b) = sum G C(b), which is exact up to rounding because C is quadratic in each bias.
* dL/dP from the windows (gradients.grad_pk) equals the central difference of L in P_j, exact for
  the linear dependence, with the RSD and magnification terms in the windows.
A gradient that dropped the transpose term, or took the whole window for the density window,
fails the second check.
"""
import numpy as np
import pytest

import synth
from oracle import fftlog, gradients


def _wl(rsd, mag):
    wl = synth.make_workload("cfg0")
    wl["ell_idx"] = wl["ell_idx"][:, ::4].copy()
    wl["n_ell"] = np.array([wl["ell_idx"].shape[1]], np.int32)
    wl["rsd"] = rsd
    if mag:
        synth.magnification_bias(wl)
    return wl


def _loss(wl, G, m):
    return float(np.sum(G * fftlog.cl(wl, 0, m)))


def _G(wl, seed):
    T = int(wl["n_tracers"][0])
    return np.random.default_rng(seed).standard_normal((int(wl["n_ell"][0]), T * (T + 1) // 2))


def test_bias_gradient_reduces_to_the_closed_form():
    wl = _wl(False, False)
    m = fftlog.method_for(wl)
    G = _G(wl, 1)
    C = fftlog.cl(wl, 0, m)
    T = int(wl["n_tracers"][0])
    ref = gradients.grad_bias(G, C, np.asarray(wl["kind"])[0, :T], np.asarray(wl["bias"])[0, :T])
    got = gradients.grad_bias_windows(wl, 0, G, m)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("mag", [False, True])
def test_bias_gradient_with_rsd_matches_central_differences(mag):
    wl = _wl(True, mag)
    m = fftlog.method_for(wl)
    G = _G(wl, 2)
    got = gradients.grad_bias_windows(wl, 0, G, m)
    T = int(wl["n_tracers"][0])
    fd = np.zeros(T)
    for t in range(T):
        h = 1e-2 * float(wl["bias"][0, t])
        up, dn = dict(wl), dict(wl)
        up["bias"] = np.array(wl["bias"], float)
        dn["bias"] = np.array(wl["bias"], float)
        up["bias"][0, t] += h
        dn["bias"][0, t] -= h
        fd[t] = (_loss(up, G, m) - _loss(dn, G, m)) / (2 * h)
    assert np.max(np.abs(got - fd)) <= 1e-8 * np.max(np.abs(fd))
    # the RSD term changes the gradient: the closed form C/b no longer holds
    C = fftlog.cl(wl, 0, m)
    cf = gradients.grad_bias(G, C, np.asarray(wl["kind"])[0, :T], np.asarray(wl["bias"])[0, :T])
    assert np.max(np.abs(cf - fd)) > 1e-3 * np.max(np.abs(fd))


def test_pk_gradient_with_rsd_and_magnification_matches_central_differences():
    wl = _wl(True, True)
    m = fftlog.method_for(wl)
    G = _G(wl, 3)
    C, W = fftlog.cl(wl, 0, m, return_windows=True)
    got = gradients.grad_pk(G, W, m)
    for j in (10, 128, 200):
        h = 1e-3 * float(wl["pk"][0, j])
        up, dn = dict(wl), dict(wl)
        up["pk"] = np.array(wl["pk"], float)
        dn["pk"] = np.array(wl["pk"], float)
        up["pk"][0, j] += h
        dn["pk"][0, j] -= h
        fd = (_loss(up, G, m) - _loss(dn, G, m)) / (2 * h)
        assert abs(got[j] - fd) <= 1e-8 * np.max(np.abs(got))
