"""Pins of the oracle's full gradient vectors dL/dn(z) and dL/dD(z) (oracle/gradients.py), CPU only.

They are the chain rule through the oracle's linear steps (window matrices of unit kernel samples,
kernels of unit n(z) samples, the natural spline of D).  Pinned against code that shares none of
that chain:
  * window_matrix reproduces the oracle's windows (A @ F = W) for every tracer kind;
  * the gradient dotted with a seeded direction v equals the directional derivative, one more
    window pass with n_t (or D) replaced by v (itself pinned to central differences);
  * L is quadratic in each n_t and in D, so the central difference of one sample is exact: single
    entries are checked that way (brute force);
  * Euler identities: sum_s D_s dL/dD_s = 2 L, and sum_s n_ts dL/dn_ts = sum over pairs holding t of
    G^{ij} C^{ij} (t counted twice in its auto pair).
The workload is the 15-tracer set restricted to two clustering bins, two lensing bins and a
CMB-lensing tracer, with intrinsic alignment on and five multipoles.
"""
import numpy as np
import pytest

import synth
from oracle import fftlog, gradients
from oracle.geometry import point_geometry

TRACERS = [0, 9, 12, 14, 15]  # clustering 0 and 9, lensing 12 and 14, the CMB-lensing tracer


@pytest.fixture(scope="module")
def case():
    wl = synth.intrinsic_alignment(synth.cmb_lensing(synth.make_workload("cfg1")))
    T = len(TRACERS)
    for key in ("nz", "kind", "bias"):
        wl[key] = np.ascontiguousarray(wl[key][:, TRACERS])
    wl["n_tracers"] = np.array([T], np.int32)
    wl["ell_idx"] = np.ascontiguousarray(wl["ell_idx"][:, [0, 20, 50, 80, 102]])
    wl["n_ell"] = np.array([5], np.int32)
    m = fftlog.method_for(wl)
    G = np.random.default_rng(3).standard_normal((5, T * (T + 1) // 2))
    C = fftlog.cl(wl, 0, m)
    return wl, m, G, C


@pytest.fixture(scope="module")
def grads(case):
    wl, m, G, C = case
    return gradients.grad_nz_full(wl, 0, G, m), gradients.grad_D_full(wl, 0, G, m)


def _loss(wl, m, G, **repl):
    w = dict(wl)
    w.update({k: v for k, v in repl.items()})
    return float(np.sum(G * fftlog.cl(w, 0, m)))


def test_window_matrix_reproduces_the_windows(case):
    wl, m, G, C = case
    geo = point_geometry(wl, 0)
    chi0, chi, F = fftlog.sampled_kernels(geo, m)
    W = fftlog.windows(wl, 0, m)
    ells = fftlog.point_ells(wl, 0)
    for li in (0, 4):
        ell = ells[li]
        for t, kind in enumerate(geo.kinds):
            A = gradients.window_matrix(ell, int(kind), chi, chi0, m)
            ref = W[li, t]
            assert np.max(np.abs(A @ F[t] - ref)) < 1e-11 * np.max(np.abs(ref)), (ell, t)


def test_full_gradients_match_directional_derivatives(case, grads):
    wl, m, G, C = case
    gn, gD = grads
    rng = np.random.default_rng(7)
    for t in range(4):  # the CMB-lensing tracer reads no n(z): its row is zero
        v = rng.standard_normal(gn.shape[1]) * wl["nz"][0, t].max()
        ref = gradients.directional_nz(wl, 0, G, t, v, m)
        assert abs(gn[t] @ v - ref) <= 1e-9 * abs(ref), t
    assert np.all(gn[4] == 0.0)
    for _ in range(2):
        v = rng.standard_normal(len(gD))
        ref = gradients.directional_D(wl, 0, G, v, m)
        assert abs(gD @ v - ref) <= 1e-9 * abs(ref)


def test_full_gradients_euler_identities(case, grads):
    wl, m, G, C = case
    gn, gD = grads
    T = len(TRACERS)
    L = float(np.sum(G * C))
    assert abs(gD @ wl["D_z"][0] - 2.0 * L) <= 1e-9 * abs(L)
    iu = np.triu_indices(T)
    for t in range(4):
        want = sum(float(np.sum(G[:, p] * C[:, p])) * (int(i == t) + int(j == t)) for p, (i, j) in enumerate(zip(*iu)))
        assert abs(gn[t] @ wl["nz"][0, t] - want) <= 1e-9 * abs(want), t


def test_full_gradients_single_entries_by_central_differences(case, grads):
    """L is quadratic in n_t(z_s) and in D(z_s): the central difference is exact up to rounding."""
    wl, m, G, C = case
    gn, gD = grads
    for t in (0, 2):
        s = int(np.argmax(np.abs(gn[t])))
        h = 1e-3 * wl["nz"][0, t].max()
        up, dn = wl["nz"].copy(), wl["nz"].copy()
        up[0, t, s] += h
        dn[0, t, s] -= h
        fd = (_loss(wl, m, G, nz=up) - _loss(wl, m, G, nz=dn)) / (2 * h)
        assert abs(fd - gn[t, s]) <= 1e-6 * np.max(np.abs(gn[t])), (t, s)
    for s in (int(np.argmax(np.abs(gD))), 300):
        h = 1e-3
        up, dn = wl["D_z"].copy(), wl["D_z"].copy()
        up[0, s] += h
        dn[0, s] -= h
        fd = (_loss(wl, m, G, D_z=up) - _loss(wl, m, G, D_z=dn)) / (2 * h)
        assert abs(fd - gD[s]) <= 1e-6 * np.max(np.abs(gD)), s
