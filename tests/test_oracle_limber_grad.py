"""Pins of the oracle's kernel gradient of the chi-node Limber rule (limber.grad_kernels_grid),
which with gradients.grad_nz_full / grad_D_full gives dL/dn(z) and dL/dD of the Limber path (CPU).

The rule is a quadratic form in the kernel samples F (g = c F / W), so
* sum_{t,m} F_t(m) dL/dF_t(m) = 2 L (Euler's identity for a homogeneous quadratic), and
* C_l is quadratic in every tracer's n(z) samples and in the D(z) samples (each kernel is linear in
  them), so a central difference of L along any direction is exact up to rounding: the n(z) and
  D(z) gradients must match it for every kind (clustering, lensing with intrinsic alignment, CMB
  lensing, whose n(z) gradient is zero).
"""
import numpy as np
import pytest

import synth
from oracle import fftlog, geometry, gradients, limber


@pytest.fixture(scope="module")
def case():
    wl = synth.intrinsic_alignment(synth.cmb_lensing(synth.make_workload("cfg2")))
    m = fftlog.method_for(wl)
    ells = fftlog.point_ells(wl, 0)[::15]
    T = int(wl["n_tracers"][0])
    G = np.random.default_rng(3).standard_normal((len(ells), T * (T + 1) // 2))
    Gf = gradients.symmetric_cotangent(G, T)
    return wl, m, ells, T, G, Gf


def _L(wl, m, ells, Gf):
    geo = geometry.point_geometry(wl, 0)
    return float(np.sum(Gf * limber.cl_limber_grid(geo, ells, m, wl["pk"][0])))


def _kern(wl, m, ells, Gf):
    return limber.grad_kernels_grid(Gf, geometry.point_geometry(wl, 0), ells, m, wl["pk"][0])


def test_limber_kernel_gradient_euler(case):
    wl, m, ells, T, G, Gf = case
    dF, F, nodes, z = _kern(wl, m, ells, Gf)
    L = _L(wl, m, ells, Gf)
    assert abs(np.sum(dF * F) - 2.0 * L) <= 1e-12 * abs(L)


def test_limber_nz_gradient_central_differences(case):
    wl, m, ells, T, G, Gf = case
    kern = _kern(wl, m, ells, Gf)
    gn = gradients.grad_nz_full(wl, 0, G, m, kern=kern)
    rng = np.random.default_rng(4)
    kinds = wl["kind"][0, :T]
    for t in (0, 9, 10, 14, T - 1):
        v = rng.standard_normal(wl["nz"].shape[-1]) * wl["nz"][0, t].max()
        eps = 1e-3
        wp, wm = dict(wl, nz=wl["nz"].copy()), dict(wl, nz=wl["nz"].copy())
        wp["nz"][0, t] += eps * v
        wm["nz"][0, t] -= eps * v
        fd = (_L(wp, m, ells, Gf) - _L(wm, m, ells, Gf)) / (2 * eps)
        if kinds[t] == geometry.KIND_CMB_LENSING:
            assert fd == 0.0 and np.all(gn[t] == 0.0)
        else:
            assert abs(gn[t] @ v - fd) <= 1e-8 * abs(fd), t


def test_limber_D_gradient_central_differences(case):
    wl, m, ells, T, G, Gf = case
    kern = _kern(wl, m, ells, Gf)
    gD = gradients.grad_D_full(wl, 0, G, m, kern=kern)
    v = np.random.default_rng(5).standard_normal(wl["D_z"].shape[-1]) * 0.01
    eps = 1e-2
    wp, wm = dict(wl, D_z=wl["D_z"].copy()), dict(wl, D_z=wl["D_z"].copy())
    wp["D_z"][0] += eps * v
    wm["D_z"][0] -= eps * v
    fd = (_L(wp, m, ells, Gf) - _L(wm, m, ells, Gf)) / (2 * eps)
    assert abs(gD @ v - fd) <= 1e-8 * abs(fd)
