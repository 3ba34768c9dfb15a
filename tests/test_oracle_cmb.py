"""Pins of the CMB-lensing oracle (Sec. 2.4), CPU only.

A CMB-lensing tracer (kind 2) carries the lensing kernel of one source plane at the last-scattering
surface, 1.5 Om (H0/c)^2 (1+z) (chi_* - chi) / (chi chi_*) D, and the convergence prefactor
l(l+1)/k^2.  Pinned against:
  * the lens efficiency of a narrow n(z) at z_*, an integral over n computed by other code;
  * the Einstein-de Sitter geometry, where chi(z) and D = a are closed forms and the window is a
    plain chi integral of the paper's formula, evaluated here by its own Gauss-Legendre panels;
  * direct quadrature on the 15-tracer workload with the geometry continued to z_* (the
    method-error floor; the kernel's corner at chi_* takes the trapezoid weight of a linear end);
  * the Limber limit, and the chi-node Limber rule against the fine-panel Limber integral.
"""
import numpy as np
import pytest
from scipy.special import jv

import synth
from oracle import fftlog, geometry, limber, quadrature
from tests.helpers import eps_metric

C_OVER_H0 = 2997.92458


@pytest.fixture(scope="module")
def wl_cmb():
    return synth.cmb_lensing(synth.make_workload("cfg1"))


def _subset_geometry(wl, tracers):
    """PointGeometry of point 0 restricted to the given tracers."""
    return geometry.PointGeometry(wl["z_geom"], wl["chi_z"][0], wl["D_z"][0], wl["omega_m"][0], wl["z_nz"],
                                  wl["nz"][0, tracers], wl["kind"][0, tracers], wl["bias"][0, tracers],
                                  z_star=wl["z_star"])


# clustering bins 0 and 9, lensing bins 12 and 14, the CMB-lensing tracer
SUBSET = [0, 9, 12, 14, 15]


def test_cmb_kernel_is_the_lens_efficiency_of_a_source_plane(wl_cmb):
    """A lensing tracer whose n(z) is a narrow Gaussian at z_s has q D / chi^2 equal to the CMB
    kernel with z_* = z_s, up to the O(sigma^2) spread of 1/chi' over the Gaussian, amplified by
    chi / (chi_* - chi): measured 2e-11 at z = 0.05, 8e-8 at z = 500."""
    zs, sig = 1000.0, 0.3
    z_nz = np.linspace(zs - 4.0, zs + 4.0, 801)
    n = np.exp(-0.5 * ((z_nz - zs) / sig) ** 2) / (sig * np.sqrt(2.0 * np.pi))
    geo = geometry.PointGeometry(wl_cmb["z_geom"], wl_cmb["chi_z"][0], wl_cmb["D_z"][0], wl_cmb["omega_m"][0],
                                 z_nz, np.array([n, n]), np.array([1, 2]), np.array([1.0, 1.0]), z_star=zs)
    z = np.array([0.05, 0.5, 2.0, 10.0, 100.0, 500.0])
    lens, cmb = geo.f_of_z(0, z), geo.f_of_z(1, z)
    assert np.all(cmb > 0)
    assert np.max(np.abs(lens / cmb - 1.0)) < 1e-6
    # nothing above the source plane
    assert np.all(geo.f_of_z(1, np.array([1000.5, 1050.0])) == 0.0)


def test_cmb_window_einstein_de_sitter():
    """Om = 1: chi = 2 (c/H0) (1 - (1+z)^-1/2) and D = a, so the window of Sec. 2.4 is
    l(l+1) 1.5 (H0/c)^2 / k^2 int_{chi_min}^{chi_*} (1/chi - 1/chi_*) j_l(k chi) dchi.  The oracle, fed
    only samples of chi(z) and D(z), matches it on the C_l metric (k^3 P weights): measured 1.4e-5
    at most (l = 229), 4e-6 at l = 2."""
    zs = 1090.0
    z = np.concatenate([np.linspace(0.01, 3.0, 1024), np.expm1(np.linspace(np.log1p(3.0), np.log1p(zs), 257))[1:]])
    chi_of = lambda zz: 2.0 * C_OVER_H0 * (1.0 - 1.0 / np.sqrt(1.0 + zz))
    geo = geometry.PointGeometry(z, chi_of(z), 1.0 / (1.0 + z), 1.0, np.linspace(0.01, 3.0, 200),
                                 np.zeros((1, 200)), np.array([2]), np.array([1.0]))
    chis, chimin = chi_of(zs), chi_of(0.01)
    x, w = np.polynomial.legendre.leggauss(16)

    def direct(ell, kk):
        npan = max(32, int(np.ceil((chis - chimin) * kk / np.pi)))
        e = np.linspace(chimin, chis, npan + 1)
        a, b = e[:-1, None], e[1:, None]
        c = (0.5 * (b - a) * x + 0.5 * (a + b)).ravel()
        wc = (0.5 * (b - a) * w).ravel()
        jl = np.sqrt(np.pi / (2.0 * kk * c)) * jv(ell + 0.5, kk * c)
        return ell * (ell + 1.0) * 1.5 / (C_OVER_H0 ** 2 * kk ** 2) * np.sum(wc * (1.0 / c - 1.0 / chis) * jl)

    k = np.geomspace(1e-4, 10.0, 1024)
    m = fftlog.Method(k, 1024)
    ells = np.array([2.0, 4.0, 15.0, 229.0, 2000.0])
    W = fftlog.windows_point(geo, ells, m)[:, 0, ::32]
    Wd = np.array([[direct(ell, kk) for kk in k[::32]] for ell in ells])
    s = (fftlog.k_weights(m) * synth.linear_pk(k, 0.3, 0.7, 0.8))[::32]
    eps = np.abs(np.sum(s * (W ** 2 - Wd ** 2), axis=1)) / np.sum(s * Wd ** 2, axis=1)
    assert eps.max() < 3e-5
    # a planted mistake: the shear prefactor in place of l(l+1) is caught at l = 2 (ratio 6 / sqrt(24))
    F2 = np.sqrt(4.0 * 3.0 * 2.0 * 1.0)
    assert abs((F2 / 6.0) ** 2 - 1.0) > 100 * eps[0]


def test_method_floor_cmb_lensing(wl_cmb):
    """FFTLog oracle against direct quadrature with the CMB tracer (tilts (-1, -1, -2) by band):
    CMB auto <= 5.8e-5 (measured at l = 2000; 1.3e-5 at l = 229, where the window turns on at
    chi_*), CMB crosses <= 4.5e-6, the other spectra at their floor without it."""
    m = fftlog.method_for(wl_cmb)
    geo = _subset_geometry(wl_cmb, SUBSET)
    ells = fftlog.point_ells(wl_cmb, 0)[[0, 9, 30, 70, 102]]
    W = fftlog.windows_point(geo, ells, m)[:, :, ::32]
    Wq = quadrature.windows_quadrature(geo, ells, m.k[::32])
    s = (fftlog.k_weights(m) * wl_cmb["pk"][0])[::32]
    eps = eps_metric(np.einsum("ltj,lsj,j->lts", W, W, s), np.einsum("ltj,lsj,j->lts", Wq, Wq, s))
    assert eps[:, 4, 4].max() < 1e-4
    assert eps[:, 4, :4].max() < 1e-5
    assert eps[:, :4, :4].max() < 3e-5


def test_cmb_limber_limit(wl_cmb):
    """The exact C_l of the CMB tracer approaches eq. Limber: the auto spectrum's relative
    difference falls from > 5% at l = 2 to < 1e-4 for l >= 200 (measured 7e-6), and the CMB row
    differs by < 2e-4 on the eps metric there (measured 7e-5: the FFTLog floor of the crosses)."""
    m = fftlog.method_for(wl_cmb)
    geo = _subset_geometry(wl_cmb, SUBSET)
    ells = fftlog.point_ells(wl_cmb, 0)[[0, 30, 50, 70, 90, 102]]
    W = fftlog.windows_point(geo, ells, m)
    C = np.einsum("ltj,lsj,j->lts", W, W, fftlog.k_weights(m) * wl_cmb["pk"][0])
    CL = limber.cl_limber(geo, ells, m.k, wl_cmb["pk"][0])
    rel = np.abs(C[:, 4, 4] / CL[:, 4, 4] - 1.0)
    assert rel[0] > 5e-2
    assert np.all(np.diff(rel[:3]) < 0)
    assert rel[ells >= 200].max() < 1e-4
    assert eps_metric(C, CL)[ells >= 200, 4, :].max() < 2e-4


def test_cmb_limber_on_the_chi_grid(wl_cmb):
    """The chi-node Limber rule (the GPU's Limber path) against the fine-panel Limber integral for
    the CMB tracer: eps < 5e-6 for l <= 500, < 1e-4 at l = 2000 (the k_max cut inside the support)."""
    m = fftlog.method_for(wl_cmb)
    geo = _subset_geometry(wl_cmb, SUBSET)
    ells = fftlog.point_ells(wl_cmb, 0)[[0, 30, 70, 80, 102]]
    CG = limber.cl_limber_grid(geo, ells, m, wl_cmb["pk"][0])
    CL = limber.cl_limber(geo, ells, m.k, wl_cmb["pk"][0])
    eps = eps_metric(CG, CL)[:, 4, :]
    assert eps[ells <= 500].max() < 5e-6
    assert eps.max() < 1e-4


def test_cmb_workload_recipe():
    """synth.cmb_lensing: geometry continued to z_*, one kind-2 tracer after each point's last
    tracer (ragged batches too), and a refusal once per-grid samples exist."""
    wl = synth.cmb_lensing(synth.make_workload("cfg3", batch=6))
    assert wl["z_geom"][-1] == 1090.0 and np.all(np.diff(wl["z_geom"]) > 0)
    assert wl["chi_z"].shape == (6, len(wl["z_geom"])) and np.all(np.diff(wl["chi_z"], axis=1) > 0)
    for b in range(6):
        T = int(wl["n_tracers"][b])
        assert wl["kind"][b, T - 1] == 2 and np.all(wl["kind"][b, :T - 1] != 2)
        assert np.all(wl["nz"][b, T - 1] == 0.0)
    with pytest.raises(ValueError):
        synth.cmb_lensing(synth.intrinsic_alignment(synth.make_workload("cfg0")))


def test_cmb_corner_is_second_order():
    """Where the window turns on at chi_* (k just above l/chi_*), the kernel's corner is all the
    window sees: with the trapezoid weight of a linear end on the last node below chi_* the error
    there falls ~4x when the grid step halves (measured 1.6e-3 -> 4.0e-4 of the window's peak at
    l = 229 from N = 1024 to 2048; the jump weight of the other kernels' edges gives 3.5e-3 ->
    1.6e-3, first order)."""
    zs = 1090.0
    z = np.concatenate([np.linspace(0.01, 3.0, 1024), np.expm1(np.linspace(np.log1p(3.0), np.log1p(zs), 257))[1:]])
    chi_of = lambda zz: 2.0 * C_OVER_H0 * (1.0 - 1.0 / np.sqrt(1.0 + zz))
    geo = geometry.PointGeometry(z, chi_of(z), 1.0 / (1.0 + z), 1.0, np.linspace(0.01, 3.0, 200),
                                 np.zeros((1, 200)), np.array([2]), np.array([1.0]))
    chis, chimin = chi_of(zs), chi_of(0.01)
    x, w = np.polynomial.legendre.leggauss(24)

    def direct(ell, kk):
        npan = max(64, 4 * int(np.ceil((chis - chimin) * kk / np.pi)))
        e = np.linspace(chimin, chis, npan + 1)
        a, b = e[:-1, None], e[1:, None]
        c = (0.5 * (b - a) * x + 0.5 * (a + b)).ravel()
        wc = (0.5 * (b - a) * w).ravel()
        jl = np.sqrt(np.pi / (2.0 * kk * c)) * jv(ell + 0.5, kk * c)
        return ell * (ell + 1.0) * 1.5 / (C_OVER_H0 ** 2 * kk ** 2) * np.sum(wc * (1.0 / c - 1.0 / chis) * jl)

    ell, err = 229.0, []
    for n in (1024, 2048):
        k = np.geomspace(1e-4, 10.0, n)
        W = fftlog.windows_point(geo, [ell], fftlog.Method(k, n))[0, 0]
        sel = np.nonzero((k > 0.75 * ell / chis) & (k < 2.5 * ell / chis))[0][::4 * n // 1024]
        Wd = np.array([direct(ell, k[j]) for j in sel])
        err.append(np.abs(W[sel] - Wd).max() / np.abs(Wd).max())
    assert err[0] < 2.5e-3
    assert err[0] / err[1] > 3.0
