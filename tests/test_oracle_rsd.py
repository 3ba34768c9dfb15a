"""Pins of the oracle's redshift-space-distortion term (eq. RSD) and of its spherical Bessel
functions, independent of the oracle's own kernel code (CPU only).

* j_l of real order (J_{l+1/2} based) against scipy's integer-order spherical_jn and against
  mpmath at real orders up to l = 3000; j_l'' (from the Bessel equation) against the derivative
  recurrence j_l' = j_{l-1} - (l+1) j_l / x differentiated once more.
* The RSD window int dchi g j_l''(k chi) of the oracle against k^-2 int dchi g'' j_l(k chi)
  (two integrations by parts; the boundary terms vanish for a bin inside the support), with
  g = -f n dz/dchi D built here from the sampled inputs and g'' by finite differences.
* The Kaiser enhancement: RSD raises the clustering autos at low l, more for narrower bins, and
  the ratio falls monotonically to 1 with l.
* A sign flip planted in the oracle's RSD kernel fails both of the last two checks.
"""
import mpmath
import numpy as np
import pytest
from scipy.interpolate import CubicSpline
from scipy.special import spherical_jn

import synth
from oracle import fftlog, geometry, quadrature


# --- spherical Bessel functions ----------------------------------------------------------------

@pytest.mark.parametrize("ell", [0, 1, 2, 7, 50, 500, 3000])
def test_spherical_jn_real_matches_scipy_integer_orders(ell):
    x = np.concatenate([np.linspace(0.05, 3.0, 40), np.linspace(0.5 * ell + 0.1, 3.0 * ell + 60.0, 400)])
    ref = spherical_jn(ell, x)
    got = quadrature.spherical_jn_real(float(ell), x)
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("ell", [0.5, 2.3, 41.7, 777.25, 2999.5])
def test_spherical_jn_real_matches_mpmath_real_orders(ell):
    mpmath.mp.dps = 30
    xs = np.array([0.9, 1.02, 1.3, 2.2]) * (ell + 0.5) + 1.0
    got = quadrature.spherical_jn_real(ell, xs)
    ref = np.array([float(mpmath.sqrt(mpmath.pi / (2 * mpmath.mpf(x))) * mpmath.besselj(mpmath.mpf(ell) + 0.5, x, maxprec=40000, maxterms=10 ** 6))
                    for x in xs])
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("ell", [1, 2, 10, 200, 3000])
def test_spherical_jn2_matches_derivative_recurrence(ell):
    """j_l'' = j_{l-1}' + (l+1) j_l / x^2 - (l+1) j_l' / x, from j_l' = j_{l-1} - (l+1) j_l / x."""
    x = np.linspace(0.3 * ell + 0.5, 2.5 * ell + 40.0, 500)
    ref = (spherical_jn(ell - 1, x, derivative=True) + (ell + 1) * spherical_jn(ell, x) / x ** 2
           - (ell + 1) * spherical_jn(ell, x, derivative=True) / x)
    got = quadrature.spherical_jn2_real(float(ell), x)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


# --- the RSD window --------------------------------------------------------------------------

def _single_bin(zc, sigma, bias):
    """Geometry of point 0 of the full-size workload with one Gaussian clustering bin."""
    wl = synth.make_workload("cfg1")
    nz = synth.gaussian_nz(wl["z_nz"], zc, sigma)
    geo = geometry.PointGeometry(wl["z_geom"], wl["chi_z"][0], wl["D_z"][0], wl["omega_m"][0], wl["z_nz"],
                                 nz[None], [0], [bias])
    return wl, nz, geo


def _by_parts_error(ells, k):
    """max |W_rsd - k^-2 int g'' j_l| / max |W_rsd| over k, for each l, of a bin at z = 0.7
    (sigma 0.05, negligible beyond z in [0.35, 1.05]); bias 0 leaves the RSD term alone."""
    wl, nz, geo = _single_bin(0.7, 0.05, 0.0)
    W = quadrature.windows_quadrature(geo, ells, k, rsd=True)[:, 0, :]
    # g(chi) = -f n dz/dchi D from the sampled inputs, continued as every sampled input is
    # (natural cubic splines); f = dln D / dln a and dz/dchi by finite differences
    chi_of_z = CubicSpline(wl["z_geom"], wl["chi_z"][0], bc_type="natural")
    D_of_z = CubicSpline(wl["z_geom"], wl["D_z"][0], bc_type="natural")
    n_of_z = CubicSpline(wl["z_nz"], nz, bc_type="natural")
    zf = np.linspace(0.3, 1.1, 400001)
    chi = np.linspace(chi_of_z(0.35), chi_of_z(1.05), 40001)
    h = chi[1] - chi[0]
    z = np.interp(chi, chi_of_z(zf), zf)
    f = np.gradient(np.log(D_of_z(z)), -np.log1p(z))
    g = -f * n_of_z(z) * np.gradient(z, h) * D_of_z(z)
    g2 = np.gradient(np.gradient(g, h), h)
    err = []
    for li, ell in enumerate(ells):
        rhs = np.array([np.trapezoid(g2 * spherical_jn(ell, kk * chi), chi) / kk ** 2 for kk in k])
        err.append(np.max(np.abs(W[li] - rhs)) / np.max(np.abs(W[li])))
    return np.array(err)


def _kaiser_ratio(zc, sigma, ells):
    """C_l^{gg} with RSD over C_l^{gg} without, bias 1.5 (FFTLog oracle on the full k grid)."""
    wl, nz, geo = _single_bin(zc, sigma, 1.5)
    w1 = dict(wl, nz=nz[None, None], kind=np.zeros((1, 1), np.int32), bias=np.array([[1.5]]),
              n_tracers=np.ones(1, np.int32))
    m = fftlog.method_for(w1)
    s = fftlog.k_weights(m) * wl["pk"][0]
    C = [np.einsum("lj,lj,j->l", W[:, 0], W[:, 0], s)
         for W in (fftlog.windows_point(geo, ells, m, rsd=r) for r in (False, True))]
    return C[1] / C[0]


_ELLS = [2, 10, 40]
_K = np.array([0.002, 0.005, 0.01, 0.03, 0.08])
_KAISER_ELLS = np.array([2, 4, 8, 16, 32, 64, 128, 256, 512], float)


def test_rsd_window_integration_by_parts():
    """Measured 1e-8 (l = 2) to 7e-7 (l = 40): the finite-difference g''."""
    assert _by_parts_error(_ELLS, _K).max() < 1e-5


def test_rsd_kaiser_enhancement():
    """Measured at l = 2: 2.17 (sigma 0.05), 1.62 (0.1), 2.43 (z = 1, 0.03); 1.0006 at l = 512."""
    r = _kaiser_ratio(0.7, 0.05, _KAISER_ELLS)
    assert r[0] > 1.5
    assert np.all(np.diff(r) < 0)
    assert np.all(r > 1.0) and r[-1] < 1.002
    wide = _kaiser_ratio(0.7, 0.1, _KAISER_ELLS[:1])
    assert 1.0 < wide[0] < r[0]


def test_planted_rsd_sign_flip_is_caught(monkeypatch):
    """With the sign of the oracle's RSD kernel flipped, the by-parts identity misses by ~2 and the
    clustering autos drop below the real-space ones at low l."""
    kernel = geometry.PointGeometry.f_rsd_of_z
    monkeypatch.setattr(geometry.PointGeometry, "f_rsd_of_z", lambda self, t, z: -kernel(self, t, z))
    assert _by_parts_error(_ELLS[:1], _K).min() > 1.0
    assert _kaiser_ratio(0.7, 0.05, _KAISER_ELLS[:2]).max() < 1.0
