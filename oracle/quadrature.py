"""The plain definition of the k-windows, by direct quadrature (oracle; FP64).

Paper, Sec. 2.1: Delta_l^i(k) = c(l) int_0^inf dchi W^i(chi) j_l(k chi), with the
kernels of Sec. 2.2 - 2.4 (see geometry.py).  Here the chi integral is written
in z on the kernel support and integrated by composite 16-point
Gauss-Legendre: panels break at every knot of the geometry and n(z) grids and
are at most pi/k wide in chi (half an oscillation of j_l).
j_l(x) = sqrt(pi / 2x) J_{l+1/2}(x) for real l (scipy.special.jv).

This is not the method: it is the exact integral the FFTLog method
approximates, and it pins the FFTLog oracle (its method-error floor).
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline
from scipy.special import jv, jvp

from .geometry import PointGeometry, ell_prefactor

_GL16 = np.polynomial.legendre.leggauss(16)


def spherical_jn_real(ell, x):
    x = np.asarray(x, float)
    return np.sqrt(np.pi / (2.0 * x)) * jv(ell + 0.5, x)


class LensingTable:
    """q_t(z) of every lensing tracer, exact on a dense z table and splined between.

    The table holds `refine` points per knot interval of the geometry and n(z)
    grids, so every spline piece lies where q is smooth.
    """

    def __init__(self, geo: PointGeometry, refine=16):
        knots = geo._knots()
        zt = np.concatenate([np.linspace(knots[i], knots[i + 1], refine + 1)[:-1]
                             for i in range(len(knots) - 1)] + [[knots[-1]]])
        self.spl = {}
        # lensing tracers, and clustering tracers too when they carry magnification
        for t in np.nonzero((geo.kinds == 1) | (geo.mag is not None))[0]:
            self.spl[int(t)] = CubicSpline(zt, geo.lensing_q(int(t), zt))

    def __call__(self, t, z):
        return self.spl[int(t)](z)


def _panels(geo: PointGeometry, k):
    """z panel edges: every knot, plus subdivisions so each panel is <= pi/k in chi."""
    knots = geo._knots()
    chi_k = geo.chi_spl(knots)
    edges = [knots[:1]]
    for i in range(len(knots) - 1):
        npan = max(1, int(np.ceil((chi_k[i + 1] - chi_k[i]) * k / np.pi)))
        edges.append(np.linspace(knots[i], knots[i + 1], npan + 1)[1:])
    return np.concatenate(edges)


def spherical_jn2_real(ell, x):
    """j_l''(x) from the spherical Bessel equation: j'' = -(2/x) j' - (1 - l(l+1)/x^2) j, with
    j' from J_nu' (scipy jvp), real order."""
    x = np.asarray(x, float)
    nu = ell + 0.5
    s = np.sqrt(np.pi / (2.0 * x))
    j = s * jv(nu, x)
    jp = s * (jvp(nu, x) - jv(nu, x) / (2.0 * x))
    return -(2.0 / x) * jp - (1.0 - ell * (ell + 1.0) / x ** 2) * j


def windows_quadrature(geo: PointGeometry, ells, k, lens_table=None, rsd=False):
    """W[l, t, j] = c_t(l, k_j) int dz (dchi/dz) f_t j_l(k_j chi(z)) for the given ells and k; with
    rsd=True the clustering tracers add int dz (dchi/dz) f_rsd j_l''(k_j chi(z)) (eq. RSD)."""
    k = np.atleast_1d(np.asarray(k, float))
    T = len(geo.kinds)
    if lens_table is None and (np.any(geo.kinds == 1) or geo.mag is not None):
        lens_table = LensingTable(geo)
    x, w = _GL16
    W = np.zeros((len(ells), T, len(k)))
    for j, kk in enumerate(k):
        e = _panels(geo, kk)
        a, b = e[:-1, None], e[1:, None]
        z = (0.5 * (b - a) * x + 0.5 * (a + b)).ravel()
        wz = (0.5 * (b - a) * w).ravel()
        chi = geo.chi_spl(z)
        D = geo.D_spl(z)
        # integrand per unit z, without j_l
        h = np.empty((T, len(z)))
        for t in range(T):
            if geo.kinds[t] == 0:
                h[t] = geo.bias[t] * geo.n_of_z(t, z) * D
            elif geo.kinds[t] == 2:
                h[t] = geo.cmb_kernel(z) * geo.chi_spl(z, 1)
            else:
                h[t] = (lens_table(t, z) * geo.chi_spl(z, 1) + geo.ia_of_z(z) * geo.n_of_z(t, z)) * D / chi ** 2
        hw = h * wz[None, :]
        if rsd:
            hr = np.array([geo.f_rsd_of_z(t, z) * geo.chi_spl(z, 1) for t in range(T)]) * wz[None, :]
        if geo.mag is not None:
            # magnification (eq. magnification bias): C_g q D / chi^2 with prefactor l(l+1)/k^2
            hm = np.array([geo.mag[t] * lens_table(t, z) * D * geo.chi_spl(z, 1) / chi ** 2 if geo.kinds[t] == 0
                           else np.zeros_like(z) for t in range(T)]) * wz[None, :]
        for li, ell in enumerate(ells):
            jl = spherical_jn_real(ell, kk * chi)
            integral = hw @ jl
            if rsd:
                integral = integral + hr @ spherical_jn2_real(ell, kk * chi)
            for t in range(T):
                W[li, t, j] = integral[t] * ell_prefactor(geo.kinds[t], ell, kk)
            if geo.mag is not None:
                W[li, :, j] += (hm @ jl) * ell * (ell + 1.0) / kk ** 2
    return W
