"""The Limber limit (paper, Sec. 2.6, eq. Limber) -- an oracle check at high l.

With j_l(x) ~ sqrt(pi/(2l+1)) delta(l + 1/2 - x) every window collapses onto
chi = (l+1/2)/k and
  C_l^{ij} ~ int dchi / chi^2 c_i c_j f_i(chi) f_j(chi) P((l+1/2)/chi),
where c = 1 for clustering and c = F(l) chi^2 / (l+1/2)^2 for lensing
(F(l)/k^2 evaluated at the Limber k).  Its error is O(1/l).

P is the user's samples, interpolated by a cubic spline in (ln k, ln P) and
set to zero outside [k_min, k_max] so that the comparison sees the same
truncated k range as the k-sum of the exact C_l.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline

from .geometry import PointGeometry
from .quadrature import LensingTable

_GL16 = np.polynomial.legendre.leggauss(16)


def cl_limber(geo: PointGeometry, ells, k, pk, n_panels=4000):
    k = np.asarray(k, float)
    lp = CubicSpline(np.log(k), np.log(pk))
    T = len(geo.kinds)
    lens = LensingTable(geo) if np.any(geo.kinds == 1) else None
    edges = np.linspace(geo.z_min, geo.z_max, n_panels + 1)
    x, w = _GL16
    a, b = edges[:-1, None], edges[1:, None]
    z = (0.5 * (b - a) * x + 0.5 * (a + b)).ravel()
    wz = (0.5 * (b - a) * w).ravel()
    chi = geo.chi_spl(z)
    dchi = geo.chi_spl(z, 1)
    D = geo.D_spl(z)
    f = np.empty((T, len(z)))
    for t in range(T):
        if geo.kinds[t] == 0:
            f[t] = geo.bias[t] * geo.n_of_z(t, z) * D / dchi
        else:
            f[t] = lens(t, z) * D / chi ** 2
    out = np.zeros((len(ells), T, T))
    for li, ell in enumerate(ells):
        nu = ell + 0.5
        kl = nu / chi
        inside = (kl >= k[0]) & (kl <= k[-1])
        P = np.where(inside, np.exp(lp(np.log(np.clip(kl, k[0], k[-1])))), 0.0)
        F = np.sqrt((ell + 2.0) * (ell + 1.0) * ell * (ell - 1.0))
        c = np.where(geo.kinds[:, None] == 1, F * chi[None, :] ** 2 / nu ** 2, 1.0)
        g = f * c
        out[li] = (g * (wz * dchi * P / chi ** 2)[None, :]) @ g.T
    return out
