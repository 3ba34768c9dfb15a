"""The Limber limit (paper, Sec. 2.6, eq. Limber) -- an oracle check at high l.

With j_l(x) ~ sqrt(pi/(2l+1)) delta(l + 1/2 - x) every window collapses onto
chi = (l+1/2)/k and
  C_l^{ij} ~ int dchi / chi^2 c_i c_j f_i(chi) f_j(chi) P((l+1/2)/chi),
where c = 1 for clustering, c = F(l) chi^2 / (l+1/2)^2 for lensing (F(l)/k^2 evaluated at the
Limber k) and c = l(l+1) chi^2 / (l+1/2)^2 for CMB lensing.  Its error is O(1/l).

P is the user's samples, interpolated by a cubic spline in (ln k, ln P) and
set to zero outside [k_min, k_max] so that the comparison sees the same
truncated k range as the k-sum of the exact C_l.

cl_limber integrates in z with fine Gauss-Legendre panels (the plain definition);
cl_limber_grid evaluates the same integral on the FFTLog log-chi grid, the rule of
the GPU's Limber path:
  C_l^{ij} = Delta sum_m w_m g_i(chi_m) g_j(chi_m) P((l+1/2)/chi_m) / chi_m,
with the edge weights w_m of the grid (reading R5: 1/2 on the lower support edge,
1/2 + theta on the last node), dchi = chi dln chi, g = c f, and P by the natural
cubic spline of ln P in ln k (zero outside the k range).
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline

from . import fftlog
from .geometry import PointGeometry
from .quadrature import LensingTable

_GL16 = np.polynomial.legendre.leggauss(16)


def _limber_prefactor(kinds, ell, chi):
    """c_t(l) at the Limber k = (l+1/2)/chi: [T, len(chi)]."""
    nu = ell + 0.5
    F = np.sqrt((ell + 2.0) * (ell + 1.0) * ell * (ell - 1.0))
    scale = np.select([kinds == 1, kinds == 2], [F, ell * (ell + 1.0)], 0.0)
    return np.where(kinds[:, None] == 0, 1.0, scale[:, None] * chi[None, :] ** 2 / nu ** 2)


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
        elif geo.kinds[t] == 2:
            f[t] = geo.cmb_kernel(z)
        else:
            f[t] = (lens(t, z) + geo.ia_of_z(z) * geo.n_of_z(t, z) / dchi) * D / chi ** 2
    out = np.zeros((len(ells), T, T))
    for li, ell in enumerate(ells):
        nu = ell + 0.5
        kl = nu / chi
        inside = (kl >= k[0]) & (kl <= k[-1])
        P = np.where(inside, np.exp(lp(np.log(np.clip(kl, k[0], k[-1])))), 0.0)
        c = _limber_prefactor(geo.kinds, ell, chi)
        g = f * c
        out[li] = (g * (wz * dchi * P / chi ** 2)[None, :]) @ g.T
    return out


def _grid_terms(geo: PointGeometry, method):
    """The chi-node rule's nodes x_m, kernel samples f_t(x_m) [T, M] and edge weights w_m (R5)."""
    chi0, chi, F = fftlog.sampled_kernels(geo, method)  # F = w_t(m) f_t(chi_m)
    nodes, Wt = fftlog.edge_weights(geo, method)
    f = np.divide(F[:, nodes], Wt, out=np.zeros_like(Wt), where=Wt > 0)
    w = np.ones(len(nodes))
    w[0] = 0.5
    if len(nodes) > 1:
        w[-1] = 0.5 + (np.log(geo.chi_max / chi0) / method.delta - nodes[-1])
    return chi[nodes], f, w


def cl_limber_grid(geo: PointGeometry, ells, method, pk):
    """eq. Limber on the log-chi grid of the FFTLog method: [L, T, T]."""
    k = method.k
    lp = CubicSpline(np.log(k), np.log(pk), bc_type="natural")
    x, f, w = _grid_terms(geo, method)
    T = len(geo.kinds)
    out = np.zeros((len(ells), T, T))
    for li, ell in enumerate(ells):
        nu = ell + 0.5
        kl = nu / x
        inside = (kl >= k[0]) & (kl <= k[-1])
        P = np.where(inside, np.exp(lp(np.log(np.clip(kl, k[0], k[-1])))), 0.0)
        c = _limber_prefactor(geo.kinds, ell, x)
        g = f * c
        out[li] = (g * (method.delta * w * P / x)[None, :]) @ g.T
    return out


def grad_pk_grid(G, geo: PointGeometry, ells, method, pk):
    """dL/dP_j of L = sum_l sum_{s,t} G[l, s, t] C_l^{st} under the chi-node rule (G full [L, T, T]).

    C is linear in P at the Limber k of every node, and ln P(k) is the natural cubic spline through
    the (ln k_j, ln P_j), linear in the ln P_j: dP(k)/dP_j = P(k) B_j(ln k) / P_j, with B_j the
    natural spline through the j-th unit vector.  Nodes whose Limber k leaves [k_min, k_max] have
    P = 0 and no gradient.
    """
    k = method.k
    lnk = np.log(k)
    lp = CubicSpline(lnk, np.log(pk), bc_type="natural")
    basis = CubicSpline(lnk, np.eye(len(k)), bc_type="natural")
    x, f, w = _grid_terms(geo, method)
    out = np.zeros(len(k))
    for li, ell in enumerate(ells):
        kl = (ell + 0.5) / x
        inside = (kl >= k[0]) & (kl <= k[-1])
        lkl = np.log(np.clip(kl, k[0], k[-1]))
        P = np.where(inside, np.exp(lp(lkl)), 0.0)
        g = f * _limber_prefactor(geo.kinds, ell, x)
        a = np.einsum("sm,st,tm->m", g, G[li], g) * method.delta * w * P / x
        out += a @ basis(lkl)
    return out / np.asarray(pk, float)


def grad_kernels_grid(G, geo: PointGeometry, ells, method, pk):
    """dL/dF_t(chi_m) [T, N] under the chi-node rule, with F = w_t(m) f_t(chi_m) the sampled kernels
    of fftlog.sampled_kernels (G full [L, T, T]); returns (dF, F, nodes, z) like
    gradients.grad_kernels, so that gradients.grad_nz_full and grad_D_full take it as `kern`.

    C_l is the quadratic form sum_m g_s g_t Delta w_m P_l(m) / chi_m in g_t(m) = c_t(l, chi_m) f_t,
    f_t = F_t(m) / W_t(m) (the tracer's own node weight, R5 / R21), so
    dL/dF_t(m) = sum_l c_t sum_s (G_ts + G_st) g_s Delta w_m P_l(m) / (chi_m W_t(m)).
    """
    k = method.k
    lp = CubicSpline(np.log(k), np.log(pk), bc_type="natural")
    chi0, chi, F, nodes, z = fftlog.sampled_kernels(geo, method, return_nodes=True)
    _, Wt = fftlog.edge_weights(geo, method)
    x, f, w = _grid_terms(geo, method)
    dF = np.zeros_like(F)
    inv_w = np.divide(1.0, Wt, out=np.zeros_like(Wt), where=Wt > 0)
    for li, ell in enumerate(ells):
        kl = (ell + 0.5) / x
        inside = (kl >= k[0]) & (kl <= k[-1])
        P = np.where(inside, np.exp(lp(np.log(np.clip(kl, k[0], k[-1])))), 0.0)
        c = _limber_prefactor(geo.kinds, ell, x)
        g = f * c
        Gs = G[li] + G[li].T
        dF[:, nodes] += c * (Gs @ g) * (method.delta * w * P / x)[None, :] * inv_w
    return dF, F, nodes, z
