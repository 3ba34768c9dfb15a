"""Derivatives of the packed C_l (oracle; FP64; test infrastructure).

The loss convention for a cotangent G packed like C (upper triangle, i <= j):
L = sum_l sum_{i<=j} G_l^{ij} C_l^{ij}.

Exact forms used (from C_l^{ij} = sum_j s_j W_i W_j, s = (2/pi) w k^3 P):
  dC^{ij}/dP_j   = (2/pi) w_j k_j^3 W_i(k_j) W_j(k_j)
  dC^{ij}/db_t   = C^{ij} (delta_it + delta_jt) / b_t   (clustering t; bias multiplies W_t)
  n(z) and D(z)  : every window is linear in n_t (clustering n, lensing q) and in
                   D, so W(x + eps v) = W(x) + eps W(v) exactly, and a directional
                   derivative is one more window pass with x replaced by v.  The full
                   gradient vectors (grad_nz_full, grad_D_full) are the chain rule through
                   the same linear steps (see the note above them).
"""
from __future__ import annotations

import numpy as np

from . import fftlog, geometry
from .geometry import PointGeometry, point_geometry


def pair_index(T):
    return np.triu_indices(T)


def grad_pk(G, W, method):
    """dL/dP_j for one point: G [L, npairs], W [L, T, Nk]."""
    iu = pair_index(W.shape[1])
    w = fftlog.k_weights(method)
    return w * np.einsum("lp,lpj->j", G, W[:, iu[0], :] * W[:, iu[1], :])


def grad_bias(G, C, kinds, bias):
    """dL/db_t (zero for lensing tracers)."""
    T = len(kinds)
    iu = pair_index(T)
    out = np.zeros(T)
    for p, (i, j) in enumerate(zip(*iu)):
        contrib = G[:, p] * C[:, p]
        for t in (i, j):
            if kinds[t] == 0:
                out[t] += np.sum(contrib) / bias[t]
    return out


def grad_bias_windows(wl, b, G, method=None):
    """dL/db_t of point b for windows that also hold terms the bias does not scale (the RSD term of
    eq. RSD, the magnification term of eq. magnification bias): a clustering window is
    b_t D_t + R_t, with D_t the density window at unit bias, so
    dC^{ij}/db_t = sum_j s_j (delta_it D_t W_j + W_i delta_jt D_t).  Zero for lensing tracers."""
    method = method or fftlog.method_for(wl)
    W = fftlog.windows(wl, b, method)
    unit = dict(wl, rsd=False, mag=None, bias=np.ones_like(np.asarray(wl["bias"], float)))
    D = fftlog.windows(unit, b, method)
    T = W.shape[1]
    kinds = np.asarray(wl["kind"])[b, :T]
    out = np.zeros(T)
    for t in range(T):
        if kinds[t] != 0:
            continue
        dW = np.zeros_like(W)
        dW[:, t] = D[:, t]
        out[t] = _dL(G, W, dW, wl["pk"][b], method)
    return out


def _dL(G, W, dW, pk, method):
    """sum_l sum_{i<=j} G^{ij} sum_j s_j (dW_i W_j + W_i dW_j)."""
    iu = pair_index(W.shape[1])
    s = fftlog.k_weights(method) * pk
    dC = (np.einsum("lpj,j->lp", dW[:, iu[0], :] * W[:, iu[1], :], s)
          + np.einsum("lpj,j->lp", W[:, iu[0], :] * dW[:, iu[1], :], s))
    return float(np.sum(G * dC))


def directional_nz(wl, b, G, t, v, method=None):
    """d/deps L(n_t + eps v) for tracer t of point b; v sampled on z_nz.  The windows are linear in
    n (through the lens efficiency and the intrinsic-alignment term alike), so dW is the window of v."""
    method = method or fftlog.method_for(wl)
    geo = point_geometry(wl, b)
    ells = fftlog.point_ells(wl, b)
    W = fftlog.windows_point(geo, ells, method)
    nz_v = np.zeros_like(geo.nz)
    nz_v[t] = v
    ia = wl.get("ia")
    gv = PointGeometry(geo.z_geom, wl["chi_z"][b], wl["D_z"][b], geo.omega_m, geo.z_nz, nz_v,
                       geo.kinds, geo.bias, ia=None if ia is None else ia[b])
    dW = fftlog.windows_point(gv, ells, method)
    mask = np.zeros(len(geo.kinds), bool)
    mask[t] = True
    dW[:, ~mask, :] = 0.0
    return _dL(G, W, dW, wl["pk"][b], method)


def directional_D(wl, b, G, v, method=None):
    """d/deps L(D + eps v), v sampled on the geometry grid."""
    method = method or fftlog.method_for(wl)
    geo = point_geometry(wl, b)
    ells = fftlog.point_ells(wl, b)
    W = fftlog.windows_point(geo, ells, method)
    T = len(geo.kinds)
    ia = wl.get("ia")
    gv = PointGeometry(geo.z_geom, wl["chi_z"][b], v, geo.omega_m, geo.z_nz, wl["nz"][b, :T],
                       geo.kinds, geo.bias, ia=None if ia is None else ia[b])
    dW = fftlog.windows_point(gv, ells, method)
    return _dL(G, W, dW, wl["pk"][b], method)


# --- full gradients in n(z) and D(z) samples ------------------------------------------------------
# Steps 2-4 of the method map the sampled kernels F_t (on the chi grid) to the windows linearly, and
# F_t is linear in the tracer's n(z) samples and in the D(z) samples.  So the whole gradient is the
# chain rule through three linear maps, each taken from the oracle's own steps:
#   dL/dW_t(l, k)  = 2 s_k sum_j Gf_tj W_j(l, k)          (L = sum_{i,j} Gf_ij C^{ij}, Gf symmetric)
#   dL/dF_t(m)     = sum_l sum_k dL/dW_t(l, k) A_l(k, m)  (A_l: the windows of unit samples, W = A_l F)
#   dL/dn_t(z_s)   = sum_m dL/dF_t(m) F_t(m)[n_t = e_s]   (the kernels of the unit n(z) sample)
#   dL/dD(z_s)     = sum_t sum_m dL/dF_t(m) F_t(m) B_s(z_m) / D(z_m)
# where B_s is the natural cubic spline through the s-th unit vector on the geometry grid: every
# kernel is a D-independent factor times D(z) (Sec. 2.2-2.4), so F_t(m) / D(z_m) is that factor.


def symmetric_cotangent(G, T):
    """Gf [L, T, T] of a packed cotangent G [L, T(T+1)/2]: L = sum_{i<=j} G^{ij} C^{ij} = sum_{i,j}
    Gf_ij C^{ij} with Gf_ii = G^{ii} and Gf_ij = Gf_ji = G^{ij} / 2."""
    Gf = np.zeros((G.shape[0], T, T))
    for p, (i, j) in enumerate(zip(*pair_index(T))):
        if i == j:
            Gf[:, i, i] = G[:, p]
        else:
            Gf[:, i, j] = Gf[:, j, i] = 0.5 * G[:, p]
    return Gf


def window_matrix(ell, kind, chi, chi0, method):
    """A [N_k, N]: the windows of the N unit kernel samples for one multipole and tracer kind
    (steps 2-4 applied to the identity), so that W_t(l, k) = A @ F_t."""
    b = method.b_of(kind, ell)
    N = method.n_chi
    n, c = fftlog.fftlog_coefficients(np.eye(N), chi, chi0, b, method)  # [N, N-1]
    p = b + 1j * 2.0 * np.pi * n / (N * method.delta)
    M = fftlog.bessel_power_integral(ell, p[None, :], method.k[:, None])  # [N_k, N-1]
    return (M @ c.T).real * geometry.ell_prefactor(kind, ell, method.k)[:, None]


def grad_kernels(wl, b, G, method=None):
    """dL/dF_t(chi_m) [T, N] of point b, and the sampled kernels, their support nodes and
    redshifts: (dF, F, nodes, z)."""
    method = method or fftlog.method_for(wl)
    if wl.get("rsd") or wl.get("mag") is not None:
        raise ValueError("the full kernel gradient covers the density windows only (no RSD or magnification)")
    geo = point_geometry(wl, b)
    ells = fftlog.point_ells(wl, b)
    chi0, chi, F, nodes, z = fftlog.sampled_kernels(geo, method, return_nodes=True)
    W = fftlog.windows_point(geo, ells, method)
    T = len(geo.kinds)
    s = fftlog.k_weights(method) * np.asarray(wl["pk"][b], float)
    dW = 2.0 * np.einsum("lij,ljk->lik", symmetric_cotangent(G, T), W) * s[None, None, :]
    dF = np.zeros((T, method.n_chi))
    for li, ell in enumerate(ells):
        for kind in np.unique(geo.kinds):
            ts = np.nonzero(geo.kinds == kind)[0]
            dF[ts] += dW[li, ts] @ window_matrix(ell, int(kind), chi, chi0, method)
    return dF, F, nodes, z


def grad_nz_full(wl, b, G, method=None, kern=None):
    """dL/dn_t(z_s) [T, n_zs] of point b: the kernels of every unit n(z) sample (the lens efficiency
    and the intrinsic-alignment term included) against dL/dF.  Zero for CMB-lensing tracers, whose
    kernel does not involve n(z) (the unit-sample rule holds for kernels linear in n only).  kern:
    grad_kernels(wl, b, G, method) if already computed."""
    method = method or fftlog.method_for(wl)
    dF = (kern or grad_kernels(wl, b, G, method))[0]
    geo = point_geometry(wl, b)
    T, ns = len(geo.kinds), len(geo.z_nz)
    ia = wl.get("ia")
    out = np.zeros((T, ns))
    for t in range(T):
        if geo.kinds[t] == geometry.KIND_CMB_LENSING:
            continue
        basis = PointGeometry(geo.z_geom, wl["chi_z"][b], wl["D_z"][b], geo.omega_m, geo.z_nz, np.eye(ns),
                              np.full(ns, geo.kinds[t]), np.full(ns, geo.bias[t]),
                              ia=None if ia is None else ia[b], z_star=wl.get("z_star"))
        Fb = fftlog.sampled_kernels(basis, method)[2]  # row s: F_t with n_t = e_s
        out[t] = Fb @ dF[t]
    return out


def grad_D_full(wl, b, G, method=None, kern=None):
    """dL/dD(z_s) [n_zg] of point b through the natural spline of D(z) at the node redshifts.  kern:
    grad_kernels(wl, b, G, method) if already computed."""
    from scipy.interpolate import CubicSpline
    method = method or fftlog.method_for(wl)
    dF, F, nodes, z = kern or grad_kernels(wl, b, G, method)
    geo = point_geometry(wl, b)
    Bz = CubicSpline(geo.z_geom, np.eye(len(geo.z_geom)), bc_type="natural")(z)  # [nodes, n_zg]
    share = np.sum(dF[:, nodes] * F[:, nodes], axis=0) / geo.D_spl(z)
    return share @ Bz
