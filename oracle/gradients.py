"""Derivatives of the packed C_l (oracle; FP64; test infrastructure).

The loss convention for a cotangent G packed like C (upper triangle, i <= j):
L = sum_l sum_{i<=j} G_l^{ij} C_l^{ij}.

Exact forms used (from C_l^{ij} = sum_j s_j W_i W_j, s = (2/pi) w k^3 P):
  dC^{ij}/dP_j   = (2/pi) w_j k_j^3 W_i(k_j) W_j(k_j)
  dC^{ij}/db_t   = C^{ij} (delta_it + delta_jt) / b_t   (clustering t; bias multiplies W_t)
  n(z) and D(z)  : every window is linear in n_t (clustering n, lensing q) and in
                   D, so W(x + eps v) = W(x) + eps W(v) exactly, and a directional
                   derivative is one more window pass with x replaced by v.
"""
from __future__ import annotations

import numpy as np

from . import fftlog
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
