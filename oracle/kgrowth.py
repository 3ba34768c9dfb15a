"""Scale-dependent growth D(k, z) by interpolation along k (Sec. 3.2), FP64 (oracle; test
infrastructure only: the tests, the smoke check and the benchmark's CPU baseline use it).

The power spectrum is factorised as P(k, chi, chi') = P(k, z_fid) D(k, z(chi)) D(k, z(chi')), and
f(chi) D(k, z(chi)) is decomposed in ln chi with coefficients that depend on k (Sec. 3.2): the chi
integral keeps its analytic form (eq. int_jl), so for every k

    Delta_l^t(k) = c(l, k) sum_n c_n^t(k) int chi^{b + i eta_n} j_l(k chi) dchi.

The coefficients are computed at N_interp nodes in k and interpolated to the other k.

Steps, in that order:
  1. at every node kappa_a: the kernels f_t(chi) D(kappa_a, z(chi)) sampled on the log-chi grid
     exactly as for scale-free growth (every kind: clustering, lensing, CMB lensing), and their
     FFTLog coefficients c_n^(a) (per tracer kind and multipole band, fftlog.fftlog_coefficients);
  2. c_n(k_j) at every k of the user's grid by interpolation along ln k;
  3. Delta_l^t(k_j) by the direct sum over n of fftlog.py, with c_n(k_j) in place of c_n;
  4. C_l by the k-sum of fftlog.py.

Readings (the paper fixes neither the node placement nor the interpolant; the HIP path takes the
same ones):
  R14 The nodes are uniform in ln k from k_min to k_max, both ends included (N_interp >= 2).
  R15 The growth at node a is given as samples D(kappa_a, z) on the geometry z grid and continued
      in z by the natural cubic spline, like D(z).
  R16 c_n(k) is continued in ln k by the natural cubic spline through the node values (real and
      imaginary parts separately).  The paper calls the interpolation smooth; the natural spline
      is the smooth interpolant of least curvature and reproduces a c_n linear in ln k exactly.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline

from . import fftlog
from .geometry import PointGeometry, ell_prefactor


def ln_nodes(method: fftlog.Method, n_interp):
    """Reading R14: ln kappa_a, a = 0..N_interp-1."""
    if int(n_interp) < 2:
        raise ValueError("N_interp must be at least 2")
    return np.linspace(np.log(method.k[0]), np.log(method.k[-1]), int(n_interp))


def node_geometries(wl, b):
    """One PointGeometry per node: the point's geometry with D(z) replaced by D(kappa_a, z)."""
    T = int(wl["n_tracers"][b])
    ia = wl.get("ia")
    geos = [PointGeometry(wl["z_geom"], wl["chi_z"][b], wl["D_kz"][b, a], wl["omega_m"][b], wl["z_nz"],
                          wl["nz"][b, :T], wl["kind"][b, :T], wl["bias"][b, :T], ia=None if ia is None else ia[b],
                          z_star=wl.get("z_star"))
            for a in range(wl["D_kz"].shape[1])]
    # every node has the point's chi(z): solve z(chi) once and share the roots
    solve = geos[0].z_of_chi
    roots = {}

    def z_of_chi(chi):
        chi = np.asarray(chi, float)
        key = chi.tobytes()
        if key not in roots:
            roots[key] = solve(chi)
        return roots[key].copy()

    for g in geos:
        g.z_of_chi = z_of_chi
    return geos


def interpolate_ln_k(x_nodes, values, x):
    """Reading R16: natural cubic spline along axis 0 (nodes x_nodes) evaluated at x."""
    re = CubicSpline(x_nodes, values.real, axis=0, bc_type="natural")(x)
    im = CubicSpline(x_nodes, values.imag, axis=0, bc_type="natural")(x)
    return re + 1j * im


def windows_point(geos, ells, method: fftlog.Method):
    """W[l, t, j] = Delta_l^t(k_j) for one parameter point; geos[a] holds node a's growth."""
    A = len(geos)
    x_nodes = ln_nodes(method, A)
    k = method.k
    N = method.n_chi
    kinds = geos[0].kinds
    T = len(kinds)
    # step 1: kernels and their coefficients at every node
    sampled = [fftlog.sampled_kernels(g, method) for g in geos]
    chi0, chi = sampled[0][0], sampled[0][1]
    W = np.zeros((len(ells), T, method.n_k))
    ells = np.asarray(ells, float)
    for kind in (0, 1, 2):
        ts = np.nonzero(kinds == kind)[0]
        if len(ts) == 0:
            continue
        bs = np.array([method.b_of(kind, ell) for ell in ells])
        for b in np.unique(bs):
            n = None
            cn = []
            for a in range(A):
                n, c = fftlog.fftlog_coefficients(sampled[a][2][ts], chi, chi0, b, method)
                cn.append(c)
            # step 2: c_n(k_j), [n_k, T_kind, N-1]
            cj = interpolate_ln_k(x_nodes, np.array(cn), np.log(k))
            p = b + 1j * 2.0 * np.pi * n / (N * method.delta)
            for li in np.nonzero(bs == b)[0]:
                ell = ells[li]
                if not (-ell - 1.0 < b < 1.0):
                    raise ValueError(f"FFTLog bias b={b} outside (-l-1, 1) at l={ell}")
                # step 3: the n-sum at every k with that k's coefficients
                Mjn = fftlog.bessel_power_integral(ell, p[None, :], k[:, None])  # [n_k, N-1]
                delta = np.einsum("jn,jtn->jt", Mjn, cj)
                W[li, ts, :] = (delta.real * ell_prefactor(kind, ell, k)[:, None]).T
    return W


def windows(wl, b, method=None):
    method = method or fftlog.method_for(wl)
    return windows_point(node_geometries(wl, b), fftlog.point_ells(wl, b), method)


def cl(wl, b, method=None, return_windows=False):
    """C_l for point b of a workload with D_kz: [L_b, T_b(T_b+1)/2] (FP64)."""
    method = method or fftlog.method_for(wl)
    W = windows(wl, b, method)
    C = fftlog.cl_from_windows(W, wl["pk"][b], method)  # step 4
    return (C, W) if return_windows else C
