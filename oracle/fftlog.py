"""The paper's FFTLog method, step by step, in FP64 (oracle; test infrastructure).

Steps, in the order of the paper (Sec. 3.1 FFTLog, Sec. 3.2 Computational Method):
  1. sample every radial kernel f(chi) (kernel x growth x bias) on a log-chi grid;
  2. FFTLog coefficients c_n of f(chi) chi^-b (eq. FFTLog and the c_n sum);
  3. the analytic integral of chi^p j_l(k chi) over chi (eq. int_jl) for p = b + i eta_n;
  4. the window Delta_l^i(k) = c(l, k) sum_n c_n int chi^{p_n} j_l(k chi) dchi,
     summed directly over n for every k of the user's grid (no inverse FFT);
  5. C_l^{ij} = (2/pi) int dk k^2 Delta_l^i Delta_l^j P(k) on the user's k nodes.

Readings (the paper is silent, garbled or inconsistent; the HIP path takes the same ones):
  R1  eq. int_jl prints Gamma((2+l+p)/2) in the denominator; the correct one is
      Gamma((2+l-p)/2).  Verified against direct quadrature in the tests.
  R2  The c_n sum is the ordinary DFT: m = 0..N-1, kernel exp(-2 pi i n m / N),
      1/N normalisation, the grid's first node chi_0 as the phase reference.
  R3  The n-sum runs over -N/2+1..N/2-1: the Nyquist coefficient is dropped.
  R4  chi grid: chi_m = chi_0 exp(m Delta) with Delta the log step of the user's
      k grid, so the k-windows land on the user's nodes; chi_0 puts the lower
      support edge chi(z_min) exactly on node m0.
  R5  Support edges: the kernel is zero below chi(z_min) and above chi(z_max).
      The node on the lower edge carries weight 1/2 (the Fourier-series value at
      a jump); the upper edge, a fraction theta of a step above node m1, gives
      node m1 the weight 1/2 + theta.  Both make the DFT a trapezoid rule of the
      cut kernel, removing the first-order error of a jump.
  R6  The FFTLog bias b (the paper's "bias b") is chosen per tracer kind and per
      band of multipoles; every l of one band uses the same c_n.
  R7  Optional "smoothing at the tails" is a cosine taper of the coefficients
      over the top fraction of |n|; zero by default.
  R8  The k integral is the trapezoid rule in ln k on the user's nodes:
      int dk k^2 g = int dln k k^3 g, weight (2/pi) Delta (1/2 at both ends).
"""
from __future__ import annotations

import numpy as np
from scipy.special import loggamma

from .geometry import PointGeometry, ell_prefactor, point_geometry

# Default FFTLog bias bands: band boundaries in l and, per tracer kind, the b of
# each band (kind 0 clustering, kind 1 lensing, kind 2 CMB lensing).  Chosen by
# measuring the method error against direct quadrature on the 15-tracer workload
# (and that workload with a CMB-lensing tracer for the third row).
DEFAULT_BAND_ELL_LO = (0.0, 3.0, 6.0)
DEFAULT_FFTLOG_B = ((0.1, -0.2, -0.5), (-1.5, -2.0, -2.5), (-1.0, -1.0, -2.0))


class Method:
    """FFTLog settings shared by the oracle and the HIP path (by statement)."""

    def __init__(self, k, n_chi, m0=None, band_ell_lo=DEFAULT_BAND_ELL_LO,
                 fftlog_b=DEFAULT_FFTLOG_B, taper_frac=0.0):
        self.k = np.asarray(k, float)
        self.n_k = len(self.k)
        self.delta = float(np.log(self.k[-1] / self.k[0]) / (self.n_k - 1))
        self.n_chi = int(n_chi)
        self.m0 = default_edge_node(self.n_chi, self.delta) if m0 is None else int(m0)
        self.band_ell_lo = tuple(float(x) for x in band_ell_lo)
        self.fftlog_b = tuple(tuple(float(x) for x in row) for row in fftlog_b)
        self.taper_frac = float(taper_frac)

    def band(self, ell):
        return int(np.searchsorted(self.band_ell_lo, ell, side="right") - 1)

    def b_of(self, kind, ell):
        """Bias b of a tracer kind at multipole l.  A table with two rows gives CMB lensing (kind 2) the
        lensing row: its kernel has the lensing 1/chi behaviour at small chi."""
        row = self.fftlog_b[kind] if kind < len(self.fftlog_b) else self.fftlog_b[1]
        return row[self.band(ell)]


def default_edge_node(n_chi, delta, support_efolds=5.0):
    """Node index of chi(z_min): centres a support of `support_efolds` e-folds in the box."""
    return int(round(0.5 * (n_chi - support_efolds / delta)))


def chi_grid(geo: PointGeometry, method: Method):
    """chi_0 and the grid chi_m = chi_0 exp(m Delta), m = 0..N-1 (reading R4)."""
    chi0 = geo.chi_min * np.exp(-method.m0 * method.delta)
    return chi0, chi0 * np.exp(np.arange(method.n_chi) * method.delta)


def edge_weights(geo: PointGeometry, method: Method):
    """Support nodes m0..m1 of the kernels and their trapezoid weights per tracer, [T, m1-m0+1].

    Reading R5: 1/2 on the lower edge chi(z_min), 1/2 + theta on node m1 when chi(z_max) lies a
    fraction theta of a step above it (the kernel is cut there: a jump).  Reading R21: a CMB-lensing
    kernel falls linearly to zero at chi_*, a corner, so its last node below chi_* takes the weight
    of a linear end, 1/2 + theta_*/2, and the nodes above it weight 0.
    """
    chi0, _ = chi_grid(geo, method)
    N, m0, d = method.n_chi, method.m0, method.delta
    u_hi = np.log(geo.chi_max / chi0) / d
    m1 = int(np.floor(u_hi))
    theta = u_hi - m1
    if m0 < 1 or m1 >= N:
        raise ValueError("kernel support does not fit in the chi box")
    nodes = np.arange(m0, m1 + 1)
    w = np.ones(len(nodes))
    w[0] = 0.5
    w[-1] = 0.5 + theta if m1 > m0 else w[-1]
    W = np.repeat(w[None, :], len(geo.kinds), axis=0)
    cmb = np.nonzero(geo.kinds == 2)[0]
    if len(cmb):
        u_s = np.log(geo.chi_star / chi0) / d
        ms = int(np.floor(u_s))
        if ms > m0:
            W[cmb, ms - m0] = 0.5 + 0.5 * (u_s - ms)
            W[cmb, ms - m0 + 1:] = 0.0
    return nodes, W


def sampled_kernels(geo: PointGeometry, method: Method, rsd=False, mag=False, return_nodes=False):
    """Step 1: w_m f_t(chi_m) on the grid, with the edge weights of readings R5 and R21 (with
    rsd=True the RSD kernels of eq. RSD instead, with mag=True the magnification kernels).

    Returns (chi0, chi_m, F) with F of shape [T, N]; with return_nodes=True also the support nodes
    m0..m1 and their redshifts z(chi_m).
    """
    chi0, chi = chi_grid(geo, method)
    nodes, W = edge_weights(geo, method)
    T = len(geo.kinds)
    F = np.zeros((T, method.n_chi))
    z = np.empty(len(nodes))
    z[0] = geo.z_min  # node m0 sits on the lower edge by construction
    z[1:] = geo.z_of_chi(np.minimum(chi[nodes[1:]], geo.chi_max))
    for t in range(T):
        F[t, nodes] = W[t] * (geo.f_rsd_of_z(t, z) if rsd else (geo.f_mag_of_z(t, z) if mag else geo.f_of_z(t, z)))
    if return_nodes:
        return chi0, chi, F, nodes, z
    return chi0, chi, F


def taper(n, N, frac):
    """Cosine taper of reading R7: 1 below x0 = 1 - frac, 1/2 (1 + cos(pi (x-x0)/frac)) above, x = |n|/(N/2)."""
    x = np.abs(n) / (N / 2.0)
    if frac <= 0:
        return np.ones_like(x)
    x0 = 1.0 - frac
    return np.where(x <= x0, 1.0, 0.5 * (1.0 + np.cos(np.pi * np.clip((x - x0) / frac, 0, 1))))


def fftlog_coefficients(F, chi, chi0, b, method: Method):
    """Step 2: c_n = (1/N) sum_m f(chi_m) chi_m^-b chi_0^{-i eta_n} e^{-2 pi i n m/N}.

    Returns (n, c) with n = -N/2+1..N/2-1 and c of shape [T, N-1].
    """
    N = method.n_chi
    n = np.arange(-N // 2 + 1, N // 2)
    eta = 2.0 * np.pi * n / (N * method.delta)
    dft = np.fft.fft(F * chi[None, :] ** (-b), axis=1) / N  # index n mod N
    c = dft[:, n % N] * np.exp(-1j * eta * np.log(chi0))[None, :]
    return n, c * taper(n, N, method.taper_frac)[None, :]


def bessel_power_integral(ell, p, k):
    """Step 3 (eq. int_jl, corrected): int_0^inf dchi chi^p j_l(k chi)
    = 2^{p-1} k^{-1-p} sqrt(pi) Gamma((1+l+p)/2) / Gamma((2+l-p)/2),  -l-1 < Re p < 1.

    Broadcasts over p and k.
    """
    p = np.asarray(p, complex)
    k = np.asarray(k, float)
    log_val = ((p - 1.0) * np.log(2.0) - (1.0 + p) * np.log(k)
               + loggamma(0.5 * (1.0 + ell + p)) - loggamma(0.5 * (2.0 + ell - p)))
    return np.sqrt(np.pi) * np.exp(log_val)


def jl2_coefficients(ell):
    """j_l'' = a j_{l-2} + b j_l + c j_{l+2}: from j_l' = (l j_{l-1} - (l+1) j_{l+1}) / (2l+1)
    applied twice (valid for real l)."""
    a = ell * (ell - 1.0) / ((2.0 * ell - 1.0) * (2.0 * ell + 1.0))
    b = -(2.0 * ell * ell + 2.0 * ell - 1.0) / ((2.0 * ell - 1.0) * (2.0 * ell + 3.0))
    c = (ell + 1.0) * (ell + 2.0) / ((2.0 * ell + 1.0) * (2.0 * ell + 3.0))
    return a, b, c


def windows_point(geo: PointGeometry, ells, method: Method, rsd=False):
    """Step 4: W[l, t, j] = Delta_l^t(k_j) for one parameter point.  rsd=True adds the RSD term of
    the clustering tracers (eq. RSD): the same steps for the RSD kernels with the integral of
    chi^p j_l'' (three terms of eq. int_jl) in place of that of chi^p j_l.  A geometry with
    lensing-bias coefficients adds the magnification term (eq. magnification bias)."""
    chi0, chi, F = sampled_kernels(geo, method)
    FR = sampled_kernels(geo, method, rsd=True)[2] if rsd else None
    mag = geo.mag is not None
    FM = sampled_kernels(geo, method, mag=True)[2] if mag else None
    T = len(geo.kinds)
    W = np.zeros((len(ells), T, method.n_k))
    coeff = {}
    k = method.k
    N = method.n_chi
    for li, ell in enumerate(ells):
        for kind in (0, 1, 2):
            ts = np.nonzero(geo.kinds == kind)[0]
            if len(ts) == 0:
                continue
            b = method.b_of(kind, ell)
            if not (-ell - 1.0 < b < 1.0):
                raise ValueError(f"FFTLog bias b={b} outside (-l-1, 1) at l={ell}")
            if (kind, b) not in coeff:
                coeff[(kind, b)] = fftlog_coefficients(F[ts], chi, chi0, b, method)
            n, c = coeff[(kind, b)]
            p = b + 1j * 2.0 * np.pi * n / (N * method.delta)
            M = bessel_power_integral(ell, p[None, :], k[:, None])  # [Nk, N-1]
            delta_lk = M @ c.T  # [Nk, T_kind], imaginary part is rounding only
            if rsd and kind == 0:
                if ("rsd", b) not in coeff:
                    coeff[("rsd", b)] = fftlog_coefficients(FR[ts], chi, chi0, b, method)
                cr = coeff[("rsd", b)][1]
                a2, a0, a4 = jl2_coefficients(ell)
                MR = sum(ai * bessel_power_integral(s, p[None, :], k[:, None])
                         for ai, s in ((a2, ell - 2.0), (a0, ell), (a4, ell + 2.0)))
                delta_lk = delta_lk + MR @ cr.T
            W[li, ts, :] = (delta_lk.real * ell_prefactor(kind, ell, k)[:, None]).T
            if mag and kind == 0:
                # magnification: a lensing-type kernel with prefactor l(l+1)/k^2, decomposed with the
                # bias b - 2 (reading R20)
                bm = b - 2.0
                if ("mag", bm) not in coeff:
                    coeff[("mag", bm)] = fftlog_coefficients(FM[ts], chi, chi0, bm, method)
                cm = coeff[("mag", bm)][1]
                pm = bm + 1j * 2.0 * np.pi * n / (N * method.delta)
                dm = bessel_power_integral(ell, pm[None, :], k[:, None]) @ cm.T
                W[li, ts, :] += (dm.real * (ell * (ell + 1.0) / k ** 2)[:, None]).T
    return W


def k_weights(method: Method):
    """Reading R8: (2/pi) Delta (1/2 at both ends) times k^3."""
    w = np.full(method.n_k, method.delta)
    w[0] *= 0.5
    w[-1] *= 0.5
    return (2.0 / np.pi) * w * method.k ** 3


def pack_upper(C):
    """[..., T, T] -> [..., T(T+1)/2], pairs (i, j) with i <= j in row-major order."""
    T = C.shape[-1]
    iu = np.triu_indices(T)
    return C[..., iu[0], iu[1]]


def cl_from_windows(W, pk, method: Method):
    """Step 5: C_l^{ij} = sum_j w_j k_j^3 P_j W_i W_j, packed upper triangle [L, T(T+1)/2]."""
    s = k_weights(method) * np.asarray(pk, float)
    C = np.einsum("ltj,lsj,j->lts", W, W, s)
    return pack_upper(C)


def method_for(wl, **kw):
    return Method(wl["k"], wl["n_chi"], **kw)


def point_ells(wl, b):
    return wl["ell"][wl["ell_idx"][b, :wl["n_ell"][b]]]


def windows(wl, b, method=None):
    method = method or method_for(wl)
    return windows_point(point_geometry(wl, b), point_ells(wl, b), method, rsd=bool(wl.get("rsd", False)))


def cl(wl, b, method=None, return_windows=False):
    """C_l for point b of a workload: [L_b, T_b(T_b+1)/2] (FP64)."""
    method = method or method_for(wl)
    W = windows(wl, b, method)
    C = cl_from_windows(W, wl["pk"][b], method)
    return (C, W) if return_windows else C
