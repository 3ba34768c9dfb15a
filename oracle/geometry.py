"""Radial kernels f_i(chi) from sampled inputs (oracle; FP64; test infrastructure).

Paper, Sec. 2.2 (galaxy clustering) and Sec. 2.3 (weak lensing):
  clustering   Delta_l^{g,D}(k) = b_1 int dchi W^{delta,g}(chi) D j_l(k chi),
               W^{delta,g}(chi) = n(z(chi)), with int dz n = 1.  The chi integral
               needs dz/dchi, so the radial kernel is f = b n(z) (dz/dchi) D(z).
  lensing      Delta_l^gamma(k) = sqrt((l+2)!/(l-2)!) k^-2 int dchi chi^-2 W^{kappa,gamma} D j_l,
               W^{kappa,gamma}(chi) = (3 Om H0^2 / 2 c^2) int_chi^inf dchi' n(chi') (chi/a) (chi'-chi)/chi'
               (eq. tomographic lens efficiency).  Written in z:
               q(chi) = 1.5 Om (H0/c)^2 chi (1+z) int_z^{z_max} dz' n(z') (1 - chi/chi(z')).
               The radial kernel is f = q D / chi^2 and c(l, k) = F(l) / k^2.
  CMB lensing  (Sec. 2.4) Delta_l^{CMB,kappa}(k) = l(l+1) (3 Om H0^2 / 2 c^2 k^2)
               int_0^{chi_*} dchi a^-1 (chi_* - chi) / (chi chi_*) D j_l(k chi): the lensing kernel
               of one source plane at chi_*, f = 1.5 Om (H0/c)^2 (1+z) (chi_* - chi) / (chi chi_*) D,
               with the convergence prefactor c(l, k) = l(l+1) / k^2 in place of F(l) / k^2.

Readings (the paper does not fix them):
  * every sampled input is continued by a natural cubic spline; n(z) is zero
    outside its sample range;
  * z(chi) is the inverse of the chi(z) spline, dz/dchi = 1 / (chi spline)';
  * the kernels are supported on [chi(z_min), chi(z_max)] of the geometry grid;
  * D(k, z) = D(z), z_fid = 0 (linear growth);
  * the last-scattering surface z_* of a CMB-lensing tracer is given with the geometry, by default
    the top of its grid; the kernel is zero above it.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline, PPoly

H0_OVER_C = 1.0 / 2997.92458  # h/Mpc
KIND_CLUSTERING, KIND_LENSING, KIND_CMB_LENSING = 0, 1, 2
_GL = np.polynomial.legendre.leggauss(12)


class PointGeometry:
    """Continuous geometry, growth and redshift distributions of one parameter point."""

    def __init__(self, z_geom, chi_z, D_z, omega_m, z_nz, nz, kinds, bias, ia=None, mag=None, z_star=None):
        self.z_geom = np.asarray(z_geom, float)
        self.z_nz = np.asarray(z_nz, float)
        self.chi_spl = CubicSpline(self.z_geom, chi_z, bc_type="natural")
        self.D_spl = CubicSpline(self.z_geom, D_z, bc_type="natural")
        # NLA amplitude A_IA(z) of the lensing tracers (Sec. 2.3), None = no intrinsic alignment
        self.ia_spl = None if ia is None else CubicSpline(self.z_geom, ia, bc_type="natural")
        # lensing-bias coefficients C_g of the clustering tracers (eq. magnification bias), or None
        self.mag = None if mag is None else np.asarray(mag, float)
        self.nz = np.asarray(nz, float)
        self.n_spl = [CubicSpline(self.z_nz, n_t, bc_type="natural") for n_t in self.nz]
        self.omega_m = float(omega_m)
        self.kinds = np.asarray(kinds, int)
        self.bias = np.asarray(bias, float)
        self.z_min, self.z_max = self.z_geom[0], self.z_geom[-1]
        self.chi_min = float(self.chi_spl(self.z_min))
        self.chi_max = float(self.chi_spl(self.z_max))
        # source plane of the CMB-lensing tracers (Sec. 2.4)
        self.z_star = self.z_max if z_star is None else float(z_star)
        if not self.z_min < self.z_star <= self.z_max:
            raise ValueError("z_star must lie inside the geometry grid")
        self.chi_star = float(self.chi_spl(self.z_star))
        self._lens_tables = {}

    # --- elementary continuous functions -------------------------------------------------
    def n_of_z(self, t, z):
        z = np.asarray(z, float)
        inside = (z >= self.z_nz[0]) & (z <= self.z_nz[-1])
        return np.where(inside, self.n_spl[t](np.clip(z, self.z_nz[0], self.z_nz[-1])), 0.0)

    def z_of_chi(self, chi):
        """Invert the chi(z) spline on the geometry range (one root per value).

        The root is that of the cubic piece whose end values bracket chi (the spline's values at
        the knots are the chi samples, increasing); should that piece not give exactly one root,
        the whole spline is solved and must give exactly one."""
        chi = np.atleast_1d(np.asarray(chi, float))
        out = np.empty_like(chi)
        knots = self.chi_spl.x
        at_knots = self.chi_spl(knots)
        for i, c in enumerate(chi):
            j = int(np.clip(np.searchsorted(at_knots, c, side="right") - 1, 0, len(knots) - 2))
            piece = PPoly(self.chi_spl.c[:, j:j + 1], knots[j:j + 2])
            r = piece.solve(c, extrapolate=False)
            if len(r) != 1:
                r = self.chi_spl.solve(c, extrapolate=False)
                r = r[(r >= self.z_min - 1e-12) & (r <= self.z_max + 1e-12)]
                if len(r) != 1:
                    raise ValueError(f"chi={c} is not inside the geometry range")
            out[i] = r[0]
        return out

    # --- lensing efficiency ----------------------------------------------------------------
    def _knots(self):
        return np.union1d(self.z_geom, self.z_nz[(self.z_nz >= self.z_min) & (self.z_nz <= self.z_max)])

    def lensing_integrals(self, t, z):
        """I0(z) = int_z^zmax n_t dz',  I1(z) = int_z^zmax n_t / chi(z') dz'.

        Gauss-Legendre (12 points) on every interval between consecutive knots
        of the geometry and n(z) grids, where the integrand is smooth; the
        interval holding z is integrated from z to its right end.
        """
        knots = self._knots()
        x, w = _GL
        a, b = knots[:-1, None], knots[1:, None]
        nodes = 0.5 * (b - a) * x + 0.5 * (a + b)
        wts = 0.5 * (b - a) * w
        nv = self.n_of_z(t, nodes)
        seg0 = np.sum(wts * nv, axis=1)
        seg1 = np.sum(wts * nv / self.chi_spl(nodes), axis=1)
        suf0 = np.concatenate([np.cumsum(seg0[::-1])[::-1], [0.0]])
        suf1 = np.concatenate([np.cumsum(seg1[::-1])[::-1], [0.0]])
        z = np.atleast_1d(np.asarray(z, float))
        i = np.clip(np.searchsorted(knots, z, side="right") - 1, 0, len(knots) - 2)
        hi = knots[i + 1]
        pn = 0.5 * (hi - z)[:, None] * x + 0.5 * (hi + z)[:, None]
        pw = 0.5 * (hi - z)[:, None] * w
        pv = self.n_of_z(t, pn)
        I0 = np.sum(pw * pv, axis=1) + suf0[i + 1]
        I1 = np.sum(pw * pv / self.chi_spl(pn), axis=1) + suf1[i + 1]
        return I0, I1

    def lensing_q(self, t, z):
        """q_t at redshift z (units h^2/Mpc^2 * Mpc/h); eq. tomographic lens efficiency in z."""
        z = np.atleast_1d(np.asarray(z, float))
        chi = self.chi_spl(z)
        I0, I1 = self.lensing_integrals(t, z)
        return 1.5 * self.omega_m * H0_OVER_C ** 2 * chi * (1.0 + z) * (I0 - chi * I1)

    def growth_rate(self, z):
        """f(z) = dln D / dln a = -(1+z) D'(z) / D(z), from the D(z) spline."""
        z = np.atleast_1d(np.asarray(z, float))
        return -(1.0 + z) * self.D_spl(z, 1) / self.D_spl(z)

    def f_rsd_of_z(self, t, z):
        """Radial kernel of the RSD term of clustering tracer t (eq. RSD), per unit chi:
        -f(z) n(z) dz/dchi D(z); it multiplies j_l'' instead of j_l.  Zero for lensing tracers."""
        z = np.atleast_1d(np.asarray(z, float))
        if self.kinds[t] != 0:
            return np.zeros_like(z)
        return -self.growth_rate(z) * self.n_of_z(t, z) * self.D_spl(z) / self.chi_spl(z, 1)

    def f_mag_of_z(self, t, z):
        """Radial kernel of the magnification term of clustering tracer t (eq. magnification bias),
        per unit chi: C_g q_t(z) D / chi^2 with q_t the lens efficiency of the tracer's own n(z); its
        prefactor is l(l+1)/k^2.  Zero for lensing tracers or without magnification."""
        z = np.atleast_1d(np.asarray(z, float))
        if self.mag is None or self.kinds[t] != 0:
            return np.zeros_like(z)
        return self.mag[t] * self.lensing_q(t, z) * self.D_spl(z) / self.chi_spl(z) ** 2

    def cmb_kernel(self, z):
        """CMB-lensing kernel per unit chi (Sec. 2.4, without l(l+1)/k^2):
        1.5 Om (H0/c)^2 (1+z) (chi_* - chi) / (chi chi_*) D(z), zero above z_*."""
        z = np.atleast_1d(np.asarray(z, float))
        chi = self.chi_spl(z)
        f = 1.5 * self.omega_m * H0_OVER_C ** 2 * (1.0 + z) * (self.chi_star - chi) / (chi * self.chi_star)
        return np.where(z <= self.z_star, f * self.D_spl(z), 0.0)

    def ia_of_z(self, z):
        """A_IA(z), 0 without intrinsic alignment."""
        z = np.atleast_1d(np.asarray(z, float))
        return np.zeros_like(z) if self.ia_spl is None else self.ia_spl(z)

    # --- radial kernels ------------------------------------------------------------------
    def f_of_z(self, t, z):
        """Radial kernel per unit chi, f_t, evaluated at redshift z (inside the support).

        Lensing tracers carry the NLA term of Sec. 2.3: the window of intrinsic alignment has the
        lensing prefactor and 1/chi^2 with n(chi) A_IA(z) in place of the lens efficiency, so
        f = (q + A_IA n dz/dchi) D / chi^2.
        """
        z = np.atleast_1d(np.asarray(z, float))
        D = self.D_spl(z)
        dzdchi = 1.0 / self.chi_spl(z, 1)
        if self.kinds[t] == KIND_CLUSTERING:
            return self.bias[t] * self.n_of_z(t, z) * dzdchi * D
        if self.kinds[t] == KIND_CMB_LENSING:
            return self.cmb_kernel(z)
        chi = self.chi_spl(z)
        return (self.lensing_q(t, z) + self.ia_of_z(z) * self.n_of_z(t, z) * dzdchi) * D / chi ** 2

    def f_of_chi(self, t, chi):
        """f_t(chi), zero outside [chi(z_min), chi(z_max)]."""
        chi = np.atleast_1d(np.asarray(chi, float))
        out = np.zeros_like(chi)
        inside = (chi >= self.chi_min) & (chi <= self.chi_max)
        if np.any(inside):
            z = self.z_of_chi(chi[inside])
            out[inside] = self.f_of_z(t, z)
        return out


def point_geometry(wl, b):
    """PointGeometry of parameter point b of a synthetic workload dict."""
    T = int(wl["n_tracers"][b])
    ia, mag = wl.get("ia"), wl.get("mag")
    return PointGeometry(wl["z_geom"], wl["chi_z"][b], wl["D_z"][b], wl["omega_m"][b], wl["z_nz"],
                         wl["nz"][b, :T], wl["kind"][b, :T], wl["bias"][b, :T],
                         ia=None if ia is None else ia[b], mag=None if mag is None else mag[b, :T],
                         z_star=wl.get("z_star"))


def ell_prefactor(kind, ell, k):
    """c(l, k): 1 for clustering, sqrt((l+2)!/(l-2)!) / k^2 for lensing, l(l+1) / k^2 for CMB
    lensing (real l)."""
    if kind == KIND_CLUSTERING:
        return np.ones_like(np.asarray(k, float))
    if kind == KIND_CMB_LENSING:
        return ell * (ell + 1.0) / np.asarray(k, float) ** 2
    F = np.sqrt((ell + 2.0) * (ell + 1.0) * ell * (ell - 1.0))
    return F / np.asarray(k, float) ** 2
