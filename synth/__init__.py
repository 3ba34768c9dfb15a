"""Seeded synthetic inputs for the beyond-Limber C_l hot path.

This module only *generates inputs*: the background tables chi(z) and D(z),
redshift distributions n(z), linear biases, the linear matter power spectrum
P(k) on a log-spaced k grid and the multipole list.  It holds none of the
method's arithmetic (no FFTLog, no Bessel integrals, no projection), so both
the oracle and the HIP path may consume what it produces.

Units: k in h/Mpc, chi in Mpc/h, P in (Mpc/h)^3, c/H0 = 2997.92458 Mpc/h.
Radiation is neglected in E(z) (flat LCDM).

Workloads (the paper's N5K 3x2pt set-up of Sec. 4.2 is reproduced in shape
only; its benchmark files are not used):
  cfg0  2 Gaussian clustering bins, 256 k, N_chi 512, 20 l in [2, 200], FP64
  cfg1  10 clustering + 5 lensing bins, 1024 k, N_chi 1024, 103 l in [2, 2000]
  cfg2  cfg1 with biases scaled by U(0.9, 1.1)
  cfg3  256 points, per-point cosmology, ragged tracer / multipole counts
  cfg4  20 clustering + 10 lensing bins, 2048 k, N_chi 2048, 200 l in [2, 3000]

scale_dependent_growth() adds growth samples D(k, z) at interpolation nodes in k to any of them,
intrinsic_alignment() an NLA amplitude A_IA(z) for the lensing tracers, cmb_lensing() a CMB-lensing
tracer with the geometry continued to the last-scattering surface.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, optimize, special

C_OVER_H0 = 2997.92458  # Mpc/h
Z_MIN, Z_MAX = 0.01, 3.0
N_ZGEOM = 1024
N_ZNZ = 200
KIND_CLUSTERING = 0
KIND_LENSING = 1
KIND_CMB_LENSING = 2

_GL8 = np.polynomial.legendre.leggauss(8)


def e_of_z(z, om):
    z = np.asarray(z, float)
    return np.sqrt(om * (1.0 + z) ** 3 + (1.0 - om))


def _cumulative_gl(fn, edges):
    """Cumulative integral of fn over consecutive intervals of `edges` (8-point GL each)."""
    x, w = _GL8
    a = edges[:-1, None]
    b = edges[1:, None]
    nodes = 0.5 * (b - a) * x[None, :] + 0.5 * (a + b)
    vals = fn(nodes)
    seg = np.sum(0.5 * (b - a) * w[None, :] * vals, axis=1)
    return np.concatenate([[0.0], np.cumsum(seg)])


def comoving_distance(z, om, refine=8):
    """chi(z) = (c/H0) int_0^z dz'/E(z') on a sorted z array (FP64)."""
    z = np.asarray(z, float)
    edges = np.concatenate([[0.0], z])
    # refine each interval so the 8-point rule is far below FP64 noise
    fine = np.concatenate([np.linspace(edges[i], edges[i + 1], refine + 1)[:-1]
                           for i in range(len(edges) - 1)] + [[edges[-1]]])
    cum = _cumulative_gl(lambda zz: 1.0 / e_of_z(zz, om), fine)
    return C_OVER_H0 * cum[::refine][1:]


def growth_factor(z, om, refine=8):
    """Linear growth D(z) normalised to D(0) = 1 (Heath integral, flat LCDM).

    D(a) is proportional to E(a) int_0^a da' / (a' E(a'))^3; in terms of a the
    integrand is a'^1.5 / (Om + (1-Om) a'^3)^1.5, regular at a' = 0.
    """
    z = np.asarray(z, float)
    a = 1.0 / (1.0 + z)
    order = np.argsort(a)
    a_sorted = a[order]
    edges = np.concatenate([[0.0], a_sorted, [1.0]])
    fine = np.concatenate([np.linspace(edges[i], edges[i + 1], refine + 1)[:-1]
                           for i in range(len(edges) - 1)] + [[1.0]])
    ol = 1.0 - om
    cum = _cumulative_gl(lambda aa: aa ** 1.5 / (om + ol * aa ** 3) ** 1.5, fine)
    cum = cum[::refine]
    i_at = np.empty_like(a)
    i_at[order] = cum[1:-1]
    i_one = cum[-1]
    return (e_of_z(z, om) * i_at) / (e_of_z(0.0, om) * i_one)


def interpolation_nodes(k, n_interp):
    """The k nodes of scale-dependent growth: n_interp points uniform in ln k from k[0] to k[-1]."""
    k = np.asarray(k, float)
    return np.exp(np.linspace(np.log(k[0]), np.log(k[-1]), int(n_interp)))


def scale_dependent_growth(wl, n_interp, f_nu=0.05, k_fs=0.1):
    """Add D(k, z) samples of a massive-neutrino-like growth suppression to workload wl.

    Below the free-streaming scale k_fs growth is the scale-free D(z); far above it the growth
    exponent is lowered by 3 f_nu / 5, so D(k, z) = D(z)^(1 - 3 f_nu / 5 * k^2 / (k^2 + k_fs^2)),
    which keeps D(k, 0) = 1.  Adds k_nodes[n_interp] and D_kz[B, n_interp, nzg] (samples on the
    geometry z grid at each node); returns wl.
    """
    kn = interpolation_nodes(wl["k"], n_interp)
    supp = 0.6 * f_nu * kn ** 2 / (kn ** 2 + k_fs ** 2)
    D = np.asarray(wl["D_z"], float)
    wl["n_interp"] = int(n_interp)
    wl["k_nodes"] = kn
    wl["D_kz"] = np.ascontiguousarray(D[:, None, :] ** (1.0 - supp[None, :, None]))
    return wl


def intrinsic_alignment(wl, a1=0.5):
    """Add the NLA amplitude of the lensing tracers, A_IA(z) = -a1 C1 rho_crit Omega_m / D(z) with
    C1 rho_crit = 0.0134 (the usual normalisation of the non-linear alignment model), sampled on the
    geometry z grid: wl["ia"] [B, nzg].  Returns wl."""
    om = np.asarray(wl["omega_m"], float)
    wl["ia"] = np.ascontiguousarray(-a1 * 0.0134 * om[:, None] / np.asarray(wl["D_z"], float))
    return wl


def magnification_bias(wl):
    """Add the lensing-bias coefficient C_g = 5 s - 2 of the clustering tracers (eq. magnification
    bias), with a number-count slope s rising from 0.2 to 0.6 over the bins in order: wl["mag"]
    [B, T], zero for lensing tracers.  Returns wl."""
    kinds = np.asarray(wl["kind"])
    mag = np.zeros(kinds.shape)
    for b in range(kinds.shape[0]):
        cl = np.nonzero(kinds[b] == KIND_CLUSTERING)[0]
        s = np.linspace(0.2, 0.6, max(len(cl), 1))[:len(cl)]
        mag[b, cl] = 5.0 * s - 2.0
    wl["mag"] = mag
    return wl


def cmb_lensing(wl, z_star=1090.0, n_high=256):
    """Add a CMB-lensing tracer (kind 2) to every point of workload wl, after its last tracer.

    The geometry grid is continued from its top to the last-scattering redshift z_star by n_high
    points uniform in ln(1 + z), and chi(z), D(z) are recomputed on it for each point's Omega_m
    (flat LCDM without radiation, as everywhere here); the tracer's n(z) row is zero and its bias 1.
    Adds z_star; returns wl.  Apply it before the modifiers that add per-grid or per-tracer samples.
    """
    for key in ("ia", "mag", "D_kz"):
        if key in wl:
            raise ValueError(f"cmb_lensing() must run before the workload gets {key!r}")
    z_lo = np.asarray(wl["z_geom"], float)
    if not z_star > z_lo[-1]:
        raise ValueError("z_star must lie above the geometry grid")
    z_hi = np.expm1(np.linspace(np.log1p(z_lo[-1]), np.log1p(z_star), n_high + 1))[1:]
    z_hi[-1] = z_star
    z_geom = np.concatenate([z_lo, z_hi])
    om = np.asarray(wl["omega_m"], float)
    B, T = np.asarray(wl["kind"]).shape
    ntr = np.asarray(wl["n_tracers"], np.int32)
    nz = np.zeros((B, T + 1, np.asarray(wl["nz"]).shape[2]))
    kinds = np.zeros((B, T + 1), np.int32)
    bias = np.ones((B, T + 1))
    nz[:, :T] = wl["nz"]
    kinds[:, :T] = wl["kind"]
    bias[:, :T] = wl["bias"]
    for b in range(B):
        t = int(ntr[b])
        nz[b, t:] = 0.0
        kinds[b, t:] = 0
        bias[b, t:] = 1.0
        nz[b, t + 1:T + 1] = np.asarray(wl["nz"])[b, t:T]
        kinds[b, t + 1:T + 1] = np.asarray(wl["kind"])[b, t:T]
        bias[b, t + 1:T + 1] = np.asarray(wl["bias"])[b, t:T]
        kinds[b, t] = KIND_CMB_LENSING
    wl.update(z_geom=z_geom, chi_z=np.array([comoving_distance(z_geom, o) for o in om]),
              D_z=np.array([growth_factor(z_geom, o) for o in om]), nz=nz, kind=kinds, bias=bias,
              n_tracers=ntr + 1, z_star=float(z_star))
    return wl


def bbks_transfer(q):
    """BBKS fitting form (Bardeen, Bond, Kaiser & Szalay 1986, eq. G3), q = k / Gamma."""
    q = np.asarray(q, float)
    return (np.log1p(2.34 * q) / (2.34 * q)
            * (1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25)


def linear_pk(k, om, h, sigma8, ns=1.0):
    """P(k) = A k^ns T_BBKS(k/Gamma)^2, Gamma = Om h, A fixed by sigma8 (top hat, R = 8 Mpc/h)."""
    gamma = om * h

    def shape(kk):
        return kk ** ns * bbks_transfer(kk / gamma) ** 2

    def integrand(lnk):
        kk = np.exp(lnk)
        x = 8.0 * kk
        wth = 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3
        return kk ** 3 * shape(kk) * wth ** 2 / (2.0 * np.pi ** 2)

    s2 = integrate.quad(integrand, np.log(1e-5), np.log(1e3), limit=500, epsabs=0, epsrel=1e-12)[0]
    return sigma8 ** 2 / s2 * shape(np.asarray(k, float))


def gaussian_nz(z, zc, sigma):
    """Gaussian n(z) normalised to unit integral over [Z_MIN, Z_MAX]."""
    z = np.asarray(z, float)
    norm = sigma * np.sqrt(np.pi / 2.0) * (special.erf((Z_MAX - zc) / (np.sqrt(2) * sigma))
                                           - special.erf((Z_MIN - zc) / (np.sqrt(2) * sigma)))
    return np.exp(-0.5 * ((z - zc) / sigma) ** 2) / norm


def _smail(z):
    return z ** 2 * np.exp(-(z / 0.28) ** 0.9)


def smail_edges(nbins):
    """Equal-count bin edges of the true-redshift Smail distribution on [Z_MIN, Z_MAX]."""
    total = integrate.quad(_smail, Z_MIN, Z_MAX, epsabs=0, epsrel=1e-13, limit=200)[0]
    edges = [Z_MIN]
    for i in range(1, nbins):
        target = total * i / nbins
        edges.append(optimize.brentq(
            lambda zz: integrate.quad(_smail, Z_MIN, zz, epsabs=0, epsrel=1e-13, limit=200)[0] - target,
            Z_MIN, Z_MAX, xtol=1e-14))
    edges.append(Z_MAX)
    return np.array(edges)


def smail_bin_nz(z, za, zb):
    """Photo-z binned Smail n(z) (sigma_z = 0.05(1+z)), normalised on [Z_MIN, Z_MAX]."""
    def raw(zz):
        s = 0.05 * (1.0 + zz)
        return _smail(zz) * 0.5 * (special.erf((zb - zz) / (np.sqrt(2) * s))
                                   - special.erf((za - zz) / (np.sqrt(2) * s)))
    norm = integrate.quad(raw, Z_MIN, Z_MAX, epsabs=0, epsrel=1e-13, limit=400)[0]
    return raw(np.asarray(z, float)) / norm


def tracer_set(n_clust, n_lens, z_nz, zc_range=(0.2, 1.2)):
    """n(z) samples, kinds and fiducial biases for n_clust Gaussian + n_lens Smail bins."""
    nz, kinds, bias = [], [], []
    for zc in (np.linspace(*zc_range, n_clust) if n_clust > 1 else [zc_range[0]]):
        nz.append(gaussian_nz(z_nz, zc, 0.05 * (1 + zc)))
        kinds.append(KIND_CLUSTERING)
        bias.append(1.0 + 0.84 * zc)
    if n_lens:
        e = smail_edges(n_lens)
        for i in range(n_lens):
            nz.append(smail_bin_nz(z_nz, e[i], e[i + 1]))
            kinds.append(KIND_LENSING)
            bias.append(1.0)  # unused for lensing tracers
    return np.array(nz), np.array(kinds, np.int32), np.array(bias)


def _points(n, seed, om_range, s8_range, bias_scale):
    rng = np.random.default_rng(seed)
    om = rng.uniform(*om_range, n) if n > 1 or om_range[0] != om_range[1] else np.full(n, om_range[0])
    s8 = rng.uniform(*s8_range, n) if n > 1 or s8_range[0] != s8_range[1] else np.full(n, s8_range[0])
    return rng, om, s8


def make_workload(name, batch=None, seed=None):
    """Return a dict of host arrays describing one synthetic workload.

    Keys: z_geom[nzg], chi_z[B,nzg], D_z[B,nzg], omega_m[B], z_nz[nzs],
    nz[B,T,nzs], bias[B,T], kind[B,T], n_tracers[B], k[Nk], pk[B,Nk],
    ell[L_union], n_ell[B], ell_idx[B,Lmax], n_chi, precision, label.
    """
    h = 0.7
    z_geom = np.linspace(Z_MIN, Z_MAX, N_ZGEOM)
    z_nz = np.linspace(Z_MIN, Z_MAX, N_ZNZ)
    out = {"z_geom": z_geom, "z_nz": z_nz, "h": h}

    if name == "cfg0":
        B = 1 if batch is None else batch
        nz1 = np.array([gaussian_nz(z_nz, 0.5, 0.1), gaussian_nz(z_nz, 1.0, 0.1)])
        kinds1 = np.array([KIND_CLUSTERING, KIND_CLUSTERING], np.int32)
        bias1 = np.array([1.5, 2.0])
        k = np.geomspace(1e-4, 10.0, 256)
        ells = [np.geomspace(2.0, 200.0, 20)] * B
        om = np.full(B, 0.3)
        s8 = np.full(B, 0.8)
        nz = np.repeat(nz1[None], B, 0)
        kinds = np.repeat(kinds1[None], B, 0)
        bias = np.repeat(bias1[None], B, 0)
        ntr = np.full(B, 2, np.int32)
        out.update(n_chi=512, precision="fp64")
    elif name in ("cfg1", "cfg2", "cfg1_batch"):
        B = 1 if batch is None else batch
        nz1, kinds1, bias1 = tracer_set(10, 5, z_nz)
        k = np.geomspace(1e-4, 10.0, 1024)
        ells = [np.geomspace(2.0, 2000.0, 103)] * B
        nz = np.repeat(nz1[None], B, 0)
        kinds = np.repeat(kinds1[None], B, 0)
        bias = np.repeat(bias1[None], B, 0).copy()
        ntr = np.full(B, 15, np.int32)
        if name == "cfg1_batch":
            rng = np.random.default_rng(1 if seed is None else seed)
            om = rng.uniform(0.25, 0.35, B)
            s8 = rng.uniform(0.7, 0.9, B)
            bias[:, :10] *= rng.uniform(0.8, 1.2, (B, 10))
        else:
            om = np.full(B, 0.3)
            s8 = np.full(B, 0.8)
        if name == "cfg2":
            rng = np.random.default_rng(2 if seed is None else seed)
            bias[:, :10] *= rng.uniform(0.9, 1.1, (B, 10))
        out.update(n_chi=1024, precision="fp32")
    elif name == "cfg3":
        B = 256 if batch is None else batch
        rng = np.random.default_rng(3 if seed is None else seed)
        om = rng.uniform(0.25, 0.35, B)
        s8 = rng.uniform(0.7, 0.9, B)
        full_nz, full_kinds, full_bias = tracer_set(10, 5, z_nz)
        choice = rng.choice([6, 10, 15], B)
        n_ell = rng.integers(50, 104, B)
        bscale = rng.uniform(0.8, 1.2, (B, 10))
        T = 15
        nz = np.zeros((B, T, N_ZNZ))
        kinds = np.zeros((B, T), np.int32)
        bias = np.ones((B, T))
        ntr = choice.astype(np.int32)
        for b in range(B):
            if choice[b] == 6:
                sel = [0, 1, 2, 3, 10, 11]
            elif choice[b] == 10:
                sel = list(range(10))
            else:
                sel = list(range(15))
            nz[b, :len(sel)] = full_nz[sel]
            kinds[b, :len(sel)] = full_kinds[sel]
            bias[b, :len(sel)] = full_bias[sel]
            for i, s in enumerate(sel):
                if s < 10:
                    bias[b, i] *= bscale[b, s]
        k = np.geomspace(1e-4, 10.0, 1024)
        ells = [np.geomspace(2.0, 2000.0, int(L)) for L in n_ell]
        out.update(n_chi=1024, precision="fp32")
    elif name == "cfg4":
        B = 64 if batch is None else batch
        rng = np.random.default_rng(4 if seed is None else seed)
        om = rng.uniform(0.25, 0.35, B)
        s8 = rng.uniform(0.7, 0.9, B)
        nz1, kinds1, bias1 = tracer_set(20, 10, z_nz)
        nz = np.repeat(nz1[None], B, 0)
        kinds = np.repeat(kinds1[None], B, 0)
        bias = np.repeat(bias1[None], B, 0).copy()
        bias[:, :20] *= rng.uniform(0.8, 1.2, (B, 20))
        ntr = np.full(B, 30, np.int32)
        k = np.geomspace(1e-4, 10.0, 2048)
        ells = [np.geomspace(2.0, 3000.0, 200)] * B
        out.update(n_chi=2048, precision="split_bf16")
    else:
        raise ValueError(f"unknown workload {name!r}")

    chi = np.array([comoving_distance(z_geom, o) for o in om])
    dz = np.array([growth_factor(z_geom, o) for o in om])
    pk = np.array([linear_pk(k, o, h, s) for o, s in zip(om, s8)])
    # union of the multipole lists, and each point's indices into it
    union = np.unique(np.concatenate(ells))
    lmax = max(len(e) for e in ells)
    ell_idx = np.zeros((B, lmax), np.int32)
    for b, e in enumerate(ells):
        ell_idx[b, :len(e)] = np.searchsorted(union, e)
    out.update(chi_z=chi, D_z=dz, omega_m=np.asarray(om, float), nz=nz, bias=bias, kind=kinds,
               n_tracers=ntr, k=k, pk=pk, ell=union, n_ell=np.array([len(e) for e in ells], np.int32),
               ell_idx=ell_idx, label=name, batch=B)
    return out
