"""Pins of the oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: independent
numerical quadrature (mpmath), an explicit O(N^2) DFT, the exact integral by
direct quadrature, the Limber limit, closed-form invariants and finite
differences.
"""
import mpmath
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import fftlog, geometry, gradients, limber, quadrature


# --- eq. int_jl (corrected denominator) -------------------------------------------------------

def _mp_power_bessel(ell, p):
    """int_0^inf x^p j_l(x) dx by mpmath oscillatory quadrature (30 digits)."""
    mpmath.mp.dps = 30
    p = mpmath.mpc(p)
    f = lambda x: x ** p * mpmath.sqrt(mpmath.pi / (2 * x)) * mpmath.besselj(ell + 0.5, x)
    return complex(mpmath.quadosc(f, [0, mpmath.inf], omega=1))


@pytest.mark.parametrize("p", [0.5, -0.3, 0.2 + 4j, -0.7 - 1.5j])
def test_power_bessel_integral_ell0_mellin_sine(p):
    """l = 0: j_0(x) = sin(x)/x and int_0^inf x^{p-1} sin x dx = Gamma(p) sin(pi p / 2), -1 < Re p < 1."""
    from scipy.special import gamma
    k = 1.7
    ref = complex(gamma(p) * np.sin(np.pi * p / 2)) * k ** (-1 - p)
    got = complex(fftlog.bessel_power_integral(0.0, p, k))
    assert abs(got - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("ell,p", [(2.0, -0.5), (7.3, -0.9), (2.0, 0.1 + 3j),
                                   (10.5, -2.0 + 5j), (3.0, -1.5 - 2j)])
def test_power_bessel_integral_matches_quadrature(ell, p):
    k = 2.0
    ref = _mp_power_bessel(ell, p) * k ** (-1 - p)  # substitution x = k chi
    got = complex(fftlog.bessel_power_integral(ell, p, k))
    # oscillatory quadrature converges slowly when the integrand decays slowly (Re p near 1)
    tol = 1e-10 if np.real(p) <= -0.5 else 1e-6
    assert abs(got - ref) <= tol * abs(ref)


def test_printed_denominator_is_a_typo():
    """The printed Gamma((2+l+p)/2) misses the quadrature value: the oracle uses (2+l-p)/2."""
    ell, p = 2.0, -0.5
    ref = _mp_power_bessel(ell, p)
    from scipy.special import gamma
    printed = 2 ** (p - 1) * np.sqrt(np.pi) * gamma(0.5 * (1 + ell + p)) / gamma(0.5 * (2 + ell + p))
    assert abs(printed - ref.real) > 0.05 * abs(ref)
    assert abs(fftlog.bessel_power_integral(ell, p, 1.0) - ref) < 1e-10 * abs(ref)


# --- the DFT step ---------------------------------------------------------------------------------

def test_fftlog_coefficients_brute_force():
    rng = np.random.default_rng(0)
    N = 32
    k = np.geomspace(1e-3, 1.0, 20)
    m = fftlog.Method(k, N, m0=4)
    chi0 = 3.0
    chi = chi0 * np.exp(np.arange(N) * m.delta)
    F = rng.standard_normal((2, N))
    b = -0.3
    n, c = fftlog.fftlog_coefficients(F, chi, chi0, b, m)
    for t in range(2):
        for i, nn in enumerate(n):
            eta = 2 * np.pi * nn / (N * m.delta)
            ref = sum(F[t, mm] * chi[mm] ** (-b) * chi0 ** (-1j * eta) * np.exp(-2j * np.pi * nn * mm / N)
                      for mm in range(N)) / N
            assert abs(c[t, i] - ref) < 1e-13 * np.abs(F).max() * chi.max() ** abs(b)
    # the series reproduces the samples away from the (dropped) Nyquist term
    recon = np.array([[np.sum(c[t] * chi[mm] ** (b + 1j * 2 * np.pi * n / (N * m.delta))) for mm in range(N)]
                      for t in range(2)])
    nyq = np.array([np.sum(F[t] * chi ** (-b) * (-1.0) ** np.arange(N)) / N for t in range(2)])
    expect = F - (nyq[:, None] * (-1.0) ** np.arange(N)[None, :]) * chi[None, :] ** b
    assert np.allclose(recon.real, expect, atol=1e-12 * np.abs(F).max() * chi.max() ** abs(b))


# --- the whole FFTLog oracle against the exact integral (method-error floor) ----------------------

def _eps(Ca, Cb):
    d = np.sqrt(np.abs(np.einsum("ltt->lt", Cb)))
    return np.abs(Ca - Cb) / (d[:, :, None] * d[:, None, :])


def _floor(wl, ell_sel, kstep, method=None):
    m = method or fftlog.method_for(wl)
    geo = geometry.point_geometry(wl, 0)
    ells = fftlog.point_ells(wl, 0)[ell_sel]
    W = fftlog.windows_point(geo, ells, m)[:, :, ::kstep]
    Wq = quadrature.windows_quadrature(geo, ells, m.k[::kstep])
    s = (fftlog.k_weights(m) * wl["pk"][0])[::kstep]
    Cf = np.einsum("ltj,lsj,j->lts", W, W, s)
    Cq = np.einsum("ltj,lsj,j->lts", Wq, Wq, s)
    return _eps(Cf, Cq)


def test_method_floor_cfg0(wl0):
    eps = _floor(wl0, [0, 9, 19], 8)
    assert eps.max() < 2e-4


def test_method_floor_cfg1(wl1):
    # l = 2 (band 0), l ~ 3.7 (band 1), then bands 2 at low, mid and top l
    eps = _floor(wl1, [0, 9, 30, 70, 102], 32)
    assert eps.max() < 3e-5


def test_method_floor_30_tracer_shape():
    """The 30-tracer shape (N_k = N_chi = 2048, l in [2, 3000]) that the split-precision parity
    tests compare against: clustering and lensing bins from both ends of each set, eps < 3e-5
    (measured 8.7e-6 at l = 2, <= 1.1e-6 from l = 4 to 3000)."""
    wl = synth.make_workload("cfg4", batch=1)
    sel = [0, 10, 19, 20, 25, 29]
    geo = geometry.PointGeometry(wl["z_geom"], wl["chi_z"][0], wl["D_z"][0], wl["omega_m"][0], wl["z_nz"],
                                 wl["nz"][0, sel], wl["kind"][0, sel], wl["bias"][0, sel])
    m = fftlog.method_for(wl)
    assert m.n_chi == 2048
    ells = fftlog.point_ells(wl, 0)[[0, 20, 60, 120, 199]]
    W = fftlog.windows_point(geo, ells, m)[:, :, ::64]
    Wq = quadrature.windows_quadrature(geo, ells, m.k[::64])
    s = (fftlog.k_weights(m) * wl["pk"][0])[::64]
    eps = _eps(np.einsum("ltj,lsj,j->lts", W, W, s), np.einsum("ltj,lsj,j->lts", Wq, Wq, s))
    assert eps.max() < 3e-5


def test_tail_taper_keeps_the_floor(wl1, monkeypatch):
    """Reading R7: the optional cosine taper acts on the top fraction of |n| only, where the
    coefficients of smooth kernels are negligible, so the floor holds with it (taper fractions 0.1
    and 0.3: eps < 3e-5, measured 8e-6 and 1e-5); the same taper planted on the low-|n| end is
    off by O(1)."""
    geo = geometry.point_geometry(wl1, 0)
    ells = fftlog.point_ells(wl1, 0)[[0, 30, 102]]
    base = fftlog.method_for(wl1)
    Wq = quadrature.windows_quadrature(geo, ells, base.k[::32])
    s = (fftlog.k_weights(base) * wl1["pk"][0])[::32]
    Cq = np.einsum("ltj,lsj,j->lts", Wq, Wq, s)

    def eps(frac):
        W = fftlog.windows_point(geo, ells, fftlog.method_for(wl1, taper_frac=frac))[:, :, ::32]
        return _eps(np.einsum("ltj,lsj,j->lts", W, W, s), Cq).max()

    assert eps(0.1) < 3e-5 and eps(0.3) < 3e-5
    orig = fftlog.taper
    monkeypatch.setattr(fftlog, "taper", lambda n, N, frac: orig(N // 2 - np.abs(n), N, frac))
    assert eps(0.1) > 0.1


def test_method_floor_cfg1_intrinsic_alignment():
    """The NLA term of the lensing tracers (Sec. 2.3) through the FFTLog oracle (geometry.f_of_z)
    and through direct quadrature (its own integrand): the same floor as without it, while IA moves
    the lensing autos by up to ~24%."""
    wl = synth.intrinsic_alignment(synth.make_workload("cfg1"))
    eps = _floor(wl, [0, 9, 30, 70, 102], 32)
    assert eps.max() < 3e-5


def test_method_floor_cfg1_rsd():
    """Redshift-space distortions of the clustering tracers (eq. RSD): the FFTLog oracle integrates
    chi^p j_l'' through the three-term recurrence and eq. int_jl, direct quadrature uses j_l'' from
    the Bessel equation.  1.5e-4 at l = 2 (the j_0 term leaves the bias b = 0.1 little room on the
    p range of eq. int_jl), 2e-5 above; RSD moves the clustering autos by up to ~95% at l = 2."""
    wl = synth.make_workload("cfg1")
    wl["rsd"] = True
    m = fftlog.method_for(wl)
    geo = geometry.point_geometry(wl, 0)
    ells = fftlog.point_ells(wl, 0)[[0, 30, 102]]
    W = fftlog.windows_point(geo, ells, m, rsd=True)[:, :, ::32]
    Wq = quadrature.windows_quadrature(geo, ells, m.k[::32], rsd=True)
    s = (fftlog.k_weights(m) * wl["pk"][0])[::32]
    eps = _eps(np.einsum("ltj,lsj,j->lts", W, W, s), np.einsum("ltj,lsj,j->lts", Wq, Wq, s))
    assert eps[0].max() < 1.5e-4
    assert eps[1:].max() < 2e-5


def test_method_floor_cfg1_magnification():
    """Magnification bias of the clustering tracers (eq. magnification bias): the FFTLog oracle
    decomposes C_g q D / chi^2 with the bias b - 2 and multiplies by l(l+1)/k^2 (reading R20), direct
    quadrature integrates the same kernel against j_l; measured 3e-5 at l = 2, 1e-5 above."""
    wl = synth.magnification_bias(synth.make_workload("cfg1"))
    eps = _floor(wl, [0, 30, 102], 32)
    assert eps.max() < 6e-5


def test_growth_rate_matches_closed_form(wl1):
    """f = dln D/dln a from the D(z) spline (the RSD kernel's growth rate) against the closed form of
    the LCDM growth integral D ~ E(a) int_0^a da' / (a' E)^3:  f = -3/2 Omega_m(a) + 1 / (a^2 E^3 I(a))."""
    geo = geometry.point_geometry(wl1, 0)
    om = float(wl1["omega_m"][0])
    z = np.array([0.1, 0.5, 1.0, 2.0, 2.9])
    a = 1.0 / (1.0 + z)
    E = synth.e_of_z(z, om)
    I = np.array([integrate.quad(lambda x: 1.0 / (x * synth.e_of_z(1.0 / x - 1.0, om)) ** 3, 1e-8, ai,
                                 epsabs=0, epsrel=1e-12)[0] for ai in a])
    f_exact = -1.5 * om * (1.0 + z) ** 3 / E ** 2 + 1.0 / (a ** 2 * E ** 3 * I)
    assert np.max(np.abs(geo.growth_rate(z) / f_exact - 1.0)) < 1e-6


def test_magnification_window_is_the_scaled_lensing_window(wl1):
    """A clustering tracer with C_g = 1 gains l(l+1)/k^2 int q D / chi^2 j_l: the lensing window of
    the same n(z) times l(l+1)/F(l).  Where b - 2 equals the lensing bias (band 2) the two are the
    same numbers; in bands 0 and 1 they differ by the method error of the two biases."""
    m = fftlog.method_for(wl1)
    nz = wl1["nz"][0, [3, 3]]
    args = (wl1["z_geom"], wl1["chi_z"][0], wl1["D_z"][0], wl1["omega_m"][0], wl1["z_nz"], nz,
            np.array([0, 1]), np.array([1.0, 1.0]))
    with_mag = geometry.PointGeometry(*args, mag=np.array([1.0, 0.0]))
    plain = geometry.PointGeometry(*args)
    ells = fftlog.point_ells(wl1, 0)[[0, 5, 9, 20, 50, 102]]
    W1 = fftlog.windows_point(with_mag, ells, m)
    W0 = fftlog.windows_point(plain, ells, m)
    F = np.sqrt((ells + 2) * (ells + 1) * ells * (ells - 1))
    ref = (ells * (ells + 1) / F)[:, None] * W0[:, 1]
    rel = np.max(np.abs((W1[:, 0] - W0[:, 0]) - ref), axis=1) / np.max(np.abs(ref), axis=1)
    band2 = np.array([m.band(l) == 2 for l in ells])
    assert rel[band2].max() < 1e-12
    assert rel[~band2].max() < 5e-5


def test_planted_edge_weight_mistake_is_caught(wl1, monkeypatch):
    """Dropping the half weight of the lower support edge must break the floor pin."""
    real = fftlog.sampled_kernels

    def wrong(geo, method):
        chi0, chi, F = real(geo, method)
        F[:, method.m0] *= 2.0
        return chi0, chi, F

    monkeypatch.setattr(fftlog, "sampled_kernels", wrong)
    eps = _floor(wl1, [0, 30], 32)
    assert eps.max() > 1e-4


# --- Limber limit (eq. Limber, error O(1/l)) -------------------------------------------------------

def test_limber_limit_high_ell(wl1):
    m = fftlog.method_for(wl1)
    geo = geometry.point_geometry(wl1, 0)
    ells_all = fftlog.point_ells(wl1, 0)
    sel = np.nonzero(ells_all >= 300)[0][::4]
    ells = ells_all[sel]
    W = fftlog.windows_point(geo, ells, m)
    s = fftlog.k_weights(m) * wl1["pk"][0]
    C = np.einsum("ltj,lsj,j->lts", W, W, s)
    CL = limber.cl_limber(geo, ells, m.k, wl1["pk"][0])
    T = len(geo.kinds)
    rel = np.array([[abs(C[i, t, t] / CL[i, t, t] - 1) for t in range(T)] for i in range(len(ells))])
    clus = rel[:, :10]
    assert clus[ells >= 500].max() < 1e-2
    # error shrinks with l: the mean over clustering autos at the top is below the bottom one
    assert clus[-1].mean() < clus[0].mean()
    # weak lensing autos (F(l)^2/(l+1/2)^4 inserted) also converge to Limber
    assert rel[ells >= 1000, 10:].max() < 2e-2


def test_limber_on_the_chi_grid_matches_the_integral(wl1):
    """eq. Limber on the FFTLog chi nodes (the GPU's rule) against fine Gauss-Legendre panels in z:
    2e-6 while P's k_max cut stays outside the kernels' support; from l ~ 600 the cut (a jump of
    the integrand) enters it and the grid's trapezoid rule sees it at first order in Delta."""
    m = fftlog.method_for(wl1)
    geo = geometry.point_geometry(wl1, 0)
    ells = fftlog.point_ells(wl1, 0)[::6]
    A = limber.cl_limber_grid(geo, ells, m, wl1["pk"][0])
    B = limber.cl_limber(geo, ells, m.k, wl1["pk"][0])
    d = np.sqrt(np.abs(np.einsum("ltt->lt", B)))
    eps = np.abs(A - B) / (d[:, :, None] * d[:, None, :])
    assert eps[ells <= 500].max() < 5e-6
    assert eps.max() < 1e-3


def test_limber_grid_gradient_in_pk(wl1):
    """dL/dP_j of the chi-node Limber rule through the natural spline of ln P: sum_j P_j dL/dP_j = L
    (scaling every P_j scales P(k) exactly), and central differences at nodes across the k range,
    those whose Limber k only some multipoles reach included."""
    m = fftlog.method_for(wl1)
    geo = geometry.point_geometry(wl1, 0)
    ells = fftlog.point_ells(wl1, 0)[[0, 30, 60, 90, 102]]
    pk = wl1["pk"][0]
    rng = np.random.default_rng(12)
    G = rng.standard_normal((len(ells), 15, 15))
    L = lambda p: float(np.sum(G * limber.cl_limber_grid(geo, ells, m, p)))
    gp = limber.grad_pk_grid(G, geo, ells, m, pk)
    assert abs(gp @ pk - L(pk)) < 1e-10 * abs(L(pk))
    for j in (40, 300, 600, 900, 1020):
        h = 1e-5 * pk[j]
        pp, pm = pk.copy(), pk.copy()
        pp[j] += h
        pm[j] -= h
        fd = (L(pp) - L(pm)) / (2 * h)
        assert abs(fd - gp[j]) <= 1e-6 * np.abs(gp).max(), j


def test_limber_rules_agree_with_intrinsic_alignment():
    """The NLA term enters the two Limber oracles by separate code (the node rule through the
    sampled kernels of geometry.f_of_z, the panel integral through its own integrand): with IA on
    they agree as without it, while IA moves the lensing autos by percents."""
    wl = synth.intrinsic_alignment(synth.make_workload("cfg1"))
    m = fftlog.method_for(wl)
    geo = geometry.point_geometry(wl, 0)
    ells = fftlog.point_ells(wl, 0)[::12]
    A = limber.cl_limber_grid(geo, ells, m, wl["pk"][0])
    B = limber.cl_limber(geo, ells, m.k, wl["pk"][0])
    d = np.sqrt(np.abs(np.einsum("ltt->lt", B)))
    eps = np.abs(A - B) / (d[:, :, None] * d[:, None, :])
    assert eps[ells <= 500].max() < 5e-6
    B0 = limber.cl_limber(geometry.point_geometry(dict(wl, ia=None), 0), ells, m.k, wl["pk"][0])
    lens = np.arange(10, 15)
    assert np.max(np.abs(B[:, lens, lens] / B0[:, lens, lens] - 1)) > 1e-2


# --- invariants of C_l -------------------------------------------------------------------------------

def _full(Cp, T):
    C = np.zeros(Cp.shape[:-1] + (T, T))
    iu = np.triu_indices(T)
    C[..., iu[0], iu[1]] = Cp
    C[..., iu[1], iu[0]] = Cp
    return C


def test_symmetric_psd_and_homogeneous(wl1):
    m = fftlog.method_for(wl1)
    wl = dict(wl1)
    wl["ell_idx"] = wl1["ell_idx"][:, ::17].copy()
    wl["n_ell"] = np.array([wl["ell_idx"].shape[1]], np.int32)
    C, W = fftlog.cl(wl, 0, m, return_windows=True)
    Cf = _full(C, 15)
    for Cl in Cf:
        ev = np.linalg.eigvalsh(Cl)
        assert ev.min() >= -1e-12 * ev.max()
    # C(alpha P) = alpha C
    C2 = fftlog.cl_from_windows(W, 3.0 * wl["pk"][0], m)
    assert _eps(_full(C2, 15), _full(3.0 * C, 15)).max() < 1e-13
    # C^{ij} proportional to b_i b_j: doubling bias 0 doubles row 0 and quadruples C^{00}
    wl["bias"] = wl1["bias"].copy()
    wl["bias"][0, 0] *= 2.0
    Cb = _full(fftlog.cl(wl, 0, m), 15)
    expect = Cf.copy()
    expect[:, 0, :] *= 2.0
    expect[:, :, 0] *= 2.0
    assert _eps(Cb, expect).max() < 1e-12


# --- geometry and growth --------------------------------------------------------------------------------

def test_comoving_distance_matches_adaptive_quad():
    z = np.array([0.01, 0.5, 1.7, 3.0])
    chi = synth.comoving_distance(z, 0.3)
    for zi, ci in zip(z, chi):
        ref = synth.C_OVER_H0 * integrate.quad(lambda x: 1 / synth.e_of_z(x, 0.3), 0, zi,
                                               epsabs=0, epsrel=1e-13)[0]
        assert abs(ci / ref - 1) < 1e-11


def test_growth_matches_ode_and_einstein_de_sitter():
    from scipy.integrate import solve_ivp
    om = 0.3
    z = np.array([0.0, 0.5, 1.0, 3.0])
    D = synth.growth_factor(z, om)
    # D'' + (3/a + dlnE/da) D' - 1.5 Om / (a^5 E^2) D = 0 in a, growing mode D ~ a early on
    def E(a):
        return np.sqrt(om / a ** 3 + 1 - om)

    def rhs(a, y):
        dlnE = -1.5 * om / a ** 4 / E(a) ** 2
        return [y[1], -(3 / a + dlnE) * y[1] + 1.5 * om / (a ** 5 * E(a) ** 2) * y[0]]

    a0 = 1e-4
    sol = solve_ivp(rhs, [a0, 1.0], [a0, 1.0], rtol=1e-12, atol=1e-16, dense_output=True)
    Dode = sol.sol(1 / (1 + z))[0] / sol.sol(1.0)[0]
    assert np.allclose(D, Dode, rtol=1e-6)
    Deds = synth.growth_factor(z, 1.0)
    assert np.allclose(Deds, 1 / (1 + z), rtol=1e-12)


def test_lensing_integrals_match_adaptive_quad(wl1):
    geo = geometry.point_geometry(wl1, 0)
    for t in (10, 14):
        for z in (0.05, 0.6, 1.9):
            I0, I1 = geo.lensing_integrals(t, np.array([z]))
            f0 = lambda zz: float(geo.n_of_z(t, zz))
            r0 = integrate.quad(f0, z, geo.z_max, limit=500, points=geo.z_nz[(geo.z_nz > z)][::10],
                                epsabs=0, epsrel=1e-12)[0]
            r1 = integrate.quad(lambda zz: f0(zz) / float(geo.chi_spl(zz)), z, geo.z_max, limit=500,
                                points=geo.z_nz[(geo.z_nz > z)][::10], epsabs=0, epsrel=1e-12)[0]
            assert abs(I0[0] - r0) < 1e-9 * abs(r0)
            assert abs(I1[0] - r1) < 1e-9 * abs(r1)


def test_lensing_table_converged(wl1):
    geo = geometry.point_geometry(wl1, 0)
    z = np.linspace(0.02, 2.9, 777)
    a = quadrature.LensingTable(geo, refine=16)
    b = quadrature.LensingTable(geo, refine=32)
    for t in (10, 12, 14):
        qa, qb = a(t, z), b(t, z)
        assert np.max(np.abs(qa - qb)) < 1e-9 * np.max(np.abs(qb))
        assert np.allclose(qa, geo.lensing_q(t, z), rtol=1e-8, atol=1e-9 * np.abs(qb).max())


def test_z_of_chi_round_trip(wl1):
    geo = geometry.point_geometry(wl1, 0)
    z = np.array([0.01, 0.3, 1.1, 2.999])
    assert np.allclose(geo.z_of_chi(geo.chi_spl(z)), z, atol=1e-12)


# --- gradients -----------------------------------------------------------------------------------------

def _small(wl, stride=25):
    w = dict(wl)
    w["ell_idx"] = wl["ell_idx"][:, ::stride].copy()
    w["n_ell"] = np.array([w["ell_idx"].shape[1]], np.int32)
    return w


def test_gradients_against_finite_differences(wl2):
    wl = _small(wl2)
    m = fftlog.method_for(wl)
    rng = np.random.default_rng(7)
    C, W = fftlog.cl(wl, 0, m, return_windows=True)
    G = rng.standard_normal(C.shape)
    L = lambda w: float(np.sum(G * fftlog.cl(w, 0, m)))
    # P: exact form vs central differences on a few nodes
    gp = gradients.grad_pk(G, W, m)
    for j in (100, 500, 900):
        h = 1e-4 * wl["pk"][0, j]
        wp, wm = dict(wl), dict(wl)
        wp["pk"] = wl["pk"].copy(); wp["pk"][0, j] += h
        wm["pk"] = wl["pk"].copy(); wm["pk"][0, j] -= h
        fd = (float(np.sum(G * fftlog.cl_from_windows(W, wp["pk"][0], m)))
              - float(np.sum(G * fftlog.cl_from_windows(W, wm["pk"][0], m)))) / (2 * h)
        assert abs(fd - gp[j]) <= 1e-7 * abs(gp).max()
    # biases
    gb = gradients.grad_bias(G, C, wl["kind"][0], wl["bias"][0])
    for t in (0, 7):
        h = 1e-4 * wl["bias"][0, t]
        wp, wm = dict(wl), dict(wl)
        wp["bias"] = wl["bias"].copy(); wp["bias"][0, t] += h
        wm["bias"] = wl["bias"].copy(); wm["bias"][0, t] -= h
        fd = (L(wp) - L(wm)) / (2 * h)
        assert abs(fd - gb[t]) <= 1e-7 * abs(gb).max()
    assert np.all(gb[10:] == 0)
    # n(z) and D(z) directional derivatives vs central differences
    v = rng.standard_normal(wl["nz"].shape[-1]) * wl["nz"][0, 12].max() * 0.1
    dn = gradients.directional_nz(wl, 0, G, 12, v, m)
    eps = 1e-3
    wp, wm = dict(wl), dict(wl)
    wp["nz"] = wl["nz"].copy(); wp["nz"][0, 12] += eps * v
    wm["nz"] = wl["nz"].copy(); wm["nz"][0, 12] -= eps * v
    fd = (L(wp) - L(wm)) / (2 * eps)
    assert abs(fd - dn) <= 1e-7 * abs(dn)
    vD = rng.standard_normal(wl["D_z"].shape[-1]) * 0.01
    dD = gradients.directional_D(wl, 0, G, vD, m)
    wp, wm = dict(wl), dict(wl)
    wp["D_z"] = wl["D_z"] + eps * vD
    wm["D_z"] = wl["D_z"] - eps * vD
    fd = (L(wp) - L(wm)) / (2 * eps)
    assert abs(fd - dD) <= 1e-7 * abs(dD)


def test_gradients_with_intrinsic_alignment():
    """With IA on, n(z) of a lensing tracer enters its kernel twice (lens efficiency and the NLA
    term) and both stay linear in n, D; the directional derivatives against central differences."""
    wl = _small(synth.intrinsic_alignment(synth.make_workload("cfg2")), 51)
    m = fftlog.method_for(wl)
    rng = np.random.default_rng(11)
    C = fftlog.cl(wl, 0, m)
    G = rng.standard_normal(C.shape)
    L = lambda w: float(np.sum(G * fftlog.cl(w, 0, m)))
    eps = 1e-3
    v = rng.standard_normal(wl["nz"].shape[-1]) * wl["nz"][0, 12].max() * 0.1
    dn = gradients.directional_nz(wl, 0, G, 12, v, m)
    wp, wm = dict(wl), dict(wl)
    wp["nz"] = wl["nz"].copy(); wp["nz"][0, 12] += eps * v
    wm["nz"] = wl["nz"].copy(); wm["nz"][0, 12] -= eps * v
    assert abs((L(wp) - L(wm)) / (2 * eps) - dn) <= 1e-7 * abs(dn)
    # the NLA term's share of the derivative is not negligible
    dn0 = gradients.directional_nz(dict(wl, ia=None), 0, G, 12, v, m)
    assert abs(dn / dn0 - 1) > 1e-3
    vD = rng.standard_normal(wl["D_z"].shape[-1]) * 0.01
    dD = gradients.directional_D(wl, 0, G, vD, m)
    wp, wm = dict(wl, D_z=wl["D_z"] + eps * vD), dict(wl, D_z=wl["D_z"] - eps * vD)
    assert abs((L(wp) - L(wm)) / (2 * eps) - dD) <= 1e-7 * abs(dD)


def test_euler_identities(wl1):
    """sum_j P_j dC/dP_j = C, and sum_s D_s dC/dD_s = 2C (C is quadratic in D)."""
    wl = _small(wl1, 34)
    m = fftlog.method_for(wl)
    C, W = fftlog.cl(wl, 0, m, return_windows=True)
    npair = C.shape[1]
    # P: with G = e_(l,p), dL/dP . P = C[l, p]
    for (l, p) in [(0, 0), (1, 17), (2, npair - 1)]:
        G = np.zeros_like(C); G[l, p] = 1.0
        assert abs(gradients.grad_pk(G, W, m) @ wl["pk"][0] - C[l, p]) < 1e-12 * abs(C[l, p])
        assert abs(gradients.directional_D(wl, 0, G, wl["D_z"][0], m) - 2 * C[l, p]) < 1e-10 * abs(C[l, p])
