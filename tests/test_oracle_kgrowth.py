"""Pins of the scale-dependent growth oracle (Sec. 3.2, k-dependent coefficients interpolated
along k) against what the mathematics fixes (CPU only).

  * growth independent of k reduces the method to scale-free FFTLog (itself pinned to direct
    quadrature of j_l in test_oracle_pins.py);
  * growth linear in ln k is reproduced exactly by the natural spline, so C_l equals scale-free
    C_l with P(k) rescaled by the square of the growth factor's k-dependence;
  * at a k node that coincides with an interpolation node the window is the scale-free window of
    that node's growth, and within the method floor of direct quadrature;
  * the interpolation converges at fourth order in the node spacing (a linear interpolant, the
    planted mistake, converges at second order and is caught).
"""
import numpy as np
import pytest

import synth
from oracle import fftlog, geometry, kgrowth, quadrature


def _eps(Ca, Cb):
    """max |Ca - Cb| / sqrt(C_ii C_jj) over packed spectra (Cb the reference)."""
    L, P = Cb.shape
    T = int(round((np.sqrt(8 * P + 1) - 1) / 2))
    iu = np.triu_indices(T)
    diag = Cb[:, [p for p, (i, j) in enumerate(zip(*iu)) if i == j]]
    den = np.sqrt(np.abs(diag[:, iu[0]] * diag[:, iu[1]]))
    return float(np.max(np.abs(Ca - Cb) / den))


@pytest.fixture(scope="module")
def wl1s():
    """The 15-tracer workload (clustering and lensing) at every 17th multipole."""
    wl = synth.make_workload("cfg1")
    wl["ell_idx"] = wl["ell_idx"][:, ::17].copy()
    wl["n_ell"] = np.array([wl["ell_idx"].shape[1]], np.int32)
    return wl


def test_scale_free_growth_is_fftlog(wl1s):
    wl = dict(wl1s)
    wl["D_kz"] = np.repeat(wl["D_z"][:, None, :], 6, 1)
    m = fftlog.method_for(wl)
    assert _eps(kgrowth.cl(wl, 0, m), fftlog.cl(wl, 0, m)) < 1e-12


def test_scale_free_growth_is_fftlog_with_intrinsic_alignment(wl1s):
    """The node geometries carry the NLA term of the lensing tracers like the scale-free one."""
    wl = synth.intrinsic_alignment(dict(wl1s))
    wl["D_kz"] = np.repeat(wl["D_z"][:, None, :], 4, 1)
    m = fftlog.method_for(wl)
    assert _eps(kgrowth.cl(wl, 0, m), fftlog.cl(wl, 0, m)) < 1e-12


def test_scale_free_growth_is_fftlog_with_cmb_lensing():
    """A CMB-lensing tracer (kind 2, its kernel linear in D) takes the node growth like the others."""
    wl = synth.cmb_lensing(synth.make_workload("cfg0"))
    wl["D_kz"] = np.repeat(wl["D_z"][:, None, :], 4, 1)
    m = fftlog.method_for(wl)
    assert _eps(kgrowth.cl(wl, 0, m), fftlog.cl(wl, 0, m)) < 1e-12


def test_growth_linear_in_ln_k_rescales_pk_with_cmb_lensing():
    wl0 = synth.cmb_lensing(synth.make_workload("cfg0"))
    wl = dict(wl0)
    m = fftlog.method_for(wl)
    x = kgrowth.ln_nodes(m, 5)
    wl["D_kz"] = wl["D_z"][:, None, :] * (1.0 + 0.03 * (x - np.log(0.05)))[None, :, None]
    ref_wl = dict(wl0)
    ref_wl["pk"] = wl0["pk"] * (1.0 + 0.03 * np.log(m.k / 0.05))[None, :] ** 2
    assert _eps(kgrowth.cl(wl, 0, m), fftlog.cl(ref_wl, 0, m)) < 1e-11


def test_growth_linear_in_ln_k_rescales_pk(wl1s):
    wl = dict(wl1s)
    m = fftlog.method_for(wl)
    eps_k, k_star = 0.04, 0.02
    A = 7
    x = kgrowth.ln_nodes(m, A)
    wl["D_kz"] = wl["D_z"][:, None, :] * (1.0 + eps_k * (x - np.log(k_star)))[None, :, None]
    got = kgrowth.cl(wl, 0, m)
    ref_wl = dict(wl1s)
    ref_wl["pk"] = wl1s["pk"] * (1.0 + eps_k * np.log(m.k / k_star))[None, :] ** 2
    assert _eps(got, fftlog.cl(ref_wl, 0, m)) < 1e-11


def test_node_columns_are_scale_free_windows_of_the_node():
    wl = synth.make_workload("cfg0")
    synth.scale_dependent_growth(wl, 16, f_nu=0.3)  # strong k-dependence
    m = fftlog.method_for(wl)
    assert (m.n_k - 1) % 15 == 0  # node a sits on k index 17 a
    geos = kgrowth.node_geometries(wl, 0)
    ells = fftlog.point_ells(wl, 0)
    W = kgrowth.windows_point(geos, ells, m)
    for a in (0, 3, 8, 15):
        j = a * (m.n_k - 1) // 15
        Wa = fftlog.windows_point(geos[a], ells, m)
        # equal up to the rounding of the n-sum, which cancels over several decades
        assert np.max(np.abs(W[:, :, j] - Wa[:, :, j])) <= 1e-9 * np.max(np.abs(Wa[:, :, j]))
        # the plain definition at that k: direct quadrature of f D(kappa_a) j_l(k chi), relative
        # to the peak of each window over k
        Wq = quadrature.windows_quadrature(geos[a], ells[::4], m.k[j:j + 1])[:, :, 0]
        rel = np.abs(W[::4, :, j] - Wq) / np.max(np.abs(Wa[::4]), axis=2)
        print(a, rel.max())
        assert rel.max() < 2e-3, (a, rel.max())


def _convergence(interp=None):
    wl = synth.make_workload("cfg0")
    m = fftlog.method_for(wl)
    Cs = {}
    for A in (17, 33, 129):
        synth.scale_dependent_growth(wl, A)
        Cs[A] = kgrowth.cl(wl, 0, m)
    e17, e33 = _eps(Cs[17], Cs[129]), _eps(Cs[33], Cs[129])
    return e17, e33


def test_interpolation_is_fourth_order():
    e17, e33 = _convergence()
    assert e33 < 1e-5
    assert e17 / e33 > 8.0, (e17, e33)


def test_planted_linear_interpolation_is_caught(monkeypatch):
    """Interpolating c_n linearly in ln k (a dropped curvature term) must fail the order pin."""
    def linear(x_nodes, values, x):
        flat = values.reshape(len(x_nodes), -1)
        out = np.stack([np.interp(x, x_nodes, flat[:, i].real) + 1j * np.interp(x, x_nodes, flat[:, i].imag)
                        for i in range(flat.shape[1])], axis=-1)
        return out.reshape((len(x),) + values.shape[1:])

    monkeypatch.setattr(kgrowth, "interpolate_ln_k", linear)
    e17, e33 = _convergence()
    assert e17 / e33 < 8.0


def test_needs_two_nodes():
    m = fftlog.method_for(synth.make_workload("cfg0"))
    with pytest.raises(ValueError):
        kgrowth.ln_nodes(m, 1)
