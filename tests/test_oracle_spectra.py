"""Pins of the oracle's spin- and polarization-resolved spectra (appendix, Bessel forms):
positivity for every pure state (fixes each term's sign and the basis handedness), the
identities that tie the separately printed forms together (F0 = w + s_f.g, the marginals
j_e and j_p of G, the sum over the four pair outcomes), and the unpolarized limits checked
against scipy's Bessel functions."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle


def unit(rng, n=1):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _scipy_bessel(x):
    ik = integrate.quad(lambda y: special.kv(1 / 3, y), x, np.inf, epsabs=0, epsrel=1e-13, limit=200)[0]
    return special.kv(1 / 3, x), special.kv(2 / 3, x), ik


def test_nlc_positivity_all_pure_states():
    """F0 - |F| >= 0 and w - |g| >= 0 for random pure (s_i, s_f), chi in [1e-2, 1e2]; the
    bound is attained (min close to zero), so a flipped term would make it negative."""
    rng = np.random.default_rng(11)
    worst = np.inf
    for _ in range(3000):
        chi = 10 ** rng.uniform(-2, 2)
        lam = 10 ** rng.uniform(-4, math.log10(1 - 1e-4)) if rng.random() < 0.5 else 1 - 10 ** rng.uniform(-4, -0.3)
        si, sf = unit(rng)[0], unit(rng)[0]
        F = oracle.nlc_F(chi, lam, si, sf)
        w = oracle.nlc_w(chi, lam, si[1])
        g = oracle.nlc_g(chi, lam, si)
        if w < 1e-250:
            continue
        assert w - np.linalg.norm(g) >= -1e-12 * w
        margin = (F[0] - np.linalg.norm(F[1:])) / w
        assert margin >= -1e-12
        worst = min(worst, margin)
    assert worst < 0.02


def test_nbw_positivity_all_pure_states():
    rng = np.random.default_rng(12)
    worst = np.inf
    for _ in range(3000):
        chi = 10 ** rng.uniform(-1, 2)
        lam = rng.uniform(1e-3, 1 - 1e-3)
        se, sp = unit(rng)[0], unit(rng)[0]
        G = oracle.nbw_G(chi, lam, se, sp)
        w0, _, _ = oracle.nbw_j(chi, lam, np.zeros(3))
        if w0 < 1e-250:
            continue
        margin = (G[0] - np.linalg.norm(G[1:])) / w0
        assert margin >= -1e-12
        worst = min(worst, margin)
    assert worst < 0.02


def test_nlc_forms_agree():
    """F0 printed in full equals w + s_f . g with w and g printed separately; F is linear in s_f."""
    rng = np.random.default_rng(13)
    for _ in range(200):
        chi, lam = 10 ** rng.uniform(-2, 2), rng.uniform(1e-3, 0.99)
        si = unit(rng)[0] * rng.uniform(0, 1)
        sf = unit(rng)[0]
        F = oracle.nlc_F(chi, lam, si, sf)
        w = oracle.nlc_w(chi, lam, si[1])
        g = oracle.nlc_g(chi, lam, si)
        assert abs(F[0] - (w + sf @ g)) <= 1e-13 * abs(w)
        Fp, Fm, F0 = (oracle.nlc_F(chi, lam, si, v) for v in (sf, -sf, np.zeros(3)))
        np.testing.assert_allclose(0.5 * (Fp + Fm), F0, rtol=0, atol=1e-13 * abs(w))
        assert abs(F0[0] - w) <= 1e-13 * abs(w)


def test_nlc_unpolarized_limit_vs_scipy():
    """s_i = s_f = 0: F = (-IntK + kappa K23, 0, 0, K23); photons carry only xi3 (NLC appendix)."""
    for chi, lam in [(0.1, 0.03), (1.0, 0.2), (10.0, 0.7), (99.0, 0.95)]:
        z = np.zeros(3)
        F = oracle.nlc_F(chi, lam, z, z)
        K1, K2, I = _scipy_bessel(2 * lam / (1 - lam) / (3 * chi))
        kap = 1 / (1 - lam) + (1 - lam)
        np.testing.assert_allclose(F, [-I + kap * K2, 0, 0, K2], rtol=1e-10, atol=0)
        # spin dependence of the rate enters only through s_beta with lam K_1/3 (w)
        assert abs(oracle.nlc_w(chi, lam, 0.7) - (-I + kap * K2 + 0.7 * lam * K1)) < 1e-10 * abs(F[0])


def test_nbw_sum_rules_and_marginals():
    """sum over the four (positron, electron) outcomes of G0 + xi.G = 4 w0, and the marginals over
    the other lepton's spin reproduce w0 + s.j with j_e, j_p printed separately."""
    rng = np.random.default_rng(14)
    for _ in range(200):
        chi, lam = 10 ** rng.uniform(-1, 2), rng.uniform(1e-3, 1 - 1e-3)
        xi = unit(rng)[0] * rng.uniform(0, 1)
        w0, je, jp = oracle.nbw_j(chi, lam, xi)
        Se, Sp = unit(rng)[0], unit(rng)[0]
        full = lambda e, p: (lambda G: G[0] + xi @ G[1:])(oracle.nbw_G(chi, lam, e, p))
        tot = sum(full(a * Se, b * Sp) for a in (-1, 1) for b in (-1, 1))
        assert abs(tot - 4 * w0) <= 1e-12 * abs(w0)
        assert abs(0.5 * (full(Se, Sp) + full(Se, -Sp)) - (w0 + Se @ je)) <= 1e-12 * abs(w0)
        assert abs(0.5 * (full(Se, Sp) + full(-Se, Sp)) - (w0 + Sp @ jp)) <= 1e-12 * abs(w0)


def test_nbw_unpolarized_limit_vs_scipy():
    """s_e = s_p = 0: G = (IntK + rho K23, 0, 0, -K23); for an unpolarized photon the positron
    spin axis is along beta only (validation section on NBW spectra)."""
    for chi, lam in [(0.5, 0.3), (1.0, 0.5), (10.0, 0.1), (99.0, 0.9)]:
        z = np.zeros(3)
        G = oracle.nbw_G(chi, lam, z, z)
        ut = 1 / lam + 1 / (1 - lam)
        K1, K2, I = _scipy_bessel(2 * ut / (3 * chi))
        rho = (1 - lam) / lam + lam / (1 - lam)
        np.testing.assert_allclose(G, [I + rho * K2, 0, 0, -K2], rtol=1e-10, atol=0)
        w0, je, jp = oracle.nbw_j(chi, lam, z)
        assert jp[0] == 0 and jp[2] == 0 and je[0] == 0 and je[2] == 0
        np.testing.assert_allclose([jp[1], je[1]], [-K1 / lam, K1 / (1 - lam)], rtol=1e-10)


def test_nlc_mean_stokes_unpolarized():
    """<xi3> = K23 / (-IntK + kappa K23) for an unpolarized lepton (NLC appendix)."""
    for chi, lam in [(1.0, 0.1), (5.0, 0.5)]:
        z = np.zeros(3)
        F = oracle.nlc_F(chi, lam, z, z)
        K1, K2, I = _scipy_bessel(2 * lam / (1 - lam) / (3 * chi))
        assert abs(F[3] / F[0] - K2 / (-I + (1 / (1 - lam) + 1 - lam) * K2)) < 1e-10


def test_classical_polarization_limits():
    """chi -> 0: photon-number-weighted <xi3> -> 3/5 and energy-weighted <xi3> -> 3/4 (7:1 sigma:pi)."""
    chi = 1e-4
    z = np.zeros(3)

    def moments(nu):
        lam = special.expit(nu)
        F = oracle.nlc_F(chi, lam, z, z)
        jac = lam * special.expit(-nu)
        return np.array([F[0], F[3], lam * F[0], lam * F[3]]) * jac
    pts = np.linspace(-40, math.log(1.5 * chi * 700), 25)
    m = np.zeros(4)
    for a, b in zip(pts[:-1], pts[1:]):
        for k in range(4):
            m[k] += integrate.quad(lambda v: moments(v)[k], a, b, epsabs=0, epsrel=1e-10)[0]
    assert abs(m[1] / m[0] - 0.6) < 2e-3
    assert abs(m[3] / m[2] - 0.75) < 2e-3
