"""Pins of the oracle's field-dependent anomalous moment (loop appendix): the Scorer function Gi
against mpmath and its defining differential equation, a(chi)/a(0) against an mpmath quadrature
of the Airy-Scorer form, its limits (Schwinger's constant at chi -> 0, the chi^(-2/3) law at large
chi), the table's interpolation error, and the T-BMT precession it drives in a constant B field."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth

EPS = synth.EPS_R
A_E = oracle.ALPHA / (2 * math.pi)


@pytest.fixture(scope="module")
def tables():
    return oracle.OracleTables()


# ------------------------------------------------------------------ Scorer function
@pytest.mark.parametrize("z", [0.0, 0.3, 1.0, 2.5, 7.0, 15.0, 19.999, 20.001, 40.0, 1e3, 1e6])
def test_scorer_gi_against_mpmath(z):
    ref = float(mp.scorergi(mp.mpf(z)))
    assert abs(oracle.scorer_gi(z) / ref - 1) < 2e-14


def test_scorer_gi_closed_forms():
    # Gi(0) = 1 / (3^(7/6) Gamma(2/3)); Gi'(0) = 1 / (3^(5/6) Gamma(1/3))
    assert abs(oracle.scorer_gi(0.0) - 1 / (3 ** (7 / 6) * math.gamma(2 / 3))) < 1e-15
    h = 1e-4
    d0 = (oracle.scorer_gi(h) - oracle.scorer_gi(0.0)) / h
    d2 = (oracle.scorer_gi(2 * h) - 2 * oracle.scorer_gi(h) + oracle.scorer_gi(0.0)) / h ** 2
    assert abs(d0 - h / 2 * d2 - 1 / (3 ** (5 / 6) * math.gamma(1 / 3))) < 1e-7
    # Gi'' - z Gi = -1/pi on both sides of the switch to the large-argument expansion
    for z in [0.5, 2.0, 8.0, 19.9, 20.1, 30.0]:
        h = 1e-3 * max(1.0, z / 10)
        d2 = (oracle.scorer_gi(z + h) - 2 * oracle.scorer_gi(z) + oracle.scorer_gi(z - h)) / h ** 2
        assert abs(d2 - z * oracle.scorer_gi(z) + 1 / math.pi) < 1e-6
    # large argument: Gi ~ 1/(pi z)
    assert abs(oracle.scorer_gi(1e8) * math.pi * 1e8 - 1) < 1e-15


# ------------------------------------------------------------------ a(chi)/a(0)
def _gfac_mp(chi):
    mp.mp.dps = 25
    c = mp.mpf(chi)
    f = lambda u: (u / c) ** (mp.mpf(2) / 3) * mp.scorergi((u / c) ** (mp.mpf(2) / 3)) / (1 + u) ** 3
    return float(2 * mp.pi * mp.quad(f, [0, c * 1e-3, c, 1, 10, mp.inf]))


@pytest.mark.parametrize("chi", [1e-4, 1e-2, 0.3, 1.0, 7.0, 100.0, 1e4])
def test_gfactor_ratio_against_mpmath(chi):
    assert abs(oracle.gfactor_ratio(chi) / _gfac_mp(chi) - 1) < 1e-12


def test_gfactor_limits():
    # chi -> 0: Schwinger's alpha/(2 pi); the deviation is of order chi^2 ln(1/chi)
    assert abs(oracle.gfactor_ratio(1e-9) - 1) < 1e-15
    d5, d6 = 1 - oracle.gfactor_ratio(1e-5), 1 - oracle.gfactor_ratio(1e-6)
    assert 0 < d6 < d5 and 0.008 < d6 / d5 < 0.0125
    # chi -> inf: 2 pi Gi(0) B(5/3, 4/3) chi^(-2/3) = 2 pi Gamma(1/3) / (9 3^(7/6)) chi^(-2/3)
    c = 2 * math.pi * math.gamma(1 / 3) / (9 * 3 ** (7 / 6))
    r = [oracle.gfactor_ratio(x) / (c * x ** (-2 / 3)) for x in (1e4, 1e6, 1e8)]
    assert r[0] > r[1] > r[2] > 1 and r[2] - 1 < 1e-5
    # decreasing in chi
    g = [oracle.gfactor_ratio(x) for x in np.logspace(-4, 4, 33)]
    assert all(b < a for a, b in zip(g, g[1:]))


def test_gfactor_table(tables):
    nodes = tables.lngfac_nodes()
    assert nodes.shape == (oracle.GF_N,)
    for i in (0, 100, 352, 600, oracle.GF_N - 1):
        chi = math.exp(oracle.GF_LNCHI0 + i * oracle.GF_DLNCHI)
        assert abs(nodes[i] - math.log(oracle.gfactor_ratio(chi))) < 1e-15
    lc = oracle.GF_LNCHI0 + (np.arange(0, oracle.GF_N - 1, 7) + 0.5) * oracle.GF_DLNCHI
    err = max(abs(tables.gfac(math.exp(x)) / oracle.gfactor_ratio(math.exp(x)) - 1) for x in lc)
    assert err < 5e-9
    assert tables.gfac(0.0) == 1.0 and tables.gfac(1e-8) == 1.0
    for chi in (3e4, 1e6):      # beyond the table: the chi^(-2/3) law from the last node
        assert abs(tables.gfac(chi) / oracle.gfactor_ratio(chi) - 1) < 5e-3


# ------------------------------------------------------------------ T-BMT with a(chi)
def _angle_in_plane(a, b):
    return math.atan2(a[0] * b[1] - a[1] * b[0], a[0] * b[0] + a[1] * b[1])


def test_push_gchi_precession_in_constant_B(tables):
    """p and s normal to B: per step p turns by phi_p = 2 atan(B dt / (2 gamma)) and s by
    2 atan((a + 1/gamma) B dt / 2) with a = a_e a(chi)/a(0) at the mid-step chi, which in a pure
    B field is eps_r |p| cos(phi_p/2) B (the mean of the momenta before and after the rotation)."""
    B, dt, n = 300.0, 0.01, 400
    p = np.array([1000.0, 0.0, 0.0]); s = np.array([0.6, 0.8, 0.0]); x = np.zeros(3)
    gamma = math.sqrt(1 + p @ p)
    phi_p = 2 * math.atan(B * dt / (2 * gamma))
    chi = EPS * math.sqrt(p @ p) * math.cos(phi_p / 2) * B
    assert 0.5 < chi < 2
    a = A_E * tables.gfac(chi)
    phi_s = 2 * math.atan((a + 1 / gamma) * B * dt / 2)
    ang0 = _angle_in_plane(p, s)
    for _ in range(n):
        p, s, x = oracle.push_one(-1, A_E, np.zeros(3), np.array([0, 0, B]), dt, oracle.F_TBMT | oracle.F_GCHI,
                                  p, s, x, tables=tables, eps_r=EPS)
    d = lambda v: (v + math.pi) % (2 * math.pi) - math.pi
    turned = d(_angle_in_plane(p, s) - ang0)
    assert abs(turned - d(n * (phi_s - phi_p))) < 1e-10
    # the field dependence is visible: a constant a_e would turn the spin about twice as far
    phi_s0 = 2 * math.atan((A_E + 1 / gamma) * B * dt / 2)
    assert abs(turned - d(n * (phi_s0 - phi_p))) > 0.3


def test_push_gchi_weak_field_is_constant_moment(tables):
    """Below chi = 1e-7 the push equals the constant-moment push bit for bit; at chi ~ 2e-5 the
    spins differ by about a_e (1 - a/a(0)) |B| dt."""
    E = np.array([0.01, 0.0, 0.0]); s0 = np.array([0.0, 0.6, 0.8])
    for p0, B, exact in ((np.array([0.3, 0.1, 0.0]), np.array([0.0, 0.0, 0.05]), True),
                         (np.array([3.0, 1.0, 0.0]), np.array([0.0, 0.0, 2.0]), False)):
        pa, sa, _ = oracle.push_one(-1, A_E, E, B, 0.05, oracle.F_TBMT, p0, s0, np.zeros(3))
        pb, sb, _ = oracle.push_one(-1, A_E, E, B, 0.05, oracle.F_TBMT | oracle.F_GCHI, p0, s0, np.zeros(3),
                                    tables=tables, eps_r=EPS)
        np.testing.assert_array_equal(pa, pb)
        chi = EPS * np.linalg.norm(p0) * np.linalg.norm(B)
        if exact:
            assert chi < 1e-7
            np.testing.assert_array_equal(sa, sb)
        else:
            bound = 2 * A_E * (1 - oracle.gfactor_ratio(chi)) * np.linalg.norm(B) * 0.05
            assert 0 < np.max(np.abs(sa - sb)) < bound
