"""Pins of the oracle's random numbers, special functions, rates and inverse CDFs against
things other than itself: published known-answer vectors, mpmath / scipy Bessel functions,
closed-form integrals, and the small-lambda law of the emission spectrum."""
import math
from pathlib import Path

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle

GOLD = Path(__file__).parent / "golden"


# ------------------------------------------------------------------ Philox4x32-10
def test_philox_known_answers():
    rows = [l.split() for l in (GOLD / "philox4x32_10_kat.txt").read_text().splitlines()
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(h, 16) for h in r]
        assert oracle.philox(v[0:4], v[4:6]) == v[6:10]


def test_uniform_maps():
    # 53-bit map: open interval, midpoint offsets; 24-bit map: exactly representable in float32
    assert oracle.u01_53(0, 0) == 0.5 * 2.0 ** -53
    assert oracle.u01_53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 0.5 * 2.0 ** -53
    assert oracle.u01_24(0) == 2.0 ** -24
    assert oracle.u01_24(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(0)
    for hi, lo in rng.integers(0, 2 ** 32, size=(2000, 2)):
        a, b = oracle.u01_53(int(hi), int(lo)), oracle.u01_24(int(hi))
        assert np.float32(b) == b
        assert abs(a - b) < 2.0 ** -23
    # uniformity of the generator over a run of counters (KS, 2e4 draws)
    u = [oracle.u01_53(*oracle.philox([i, 0, 7, 0], [1, 0])[:2]) for i in range(20000)]
    assert stats.kstest(u, "uniform").pvalue > 1e-3


# ------------------------------------------------------------------ Bessel functions
@pytest.mark.parametrize("x", [1e-30, 1e-8, 1e-3, 0.05, 0.0999, 0.1, 0.1001, 0.3, 1.0, 2.5, 7.0, 20.0,
                               60.0, 150.0, 400.0, 699.0])
def test_bessel_K_vs_mpmath(x):
    mp.mp.dps = 30
    k13, k23, _ = oracle.bessel3(x)
    assert abs(k13 / float(mp.besselk(mp.mpf(1) / 3, x)) - 1) < 3e-15
    assert abs(k23 / float(mp.besselk(mp.mpf(2) / 3, x)) - 1) < 4e-15


@pytest.mark.parametrize("x", [1e-8, 1e-3, 0.05, 0.0999, 0.1001, 0.3, 1.0, 2.5, 7.0, 20.0])
def test_intk_vs_mpmath(x):
    mp.mp.dps = 30
    ref = mp.quad(lambda y: mp.besselk(mp.mpf(1) / 3, y), [x, x + 1, x + 10, mp.inf])
    assert abs(oracle.bessel3(x)[2] / float(ref) - 1) < 3e-15


def test_intk_closed_forms():
    # int_0^inf K_1/3 = pi / (2 cos(pi/6)) = pi / sqrt(3)
    assert abs(oracle.bessel3(1e-300)[2] / (math.pi / math.sqrt(3)) - 1) < 1e-15
    # d/dx IntK_1/3(x) = -K_1/3(x), at large x where mpmath's quadrature is not trustworthy
    for x in (60.0, 300.0):
        h = 1e-3
        d = [(oracle.bessel3(x - k * h)[2] - oracle.bessel3(x + k * h)[2]) / (2 * k * h) for k in (1, 2)]
        deriv = (4 * d[0] - d[1]) / 3.0               # Richardson
        assert abs(deriv / oracle.bessel3(x)[0] - 1) < 1e-8
    assert oracle.bessel3(700.0) == (0.0, 0.0, 0.0)


@pytest.mark.parametrize("nu_idx,nu", [(0, 1.0 / 3.0), (1, 2.0 / 3.0)])
def test_bessel_integral_closed_form(nu_idx, nu):
    # int_0^inf K_nu(x) dx = pi / (2 cos(nu pi / 2))
    f = lambda x: oracle.bessel3(x)[nu_idx]
    val = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=200)[0]
              for a, b in [(0, 1e-6), (1e-6, 1e-2), (1e-2, 1), (1, 10), (10, 60)])
    assert abs(val / (math.pi / (2 * math.cos(nu * math.pi / 2))) - 1) < 1e-10


# ------------------------------------------------------------------ rates (independent quadrature)
def _scipy_intk(x):
    if x > 700:
        return 0.0
    return integrate.quad(lambda y: special.kv(1 / 3, y), x, np.inf, epsabs=0, epsrel=1e-13, limit=200)[0]


def _scipy_nlc_rate(chi, sb):
    """int_0^1 [-IntK(u') + kappa K_2/3(u') + sb lam K_1/3(u')] dlam with scipy's Bessel functions,
    integrated in nu = logit(lam)."""
    def f(nu):
        lam, oml = special.expit(nu), special.expit(-nu)
        up = 2.0 * math.exp(nu) / (3.0 * chi)
        if up > 700:
            return 0.0
        kap = 1.0 / oml + oml
        return (-_scipy_intk(up) + kap * special.kv(2 / 3, up) + sb * lam * special.kv(1 / 3, up)) * lam * oml
    hi = math.log(1.5 * chi * 700)
    pts = np.linspace(-40.0, hi, 12)
    body = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-11, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
    lam0 = special.expit(-40.0)
    tail = 3 * special.gamma(2 / 3) * (3 * chi) ** (2 / 3) * lam0 ** (1 / 3)
    return body + tail


def _scipy_nbw_rate(chi, xi3):
    def f(nu):
        lam, oml = special.expit(nu), special.expit(-nu)
        ut = 1.0 / lam + 1.0 / oml
        up = 2.0 * ut / (3.0 * chi)
        if up > 700:
            return 0.0
        rho = oml / lam + lam / oml
        return (_scipy_intk(up) + rho * special.kv(2 / 3, up) - xi3 * special.kv(2 / 3, up)) * lam * oml
    m = math.acosh(max(1.0, 0.75 * chi * 700 - 1))
    pts = np.linspace(-m, m, 10)
    return sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-11, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))


@pytest.mark.parametrize("chi", [0.1, 1.0, 10.0])
def test_nlc_rates_vs_scipy(chi):
    for ch, sb in ((oracle.NLC_DOWN, -1.0), (oracle.NLC_UP, 1.0)):
        assert abs(oracle.rate_integral(ch, chi) / _scipy_nlc_rate(chi, sb) - 1) < 1e-9


@pytest.mark.parametrize("chi", [0.5, 1.0, 10.0])
def test_nbw_rates_vs_scipy(chi):
    for ch, x3 in ((oracle.NBW_MINUS, -1.0), (oracle.NBW_PLUS, 1.0)):
        assert abs(oracle.rate_integral(ch, chi) / _scipy_nbw_rate(chi, x3) - 1) < 1e-9


def test_nlc_classical_limits():
    """Low-chi limits of the spin-averaged photon number and power (known expansions):
    number rate -> (5 pi chi / 2)(1 - 8 sqrt3 chi / 15), power -> (2/3) chi^2 (1 - 55 sqrt3 chi / 16 + 48 chi^2)
    in units of the prefactor alpha / (sqrt3 pi eps_r gamma)."""
    chi = 1e-3
    ibar = 0.5 * (oracle.rate_integral(0, chi) + oracle.rate_integral(1, chi))
    assert abs(ibar / (2.5 * math.pi * chi * (1 - 8 * math.sqrt(3) * chi / 15)) - 1) < 5 * chi ** 2

    def lamw(nu):
        lam = special.expit(nu)
        return lam * 0.5 * (oracle.density_nu(0, chi, nu) + oracle.density_nu(1, chi, nu))
    pts = np.linspace(-40, math.log(1.5 * chi * 700), 20)
    power = sum(integrate.quad(lamw, a, b, epsabs=0, epsrel=1e-12)[0] for a, b in zip(pts[:-1], pts[1:]))
    ref = (2.0 / 3.0) * math.sqrt(3) * math.pi * chi ** 2 * (1 - 55 * math.sqrt(3) / 16 * chi + 48 * chi ** 2)
    assert abs(power / ref - 1) < 5e-6


def test_nbw_low_chi_limits():
    """J_-/J_+ -> 2 and the Erber law J -> sqrt3 pi (3 sqrt3 / (16 sqrt2)) chi exp(-8/(3 chi)) as chi -> 0."""
    prev = None
    for chi in (0.2, 0.1, 0.05):
        jm, jp = oracle.rate_integral(2, chi), oracle.rate_integral(3, chi)
        erber = math.sqrt(3) * math.pi * 3 * math.sqrt(3) / (16 * math.sqrt(2)) * chi * math.exp(-8 / (3 * chi))
        dev = abs(0.5 * (jm + jp) / erber - 1)
        assert dev < 0.2 * chi
        assert abs(jm / jp - 2) < 0.3 * chi
        if prev is not None:
            assert dev < prev
        prev = dev


# ------------------------------------------------------------------ inverse CDFs
@pytest.mark.parametrize("ch,chi", [(0, 1.0), (1, 1e-3), (1, 30.0), (2, 0.05), (3, 1.0), (2, 100.0)])
def test_icdf_inverts_cdf(ch, chi):
    for rho in np.linspace(-37.5, 37.5, 13):
        nu = oracle.icdf_nu(ch, chi, rho)
        lam = special.expit(nu)
        if rho <= 0:
            assert abs(oracle.cdf(ch, chi, lam) / special.expit(rho) - 1) < 1e-11
        else:
            assert abs(oracle.ccdf(ch, chi, lam) / special.expit(-rho) - 1) < 1e-10


def test_icdf_vs_independent_cdf():
    """CDF(ICDF(r)) = r with a CDF integrated by scipy from scipy's Bessel functions."""
    chi = 1.0
    total = _scipy_nlc_rate(chi, 1.0)
    for rho in (-2.0, 0.0, 1.5):
        nu = oracle.icdf_nu(1, chi, rho)

        def f(v):
            lam, oml = special.expit(v), special.expit(-v)
            up = 2.0 * math.exp(v) / (3.0 * chi)
            return (-_scipy_intk(up) + (1 / oml + oml) * special.kv(2 / 3, up) + lam * special.kv(1 / 3, up)) * lam * oml
        pts = np.linspace(-40.0, nu, 10)
        part = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-11)[0] for a, b in zip(pts[:-1], pts[1:]))
        part += 3 * special.gamma(2 / 3) * (3 * chi) ** (2 / 3) * special.expit(-40.0) ** (1 / 3)
        assert abs(part / total / special.expit(rho) - 1) < 1e-8


def test_icdf_small_lambda_law():
    """For r -> 0 the NLC spectrum gives lam = (r I / (3 Gamma(2/3) (3 chi)^(2/3)))^3."""
    for chi in (1e-2, 1.0, 50.0):
        for ch in (0, 1):
            total = oracle.rate_integral(ch, chi)
            for rho in (-30.0, -20.0):
                r = special.expit(rho)
                lam = special.expit(oracle.icdf_nu(ch, chi, rho))
                ref = (r * total / (3 * special.gamma(2 / 3) * (3 * chi) ** (2 / 3))) ** 3
                assert abs(lam / ref - 1) < 1e-6


def test_nbw_icdf_symmetry():
    # the NBW spectrum is symmetric under lam <-> 1 - lam, so nu(-rho) = -nu(rho)
    for ch in (2, 3):
        for chi in (0.1, 2.0, 50.0):
            for rho in (0.3, 5.0, 30.0):
                assert abs(oracle.icdf_nu(ch, chi, rho) + oracle.icdf_nu(ch, chi, -rho)) < 1e-12 * max(
                    1, abs(oracle.icdf_nu(ch, chi, rho)))


def test_tables_interpolation_error(otables):
    """Method error of the contract grid against the exact inverse CDF and rates (reported, bounded)."""
    rng = np.random.default_rng(5)
    worst_nu, worst_rate = 0.0, 0.0
    for _ in range(40):
        ch = int(rng.integers(0, 4))
        lo, hi = ((math.log(1e-3), math.log(1e2)) if ch < 2 else (math.log(0.05), math.log(1e2)))
        lnchi = rng.uniform(lo, hi)
        rho = rng.uniform(-30, 30)
        worst_nu = max(worst_nu, abs(otables.nu(ch, lnchi, rho) - oracle.icdf_nu(ch, math.exp(lnchi), rho)))
        ex = math.log(oracle.rate_integral(ch, math.exp(lnchi)))
        worst_rate = max(worst_rate, abs(otables.lnrate(ch, lnchi) - ex))
    # measured over 2000 points per channel: 4.5e-5 in nu (NBW xi3 = +1; the others 4e-7) and
    # 1.1e-8 in ln rate (the pair rows carry the Erber exponent 8/(3 chi) taken out)
    assert worst_nu < 1e-4
    assert worst_rate < 3e-8


@pytest.mark.parametrize("ch,chi", [(2, 0.0537), (3, 0.3), (3, 5.0), (0, 1e-3), (1, 0.05), (0, 10.0), (1, 100.0)])
def test_icdf_tails_vs_independent_quadrature(ch, chi):
    """Tail probabilities at the extreme table nodes (rho = +-37.5, |r - 0 or 1| ~ 5e-17), where
    the density falls by ~e^50 per unit nu, against scipy's adaptive quadrature of the
    density between the root and a point far in the tail."""
    tot = oracle.rate_integral(ch, chi)
    f = lambda v: oracle.density_nu(ch, chi, v)
    for rho in (-37.5, -30.0, 30.0, 37.5):
        nu = oracle.icdf_nu(ch, chi, rho)
        if rho > 0:
            pts = np.linspace(nu, nu + 8.0, 200)
            target = special.expit(-rho)
        else:
            if ch < 2 and nu < -60:
                continue          # below nu = -60 the small-lambda law (pinned separately) is used
            pts = np.linspace(nu - 8.0 if ch >= 2 else -60.0, nu, 200)
            target = special.expit(rho)
        val = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=300)[0] for a, b in zip(pts[:-1], pts[1:]))
        if rho < 0 and ch < 2:
            lam0 = special.expit(-60.0)
            val += 3 * special.gamma(2 / 3) * (3 * chi) ** (2 / 3) * lam0 ** (1 / 3) - math.pi / math.sqrt(3) * lam0
        assert abs(val / tot / target - 1) < 1e-12, (rho, val / tot / target - 1)
