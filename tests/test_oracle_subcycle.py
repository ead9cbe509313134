"""Pins of the oracle's per-particle sub-cycling of the lepton step (F_SUB; the decision-making
section asks for W dt << 1): no change where W dt <= 0.1; binomial emission counts with m
sub-steps at constant W (including the cap of 16); the exact Sokolov-Ternov recursion over the
sub-steps in the test-particle workload, whose W dt is about 0.95."""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
import synth

EPS = synth.EPS_R
CE = lambda gamma: oracle.ALPHA / (math.sqrt(3) * math.pi * EPS * gamma)


def _run(otables, flags, p, s, B, dt, step=5, seed=3, track=(False, False, False)):
    n = p.shape[1]
    L = oracle.LeptonSet(0, n, track=track)
    L.set(np.zeros((3, n)), p, s)
    G = oracle.PhotonSet(40 * n, track=track)
    F = oracle.make_fields(oracle.FIELD_UNIFORM, B0=(0, 0, B))
    ctr = oracle.Counters()
    prm = oracle.make_params(dt, EPS, step=step, seed=seed, flags=flags)
    oracle.lepton_step(otables, prm, F, L, G, ctr)
    return L, G, ctr


def _wbar_dt(otables, chi, gamma, dt):
    lc = math.log(chi)
    return CE(gamma) * 0.5 * (math.exp(otables.lnrate(0, lc)) + math.exp(otables.lnrate(1, lc))) * dt


def test_subcycling_changes_nothing_below_threshold(otables):
    """Every lepton below W dt = 0.1 takes one sub-step with the step's own draws and photon ids:
    the step is bit for bit the plain one."""
    rng = np.random.default_rng(4)
    n = 3000
    g = np.exp(rng.uniform(math.log(300), math.log(3000), n))
    p = synth.random_unit_vectors(rng, n) * np.sqrt(g * g - 1)
    s = synth.random_unit_vectors(rng, n) * rng.uniform(0, 1, n)
    B = 40.0
    # chi <= eps_r |p| B and W_s <= 1.2 W-bar: the largest W dt is kept at 0.08
    wmax = max(_wbar_dt(otables, EPS * math.sqrt(gi * gi - 1) * B, gi, 1.0) for gi in g)
    dt = 0.08 / (1.2 * wmax)
    flags = oracle.F_ALL & ~oracle.F_PAIR
    a = _run(otables, flags, p, s, B, dt)
    b = _run(otables, flags | oracle.F_SUB, p, s, B, dt)
    assert a[2].n_emit > 100 and a[2].n_emit == b[2].n_emit
    for u, v in zip(a[0].arrays(), b[0].arrays()):
        np.testing.assert_array_equal(u, v)
    for u, v in zip(a[1].arrays(), b[1].arrays()):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("wdt, m", [(0.7, 8), (3.0, 16)])
def test_subcycled_emission_counts_are_binomial(otables, wdt, m):
    """Constant W (no recoil, no spin change, unpolarized): the photons of one lepton in one step
    follow Binomial(m, W dt / m), m the smallest power of two with W dt / m <= 0.1, at most 16;
    the rounds in their ids are the multiples of 16/m."""
    n, gamma, chi = 40_000, 2000.0, 1.0
    pm = math.sqrt(gamma ** 2 - 1)
    B = chi / (EPS * pm)
    dt = wdt / _wbar_dt(otables, chi, gamma, 1.0)
    p = np.zeros((3, n)); p[0] = pm
    flags = oracle.F_EMIT | oracle.F_SUB
    L, G, ctr = _run(otables, flags, p, np.zeros((3, n)), B, dt)
    ids = G.arrays()[3][:G.n].astype(np.uint64)
    parent = ((ids >> np.uint64(24)) & np.uint64((1 << 33) - 1)).astype(np.int64)
    rnd = ((ids >> np.uint64(57)) & np.uint64(15)).astype(np.int64)
    assert set(np.unique(rnd)) <= set(range(0, 16, 16 // m))
    counts = np.bincount(parent, minlength=n)
    q = wdt / m
    assert ctr.n_prob_clamped == 0
    assert abs(counts.mean() - wdt) < 5 * math.sqrt(m * q * (1 - q) / n)
    kmax = 5
    obs = np.array([np.sum(counts == k) for k in range(kmax)] + [np.sum(counts >= kmax)])
    pk = np.array([stats.binom.pmf(k, m, q) for k in range(kmax)] + [stats.binom.sf(kmax - 1, m, q)])
    chi2 = np.sum((obs - n * pk) ** 2 / (n * pk))
    assert chi2 < stats.chi2.ppf(0.999, len(pk) - 1), (obs, n * pk)


def _psi(chi):
    def f(u, k):
        up = 2 * u / (3 * chi)
        return u * u / (1 + u) ** 3 * (special.kv(2 / 3, up) if k == 1 else special.kv(1 / 3, up))
    pts = [0, 0.1, 1, 10, 100, 2000]
    return [sum(integrate.quad(f, a, b, args=(k,), epsabs=0, epsrel=1e-11)[0] for a, b in zip(pts[:-1], pts[1:]))
            for k in (1, 3)]


def test_subcycled_sokolov_ternov_recursion(otables):
    """The test-particle workload (W dt = 0.95, so 16 sub-steps) with recoil off and an
    unpolarized start: the mean of s.beta after n steps is exactly
    (psi3/psi1)(1 - (1 - C_e psi1 dt/16)^(16 n)), the per-step recursion over the sub-steps."""
    w = synth.c1(n=30_000)
    gamma = w.extra["gamma0"]
    assert 0.8 < _wbar_dt(otables, 1.0, gamma, w.dt) < 1.0
    psi1, psi3 = _psi(1.0)
    L = oracle.LeptonSet(0, w.n, track=w.track)
    L.set(w.x, w.p, np.zeros_like(w.s))
    G = oracle.PhotonSet(40 * w.n, track=w.track)
    F = oracle.make_fields(w.field_kind, B0=w.B0)
    flags = oracle.F_PUSH | oracle.F_TBMT | oracle.F_EMIT | oracle.F_SPIN | oracle.F_NOEMIT | oracle.F_SUB
    ctr = oracle.Counters()
    h = w.dt / 16
    for n in range(1, 13):
        prm = oracle.make_params(w.dt, EPS, step=n, t=n * w.dt, seed=7, flags=flags)
        G.n = 0
        oracle.lepton_step(otables, prm, F, L, G, ctr)
        if n in (1, 4, 12):
            _, p, s = L.arrays()
            sb = -s[2]
            exp_n = psi3 / psi1 * (1 - (1 - CE(gamma) * psi1 * h) ** (16 * n))
            sigma = np.std(sb) / math.sqrt(w.n)
            assert abs(sb.mean() - exp_n) < 5 * sigma + 2e-3, (n, sb.mean(), exp_n)
    assert ctr.n_norm_clamped == 0 and ctr.n_prob_clamped == 0
