"""Pins of the oracle's rejection-sampling mode (spectrum-sampling section): the candidate
lambda = r1^3 is accepted with probability 3 r1^2 dW/dlambda dt, so per step an electron emits
with probability W_s dt, and the accepted lambda follow the spectrum of its spin state.  Both
are checked against the oracle's quadrature rate and CDF (an independent route: they integrate
the spectrum, the rejection step only evaluates it), on electrons at chi = 1 in a uniform B."""
import math

import numpy as np

import oracle
import synth

EPS = synth.EPS_R


def _run(otables, sb, n, dt, seed):
    gamma = 2000.0
    B = np.array([0.0, 0.0, 1.0 / (EPS * math.sqrt(gamma * gamma - 1.0))])      # chi = 1
    p = np.array([math.sqrt(gamma * gamma - 1.0), 0.0, 0.0])
    chi, e, b, k = oracle.basis(-1, EPS, np.zeros(3), B, p)
    L = oracle.LeptonSet(0, n, track=(False, False, False))
    L.set(np.zeros((3, n)), np.repeat(p[:, None], n, axis=1), np.repeat((sb * b)[:, None], n, axis=1))
    G = oracle.PhotonSet(n, track=(False, False, False))
    F = oracle.make_fields(oracle.FIELD_UNIFORM, B0=B)
    ctr = oracle.Counters()
    prm = oracle.make_params(dt, EPS, step=0, seed=seed, flags=oracle.F_EMIT | oracle.F_REJECT)
    oracle.lepton_step(otables, prm, F, L, G, ctr)
    lam = np.linalg.norm(np.stack([G.k[c][:G.n] for c in range(3)]), axis=0) / np.linalg.norm(p)
    return chi, gamma, lam, ctr


def test_rejection_rate_and_spectrum(otables):
    n = 30_000
    for sb, ch in ((1.0, oracle.NLC_UP), (-1.0, oracle.NLC_DOWN)):
        gamma = 2000.0
        ce = oracle.ALPHA / (math.sqrt(3) * math.pi * EPS * gamma)
        W = ce * oracle.rate_integral(ch, 1.0)
        dt = 0.25 / W
        # the acceptance probability stays below 1 for every candidate
        r = np.linspace(1e-4, 1 - 1e-4, 4001)
        A = np.array([3 * x * x * ce * oracle.nlc_w(1.0, x ** 3, sb) * dt for x in r])
        assert A.max() < 1.0
        chi, gamma, lam, ctr = _run(otables, sb, n, dt, seed=31 + int(sb > 0))
        assert abs(chi - 1.0) < 1e-12
        f = lam.size / n
        assert abs(f - 0.25) < 4 * math.sqrt(0.25 * 0.75 / n), (sb, f)
        assert ctr.n_prob_clamped == 0
        # empirical CDF of the accepted lambda against the quadrature CDF of the spin state
        for q in (1e-4, 1e-3, 1e-2, 0.05, 0.1, 0.2, 0.3, 0.5, 0.7, 0.9):
            c = oracle.cdf(ch, 1.0, q)
            emp = np.mean(lam <= q)
            assert abs(emp - c) < 4 * math.sqrt(c * (1 - c) / lam.size) + 1e-12, (sb, q, emp, c)


def test_rejection_spin_asymmetry(otables):
    """The two spin states emit at different rates (the spin-resolved spectrum's lambda s K1/3
    term): the frequencies at one dt differ by the ratio of the up and down rate integrals."""
    gamma = 2000.0
    ce = oracle.ALPHA / (math.sqrt(3) * math.pi * EPS * gamma)
    Wu, Wd = ce * oracle.rate_integral(oracle.NLC_UP, 1.0), ce * oracle.rate_integral(oracle.NLC_DOWN, 1.0)
    dt = 0.2 / max(Wu, Wd)
    n = 30_000
    fu = _run(otables, 1.0, n, dt, seed=41)[2].size / n
    fd = _run(otables, -1.0, n, dt, seed=42)[2].size / n
    for f, W in ((fu, Wu), (fd, Wd)):
        assert abs(f - W * dt) < 4 * math.sqrt(W * dt * (1 - W * dt) / n)
    assert (fu > fd) == (Wu > Wd)
