"""Pins of the oracle's particle dynamics: Boris + T-BMT closed forms, the rest-frame basis and
chi against a Lorentz transformation, the photon P-vector (photon-polarization section), and
statistical laws that hold exactly in expectation for the whole Monte-Carlo step:
the Sokolov-Ternov recursion, the means of the collapsed spin / Stokes vectors and pair spins,
and the equal evolution of differently built "unpolarized" photon beams (non-transition section)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import synth

EPS = synth.EPS_R
A_E = oracle.ALPHA / (2 * math.pi)
CE = lambda gamma: oracle.ALPHA / (math.sqrt(3) * math.pi * EPS * gamma)


# ------------------------------------------------------------------ push + T-BMT
def _angle_in_plane(a, b):
    return math.atan2(a[0] * b[1] - a[1] * b[0], a[0] * b[0] + a[1] * b[1])


def test_g2_keeps_spin_momentum_angle():
    rng = np.random.default_rng(1)
    B = np.array([0.0, 0.0, 3.7])
    p = np.array([40.0, -15.0, 6.0])
    s = rng.normal(size=3); s /= np.linalg.norm(s)
    c0 = s @ p / np.linalg.norm(p)
    x = np.zeros(3)
    for _ in range(1000):
        p, s, x = oracle.push_one(-1, 0.0, np.zeros(3), B, 0.05, oracle.F_TBMT, p, s, x)
    assert abs(s @ p / np.linalg.norm(p) - c0) < 1e-12
    assert abs(np.linalg.norm(s) - 1) < 1e-13


def test_anomalous_moment_closed_form():
    """p and s in the plane normal to B: per step p turns by 2 atan(B dt / (2 gamma)) and s by
    2 atan((a + 1/gamma) B dt / 2) (Cayley rotations), so their angle changes by the difference."""
    B, dt, a = 2.0, 0.03, 0.05
    p = np.array([30.0, 0.0, 0.0]); s = np.array([0.6, 0.8, 0.0]); x = np.zeros(3)
    gamma = math.sqrt(1 + p @ p)
    phi_p = 2 * math.atan(B * dt / (2 * gamma))
    phi_s = 2 * math.atan((a + 1 / gamma) * B * dt / 2)
    ang0 = _angle_in_plane(p, s)
    p0 = p.copy()
    n = 500
    for _ in range(n):
        p, s, x = oracle.push_one(-1, a, np.zeros(3), np.array([0, 0, B]), dt, oracle.F_TBMT, p, s, x)
    d = lambda v: (v + math.pi) % (2 * math.pi) - math.pi
    assert abs(d(_angle_in_plane(p0, p) - d(n * phi_p))) < 1e-10
    assert abs(d(_angle_in_plane(p, s) - ang0 - n * (phi_s - phi_p))) < 1e-10


def test_push_electric_field_and_position():
    E = np.array([0.3, -0.2, 0.1]); dt = 0.1
    p = np.array([1.0, 2.0, -0.5]); s = np.array([0, 0, 1.0]); x = np.zeros(3)
    p1, s1, x1 = oracle.push_one(+1, A_E, E, np.zeros(3), dt, 0, p, s, x)
    np.testing.assert_allclose(p1, p + dt * E, rtol=0, atol=1e-15)
    np.testing.assert_allclose(x1, p1 / math.sqrt(1 + p1 @ p1) * dt, rtol=1e-15)
    np.testing.assert_array_equal(s1, s)      # T-BMT off: spin untouched


# ------------------------------------------------------------------ basis and chi
def _rest_frame_E(E, B, p):
    g = math.sqrt(1 + p @ p); v = p / g
    return g * (E + np.cross(v, B)) - g * g / (g + 1) * v * (v @ E)


def test_basis_and_chi():
    rng = np.random.default_rng(2)
    for _ in range(200):
        E, B = rng.normal(size=3) * 10, rng.normal(size=3) * 10
        p = rng.normal(size=3) * 10 ** rng.uniform(0, 4)
        for q in (-1, 1):
            chi, e, b, k = oracle.basis(q, EPS, E, B, p)
            np.testing.assert_allclose([e @ e, b @ b, k @ k, e @ b, e @ k, b @ k], [1, 1, 1, 0, 0, 0], atol=1e-13)
            np.testing.assert_allclose(np.cross(e, b), k, atol=1e-13)            # right-handed
            assert abs(chi / (EPS * np.linalg.norm(_rest_frame_E(E, B, p))) - 1) < 1e-9
        chi_g, e, b, k = oracle.basis(0, EPS, E, B, p)
        pn = np.linalg.norm(p)
        ref = EPS * math.sqrt(max(0, np.sum((pn * E + np.cross(p, B)) ** 2) - (p @ E) ** 2))
        assert abs(chi_g / ref - 1) < 1e-12


def test_basis_orientation_in_magnetic_field():
    """Electron moving along x in B_z: eps = -y, beta = -z (against B); positron: beta = +z."""
    B = np.array([0, 0, 5.0]); p = np.array([100.0, 0, 0])
    _, e, b, _ = oracle.basis(-1, EPS, np.zeros(3), B, p)
    np.testing.assert_allclose(e, [0, -1, 0], atol=1e-15); np.testing.assert_allclose(b, [0, 0, -1], atol=1e-15)
    _, e, b, _ = oracle.basis(1, EPS, np.zeros(3), B, p)
    np.testing.assert_allclose(e, [0, 1, 0], atol=1e-15); np.testing.assert_allclose(b, [0, 0, 1], atol=1e-15)


# ------------------------------------------------------------------ P-vector
def test_pvector_round_trip_and_rotation():
    rng = np.random.default_rng(3)
    for _ in range(500):
        xi = rng.normal(size=3); xi *= rng.uniform(0, 1) / np.linalg.norm(xi)
        k = rng.normal(size=3); k /= np.linalg.norm(k)
        e = np.cross(k, rng.normal(size=3)); e /= np.linalg.norm(e)
        b = np.cross(k, e)
        P = oracle.stokes_to_P(xi, e, b, k)
        assert abs(np.linalg.norm(P) - np.linalg.norm(xi)) < 1e-14
        np.testing.assert_allclose(oracle.P_to_stokes(P, e, b, k), xi, atol=1e-13)
        phi = rng.uniform(-math.pi, math.pi)
        o1 = e * math.cos(phi) + b * math.sin(phi); o2 = -e * math.sin(phi) + b * math.cos(phi)
        ref = [xi[0] * math.cos(2 * phi) - xi[2] * math.sin(2 * phi), xi[1],
               xi[0] * math.sin(2 * phi) + xi[2] * math.cos(2 * phi)]
        np.testing.assert_allclose(oracle.P_to_stokes(P, o1, o2, k), ref, atol=1e-13)


# ------------------------------------------------------------------ exact-in-expectation laws
def _psi(chi):
    """psi1 = int (kappa-2) K_2/3(u') dlam, psi3 = int (u - lam) K_1/3(u') dlam with scipy's Bessel."""
    def f(nu, which):
        lam, oml = special.expit(nu), special.expit(-nu)
        up = 2 * math.exp(nu) / (3 * chi)
        if up > 700:
            return 0.0
        w = (lam * lam / oml) * (special.kv(2 / 3, up) if which == 1 else special.kv(1 / 3, up))
        return w * lam * oml
    pts = np.linspace(-40, math.log(1.5 * chi * 700), 15)
    return [sum(integrate.quad(f, a, b, args=(k,), epsabs=0, epsrel=1e-11)[0] for a, b in zip(pts[:-1], pts[1:]))
            for k in (1, 3)]


def test_sokolov_ternov_recursion(otables):
    """Recoil off, constant B, unpolarized start (s = 0): the mean of s.beta after n steps is exactly
    (psi3/psi1)(1 - (1 - C_e psi1 dt)^n) for the per-step algorithm (decision, mixture, collapse with
    mean g/w, no-emission update)."""
    w = synth.c1(n=50_000)
    gamma = w.extra["gamma0"]
    psi1, psi3 = _psi(1.0)
    L = oracle.LeptonSet(0, w.n, track=w.track)
    L.set(w.x, w.p, np.zeros_like(w.s))
    G = oracle.PhotonSet(w.n, track=w.track)
    F = oracle.make_fields(w.field_kind, B0=w.B0)
    flags = oracle.F_PUSH | oracle.F_TBMT | oracle.F_EMIT | oracle.F_SPIN | oracle.F_NOEMIT
    ctr = oracle.Counters()
    for n in range(1, 41):
        prm = oracle.make_params(w.dt, EPS, step=n, t=n * w.dt, seed=7, flags=flags)
        G.n = 0
        oracle.lepton_step(otables, prm, F, L, G, ctr)
        if n in (3, 10, 25, 40):
            _, p, s = L.arrays()
            sb = -s[2]                                    # beta = -z for electrons in B_z
            exp_n = psi3 / psi1 * (1 - (1 - CE(gamma) * psi1 * w.dt) ** n)
            sigma = np.std(sb) / math.sqrt(w.n)
            assert abs(sb.mean() - exp_n) < 5 * sigma + 2e-3, (n, sb.mean(), exp_n)
    assert ctr.n_norm_clamped == 0 and ctr.n_prob_clamped == 0


def _one_step_emitters(otables, s0, chi=1.0, n=40_000, flags=None):
    gamma = 2000.0
    pm = math.sqrt(gamma ** 2 - 1)
    B = chi / (EPS * pm)
    L = oracle.LeptonSet(0, n, track=(False, False, False))
    p = np.zeros((3, n)); p[0] = pm
    L.set(np.zeros((3, n)), p, np.tile(np.asarray(s0, float)[:, None], (1, n)))
    G = oracle.PhotonSet(n, track=(False, False, False))
    F = oracle.make_fields(oracle.FIELD_UNIFORM, B0=(0, 0, B))
    dt = 0.6 / (CE(gamma) * 5.6)
    flags = flags or (oracle.F_EMIT | oracle.F_SPIN | oracle.F_PHOTON_POL | oracle.F_NOEMIT)
    prm = oracle.make_params(dt, EPS, step=3, seed=11, flags=flags)
    oracle.lepton_step(otables, prm, F, L, G, oracle.Counters())
    _, e, b, k = oracle.basis(-1, EPS, np.zeros(3), np.array([0, 0, B]), p[:, 0])
    return L, G, (e, b, k)


def _lam_means(chi, si):
    """(int g dlam, int F(s_f = 0) dlam) / int w dlam, components in (eps, beta, k)."""
    def comp(nu, j):
        lam = special.expit(nu)
        jac = lam * special.expit(-nu)
        if j < 3:
            return oracle.nlc_g(chi, lam, si)[j] * jac
        if j < 6:
            return oracle.nlc_F(chi, lam, si, np.zeros(3))[j - 2] * jac
        return oracle.nlc_w(chi, lam, si[1]) * jac
    pts = np.linspace(-40, math.log(1.5 * chi * 700), 15)
    v = [sum(integrate.quad(comp, a, b, args=(j,), epsabs=1e-14, epsrel=1e-9)[0]
             for a, b in zip(pts[:-1], pts[1:])) for j in range(7)]
    return np.array(v[:3]) / v[6], np.array(v[3:6]) / v[6]


@pytest.mark.parametrize("s0", [(0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.6, 0.0, 0.8)])
def test_collapse_means(otables, s0):
    """Mean final spin over emitters = int g / int w; mean photon Stokes = int F(s_f=0) / int w."""
    L, G, (e, b, k) = _one_step_emitters(otables, s0)
    _, _, s = L.arrays()
    emitted = G.id[:G.n] != 0
    assert emitted.sum() > 10_000
    par = oracle.nlc_g  # noqa: F841  (documentation: the reference uses the printed g and F)
    si = np.array([np.dot(s0, e), np.dot(s0, b), np.dot(s0, k)])
    mg, mF = _lam_means(1.0, si)
    # emitters are the leptons whose index appears as a photon parent
    parents = ((G.id[:G.n].astype(np.uint64) >> np.uint64(24)) & np.uint64((1 << 33) - 1)).astype(np.int64)
    sf = s[:, parents]
    comp = np.stack([e @ sf, b @ sf, k @ sf])
    xi = np.stack([oracle.P_to_stokes(np.array([G.P[i][j] for i in range(3)]), e, b, k) for j in range(G.n)]).T
    tol = 5 / math.sqrt(emitted.sum()) + 2e-3
    np.testing.assert_allclose(comp.mean(axis=1), mg, atol=tol)
    np.testing.assert_allclose(xi.mean(axis=1), mF, atol=tol)
    assert np.all(np.abs(np.linalg.norm(sf, axis=0) - 1) < 1e-12)       # pure final spins
    assert np.all(np.abs(np.linalg.norm(xi, axis=0) - 1) < 1e-12)       # pure photon states


def _photon_beam(n, chi, xi_half, wdt, k0=1e4):
    B = chi / (EPS * k0)
    G = oracle.PhotonSet(2 * n, track=(False, False, False))
    k = np.array([k0, 0.0, 0.0])
    _, e, b, kh = oracle.basis(0, EPS, np.zeros(3), np.array([0, 0, B]), k)
    Pp = oracle.stokes_to_P(np.asarray(xi_half, float), e, b, kh)
    Pm = oracle.stokes_to_P(-np.asarray(xi_half, float), e, b, kh)
    for i in range(3):
        G.k[i][:2 * n] = k[i]
        G.P[i][:n], G.P[i][n:2 * n] = Pp[i], Pm[i]
    G.id[:2 * n] = (np.uint64(1) << np.uint64(63)) | (np.arange(2 * n, dtype=np.uint64) << np.uint64(24))
    G.n = G.n_prev = 2 * n
    jbar = 0.5 * (oracle.rate_integral(2, chi) + oracle.rate_integral(3, chi))
    dt = wdt / (oracle.ALPHA / (math.sqrt(3) * math.pi * EPS * k0) * jbar)
    return G, oracle.make_fields(oracle.FIELD_UNIFORM, B0=(0, 0, B)), dt, (e, b, kh)


def _xi3_of(G, mask, basis):
    # the P-vector decode of the photon-polarization section, vectorized for the test's measurement
    e, b, _ = basis
    P = np.stack([G.P[i][:G.n][mask] for i in range(3)])
    d = np.linalg.norm(P, axis=0)
    p1, p2 = (e @ P) / d, (b @ P) / d
    r = np.sqrt(p1 * p1 + p2 * p2)
    return np.where(r > 0, d * (p1 * p1 - p2 * p2) / np.where(r > 0, r, 1.0), 0.0)


def test_unpolarized_photon_beams_evolve_alike(otables):
    """Three 'unpolarized' beams (opposite linear / circular / diagonal halves) give the same
    survivor count and mean xi3 with the no-pair update, equal to the linear recursion for
    (count, sum xi3); without it they differ (non-transition section, second example)."""
    chi, n, steps = 1.0, 20_000, 8
    res = {}
    for upd in (True, False):
        for name, xh in (("lin", (0, 0, 1)), ("circ", (0, 1, 0)), ("diag", (1, 0, 0))):
            G, F, dt, basis = _photon_beam(n, chi, xh, 0.05)
            flags = oracle.F_PAIR | (oracle.F_NOPAIR if upd else 0)
            Le, Lp = oracle.LeptonSet(0, 2 * n), oracle.LeptonSet(1, 2 * n)
            for st in range(steps):
                oracle.photon_step(otables, oracle.make_params(dt, EPS, step=st, seed=5, flags=flags), F, G, Le, Lp,
                                   oracle.Counters())
            alive = G.id[:G.n] != 0
            x3 = _xi3_of(G, alive, basis)
            res[(upd, name)] = (alive.mean(), x3.sum() / (2 * n))
    Jm, Jp = oracle.rate_integral(2, chi), oracle.rate_integral(3, chi)
    wbar_dt = 0.05
    dW_dt = wbar_dt * (Jp - Jm) / (Jp + Jm)
    A, X = 1.0, 0.0
    for _ in range(steps):
        A, X = A * (1 - wbar_dt) - dW_dt * X, X * (1 - wbar_dt) - dW_dt * A
    tol = 5 / math.sqrt(2 * n)
    for name in ("lin", "circ", "diag"):
        a, x = res[(True, name)]
        assert abs(a - A) < tol and abs(x - X) < tol, (name, a, A, x, X)
    # without the update the linear and circular beams separate
    assert abs(res[(False, "lin")][1] - res[(False, "circ")][1]) > 2 * tol


def test_pair_spin_means(otables):
    """Mean produced-lepton spins over pair events = int j / int w0 (NBW section)."""
    chi, n = 2.0, 30_000
    xi0 = np.array([0.3, 0.5, -0.4])
    G, F, dt, (e, b, kh) = _photon_beam(n, chi, xi0, 0.5)
    for j in range(n, 2 * n):      # make the whole beam the same state
        for i in range(3):
            G.P[i][j] = G.P[i][0]
    Le, Lp = oracle.LeptonSet(0, 2 * n), oracle.LeptonSet(1, 2 * n)
    oracle.photon_step(otables, oracle.make_params(dt, EPS, step=1, seed=9, flags=oracle.F_PAIR | oracle.F_PAIR_SPIN),
                       F, G, Le, Lp, oracle.Counters())
    assert Le.n > 10_000

    def comp(nu, j):
        lam = special.expit(nu)
        w0, je, jp = oracle.nbw_j(chi, lam, xi0)
        v = [*je, *jp, w0][j]
        return v * lam * special.expit(-nu)
    m = math.acosh(0.75 * chi * 700 - 1)
    pts = np.linspace(-m, m, 12)
    v = [sum(integrate.quad(comp, a, c, args=(j,), epsabs=1e-15, epsrel=1e-9)[0] for a, c in zip(pts[:-1], pts[1:]))
         for j in range(7)]
    _, _, se = Le.arrays(); _, _, sp = Lp.arrays()
    tol = 5 / math.sqrt(Le.n) + 2e-3
    np.testing.assert_allclose([e @ se.mean(1), b @ se.mean(1), kh @ se.mean(1)], np.array(v[0:3]) / v[6], atol=tol)
    np.testing.assert_allclose([e @ sp.mean(1), b @ sp.mean(1), kh @ sp.mean(1)], np.array(v[3:6]) / v[6], atol=tol)
    # momentum conservation: p_e + p_p = k for every pair
    _, pe, _ = Le.arrays(); _, pp, _ = Lp.arrays()
    np.testing.assert_allclose(pe + pp, np.tile([[1e4], [0], [0]], (1, Le.n)), rtol=1e-14)


# ------------------------------------------------------------------ array-step semantics
def test_array_step_bookkeeping(otables):
    w = synth.c1(n=64)
    L = oracle.LeptonSet(0, 64, track=w.track); L.set(w.x, w.p, w.s)
    G = oracle.PhotonSet(150, track=w.track)
    F = oracle.make_fields(w.field_kind, B0=w.B0)
    ctr = oracle.Counters()
    for n in range(3):
        oracle.lepton_step(otables, oracle.make_params(w.dt, EPS, step=n, seed=1, flags=oracle.F_ALL), F, L, G, ctr)
    assert G.n == 150 and ctr.n_capacity_overflow == ctr.n_emit - 150
    ids = G.id[:G.n].astype(np.uint64)
    step = (ids & np.uint64(0xFFFFFF)).astype(np.int64)
    parent = ((ids >> np.uint64(24)) & np.uint64((1 << 33) - 1)).astype(np.int64)
    order = step * 1000 + parent
    assert np.all(np.diff(order) > 0)                   # appended by step, then by parent index
    assert np.all(ids >> np.uint64(63) == 1)
    # retirement at birth leaves dead slots; compaction keeps the order of the survivors
    G2 = oracle.PhotonSet(1000, track=w.track)
    for n in range(3):
        oracle.lepton_step(otables, oracle.make_params(w.dt, EPS, step=n, seed=1, flags=oracle.F_ALL, k_retire=150.0),
                           F, L, G2, ctr)
    live = G2.id[:G2.n][G2.id[:G2.n] != 0].copy()
    assert 0 < live.size < G2.n
    oracle.compact(G2)
    assert G2.n == live.size and G2.n_prev == live.size
    np.testing.assert_array_equal(G2.id[:G2.n], live)


def test_optical_depth_decision_is_memoryless(otables):
    """Optical-depth decision with a constant rate (recoil off, unpolarized electrons that stay
    unpolarized, chi = 1 held by a pure B): tau restarts at 0 after each emission, so an emission in
    a step is Bernoulli with probability 1 - exp(-W dt), independent of the past; the per-step
    draw gives W dt.  W from scipy quadrature of scipy's Bessel functions."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_special import _scipy_nlc_rate
    w = synth.c1(n=20_000)
    gamma = w.extra["gamma0"]
    P = CE(gamma) * 0.5 * (_scipy_nlc_rate(1.0, 1.0) + _scipy_nlc_rate(1.0, -1.0)) * w.dt
    base = oracle.F_PUSH | oracle.F_TBMT | oracle.F_EMIT
    F = oracle.make_fields(w.field_kind, B0=w.B0)
    for mode, expect in ((oracle.F_TAU, 1.0 - math.exp(-P)), (0, P)):
        L = oracle.LeptonSet(0, w.n, track=w.track, tau=True)
        L.set(w.x, w.p, np.zeros_like(w.s))
        G = oracle.PhotonSet(w.n, track=w.track)
        hist = []
        for k in range(8):
            prm = oracle.make_params(w.dt, EPS, step=k, t=k * w.dt, seed=5, flags=base | mode)
            G.n = 0
            oracle.lepton_step(otables, prm, F, L, G, oracle.Counters())
            par = (G.id[:G.n] >> np.uint64(24)) & np.uint64((1 << 33) - 1)
            e = np.zeros(w.n, bool)
            e[par.astype(np.int64)] = True
            hist.append(e)
        h = np.array(hist)
        sigma = math.sqrt(expect * (1 - expect) / h.size)
        assert abs(h.mean() - expect) < 5 * sigma, (mode, h.mean(), expect)
        if mode:
            # independence of consecutive steps
            both = (h[1:] & h[:-1]).mean()
            assert abs(both - expect ** 2) < 5 * math.sqrt(expect ** 2 * (1 - expect ** 2) / h[1:].size)
            assert np.all(L.tau[:w.n] >= 0) and np.all(L.tau_target[:w.n] > 0)


def test_grid_fields_bilinear_and_periodic():
    """Grid field model: reproduces a field linear in x and y exactly inside the grid (bilinear
    interpolation is exact for it), returns node values at nodes, and is periodic."""
    nx, ny, dx, dy, x0, y0 = 7, 5, 0.3, 0.45, -1.0, 2.0
    X, Y = np.meshgrid(x0 + dx * np.arange(nx), y0 + dy * np.arange(ny))
    coef = np.array([[1.0, 2.0, -0.5], [0.3, -1.0, 0.7], [-2.0, 0.1, 0.2], [0.5, 0.5, 0.5], [1.5, -0.2, 0.0],
                     [0.0, 1.0, -1.0]])
    grid = np.stack([c[0] + c[1] * X + c[2] * Y for c in coef]).astype(np.float32)
    F = oracle.make_fields(oracle.FIELD_GRID2D, E0=(0.1, 0, 0), grid=grid, dx=dx, dy=dy, x0=x0, y0=y0)
    rng = np.random.default_rng(0)
    for _ in range(50):
        x = x0 + dx * rng.uniform(0, nx - 1)
        y = y0 + dy * rng.uniform(0, ny - 1)
        E, B = oracle.fields_eval(F, [x, y, 0.3], 0.7)
        want = np.array([c[0] + c[1] * x + c[2] * y for c in coef])
        # the grid holds float32 node values of the linear function
        assert np.allclose(np.concatenate([E - [0.1, 0, 0], B]), want, atol=2e-5)
    for i in range(nx):
        for j in range(ny):
            E, B = oracle.fields_eval(F, [x0 + i * dx, y0 + j * dy, 0.0], 0.0)
            np.testing.assert_allclose(np.concatenate([E - [0.1, 0, 0], B]), grid[:, j, i], rtol=0, atol=1e-12)
    x, y = 0.37, 2.81
    E1, B1 = oracle.fields_eval(F, [x, y, 0], 0)
    E2, B2 = oracle.fields_eval(F, [x + 3 * nx * dx, y - 2 * ny * dy, 0], 0)
    np.testing.assert_allclose(np.concatenate([E1, B1]), np.concatenate([E2, B2]), atol=1e-12)


def test_rotating_field_classical_orbit(otables):
    """The rotating-field model of the cascade setup (polarized-cascade section): without QED an
    electron (q = -1) released at rest at t = 0 in E = a0 (cos t, sin t, 0) has
    p(t) = q a0 (sin t, 1 - cos t, 0), so |p| = 2 a0 |sin(t/2)| (the classical advection the
    section's phase-space figure draws).  Pushed step by step over one period with the fields at
    the start of each step, the oracle's error is first order in dt: it halves with dt."""
    a0, T = 1000.0, 2 * math.pi
    F = oracle.make_fields(oracle.FIELD_ROTATING_E, a0=a0)
    errs = []
    for dt in (2e-2, 1e-2):
        L = oracle.LeptonSet(0, 1, track=(False, False, False))
        L.set(np.zeros((3, 1)), np.zeros((3, 1)), np.array([[0.0], [0.0], [1.0]]))
        G = oracle.PhotonSet(1, track=(False, False, False))
        n = int(round(T / dt))
        worst = 0.0
        for k in range(n):
            prm = oracle.make_params(dt, EPS, step=k, t=k * dt, seed=1, flags=oracle.F_PUSH)
            oracle.lepton_step(otables, prm, F, L, G, oracle.Counters())
            t = (k + 1) * dt
            exact = -a0 * np.array([math.sin(t), 1 - math.cos(t), 0.0])
            got = np.array([L.p[c][0] for c in range(3)])
            worst = max(worst, float(np.abs(got - exact).max()))
            if k + 1 == n // 2:                        # t = pi: the left-point error of p_x is q a0 dt
                assert abs((got[0] - exact[0]) / (-a0 * dt) - 1) < 0.1
        errs.append(worst)
        assert worst < 1.05 * a0 * dt                  # left-point rule: a0 dt (1 + O(dt)) at cos t = -1
    assert 1.8 < errs[0] / errs[1] < 2.2


def test_multiply_add_build_is_the_same_algorithm(otables):
    """The oracle's second build (contracted multiply-adds) makes the same decisions as the plain
    build and differs from it only at the rounding level on a short run; the conditioning it
    records for collapses is at least 1 (a sum of absolute terms is never below the norm)."""
    import synth
    from parity import oracle_run, sensitivity_run
    w = synth.subsample(synth.c1(n=64), np.arange(64))
    ref = oracle_run(otables, w, 20, oracle.F_ALL & ~oracle.F_PAIR, cap_g=64 * 20, k_retire=0.0)
    alt = sensitivity_run(otables, w, 20, oracle.F_ALL & ~oracle.F_PAIR, ref, cap_g=64 * 20, k_retire=0.0)
    _, p0, s0 = ref["E"].arrays()
    _, p1, s1 = alt["E"].arrays()
    d = np.linalg.norm(p0 - p1, axis=0) / np.linalg.norm(p0, axis=0)
    assert 0 < d.max() < 1e-12 and np.abs(s0 - s1).max() < 1e-12
    c = ref["E"].cond[:64]
    assert (c >= 1.0).all() and ref["ctr"]["n_emit"] > 500
    assert (ref["G"].cond[:ref["G"].n] >= 1.0).all()
