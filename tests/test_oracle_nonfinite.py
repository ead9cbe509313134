"""The non-finite input rule of the step, pinned in the oracle by independence: a lepton whose
state or fields hold a NaN or an infinity keeps its stored state (or only its push) and is
counted; a photon whose k or x is not finite is removed, one whose P is not finite is stepped
as unpolarized, each counted; every other particle steps exactly as it does in a run without the bad ones, since
particles do not interact within a step and keep their Philox ids."""
import math

import numpy as np

import oracle
import synth

NAN, INF = float("nan"), float("inf")


def _leptons(n, seed):
    rng = np.random.default_rng(seed)
    d = synth.random_unit_vectors(rng, n)
    g = np.exp(rng.uniform(math.log(500.0), math.log(5000.0), n))
    p = d * np.sqrt(g * g - 1)
    s = synth.random_unit_vectors(rng, n)
    x = np.stack([rng.uniform(0, 50, n), rng.uniform(-5, 5, n), rng.uniform(-5, 5, n)])
    return x, p, s


def _step(T, x, p, s, index, flags, fields):
    n = p.shape[1]
    L = oracle.LeptonSet(0, n, track=(True, True, True))
    L.set(x, p, s, index=index)
    G = oracle.PhotonSet(2 * n + 8, track=(True, True, True))
    c = oracle.Counters()
    prm = oracle.make_params(0.3, synth.EPS_R, step=5, seed=4, flags=flags, k_retire=0.0)
    oracle.lepton_step(T, prm, fields, L, G, c, 4)
    return L, G, c.as_dict()


def test_nonfinite_leptons_are_left_alone_and_counted(otables):
    n = 400
    x, p, s = _leptons(n, 1)
    bad = {3: ("p", 0, NAN), 17: ("s", 2, INF), 55: ("x", 0, -INF), 300: ("p", 1, -INF)}
    xb, pb, sb = x.copy(), p.copy(), s.copy()
    for j, (a, c, v) in bad.items():
        {"x": xb, "p": pb, "s": sb}[a][c, j] = v
    f = oracle.make_fields(oracle.FIELD_UNIFORM, E0=(0.0, 30.0, 0.0), B0=(0.0, 0.0, 120.0))
    flags = oracle.F_ALL & ~oracle.F_PAIR
    L, G, c = _step(otables, xb, pb, sb, np.arange(n), flags, f)
    assert c["n_nonfinite"] == len(bad)
    xo, po, so = L.arrays()
    bj = np.array(sorted(bad))
    for arr, src in ((xo, xb), (po, pb), (so, sb)):                   # kept bit for bit (NaN as NaN)
        np.testing.assert_array_equal(arr[:, bj], src[:, bj])
    good = np.setdiff1d(np.arange(n), bj)
    L2, G2, c2 = _step(otables, x[:, good], p[:, good], s[:, good], good, flags, f)
    for a, b in zip(L.arrays(), L2.arrays()):
        np.testing.assert_array_equal(a[:, good], b)
    assert c2["n_emit"] == c["n_emit"] > 50 and c2["n_nonfinite"] == 0
    _, k1, P1, id1 = G.arrays()
    _, k2, P2, id2 = G2.arrays()
    np.testing.assert_array_equal(id1, id2)
    np.testing.assert_array_equal(k1, k2)
    assert np.isfinite(k1).all() and np.isfinite(P1).all()


def test_nonfinite_fields_stop_the_step(otables):
    """NaN in the uniform field: no lepton is pushed, none does QED, all are counted."""
    n = 64
    x, p, s = _leptons(n, 2)
    f = oracle.make_fields(oracle.FIELD_UNIFORM, E0=(0.0, NAN, 0.0), B0=(0.0, 0.0, 120.0))
    L, G, c = _step(otables, x, p, s, np.arange(n), oracle.F_ALL & ~oracle.F_PAIR, f)
    assert c["n_nonfinite"] == n and c["n_emit"] == 0 and G.n == 0
    for a, b in zip(L.arrays(), (x, p, s)):
        np.testing.assert_array_equal(a, b)


def test_nonfinite_photons_are_removed(otables):
    rng = np.random.default_rng(5)
    n = 300
    d = synth.random_unit_vectors(rng, n)
    k = d * np.exp(rng.uniform(math.log(2e3), math.log(2e4), n))
    P = synth.random_unit_vectors(rng, n) * 0.8
    x = rng.uniform(0, 10, (3, n))
    ids = (np.uint64(1) << np.uint64(63)) | (np.arange(n, dtype=np.uint64) << np.uint64(24)) | np.uint64(3)
    k[0, 4] = NAN
    x[1, 9] = INF
    P[2, 20] = NAN                     # chi_gamma >= chi_min here: stepped as unpolarized
    k[:, 30] = 0.0                     # no direction: removed
    f = oracle.make_fields(oracle.FIELD_UNIFORM, E0=(0.0, 0.0, 0.0), B0=(0.0, 0.0, 150.0))

    def run(mask):
        G = oracle.PhotonSet(n, track=(True, True, True))
        m = int(mask.sum())
        for i in range(3):
            G.x[i][:m], G.k[i][:m], G.P[i][:m] = x[i][mask], k[i][mask], P[i][mask]
        G.id[:m] = ids[mask]
        G.n = G.n_prev = m
        E = oracle.LeptonSet(0, 2 * n, track=(True, True, True))
        Pp = oracle.LeptonSet(1, 2 * n, track=(True, True, True))
        c = oracle.Counters()
        prm = oracle.make_params(0.4, synth.EPS_R, step=2, seed=8, flags=oracle.F_ALL, k_retire=0.0)
        oracle.photon_step(otables, prm, f, G, E, Pp, c, 4)
        return G, c.as_dict()

    allm = np.ones(n, bool)
    G, c = run(allm)
    assert c["n_nonfinite"] == 4
    assert (G.id[[4, 9, 30]] == 0).all()
    if G.id[20] != 0:                                    # survived: stepped as unpolarized, finite now
        assert np.isfinite([G.P[i][20] for i in range(3)]).all()
    good = allm.copy()
    good[[4, 9, 30]] = False
    P[:, 20] = 0.0                                       # the same photon given as unpolarized
    G2, c2 = run(good)
    assert c2["n_nonfinite"] == 0 and c2["n_pair"] == c["n_pair"]
    live = G.id[:n] != 0
    np.testing.assert_array_equal(G.id[:n][live], G2.id[:G2.n][G2.id[:G2.n] != 0])
    for i in range(3):
        np.testing.assert_array_equal(G.P[i][:n][live], G2.P[i][:G2.n][G2.id[:G2.n] != 0])
