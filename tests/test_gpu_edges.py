"""Degenerate inputs of the step on the GPU, per-species calls and merged step, FP64 and FP32,
against the oracle: leptons at rest without the push (chi is defined but the emission basis is
not: no QED), leptons moving along B and photons along B (chi = 0), zero fields, and fully
unpolarized leptons and photons.  Nothing may become NaN, nothing may be emitted or decay where
chi = 0, and every particle must equal the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_leptons, compare_photons, oracle_run

pytestmark = pytest.mark.gpu
EPS = synth.EPS_R


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2511_08929_amd as q
    q.lib()
    return q


@pytest.fixture(scope="module")
def tabs(q):
    return {"fp64": q.Tables(precision=q.QED_F64), "fp32": q.Tables(precision=q.QED_F32)}


def _workload(E0, B0, p, s):
    n = p.shape[1]
    w = synth.Workload("degenerate", n, 1, 0.05, 9, synth.FIELD_UNIFORM, E0=E0, B0=B0, track=(True, True, True))
    w.x = np.zeros((3, n)); w.p = p; w.s = s
    return w


def _run(q, tab, w, flags, merged):
    from paper_2511_08929_amd.sim import Simulation
    f = q.make_fields(w.field_kind, E0=w.E0, B0=w.B0)
    n = w.p.shape[1]
    sim = Simulation(tab, cap_e=2 * n + 64, cap_p=n + 64, cap_g=4 * n + 64, track=w.track, fields=f, dt=w.dt,
                     eps_r=EPS, seed=w.seed, flags=flags, k_retire=0.0, device_clock=merged, merged=merged)
    sim.e.load(w.x, w.p, w.s)
    sim.step()
    return sim


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("merged", [False, True])
def test_leptons_at_rest_and_along_B(q, tabs, prec, merged):
    """No push: 100 leptons at rest in strong parallel E and B (the rest-frame field is E, but
    there is no emission direction), then 100 leptons moving along a pure B field (gamma 1000,
    chi = 0): neither group does any QED, nothing is emitted and the spins stay as they are."""
    rng = np.random.default_rng(3)
    n = 100
    flags = q.QED_ALL & ~q.QED_PUSH & ~q.QED_PAIR
    tol = 1e-12 if prec == "fp64" else 1e-6
    p_along = np.zeros((3, n)); p_along[2] = 1000.0
    for E0, B0, p in (((0.0, 0.0, 400.0), (0.0, 0.0, 300.0), np.zeros((3, n))),
                      ((0.0, 0.0, 0.0), (0.0, 0.0, 300.0), p_along)):
        s = synth.random_unit_vectors(rng, n) * 0.7
        w = _workload(E0, B0, p, s)
        sim = _run(q, tabs[prec], w, flags, merged)
        x, pg, sg = sim.e.arrays()
        assert np.isfinite(x).all() and np.isfinite(pg).all() and np.isfinite(sg).all()
        c = q.counters_dict(sim.ctr)
        assert c["n_emit"] == 0 and sim.g.n() == 0, c
        np.testing.assert_array_equal(pg, p)
        assert np.abs(sg - w.s).max() < tol
        ref = oracle_run(oracle_tables(), w, 1, flags, cap_g=64, k_retire=0.0)
        assert ref["ctr"]["n_emit"] == 0
        compare_leptons((x, pg, sg), ref["E"].arrays(), np.zeros(n, bool), tol, tol, rtol_x=tol,
                        what="at rest / along B")


_OT = None


def oracle_tables():
    global _OT
    if _OT is None:
        _OT = oracle.OracleTables()
    return _OT


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("merged", [False, True])
def test_zero_field_step(q, tabs, prec, merged):
    """Zero field: the push only moves x, nothing is emitted, spins stay as they are."""
    n = 130
    rng = np.random.default_rng(5)
    p = synth.random_unit_vectors(rng, n) * 500.0
    s = synth.random_unit_vectors(rng, n)
    w = _workload((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), p, s)
    sim = _run(q, tabs[prec], w, q.QED_ALL, merged)
    x, pg, sg = sim.e.arrays()
    c = q.counters_dict(sim.ctr)
    assert c["n_emit"] == 0 and np.isfinite(x).all() and np.isfinite(sg).all()
    pw = p.astype(np.float32).astype(np.float64) if prec == "fp32" else p
    rel = np.abs(x - w.dt * pw / np.sqrt(1 + np.sum(pw * pw, axis=0))).max()
    assert rel < (1e-15 if prec == "fp64" else 1e-7)
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert np.abs(sg - w.s).max() < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_photons_along_B_and_unpolarized(q, tabs, prec):
    """qed_pair on 96 photons in a pure B field: 48 along B (chi_gamma = 0: no decay, no update,
    P stays as given) and 48 across it (chi_gamma about 5), half of each unpolarized (P = 0),
    against the oracle."""
    import torch
    from paper_2511_08929_amd.sim import Simulation
    m = 96
    rng = np.random.default_rng(8)
    k = np.zeros((3, m)); k[2, :48] = 3000.0; k[0, 48:] = 3000.0
    P = np.zeros((3, m))
    P[:, 24:48] = synth.random_unit_vectors(rng, 24) * 0.8
    P[:, 72:] = synth.random_unit_vectors(rng, 24) * 0.8
    x = np.zeros((3, m))
    ids = (np.uint64(1) << np.uint64(63)) | np.arange(1, m + 1, dtype=np.uint64)
    if prec == "fp32":
        P = P.astype(np.float32).astype(np.float64)
    B0 = (0.0, 0.0, 5.0 / (EPS * 3000.0))
    w = synth.Workload("photons_along_B", 0, 1, 0.5, 4, synth.FIELD_UNIFORM, B0=B0, track=(True, True, True))
    tab = tabs[prec]
    f = q.make_fields(w.field_kind, B0=B0)
    sim = Simulation(tab, cap_e=2 * m, cap_p=2 * m, cap_g=m, track=w.track, fields=f, dt=w.dt, eps_r=EPS,
                     seed=w.seed, flags=q.QED_ALL, k_retire=0.0)
    for i in range(3):
        sim.g.x[i][:m] = torch.as_tensor(x[i]); sim.g.k[i][:m] = torch.as_tensor(k[i])
        sim.g.P[i][:m] = torch.as_tensor(P[i])
    sim.g.id[:m] = torch.as_tensor(ids.view(np.int64))
    sim.g.count.fill_(m); sim.g.count_prev.fill_(m)
    q.qed_pair(tab, sim.g, sim.fields, sim.step_params(0), sim.e, sim.p, sim.ctr, sim.ws)
    xg, kg, Pg, idg = sim.g.arrays()
    assert np.isfinite(kg).all() and np.isfinite(Pg).all() and np.isfinite(xg).all()
    np.testing.assert_array_equal(idg[:48], ids[:48])             # none of those decayed
    np.testing.assert_array_equal(Pg[:, :48], P[:, :48])          # nor changed polarization
    G = oracle.PhotonSet(m, track=w.track)
    for i in range(3):
        G.x[i][:m], G.k[i][:m], G.P[i][:m] = x[i], k[i], P[i]
    G.id[:m] = ids; G.n = G.n_prev = m
    Le, Lp = oracle.LeptonSet(0, 2 * m), oracle.LeptonSet(1, 2 * m)
    ctr = oracle.Counters()
    fp32 = prec == "fp32"
    prm = oracle.make_params(w.dt, EPS, step=0, seed=w.seed, flags=q.QED_ALL, near_tol=1e-5 if fp32 else 1e-10,
                             u24=fp32)
    oracle.photon_step(oracle_tables(), prm, oracle.make_fields(w.field_kind, B0=B0), G, Le, Lp, ctr)
    assert ctr.n_pair == q.counters_dict(sim.ctr)["n_pair"] > 0
    tol = 1e-5 if fp32 else 1e-12
    compare_photons(sim.g.arrays(), G.arrays(), set(), tol, tol, what="photons along and across B")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("merged", [False, True])
def test_nonfinite_inputs(q, tabs, prec, merged):
    """NaN and infinity in lepton and photon states (and k = 0) in one step with both channels:
    the leptons keep their stored values bit for bit, the photons with bad k or x become dead
    slots, the one with a NaN P-vector is stepped as unpolarized; every one is counted in
    n_nonfinite as by the oracle, nothing else becomes non-finite, and every other particle
    equals the oracle's."""
    import math

    import torch
    rng = np.random.default_rng(12)
    n, m = 400, 300
    d = synth.random_unit_vectors(rng, n)
    g = np.exp(rng.uniform(math.log(500.0), math.log(5000.0), n))
    p = d * np.sqrt(g * g - 1)
    s = synth.random_unit_vectors(rng, n)
    x = np.stack([rng.uniform(0, 50, n), rng.uniform(-5, 5, n), rng.uniform(-5, 5, n)])
    for j, (arr, c, v) in {3: (p, 0, np.nan), 17: (s, 2, np.inf), 55: (x, 0, -np.inf), 300: (p, 1, -np.inf)}.items():
        arr[c, j] = v
    kd = synth.random_unit_vectors(rng, m) * np.exp(rng.uniform(math.log(2e3), math.log(2e4), m))
    P = synth.random_unit_vectors(rng, m) * 0.8
    xg = rng.uniform(0, 10, (3, m))
    ids = (np.uint64(1) << np.uint64(63)) | (np.arange(m, dtype=np.uint64) << np.uint64(24)) | np.uint64(3)
    kd[0, 4] = np.nan
    xg[1, 9] = np.inf
    P[2, 20] = np.nan
    kd[:, 30] = 0.0
    if prec == "fp32":
        p, s, x, kd, P, xg = (a.astype(np.float32).astype(np.float64) for a in (p, s, x, kd, P, xg))
    E0, B0 = (0.0, 30.0, 0.0), (0.0, 0.0, 120.0)
    w = _workload(E0, B0, p, s)
    w.x, w.dt = x, 0.5
    from paper_2511_08929_amd.sim import Simulation
    f = q.make_fields(w.field_kind, E0=E0, B0=B0)
    sim = Simulation(tabs[prec], cap_e=3 * n, cap_p=2 * n, cap_g=m + 2 * n, track=w.track, fields=f, dt=w.dt,
                     eps_r=EPS, seed=w.seed, flags=q.QED_ALL, k_retire=0.0, device_clock=merged, merged=merged)
    sim.e.load(x, p, s)
    sim.g.load(xg, kd, P, ids)
    sim.step()
    torch.cuda.synchronize()
    c = q.counters_dict(sim.ctr)
    # the oracle on the same inputs, in the same order
    T = oracle_tables()
    E = oracle.LeptonSet(0, 3 * n, track=w.track)
    E.set(x, p, s)
    Pp = oracle.LeptonSet(1, 2 * n, track=w.track)
    G = oracle.PhotonSet(m + 2 * n, track=w.track)
    for i in range(3):
        G.x[i][:m], G.k[i][:m], G.P[i][:m] = xg[i], kd[i], P[i]
    G.id[:m] = ids
    G.n = G.n_prev = m
    fo = oracle.make_fields(oracle.FIELD_UNIFORM, E0=E0, B0=B0)
    prm = oracle.make_params(w.dt, EPS, step=0, seed=w.seed, flags=q.QED_ALL, k_retire=0.0,
                             near_tol=1e-10 if prec == "fp64" else 1e-5, u24=prec == "fp32")
    ctr = oracle.Counters()
    oracle.lepton_step(T, prm, fo, E, G, ctr, 8)
    near = E.near[:n].astype(bool).copy()
    oracle.lepton_step(T, prm, fo, Pp, G, ctr, 8)
    oracle.photon_step(T, prm, fo, G, E, Pp, ctr, 8)
    oc = ctr.as_dict()
    print(prec, merged, c, oc)
    assert c["n_nonfinite"] == oc["n_nonfinite"] == 4 + 4
    assert c["n_emit"] == oc["n_emit"] > 50 and c["n_pair"] == oc["n_pair"] > 0
    xo_, po_, so_ = sim.e.arrays()
    bj = np.array([3, 17, 55, 300])
    for a, b in ((xo_, x), (po_, p), (so_, s)):
        np.testing.assert_array_equal(a[:, bj], b[:, bj])
    good = np.setdiff1d(np.arange(sim.e.n()), bj)
    assert all(np.isfinite(a[:, good]).all() for a in (xo_, po_, so_))
    tol = 1e-12 if prec == "fp64" else 1e-5
    oa = E.arrays()
    ex = np.zeros(sim.e.n(), bool)
    ex[:n] = near
    ex[bj] = True
    compare_leptons((xo_, po_, so_), oa, ex, tol, tol, rtol_x=tol, what="leptons beside non-finite ones")
    ga = sim.g.arrays()
    assert (ga[3][[4, 9, 30]] == 0).all()
    live = ga[3] != 0
    assert np.isfinite(ga[1][:, live]).all() and np.isfinite(ga[2][:, live]).all()
    compare_photons(ga, G.arrays(), {(0, int(i)) for i in np.nonzero(near)[0]}, tol, tol, what="photons")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("merged", [False, True])
def test_nonfinite_grid_node(q, tabs, prec, merged):
    """A NaN at one node of a grid field: leptons that interpolate it in the push keep their state,
    those that meet it only at t + dt are pushed without a QED part, photons there get no QED
    part; all counted as by the oracle, and every particle equals the oracle's."""
    import torch
    w = synth.c3(n=4000, steps=1, nx=16, ny=8)
    grid = w.extra["grid"].copy()
    grid[1, 3, 5] = np.nan                     # Ey at node (i = 5, j = 3)
    dx = w.extra["dx"]
    # half the electrons inside the cells around that node
    rng = np.random.default_rng(4)
    w.x[0, :2000] = dx * rng.uniform(4.0, 6.0, 2000)
    w.x[1, :2000] = dx * rng.uniform(2.0, 4.0, 2000)
    if prec == "fp32":
        w.x, w.p, w.s = (a.astype(np.float32).astype(np.float64) for a in (w.x, w.p, w.s))
    fg = q.make_fields(q.QED_FIELD_GRID2D, grid=torch.as_tensor(grid, device="cuda"), dx=dx, dy=dx)
    fo = oracle.make_fields(oracle.FIELD_GRID2D, grid=grid, dx=dx, dy=dx)
    from paper_2511_08929_amd.sim import Simulation
    sim = Simulation(tabs[prec], cap_e=3 * w.n, cap_p=2 * w.n, cap_g=4 * w.n, track=w.track, fields=fg, dt=w.dt,
                     eps_r=EPS, seed=w.seed, flags=q.QED_ALL, k_retire=0.0, device_clock=merged, merged=merged)
    sim.e.load(w.x, w.p, w.s)
    for _ in range(2):
        sim.step()
    torch.cuda.synchronize()
    ref = oracle_run(oracle_tables(), w, 2, q.QED_ALL, cap_e=3 * w.n, cap_p=2 * w.n, cap_g=4 * w.n, k_retire=0.0,
                     fields=fo, u24=prec == "fp32", near_tol=1e-10 if prec == "fp64" else 1e-5,
                     round32=prec == "fp32")
    c = q.counters_dict(sim.ctr)
    print(prec, merged, c, ref["ctr"])
    assert c["n_nonfinite"] == ref["ctr"]["n_nonfinite"] > 100
    assert c["n_emit"] == ref["ctr"]["n_emit"] and c["n_pair"] == ref["ctr"]["n_pair"]
    tol = 1e-12 if prec == "fp64" else 1e-5
    x, p, s = sim.e.arrays()
    assert np.isfinite(p).all() and np.isfinite(s).all()
    compare_leptons((x, p, s), ref["E"].arrays(), ref["near_e"], tol, tol, rtol_x=tol, what="electrons by a NaN node")
    compare_photons(sim.g.arrays(), ref["G"].arrays(), {(0, int(i)) for i in np.nonzero(ref["near_e"])[0]}, tol, tol,
                    what="photons by a NaN node")


def test_nonfinite_field_parameters_are_rejected(q, tabs):
    """An analytic field model with a NaN or infinite parameter is refused on the host."""
    import torch
    n = 8
    e = q.LeptonBuffers(0, n, torch.float32, track=(True, False, False))
    g = q.PhotonBuffers(n, torch.float32, track=(True, False, False))
    ws = q.new_workspace(q.qed_workspace_size(n))
    sp = q.make_step(0.1, EPS)
    for f in (q.make_fields(q.QED_FIELD_UNIFORM, E0=(0.0, np.nan, 0.0)),
              q.make_fields(q.QED_FIELD_PLANE_LP, a0=np.inf, phase_len=100.0),
              q.make_fields(q.QED_FIELD_UNIFORM, B0=(0.0, 0.0, 1e31))):
        with pytest.raises(q.QedError, match="status -1"):
            q.qed_emit(tabs["fp32"], e, f, sp, g, q.new_counters(), ws)
