"""GPU runs against the oracle on whole states: the decision mismatch count at the peak of the
head-on collision (every particle of the full-size run, one step, both precisions), multi-step
single-precision runs through the peak of the pulse (merged and per-species steps, the
optical-depth decision), and the batched plan with several instances of the ensemble recipe in
both precisions.

Tolerances.  FP64: tol_k(n) = 1e-12 max(1, n/250) as in test_gpu_parity.  FP32: one step's
single-precision arithmetic moves a stored quantity by at most about 1e-6 relative (the Boris
rotation and the no-transition update are a few dependent operations of unit roundoff 6e-8 each),
and the state is stored in FP32 between steps on both sides (the oracle rounds it), so the
differences add up step by step: tol32(n) = max(1e-5, n 1e-6).  Spins and P-vectors get
tol max(1, kappa), kappa the conditioning of their collapse axes recorded by the oracle.
Decisions: a lepton or photon whose draw the oracle flagged as a near tie (within 1e-5 (FP32)
or 1e-10 (FP64) of a threshold) may come out the other way, and then so may everything that
follows from it; every other decision must agree, and the number of near ties that did flip is
printed and bounded.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import (compare_leptons, compare_photons, decision_flips, near_tie_outcomes, oracle_advance,
                    oracle_sets_from_snapshot, photon_parent)

pytestmark = pytest.mark.gpu
EPS = synth.EPS_R


def tol_k(steps):
    return 1e-12 * max(1.0, steps / 250.0)


def tol32(steps):
    return max(1e-5, steps * 1e-6)


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


def _sim(q, tab, w, cap_e, cap_p, cap_g, flags=None, merged=True, tau=False, ppb=0):
    from paper_2511_08929_amd.sim import Simulation
    f = q.make_fields(w.field_kind, E0=w.E0, B0=w.B0, a0=w.a0, phase_len=w.phase_len)
    return Simulation(tab, cap_e=cap_e, cap_p=cap_p, cap_g=cap_g, track=w.track, fields=f, dt=w.dt, eps_r=EPS,
                      seed=w.seed, flags=q.QED_ALL if flags is None else flags, k_retire=w.k_retire,
                      device_clock=True, merged=merged, optical_depth=tau, particles_per_block=ppb)


def _run_to(sim, w, k0, every=50):
    """k0 steps from the workload's initial state (graph replays of `every` steps and a compaction)"""
    import torch
    sim.e.load(w.x, w.p, w.s)
    g = sim.capture(every)
    for _ in range(k0 // every):
        sim.replay(g)
    for _ in range(k0 % every):
        sim.step()
    torch.cuda.synchronize()
    del g


# ------------------------------------------------------------------ decision mismatches
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_decision_mismatch_at_the_peak_full_size(q, tabs, otables, prec):
    """All 10^6 electrons of the head-on collision run to the peak of the pulse (step 850) in the
    benchmark's launch configuration; then one step of every lepton and photon on the GPU and in
    the oracle from that state.  Every emit / no-emit and pair / no-pair decision agrees except
    where the oracle flags a near tie; emission energies agree (the spin-down / spin-up branch)."""
    import torch
    w = synth.c2()
    k0 = 850
    sim = _sim(q, tabs[prec], w, w.n + w.n // 5, w.n // 5, 30 * w.n, ppb=1024)
    _run_to(sim, w, k0)
    st = sim.snapshot(device=False)
    del sim
    torch.cuda.empty_cache()
    u24 = prec == "fp32"
    r = decision_flips(q, tabs[prec], w, st, k0, otables, 16, u24=u24, near_tol=1e-5 if u24 else 1e-10)
    print(prec, r)
    assert r["emissions_gpu"] > 50_000 and r["photons"] > 1_000_000
    assert r["lepton_flips_not_near"] == 0 and r["photon_flips_not_near"] == 0
    assert r["energy_mismatch_not_near"] == 0
    assert r["lepton_flips"] <= r["lepton_near_ties"] and r["photon_flips"] <= r["photon_near_ties"]
    if not u24:
        assert r["lepton_flips"] == 0 and r["photon_flips"] == 0 and r["pairs_gpu"] == r["pairs_oracle"]
    assert r["flip_rate"] < 1e-5


# ------------------------------------------------------------------ single precision through the peak
def _compare_state(q, sim, E, P, G, res, tol, what, st, compare_pairs=True):
    """The GPU sets after the window against the oracle's.  Leptons by index, photons by id.  A
    near-tie pair decision shifts the indices of every later pair, so then only the leptons that
    existed at the start of the window (and their photons) are compared."""
    ne0, np0 = st["e"]["count"], st["p"]["count"]
    near_pairs = res["near_photon_ids"].size > 0
    full = compare_pairs and not near_pairs
    xg, pg, sg = sim.e.arrays()
    m = E.n if full else ne0
    compare_leptons(tuple(a[:, :m] for a in (xg, pg, sg)), tuple(a[:, :m] for a in E.arrays()),
                    res["near_e"][:m], tol, tol, rtol_x=tol, what=f"{what} electrons", cond=E.cond[:m])
    xp, pp, sp = sim.p.arrays()
    mp = P.n if full else np0
    compare_leptons(tuple(a[:, :mp] for a in (xp, pp, sp)), tuple(a[:, :mp] for a in P.arrays()),
                    res["near_p"][:mp], tol, tol, rtol_x=tol, what=f"{what} positrons", cond=P.cond[:mp])
    if full:
        assert sim.e.n() == E.n and sim.p.n() == P.n, f"{what}: lepton counts"
    excl = {(0, int(i)) for i in np.nonzero(res["near_e"])[0]} | {(1, int(i)) for i in np.nonzero(res["near_p"])[0]}
    if not full:                              # leptons made in the window, whose indices may differ
        excl |= {(0, i) for i in range(ne0, max(E.n, sim.e.n()))} | {(1, i) for i in range(np0, max(P.n, sim.p.n()))}
    ga, oa = sim.g.arrays(), G.arrays()
    wp = compare_photons(ga, oa, excl, tol, tol, what=f"{what} photons", near_photons=res["near_photon_ids"])
    nt, flipped, other = near_tie_outcomes(ga[3], oa[3], res["near_e"], res["near_p"])
    print(f"{what}: near-tie leptons {nt}, ended differently {flipped}; near-tie photons "
          f"{res['near_photon_ids'].size}; photons {wp}")
    if full:
        assert other == 0
    return wp


@pytest.mark.parametrize("merged", [True, False])
def test_head_on_fp32_through_the_peak(q, tabs, otables, merged):
    """3000 electrons of the head-on collision, single precision: the GPU runs to step 740, then
    60 more steps across the peak of the pulse; the oracle takes the GPU's state at step 740 and
    runs the same 60 steps in its 24-bit-uniform mode, rounding the stored state to FP32 after
    every step."""
    import torch
    w = synth.subsample(synth.c2(), np.arange(3000))
    k0, n = 740, 60
    sim = _sim(q, tabs["fp32"], w, 4 * w.n, 3 * w.n, 200 * w.n, merged=merged)
    _run_to(sim, w, k0)
    st = sim.snapshot(device=False)
    for _ in range(n):
        sim.step()
    torch.cuda.synchronize()
    E, P, G = oracle_sets_from_snapshot(st, w.track, extra_e=2 * w.n, extra_g=200 * w.n)
    res = oracle_advance(otables, w, E, P, G, n, q.QED_ALL, k0, u24=True, near_tol=1e-5, round32=True)
    print("counters", q.counters_dict(sim.ctr), res["ctr"])
    assert res["ctr"]["n_emit"] > 2000
    wp = _compare_state(q, sim, E, P, G, res, tol32(n), f"fp32 {'merged' if merged else 'per-species'}", st)
    assert wp["matched"] > 1000


def test_optical_depth_fp32_vs_oracle(q, tabs, otables):
    """The optical-depth decision in single precision (merged step): 1500 electrons of the head-on
    collision from the GPU's state at step 740 through 60 steps; tau (FP64 on both sides, summed
    from single-precision W dt on the GPU) within tol32 relative, targets (drawn in FP64 from the
    same Philox words) to 1e-12."""
    import torch
    w = synth.subsample(synth.c2(), np.arange(1500))
    k0, n = 740, 60
    flags = q.QED_ALL | q.QED_OPTICAL_DEPTH
    sim = _sim(q, tabs["fp32"], w, 4 * w.n, 3 * w.n, 200 * w.n, flags=flags, tau=True)
    _run_to(sim, w, k0)
    st = sim.snapshot(device=False)
    for _ in range(n):
        sim.step()
    torch.cuda.synchronize()
    E, P, G = oracle_sets_from_snapshot(st, w.track, extra_e=2 * w.n, extra_g=200 * w.n, tau=True)
    res = oracle_advance(otables, w, E, P, G, n, flags, k0, u24=True, near_tol=1e-5, round32=True)
    assert res["ctr"]["n_emit"] > 1000
    _compare_state(q, sim, E, P, G, res, tol32(n), "optical depth fp32", st, compare_pairs=False)
    keep = ~res["near_e"][:w.n]
    tg, ttg = sim.e.tau_arrays()
    to, tto = E.tau[:w.n], E.tau_target[:w.n]
    dt_ = np.abs(tg[:w.n] - to) / np.maximum(np.abs(to), 1e-3)
    dtt = np.abs(ttg[:w.n] - tto) / np.maximum(np.abs(tto), 1e-300)
    print("tau rel err", dt_[keep].max(), "target rel err", dtt[keep].max())
    assert dt_[keep].max() <= tol32(n) and dtt[keep].max() <= 1e-12


# ------------------------------------------------------------------ batched plan
def _batch(q, tab, ws, ppb=128):
    from paper_2511_08929_amd.sim import Batch
    specs = [dict(cap_e=4 * w.n + 2000, cap_p=3 * w.n + 2000, cap_g=120 * w.n + 20_000, track=w.track,
                  fields=dict(kind=w.field_kind, a0=w.a0, phase_len=w.phase_len), dt=w.dt, eps_r=EPS, seed=w.seed,
                  flags=q.QED_ALL, k_retire=w.k_retire) for w in ws]
    bat = Batch(tab, specs, particles_per_block=ppb)
    for w, inst in zip(ws, bat.inst):
        inst["e"].load(w.x, w.p, w.s)
    return bat


def _inst_arrays(inst):
    return inst["e"], inst["p"], inst["g"]


def test_batched_plan_vs_oracle_fp64(q, tabs, otables):
    """Four instances of the ensemble recipe (N ~ LogUniform, a0 ~ U[20, 200], gamma0 ~
    U[500, 1e4], partial spin polarization along a random transverse axis) in one plan, replayed
    from a HIP graph of 50 steps and a compaction, 1600 steps through the whole pulse; each
    instance against its own oracle run, every particle."""
    import torch
    ws = synth.c5(n_instances=4, seed=17, n_min=200, n_max=800)
    steps = 1600
    bat = _batch(q, tabs["fp64"], ws)
    g = bat.capture(50)
    for _ in range(steps // 50):
        bat.replay(g)
    torch.cuda.synchronize()
    t = tol_k(steps)
    for j, (w, inst) in enumerate(zip(ws, bat.inst)):
        from parity import oracle_run
        ref = oracle_run(otables, w, steps, q.QED_ALL, cap_e=4 * w.n + 2000, cap_p=3 * w.n + 2000,
                         cap_g=120 * w.n + 20_000)
        c = q.counters_dict(inst["ctr"])
        print(f"instance {j}: n {w.n} a0 {w.a0:.1f} gamma0 {w.extra['gamma0']:.0f}", c, ref["ctr"])
        assert not ref["near_e"].any() and not ref["near_g"].any()
        assert c["n_emit"] == ref["ctr"]["n_emit"] and c["n_pair"] == ref["ctr"]["n_pair"]
        e, p, gph = _inst_arrays(inst)
        compare_leptons(e.arrays(), ref["E"].arrays(), np.zeros(ref["E"].n, bool), t, t, rtol_x=t,
                        what=f"instance {j} electrons")
        compare_leptons(p.arrays(), ref["P"].arrays(), np.zeros(ref["P"].n, bool), t, t, rtol_x=t,
                        what=f"instance {j} positrons")
        compare_photons(gph.arrays(), ref["G"].arrays(), set(), t, t, what=f"instance {j} photons")
    assert sum(q.counters_dict(i["ctr"])["n_emit"] for i in bat.inst) > 20_000


def test_batched_plan_vs_oracle_fp32(q, tabs, otables):
    """The same recipe in single precision: the plan runs to step 740, then 60 steps across the
    peak; each instance against the oracle from the plan's own state at step 740."""
    import torch
    ws = synth.c5(n_instances=4, seed=19, n_min=300, n_max=1500)
    k0, n = 740, 60
    bat = _batch(q, tabs["fp32"], ws)
    g = bat.capture(50)
    for _ in range(k0 // 50):
        bat.replay(g)
    for _ in range(k0 % 50):
        bat.step()
    torch.cuda.synchronize()
    del g
    snaps = bat.snapshot(device=False)
    for _ in range(n):
        bat.step()
    torch.cuda.synchronize()
    emitted = 0
    for j, (w, inst, st) in enumerate(zip(ws, bat.inst, snaps)):
        E, P, G = oracle_sets_from_snapshot(st, w.track, extra_e=2 * w.n, extra_g=120 * w.n)
        res = oracle_advance(otables, w, E, P, G, n, q.QED_ALL, k0, u24=True, near_tol=1e-5, round32=True)
        emitted += res["ctr"]["n_emit"]

        class View:                               # the instance's sets as _compare_state reads them
            e, p, g = _inst_arrays(inst)
        _compare_state(q, View, E, P, G, res, tol32(n), f"batched fp32 instance {j}", st)
    assert emitted > 1000
