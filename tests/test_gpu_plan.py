"""Merged and batched steps (qed_plan_step) against the per-species calls, bit for bit.

A plan step of an instance is defined as qed_emit(electrons), qed_emit(positrons),
qed_pair(photons), clock + 1; the per-species calls are themselves checked against the oracle
in test_gpu_parity.  So equality here, particle by particle and counter by counter, carries the
oracle parity over to the plan path.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

EPS = synth.EPS_R


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_08929_amd as q
    return q


@pytest.fixture(scope="module")
def tabs(q):
    return {"fp64": q.Tables(precision=q.QED_F64), "fp32": q.Tables(precision=q.QED_F32)}


def _sim(q, tab, w, merged, cap_e, cap_p, cap_g, flags=None, ppb=0, tau=False, maxb=0, fields=None, pvar=0):
    from paper_2511_08929_amd.sim import Simulation
    f = fields or q.make_fields(w.field_kind, E0=w.E0, B0=w.B0, a0=w.a0, phase_len=w.phase_len)
    sim = Simulation(tab, cap_e=cap_e, cap_p=cap_p, cap_g=cap_g, track=w.track, fields=f, dt=w.dt, eps_r=EPS,
                     seed=w.seed, flags=q.QED_ALL if flags is None else flags, k_retire=w.k_retire,
                     device_clock=True, merged=merged, particles_per_block=ppb, optical_depth=tau,
                     max_blocks_per_set=maxb, photon_variant=pvar)
    sim.e.load(w.x, w.p, w.s)
    return sim


def _state(q, sim):
    return sim.e.arrays() + sim.p.arrays() + sim.g.arrays() + (q.counters_dict(sim.ctr),)


def _assert_same(a, b, what):
    assert len(a) == len(b)
    for j, (x, y) in enumerate(zip(a, b)):
        if isinstance(x, dict):
            assert x == y, f"{what}: counters {x} vs {y}"
        else:
            assert x.shape == y.shape, f"{what}: array {j} shape {x.shape} vs {y.shape}"
            np.testing.assert_array_equal(x, y, err_msg=f"{what}: array {j}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plan_equals_per_species_head_on(q, tabs, prec):
    """2000 electrons of the head-on collision through the pulse (emission, pairs, retirement,
    compaction every 25 steps), checked at five points."""
    import torch
    w = synth.subsample(synth.c2(), np.arange(2000))
    a = _sim(q, tabs[prec], w, False, w.n + 3000, 3000, 150_000)
    b = _sim(q, tabs[prec], w, True, w.n + 3000, 3000, 150_000)
    for k in range(1, 1001):
        a.step(); b.step()
        if k % 25 == 0:
            a.compact(); b.compact()
        if k % 200 == 0:
            torch.cuda.synchronize()
            _assert_same(_state(q, a), _state(q, b), f"{prec} step {k}")
    c = q.counters_dict(b.ctr)
    print(prec, c)
    assert c["n_emit"] > 10_000 and c["n_pair"] > 0 and c["n_retired"] > 0
    assert int(a.clock.item()) == int(b.clock.item()) == 1000


@pytest.mark.parametrize("pvar", [1, 2])
def test_plan_photon_variants_equal_per_species(q, tabs, pvar):
    """The photon pass's launch variants (512-slot tiles; 1024-slot tiles at three waves per SIMD)
    give the per-species results bit for bit: 2000 electrons of the head-on collision in FP32
    through the pulse, compaction every 25 steps, with many photon tiles per block (particles per
    block 4096)."""
    import torch
    w = synth.subsample(synth.c2(), np.arange(2000))
    a = _sim(q, tabs["fp32"], w, False, w.n + 3000, 3000, 150_000)
    b = _sim(q, tabs["fp32"], w, True, w.n + 3000, 3000, 150_000, ppb=4096, pvar=pvar)
    for k in range(1, 1001):
        a.step(); b.step()
        if k % 25 == 0:
            a.compact(); b.compact()
        if k % 250 == 0:
            torch.cuda.synchronize()
            _assert_same(_state(q, a), _state(q, b), f"variant {pvar} step {k}")
    assert q.counters_dict(b.ctr)["n_photon_steps"] > 1_000_000


def test_plan_rejects_unknown_photon_variant(q, tabs):
    w = synth.subsample(synth.c2(), np.arange(64))
    with pytest.raises(Exception):
        _sim(q, tabs["fp32"], w, True, 1000, 1000, 1000, pvar=3).step()


def test_plan_equals_per_species_pair_overflow(q, tabs):
    """Positron store of four slots: pairs beyond it are counted as overflow and not stored, in
    the plan as in the per-species calls (the pair append bases and the capacity clamp of the
    processing launch's own bookkeeping)."""
    import torch
    w = synth.subsample(synth.c2(), np.arange(3000))
    a = _sim(q, tabs["fp32"], w, False, w.n + 4, 4, 200_000)
    b = _sim(q, tabs["fp32"], w, True, w.n + 4, 4, 200_000)
    for k in range(1, 1201):
        a.step(); b.step()
        if k % 50 == 0:
            a.compact(); b.compact()
    torch.cuda.synchronize()
    _assert_same(_state(q, a), _state(q, b), "pair overflow")
    c = q.counters_dict(b.ctr)
    assert b.p.n() == 4 and c["n_pair"] > 4 and c["n_capacity_overflow"] == c["n_pair"] - 4


def test_plan_equals_per_species_rejection(q, tabs):
    """Rejection sampling of the emission in the merged step: 2000 electrons of the head-on
    collision, FP32, 800 steps, against the per-species calls bit for bit."""
    import torch
    w = synth.subsample(synth.c2(), np.arange(2000))
    flags = q.QED_ALL | q.QED_REJECTION
    a = _sim(q, tabs["fp32"], w, False, w.n + 3000, 3000, 150_000, flags)
    b = _sim(q, tabs["fp32"], w, True, w.n + 3000, 3000, 150_000, flags)
    for k in range(1, 801):
        a.step(); b.step()
        if k % 50 == 0:
            a.compact(); b.compact()
    torch.cuda.synchronize()
    _assert_same(_state(q, a), _state(q, b), "rejection")
    assert q.counters_dict(b.ctr)["n_emit"] > 10_000


def test_plan_equals_per_species_optical_depth(q, tabs):
    """Optical-depth decision in the merged step: 1500 electrons of the head-on collision, FP32,
    tau and targets compared too."""
    import torch
    w = synth.subsample(synth.c2(), np.arange(1500))
    flags = q.QED_ALL | q.QED_OPTICAL_DEPTH
    a = _sim(q, tabs["fp32"], w, False, w.n + 3000, 3000, 120_000, flags, tau=True)
    b = _sim(q, tabs["fp32"], w, True, w.n + 3000, 3000, 120_000, flags, tau=True)
    for k in range(1, 1001):
        a.step(); b.step()
        if k % 50 == 0:
            a.compact(); b.compact()
    torch.cuda.synchronize()
    _assert_same(_state(q, a) + a.e.tau_arrays() + a.p.tau_arrays(),
                 _state(q, b) + b.e.tau_arrays() + b.p.tau_arrays(), "optical depth")
    assert q.counters_dict(b.ctr)["n_pair"] > 0


def test_plan_equals_per_species_dense_emission(q, tabs):
    """Test-particle case (about 95 % emitters per step, no pairs): every block of the process
    pass has a full list; small blocks (64 particles each) and a photon store that overflows."""
    w = synth.c1(n=3000)
    flags = q.QED_ALL & ~q.QED_PAIR
    a = _sim(q, tabs["fp64"], w, False, w.n, 1, 40_000, flags)
    b = _sim(q, tabs["fp64"], w, True, w.n, 1, 40_000, flags, ppb=64)
    assert b.plan is None
    for _ in range(16):
        a.step(); b.step()
    assert b.plan.blocks == 3000 // 64 + 1
    _assert_same(_state(q, a), _state(q, b), "c1")
    c = q.counters_dict(b.ctr)
    assert c["n_capacity_overflow"] > 0 and b.g.n() == 40_000


def test_plan_batched_instances(q, tabs):
    """Three instances of different sizes, fields and seeds in one plan, each equal to its own
    per-species run; then the same plan captured in a HIP graph and replayed, with eager work
    between the replays, equal to further per-species steps after every replay."""
    import torch
    from paper_2511_08929_amd.sim import Batch
    ws = synth.c5(n_instances=3, seed=11, n_min=300, n_max=3000)
    tab = tabs["fp32"]
    specs = []
    for w in ws:
        specs.append(dict(cap_e=w.n * 2 + 2000, cap_p=w.n + 2000, cap_g=80 * w.n + 20_000, track=w.track,
                          fields=dict(kind=w.field_kind, a0=w.a0, phase_len=w.phase_len), dt=w.dt, eps_r=EPS,
                          seed=w.seed, flags=q.QED_ALL, k_retire=w.k_retire))
    bat = Batch(tab, specs, particles_per_block=128)
    for w, inst in zip(ws, bat.inst):
        inst["e"].load(w.x, w.p, w.s)
    ref = [_sim(q, tab, w, False, s["cap_e"], s["cap_p"], s["cap_g"]) for w, s in zip(ws, specs)]

    def check(what):
        torch.cuda.synchronize()
        for j, (r, inst) in enumerate(zip(ref, bat.inst)):
            got = inst["e"].arrays() + inst["p"].arrays() + inst["g"].arrays() + (q.counters_dict(inst["ctr"]),)
            _assert_same(_state(q, r), got, f"{what} instance {j}")

    for k in range(1, 601):
        bat.step()
        for r in ref:
            r.step()
        if k % 50 == 0:
            bat.compact()
            for r in ref:
                r.compact()
    check("eager")
    g = bat.capture(50)
    for rep in range(4):
        bat.replay(g)
        for r in ref:
            for _ in range(50):
                r.step()
            r.compact()
        torch.cuda.synchronize()
        check(f"replay {rep}")
    tot = [q.counters_dict(i["ctr"]) for i in bat.inst]
    print(tot)
    assert sum(t["n_emit"] for t in tot) > 1000


def test_plan_equals_per_species_many_blocks(q, tabs):
    """All 10^6 electrons of the head-on collision in blocks of 64 particles and no cap on the
    blocks of a set: about 47 000 main blocks, so the bookkeeping scan runs over several LDS
    chunks of block counts."""
    w = synth.c2()
    a = _sim(q, tabs["fp32"], w, False, w.n + 20_000, 20_000, 2_000_000)
    b = _sim(q, tabs["fp32"], w, True, w.n + 20_000, 20_000, 2_000_000, ppb=64, maxb=1 << 20)
    for _ in range(40):
        a.step(); b.step()
    assert b.plan.blocks > 2 * 8192
    _assert_same(_state(q, a), _state(q, b), "many blocks")
    assert q.counters_dict(b.ctr)["n_emit"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plan_equals_per_species_grid(q, tabs, prec):
    """Grid fields in the merged step, which interpolates from its own node-interleaved copy of the
    grid (refreshed every step), against the per-species calls, which read the caller's six
    arrays: 20000 electrons of the grid workload over 60 steps with pairs, bit for bit; the
    grid is then changed between steps and both must follow it."""
    import torch
    w = synth.c3(n=20_000, steps=60)
    grid = torch.as_tensor(w.extra["grid"], device="cuda")
    f = q.make_fields(q.QED_FIELD_GRID2D, grid=grid, dx=w.extra["dx"], dy=w.extra["dy"])
    a = _sim(q, tabs[prec], w, False, 4 * w.n, 2 * w.n, 40 * w.n, fields=f)
    b = _sim(q, tabs[prec], w, True, 4 * w.n, 2 * w.n, 40 * w.n, fields=f)
    for k in range(1, 61):
        if k == 31:
            grid.mul_(1.25)                  # the field changes between steps
            torch.cuda.synchronize()
        a.step(); b.step()
        if k % 20 == 0:
            a.compact(); b.compact()
    torch.cuda.synchronize()
    _assert_same(_state(q, a), _state(q, b), f"grid {prec}")
    c = q.counters_dict(b.ctr)
    assert c["n_emit"] > 10_000 and c["n_pair"] > 0, c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checkpoint_resume_is_bit_identical(q, tabs, prec, tmp_path):
    """Run N steps; separately run k steps, save a checkpoint to disk, load it into a fresh
    simulation and run N - k: the two end states are equal bit for bit (Philox is counter-based,
    the state is the SoA arrays, the counts, the counters and the step index)."""
    import torch
    w = synth.subsample(synth.c2(), np.arange(1500))
    N, k = 900, 370
    caps = (w.n + 3000, 3000, 120_000)

    def run(sim, a, b):
        for j in range(a, b):
            sim.step()
            if (j + 1) % 50 == 0:
                sim.compact()

    a = _sim(q, tabs[prec], w, True, *caps)
    run(a, 0, N)
    b = _sim(q, tabs[prec], w, True, *caps)
    run(b, 0, k)
    path = str(tmp_path / "ckpt.npz")
    b.save(path)
    del b
    c = _sim(q, tabs[prec], w, True, *caps)
    c.load_checkpoint(path)
    assert c.n == k
    run(c, k, N)
    torch.cuda.synchronize()
    _assert_same(_state(q, a), _state(q, c), f"resume {prec}")
    assert int(a.clock.item()) == int(c.clock.item()) == N
    cc = q.counters_dict(c.ctr)
    assert cc["n_emit"] > 1000 and cc["n_pair"] > 0
