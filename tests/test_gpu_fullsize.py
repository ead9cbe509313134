"""The head-on collision at its full size (10^6 electrons) in the launch configuration the
benchmark times (merged step, 1024 particles per block, graph replay with a compaction every 50
steps), against the oracle on sampled electrons: FP64 through the whole pulse, and FP32 for two
steps from the state at the peak of the pulse.  Electrons are independent of one another given
the fields, so the oracle recomputes a sample of them (with their original Philox ids) and the
photons they emit; pair products are left out (their slots depend on every photon)."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_leptons, compare_photons, oracle_run, photon_parent

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


def _sim(q, tab, w, t0=0.0):
    from paper_2511_08929_amd.sim import Simulation
    cap_p = w.n // 5
    f = q.make_fields(w.field_kind, a0=w.a0, phase_len=w.phase_len)
    return Simulation(tab, cap_e=w.n + cap_p, cap_p=cap_p, cap_g=30 * w.n, track=w.track, fields=f, dt=w.dt,
                      eps_r=EPS, seed=w.seed, flags=q.QED_ALL, k_retire=w.k_retire, t0=t0, device_clock=True,
                      merged=True, particles_per_block=1024)


def _sample(n):
    return np.sort(np.random.default_rng(1234).choice(np.arange(10_000, n), 256, replace=False))


def _own_photons(arrays, idx):
    """the live photons of the sampled electrons (with the oracle's conditioning when present)"""
    x, k, P, ids = arrays
    sp, par = photon_parent(ids)
    mine = (ids != 0) & (sp == 0) & np.isin(par, idx)
    out = oracle.SetArrays((x[:, mine], k[:, mine], P[:, mine], ids[mine]))
    out.cond = arrays.cond[mine] if getattr(arrays, "cond", None) is not None else None
    return out


def test_head_on_full_size_graph_fp64(q, otables):
    import torch
    w = synth.c2()
    steps = 1700                                   # through the whole pulse
    sim = _sim(q, q.Tables(precision=q.QED_F64), w)
    sim.e.load(w.x, w.p, w.s)
    g = sim.capture(50)
    for _ in range(steps // 50):
        sim.replay(g)
    torch.cuda.synchronize()
    c = q.counters_dict(sim.ctr)
    print("full size fp64:", c)
    assert c["n_capacity_overflow"] == 0 and c["n_emit"] > 10_000_000
    idx = _sample(w.n)
    sub = synth.subsample(w, idx)
    ref = oracle_run(otables, sub, steps, q.QED_ALL, cap_e=2000, cap_p=2000, cap_g=60_000, index=idx)
    ex = ref["near_e"][:256]
    x, p, s = sim.e.arrays()
    t = 1e-12 * steps / 250
    compare_leptons((x[:, idx], p[:, idx], s[:, idx]), tuple(a[:, :256] for a in ref["E"].arrays()), ex, t, t,
                    rtol_x=t, what="sampled electrons", cond=ref["E"].cond[:256])
    compare_photons(_own_photons(sim.g.arrays(), idx), _own_photons(ref["G"].arrays(), idx),
                    {(0, int(i)) for i in idx[ex]}, t, t, what="their photons")


def test_head_on_full_size_peak_fp32(q, otables):
    """The FP64 state at the peak of the pulse (step 850), stored in FP32, then two FP32 merged
    steps; the oracle takes the same FP32 inputs in its 24-bit-uniform mode."""
    import torch
    w = synth.c2()
    k0 = 850
    s64 = _sim(q, q.Tables(precision=q.QED_F64), w)
    s64.e.load(w.x, w.p, w.s)
    g = s64.capture(50)
    for _ in range(k0 // 50):
        s64.replay(g)
    torch.cuda.synchronize()
    # the primary electrons only (pair-born ones sit behind them)
    x, p, s = (a[:, :w.n].astype(np.float32).astype(np.float64) for a in s64.e.arrays())
    del s64, g
    torch.cuda.empty_cache()
    w2 = synth.subsample(w, np.arange(w.n))
    w2.x, w2.p, w2.s = x, p, s
    sim = _sim(q, q.Tables(precision=q.QED_F32), w2, t0=k0 * w.dt)
    sim.e.load(x, p, s)
    for _ in range(2):
        sim.step()
    torch.cuda.synchronize()
    c = q.counters_dict(sim.ctr)
    print("full size fp32 at the peak:", c)
    assert c["n_emit"] > 20_000
    idx = _sample(w.n)
    sub = synth.subsample(w2, idx)
    ref = oracle_run(otables, sub, 2, q.QED_ALL, cap_e=1000, cap_p=1000, cap_g=2000, index=idx, t0=k0 * w.dt,
                     u24=True, near_tol=1e-5, round32=True)
    ex = ref["near_e"][:256]
    xg, pg, sg = sim.e.arrays()
    compare_leptons((xg[:, idx], pg[:, idx], sg[:, idx]), tuple(a[:, :256] for a in ref["E"].arrays()), ex, 1e-5, 1e-5,
                    what="sampled electrons fp32", cond=ref["E"].cond[:256])
    compare_photons(_own_photons(sim.g.arrays(), idx), _own_photons(ref["G"].arrays(), idx),
                    {(0, int(i)) for i in idx[ex]}, 1e-5, 1e-5, what="their photons fp32")
