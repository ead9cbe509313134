"""The learned inverse CDF (qed_surrogate_*): the GPU training kernels' gradients against the FP64
reference network (oracle/mlp.py, itself pinned by finite differences); the trained surrogate
(coarse table + network for its residual) against the fine inverse-CDF tables it stands in for,
with the tables as judge and fallback; what the network gains (error against its coarse table
alone, memory against the fine tables, and a plain table of the same bytes beside it); and the
merged step with it (same decisions, photon energies within the stated error, replayable in a
graph)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from oracle import mlp

pytestmark = pytest.mark.gpu

EPS = synth.EPS_R
JUDGE_BOUND = 0.01          # |dnu| above which a coarse cell falls back to the table inverse CDF


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_08929_amd as q
    return q


@pytest.fixture(scope="module")
def t32(q):
    return q.Tables(precision=q.QED_F32)


@pytest.fixture(scope="module")
def trained(q, t32):
    out = {}
    for proc in (0, 1):
        s = q.Surrogate(t32, proc, seed=1)
        loss = s.fit().cpu().numpy()
        err, nm = s.judge(JUDGE_BOUND)
        out[proc] = (s, loss, err, nm)
    return out


def _bf16(a):
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _inputs(q, s, n, seed, rho_max=16.0):
    import torch
    m, h, rs, os_ = s.norm()
    rng = np.random.default_rng(seed)
    x = np.column_stack([m + h * rng.uniform(-1, 1, n), rng.uniform(-rho_max, rho_max, n), rng.choice([-1.0, 1.0], n)])
    return torch.tensor(x, dtype=torch.float32, device="cuda").contiguous()


@pytest.mark.parametrize("proc", [0, 1])
def test_surrogate_gradient_matches_fp64_reference(q, t32, proc):
    import torch
    s = q.Surrogate(t32, proc, seed=5)
    m, h, rs, os_ = s.norm()
    n = 4096
    x = _inputs(q, s, n, 2)
    y = np.random.default_rng(3).normal(0.0, 0.5, n).astype(np.float32)
    g = s.gradient(x, torch.tensor(y, device="cuda")).cpu().numpy().astype(np.float64)
    theta = _bf16(s.get_params().cpu().numpy())            # the network runs on BF16 weights
    xf = x.cpu().numpy()
    X = np.column_stack([(xf[:, 0] - np.float32(m)) / np.float32(h), xf[:, 1] / np.float32(rs), xf[:, 2]])
    L, go = mlp.loss_and_grad(theta, X.astype(np.float64), y.astype(np.float64))
    o = 0
    for name, shp in mlp.SHAPES:
        k = int(np.prod(shp))
        a, b = g[o:o + k], go[o:o + k]
        o += k
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert rel < 5e-3, (name, rel)
    assert abs(g[-1] / L - 1) < 1e-3


def _lagrange(t):
    return np.stack([-(t - 1) * (t - 2) * (t - 3) / 6, t * (t - 2) * (t - 3) / 2, -t * (t - 1) * (t - 3) / 2,
                     t * (t - 1) * (t - 2) / 6], -1)


def _interp(nodes, x0, dx, y0, dy, x, y):
    """4-point Lagrange in both axes on a node array (one-sided at the ends, clamped), vectorized"""
    nx, ny = nodes.shape
    fx = np.clip((x - x0) / dx, 0, nx - 1)
    fy = np.clip((y - y0) / dy, 0, ny - 1)
    ix = np.clip(np.floor(fx).astype(int) - 1, 0, nx - 4)
    iy = np.clip(np.floor(fy).astype(int) - 1, 0, ny - 4)
    Lx, Ly = _lagrange(fx - ix), _lagrange(fy - iy)
    out = np.zeros_like(x)
    for a in range(4):
        for b in range(4):
            out += Lx[:, a] * Ly[:, b] * nodes[ix + a, iy + b]
    return out


def _fine(otables, ch, lnchi, rho):
    sp = otables.spec
    g = 0 if ch < 2 else 1
    return _interp(otables.nu_nodes(ch), sp["lnchi0"][g], sp["dlnchi"][g], sp["rho0"], sp["drho"], lnchi, rho)


def _sampling_inputs(q, s, n, seed):
    """(ln chi, rho, c) with ln chi uniform over the table range and rho = logit r of a 24-bit
    uniform r: the distribution the step draws rho from"""
    import torch
    m, h, _, _ = s.norm()
    rng = np.random.default_rng(seed)
    r = (2 * rng.integers(0, 2**23, n) + 1) * 2.0**-24
    x = np.column_stack([m + h * rng.uniform(-1, 1, n), np.log(r) - np.log1p(-r), rng.choice([-1.0, 1.0], n)])
    return torch.tensor(x, dtype=torch.float32, device="cuda").contiguous()


@pytest.mark.parametrize("proc", [0, 1])
def test_surrogate_judged_error(q, t32, trained, otables, proc):
    """The surrogate against the fine tables at the rho the sampling draws: the network alone
    (base + net everywhere), and as the step uses it (table inverse CDF in the cells the judgement
    marked), whose error stays at the judge's bound; the judgement marks few cells, and the marked
    cells return exactly the table's nu."""
    s, loss, cell_err, nm = trained[proc]
    info = s.info()
    assert np.sqrt(loss[-1]) * info.out_s < 2e-3 < np.sqrt(loss[0]) * info.out_s    # training mse, in nu
    assert info.n_masked == nm and info.bound == pytest.approx(JUDGE_BOUND) and cell_err.shape == (info.n_cells,)
    x = _sampling_inputs(q, s, 200_000, 7)
    xf = x.cpu().numpy().astype(np.float64)
    ch = 2 * proc + (xf[:, 2] > 0)
    ref = np.where(ch % 2 == 1, _fine(otables, 2 * proc + 1, xf[:, 0], xf[:, 1]),
                   _fine(otables, 2 * proc, xf[:, 0], xf[:, 1]))
    lam = lambda v: 1 / (1 + np.exp(-v))            # noqa: E731
    stats = {}
    for name, mode in (("base", q.SURROGATE_BASE), ("network", q.SURROGATE_NETWORK), ("as used", q.SURROGATE_AS_USED)):
        nu = s.eval(x, mode).cpu().numpy().astype(np.float64)
        d = np.abs(nu - ref)
        rel = np.abs(lam(nu) - lam(ref)) / lam(ref)
        stats[name] = d
        print(f"process {proc} {name}: |dnu| rms {np.sqrt(np.mean(d * d)):.3g} p99.9 {np.quantile(d, 0.999):.3g} "
              f"max {d.max():.3g}; lambda rel median {np.median(rel):.3g} p99 {np.quantile(rel, 0.99):.3g}")
    print(f"process {proc}: {nm} of {info.n_cells} cells marked at |dnu| > {JUDGE_BOUND}")
    assert nm <= 0.05 * info.n_cells
    # the judge's 8 x 8 points per cell bound the error between them to within a small margin
    assert np.quantile(stats["as used"], 0.999) < JUDGE_BOUND and stats["as used"].max() < 2 * JUDGE_BOUND
    assert np.sqrt(np.mean(stats["network"] ** 2)) < 5e-3
    # marked cells: the table inverse CDF itself (FP64 lookup of the same tables, stored in FP32)
    used = s.eval(x, q.SURROGATE_AS_USED).cpu().numpy().astype(np.float64)
    net = s.eval(x, q.SURROGATE_NETWORK).cpu().numpy().astype(np.float64)
    fb = used != net
    print(f"process {proc}: {fb.sum()} of {fb.size} samples in marked cells")
    if nm:
        assert (np.abs(used[fb] - ref[fb]) <= 1e-6 * np.maximum(1, np.abs(ref[fb]))).all()


@pytest.mark.parametrize("proc", [0, 1])
def test_what_the_network_gains(q, t32, trained, otables, proc):
    """What the trained network adds to the method without it.  Against its own coarse table it
    cuts the error several times (that is what it learns); against the fine tables of the step it
    needs a small fraction of their memory at the stated error.  Beside it, a plain table of the
    same bytes as network + coarse table + mask, on the fine tables' own values: in this
    two-variable inverse CDF such a table is more accurate than the network, so the gain is
    memory against the fine tables, not accuracy per byte (reported, not asserted)."""
    s, _, _, _ = trained[proc]
    info = s.info()
    x = _sampling_inputs(q, s, 200_000, 11)
    xf = x.cpu().numpy().astype(np.float64)
    up = xf[:, 2] > 0
    ref = np.where(up, _fine(otables, 2 * proc + 1, xf[:, 0], xf[:, 1]), _fine(otables, 2 * proc, xf[:, 0], xf[:, 1]))
    rms = lambda d: float(np.sqrt(np.mean(d * d)))   # noqa: E731
    e_base = rms(s.eval(x, q.SURROGATE_BASE).cpu().numpy() - ref)
    e_net = rms(s.eval(x, q.SURROGATE_NETWORK).cpu().numpy() - ref)
    sp = otables.spec
    g = 0 if proc == 0 else 1
    fine_bytes = 2 * sp["n_chi"][g] * sp["n_rho"] * 8
    sur_bytes = info.bytes_network + info.bytes_base + info.bytes_mask
    # the equal-bytes plain table: FP32 nodes over the same ln chi range and rho in [-20, 20], with
    # the coarse table's aspect (nodes per unit of ln chi / per unit of rho) kept
    n_nodes = sur_bytes // 4 // 2
    lo = info.base_lnchi0
    hi = lo + (info.base_n_chi - 1) * info.base_dlnchi
    aspect = (info.base_n_chi - 1) / (info.base_n_rho - 1)
    nr = int(np.sqrt(n_nodes / aspect))
    nx = n_nodes // nr
    gx, gy = np.linspace(lo, hi, nx), np.linspace(-20, 20, nr)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    eq = {}
    for c in (0, 1):
        nodes = _fine(otables, 2 * proc + c, X.ravel(), Y.ravel()).reshape(X.shape).astype(np.float32)
        eq[c] = _interp(nodes.astype(np.float64), lo, gx[1] - gx[0], -20.0, gy[1] - gy[0], xf[:, 0], xf[:, 1])
    e_eq = rms(np.where(up, eq[1], eq[0]) - ref)
    print(f"process {proc}: rms |dnu| coarse table {e_base:.3g} ({info.bytes_base} B) -> with the network "
          f"{e_net:.3g} ({sur_bytes} B in all: {e_base / e_net:.1f}x lower); fine tables {fine_bytes} B "
          f"({fine_bytes / sur_bytes:.0f}x the surrogate); a plain {nx} x {nr} FP32 table of the same bytes: {e_eq:.3g}")
    assert e_net < e_base / 4
    assert fine_bytes > 50 * sur_bytes


def test_merged_step_with_surrogate(q, t32, trained):
    """Head-on collision, 4000 electrons, FP32: one step from the same state gives the same
    decisions with and without the network and photon energies within its stated error; the
    surrogate plan replayed in a HIP graph equals its eager steps."""
    import torch
    from paper_2511_08929_amd.sim import Simulation
    w = synth.subsample(synth.c2(), np.arange(4000))
    w.k_retire = 0.0                           # keep every photon, soft ones included
    f = q.make_fields(w.field_kind, a0=w.a0, phase_len=w.phase_len)
    sur = (trained[0][0], trained[1][0])

    def mk(use):
        sim = Simulation(t32, cap_e=w.n + 3000, cap_p=3000, cap_g=400_000, track=w.track, fields=f, dt=w.dt,
                         eps_r=EPS, seed=w.seed, flags=q.QED_ALL, k_retire=w.k_retire, device_clock=True,
                         merged=True, surrogates=sur if use else (None, None))
        sim.e.load(w.x, w.p, w.s)
        return sim

    a, b = mk(False), mk(True)
    for k in range(700):                       # into the pulse, eagerly, same state on both
        a.step()
        if (k + 1) % 50 == 0:
            a.compact()
    for L, M in ((a.e, b.e), (a.p, b.p)):
        for i in range(3):
            M.p[i].copy_(L.p[i]); M.s[i].copy_(L.s[i])
            if L.x[i] is not None:
                M.x[i].copy_(L.x[i])
        M.count.copy_(L.count)
    for i in range(3):
        b.g.k[i].copy_(a.g.k[i]); b.g.P[i].copy_(a.g.P[i])
        if a.g.x[i] is not None:
            b.g.x[i].copy_(a.g.x[i])
    b.g.id.copy_(a.g.id); b.g.count.copy_(a.g.count); b.g.count_prev.copy_(a.g.count_prev)
    b.clock.copy_(a.clock); b.n = a.n
    n0 = a.g.n()
    a.step(); b.step()
    torch.cuda.synchronize()
    ida, idb = a.g.id[n0:a.g.n()].cpu().numpy(), b.g.id[n0:b.g.n()].cpu().numpy()
    assert ida.shape == idb.shape                              # same emitters: same slots
    # a photon born below the retirement energy is stored as a dead slot (id 0): near that
    # energy the network's lambda may decide differently
    both = (ida != 0) & (idb != 0)
    np.testing.assert_array_equal(ida[both], idb[both])
    assert ((ida != 0) != (idb != 0)).mean() < 0.05
    ka = np.stack([a.g.k[i][n0:a.g.n()].double().cpu().numpy() for i in range(3)])
    kb = np.stack([b.g.k[i][n0:b.g.n()].double().cpu().numpy() for i in range(3)])
    live = both
    rel = np.linalg.norm(kb[:, live] - ka[:, live], axis=0) / np.linalg.norm(ka[:, live], axis=0)
    print(f"one step: {live.sum()} photons, energy rel err median {np.median(rel):.3g} p99 {np.quantile(rel, 0.99):.3g}")
    # photon energy = lambda |p|: its relative error is that of lambda, (1 - lambda) |dnu| <= |dnu|
    assert live.sum() > 200 and np.median(rel) < 2e-3 and np.quantile(rel, 0.99) < JUDGE_BOUND
    # graph replay of the surrogate plan equals its eager steps
    c = mk(True)
    for k in range(650):
        c.step()
        if (k + 1) % 50 == 0:
            c.compact()
    d = mk(True)
    for k in range(600):
        d.step()
        if (k + 1) % 50 == 0:
            d.compact()
    g = d.capture(50)
    d.replay(g)
    torch.cuda.synchronize()
    for x, y in zip(c.e.arrays() + c.g.arrays(), d.e.arrays() + d.g.arrays()):
        np.testing.assert_array_equal(x, y)


def test_surrogate_step_full_size(q, t32, trained):
    """The learned-inverse-CDF workload at its stated size: all 10^8 electrons of the head-on
    collision, FP32, started at the centre of the pulse.  One step from the same state with the
    tables and with the network: the same emitters (the same photon ids in the same slots), photon
    energies within the network's stated error, and every electron that did not emit equal bit for
    bit (its step does not involve the inverse CDF)."""
    import torch
    from paper_2511_08929_amd.sim import Simulation
    w = synth.c2(n=100_000_000)
    f = q.make_fields(w.field_kind, a0=w.a0, phase_len=w.phase_len)
    t0 = 0.5 * w.phase_len + math.pi            # electron phases t + x in the middle of the pulse
    sur = (trained[0][0], trained[1][0])

    def mk(use):
        sim = Simulation(t32, cap_e=w.n + 1000, cap_p=1000, cap_g=w.n // 4, track=w.track, fields=f, dt=w.dt,
                         eps_r=EPS, seed=w.seed, flags=q.QED_ALL, k_retire=0.0, t0=t0, device_clock=True,
                         merged=True, surrogates=sur if use else (None, None))
        sim.e.load(w.x, w.p, w.s)
        return sim

    a = mk(False)
    a.step()
    torch.cuda.synchronize()
    ca = q.counters_dict(a.ctr)
    ng = a.g.n()
    ida = a.g.id[:ng].cpu().numpy()
    ka = np.stack([a.g.k[i][:ng].double().cpu().numpy() for i in range(3)])
    pa = [a.e.p[i][:w.n].cpu().numpy() for i in range(3)]
    del a
    torch.cuda.empty_cache()
    b = mk(True)
    b.step()
    torch.cuda.synchronize()
    cb = q.counters_dict(b.ctr)
    assert ca["n_capacity_overflow"] == 0 and cb["n_capacity_overflow"] == 0
    assert ca["n_emit"] == cb["n_emit"] == ng == b.g.n() and ng > 10**6
    np.testing.assert_array_equal(ida, b.g.id[:ng].cpu().numpy())
    kb = np.stack([b.g.k[i][:ng].double().cpu().numpy() for i in range(3)])
    rel = np.linalg.norm(kb - ka, axis=0) / np.linalg.norm(ka, axis=0)
    print(f"10^8 electrons, one step: {ng} photons, energy rel err median {np.median(rel):.3g} "
          f"p99 {np.quantile(rel, 0.99):.3g}")
    assert np.median(rel) < 2e-3 and np.quantile(rel, 0.99) < JUDGE_BOUND
    same = np.ones(w.n, dtype=bool)
    for i in range(3):
        same &= pa[i] == b.e.p[i][:w.n].cpu().numpy()
    assert (~same).sum() <= ng                   # only emitters differ (recoil with the network's lambda)


def test_fallback_everywhere_is_the_table_path(q, t32, trained):
    """With every cell marked (judged at bound 0) the surrogate step is the table step: one merged
    step of 20000 electrons at the centre of the pulse equals the table path bit for bit, and the
    evaluation as used returns the tables' nu.  The judgement is restored afterwards."""
    import torch
    from paper_2511_08929_amd.sim import Simulation
    w = synth.subsample(synth.c2(), np.arange(20_000))
    f = q.make_fields(w.field_kind, a0=w.a0, phase_len=w.phase_len)
    t0 = 0.5 * w.phase_len + math.pi
    sur = (trained[0][0], trained[1][0])
    try:
        for s in sur:
            _, nm = s.judge(0.0)
            assert nm > 0.3 * s.info().n_cells          # every cell the 24-bit rho reaches
        x = _sampling_inputs(q, sur[0], 4096, 3)
        tab = sur[0].eval(x, q.SURROGATE_AS_USED).cpu().numpy()
        net = sur[0].eval(x, q.SURROGATE_NETWORK).cpu().numpy()
        assert (tab != net).mean() > 0.99

        def run(use):
            sim = Simulation(t32, cap_e=w.n + 1000, cap_p=1000, cap_g=w.n, track=w.track, fields=f, dt=w.dt,
                             eps_r=EPS, seed=w.seed, flags=q.QED_ALL, k_retire=0.0, t0=t0, device_clock=True,
                             merged=True, surrogates=sur if use else (None, None))
            sim.e.load(w.x, w.p, w.s)
            for _ in range(3):
                sim.step()
            torch.cuda.synchronize()
            return sim, q.counters_dict(sim.ctr)

        a, ca = run(False)
        b, cb = run(True)
        assert ca == cb and ca["n_emit"] > 500
        for u, v in zip(a.e.arrays() + a.g.arrays(), b.e.arrays() + b.g.arrays()):
            np.testing.assert_array_equal(u, v)
    finally:
        for s in sur:
            s.judge(JUDGE_BOUND)
