#!/usr/bin/env python3
"""Throughput of the spin- and polarization-resolved QED step on one MI355X.

Workload: the head-on collision -- 10^6 electrons, gamma0 ~ N(4000, 5 %), 1 mrad spread, spins
+/-y, LP plane wave along -x with a0 = 100 and a 30 fs (intensity FWHM) sin^2 envelope,
dt = lambda/(100 c), both QED channels on -- in the single-precision path with FP64 islands.

One benchmark step is one whole collision: the 3000 time steps of that workload from its
initial state, each time step the whole path over every particle (push + NLC for electrons
and positrons, NBW for photons, and the compaction of dead photon slots every 50 steps).
`--steps K` times K such collisions after `--warmup W` untimed ones; the initial state is kept
on the device and put back (device copies) at the start of each collision, inside the timed
region.  The number of time steps per collision is fixed: it is part of the workload.

value = (lepton steps + live photon steps) counted on the device over the K collisions / wall
time.  Prints one JSON line.  Besides the headline it reports the FP64 path on the same
collision, the dominant kernel's achieved HBM bandwidth (HIP events that its dispatches stamp) next
to its VALU issue and counted traffic, the whole-step bandwidth, the oracle's throughput on the
host cores (`cpu_baseline`) with the decision mismatch rate of the single-precision path and the
table method error, and extras (learned inverse CDF, batched ensembles, rejection sampling,
field-dependent g, cascade, sub-cycling, grid fields), each fail-soft and within a time budget.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
import traceback

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ = 256, 2.4
# one 64-lane VALU instruction per compute unit per cycle (four SIMD16 units, four cycles each):
# the unpacked FP32 / INT32 / FP64-FMA lane rate of the chip
VALU_PEAK_TLANE = CUS * 64 * CLOCK_GHZ * 1e9 / 1e12
METRIC = "particle-QED-steps/s (spin+pol resolved), FP32/surrogate vs FP64, at stated error"
COLLISION_STEPS = 3000                 # time steps of one head-on collision (the workload)
COMPACT_EVERY = 50
T_START = time.perf_counter()


def log(*a):
    print("[bench]", f"{time.perf_counter() - T_START:7.1f}s", *a, file=sys.stderr, flush=True)


def bytes_per_unit(es, tracked_x=1):
    """Algorithmic HBM bytes per lepton-step and per photon-step (element size es):
    lepton: read and write the tracked x components, p[3], s[3];
    photon: read id, k[3], P[3], x; write x and P[3]."""
    lep = 2 * es * (tracked_x + 6)
    pho = 8 + es * (6 + tracked_x) + es * (3 + tracked_x)
    return lep, pho


def work_of(ctr):
    return ctr["n_lepton_steps"] + ctr["n_photon_steps"]


# ----------------------------------------------------------------------------- collisions
class Collision:
    """One Simulation of the head-on collision in the benchmark's launch configuration (merged
    step, HIP graph of COMPACT_EVERY steps plus a compaction) with its initial state kept on the
    device; run() puts that state back and replays the whole collision."""

    def __init__(self, q, tab, w, cfg, surrogates=(None, None), flags=None, fields=None, caps=None,
                 photons_per_electron=30, steps=COLLISION_STEPS):
        from paper_2511_08929_amd.sim import Simulation
        cap_p = max(1000, w.n // 5)
        cap_e, cap_g = w.n + cap_p, max(100_000, photons_per_electron * w.n)
        if caps is not None:
            cap_e, cap_p, cap_g = caps
        if fields is None:
            fields = q.make_fields(w.field_kind, a0=w.a0, phase_len=w.phase_len)
        self.steps = steps
        self.sim = Simulation(tab, cap_e=cap_e, cap_p=cap_p, cap_g=cap_g, track=w.track, fields=fields, dt=w.dt,
                              eps_r=synth.EPS_R, seed=w.seed, flags=q.QED_ALL if flags is None else flags,
                              k_retire=w.k_retire, device_clock=True, merged=True, surrogates=surrogates,
                              particles_per_block=cfg.get("particles_per_block", 0),
                              process_group=cfg.get("process_group", 0),
                              max_blocks_per_set=cfg.get("max_blocks_per_set", 0),
                              photon_variant=cfg.get("photon_variant", 0))
        self.sim.e.load(w.x, w.p, w.s)
        self.init = self.sim.snapshot()
        self.graph = None

    def set_config(self, cfg):
        self.graph = None
        self.sim.set_launch_config(**cfg)

    def run(self, reps=1):
        """reps whole collisions from the initial state (no host synchronization inside)"""
        sim = self.sim
        if self.graph is None:
            sim.restore(self.init)
            self.graph = sim.capture(COMPACT_EVERY)
        for _ in range(reps):
            sim.restore(self.init, counters=False)
            done = 0
            while done + COMPACT_EVERY <= self.steps:
                sim.replay(self.graph)
                done += COMPACT_EVERY
            for _ in range(self.steps - done):
                sim.step()

    def counters(self):
        import paper_2511_08929_amd as q
        return q.counters_dict(self.sim.ctr)

    def zero_counters(self):
        self.sim.ctr.zero_()

    def timed(self, reps, warmup):
        """wall time of `reps` collisions after `warmup` untimed ones, and their counters"""
        import torch
        self.run(warmup)
        torch.cuda.synchronize()
        self.zero_counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.run(reps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, self.counters()

    def close(self):
        import torch
        self.graph = None
        self.sim.set_launch_config()
        del self.sim, self.init
        torch.cuda.empty_cache()


def profiled_collision(q, tab, w, cfg):
    """One eager collision with every launch timed by a start and a stop event that its dispatch
    stamps (the kernel's own begin and end); per-kernel
    (calls, total ms), the counters of that collision and its wall time."""
    import torch
    from paper_2511_08929_amd.sim import Simulation
    cap_p = max(1000, w.n // 5)
    sim = Simulation(tab, cap_e=w.n + cap_p, cap_p=cap_p, cap_g=max(100_000, 30 * w.n), track=w.track,
                     fields=q.make_fields(w.field_kind, a0=w.a0, phase_len=w.phase_len), dt=w.dt, eps_r=synth.EPS_R,
                     seed=w.seed, flags=q.QED_ALL, k_retire=w.k_retire, device_clock=True, merged=True,
                     particles_per_block=cfg.get("particles_per_block", 0), process_group=cfg.get("process_group", 0),
                     max_blocks_per_set=cfg.get("max_blocks_per_set", 0), photon_variant=cfg.get("photon_variant", 0))
    sim.e.load(w.x, w.p, w.s)
    init = sim.snapshot()
    sim.step()                                   # the plan is built outside the profiled region
    torch.cuda.synchronize()
    sim.restore(init)
    torch.cuda.synchronize()
    q.qed_profile_start()
    t0 = time.perf_counter()
    for k in range(COLLISION_STEPS):
        sim.step()
        if (k + 1) % COMPACT_EVERY == 0:
            sim.compact()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = q.qed_profile_stop()
    c = q.counters_dict(sim.ctr)
    sim.set_launch_config()
    del sim, init
    torch.cuda.empty_cache()
    return kt, c, wall


# ----------------------------------------------------------------------------- roofline
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "plan_photon_head_on_1e6_fp32_hbm_traffic.md")
VALU_FILE = os.path.join(ROOT, "profiles", "plan_kernels_head_on_1e6_fp32_valu.md")


def kernel_source_hash():
    """sha256 over the HIP sources; counters taken on other sources do not describe these kernels"""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2511_08929_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _summary_blob(path):
    try:
        text = open(path).read()
        return json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None


def load_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and WRITE_SIZE
    passes scaled by the copy-kernel factors), or None if absent or taken on other sources."""
    blob = _summary_blob(TRAFFIC_FILE)
    if not blob or blob.get("source_sha256") != kernel_source_hash():
        return None
    if blob.get("kernel") == kernel:
        return blob.get("traffic_bytes_per_launch")
    return (blob.get("kernels") or {}).get(kernel, {}).get("traffic_bytes_per_launch")


def load_valu(kernel):
    """VALU wave-instructions per launch of `kernel` from the committed counter summary, or None
    if absent or taken on other sources."""
    blob = _summary_blob(VALU_FILE)
    if not blob or blob.get("source_sha256") != kernel_source_hash():
        return None
    return blob.get("kernels", {}).get(kernel, {}).get("valu_per_launch")


def roofline(kt, ck, cgbs):
    """Dominant kernel (largest total time) of the profiled collision against its ceilings.
    Algorithmic bytes per launch: 56 B per lepton-step (plan_lepton) or 52 B per photon-step
    (plan_photon), FP32, times the steps counted on the device, over the launches.  The bound is
    the ceiling with the longer minimum time: HBM (algorithmic bytes / 8 TB/s) or VALU issue (the
    committed SQ_INSTS_VALU of the kernel / one wave-instruction per CU per cycle), when the VALU
    counters were taken on these sources."""
    lep_b, pho_b = bytes_per_unit(4)
    alg = {"plan_lepton": ck["n_lepton_steps"] * lep_b, "plan_photon": ck["n_photon_steps"] * pho_b}
    times = {k: v for k, v in kt.items() if k in alg}
    dom = max(times, key=lambda k: times[k][1])
    calls, ms = times[dom]
    t_launch = ms * 1e-3 / calls
    bytes_launch = alg[dom] / calls
    hbm_ach = bytes_launch / t_launch / 1e9
    valu = load_valu(dom)
    t_hbm_min = bytes_launch / (HBM_PEAK_GBS * 1e9)
    hbm = dict(achieved=round(hbm_ach, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(hbm_ach / HBM_PEAK_GBS, 4),
               min_time_us=round(t_hbm_min * 1e6, 2))
    out = dict(kernel=dom, avg_launch_us=round(t_launch * 1e6, 2), launches=calls, bytes_per_launch=round(bytes_launch),
               traffic=load_traffic(dom), copy_achieved=round(cgbs, 1), frac_of_copy=round(hbm_ach / cgbs, 4),
               hbm=hbm, kernel_ms={k: round(v[1], 3) for k, v in kt.items()})
    bound = "hbm"
    if valu:
        t_valu_min = valu / (CUS * CLOCK_GHZ * 1e9)
        lanes = valu * 64 / t_launch / 1e12
        out["alu"] = dict(achieved=round(lanes, 3), peak=round(VALU_PEAK_TLANE, 3),
                          unit="T VALU lane-instructions/s", frac=round(lanes / VALU_PEAK_TLANE, 4),
                          valu_per_launch=valu, min_time_us=round(t_valu_min * 1e6, 2))
        if t_valu_min > t_hbm_min:
            bound = "alu"
    src = out["alu"] if bound == "alu" else hbm
    out.update(bound=bound, achieved=src["achieved"], peak=src["peak"], unit=src["unit"], frac=src["frac"])
    # the whole step: every streaming kernel's algorithmic bytes over the time of all launches
    tot_ms = sum(v[1] for v in kt.values())
    step_bytes = sum(alg.values())
    out["whole_step"] = dict(algorithmic_bytes=int(step_bytes), kernel_ms=round(tot_ms, 3),
                             achieved=round(step_bytes / (tot_ms * 1e-3) / 1e9, 1),
                             frac=round(step_bytes / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             target_frac=0.6)
    # bytes the method must move (P-vector only for photons that reach the QED part)
    need = ck["n_lepton_steps"] * lep_b + ck["n_photon_steps"] * (pho_b - 24) + ck["n_photon_qed"] * 24
    out["method_bytes_per_step"] = int(need / COLLISION_STEPS)
    return out


def copy_gbs(reps=10):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy of 1 GiB (read 1 GiB,
    write 1 GiB), timed with HIP events, best of `reps`."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = float("inf")
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * (1 << 30) / (best * 1e-3) / 1e9


# ----------------------------------------------------------------------------- spectra
def spectra(q, tab, w, steps, surrogates=(None, None), flags=None):
    """Every photon emitted in `steps` steps of workload w (no retirement, no compaction: dead
    slots keep their momentum and P-vector) and the electrons' final spins."""
    import torch
    from paper_2511_08929_amd.sim import Simulation
    fields = q.make_fields(w.field_kind, a0=w.a0, phase_len=w.phase_len)
    sim = Simulation(tab, cap_e=w.n * 2 + 1000, cap_p=w.n + 1000, cap_g=120 * w.n, track=w.track, fields=fields,
                     dt=w.dt, eps_r=synth.EPS_R, seed=w.seed, flags=q.QED_ALL if flags is None else flags, k_retire=0.0,
                     device_clock=True, merged=True, surrogates=surrogates)
    sim.e.load(w.x, w.p, w.s)
    for _ in range(steps):
        sim.step()
    torch.cuda.synchronize()
    n = sim.g.n()
    k = torch.stack([c[:n].double() for c in sim.g.k]).norm(dim=0).cpu().numpy()
    P = torch.stack([c[:n].double() for c in sim.g.P]).cpu().numpy()
    kh = torch.stack([c[:n].double() for c in sim.g.k]).cpu().numpy() / np.maximum(k, 1e-300)
    xi2 = np.sum(P * kh, axis=0)                       # circular Stokes parameter (P along k)
    lin = P[1] ** 2 - P[2] ** 2                          # linear polarization along the laser E (y) vs B (z)
    s = torch.stack([c[:w.n].double() for c in sim.e.s]).cpu().numpy()
    c = q.counters_dict(sim.ctr)
    del sim
    torch.cuda.empty_cache()
    return dict(k=k, xi2=xi2, lin=lin, s_mean=s.mean(axis=1), ctr=c)


def spectrum_error(ref, got, bins_per_decade=8, min_count=10_000):
    """per-bin relative error of the photon-energy spectrum (8 bins per decade) over bins holding at
    least min_count photons; per bin, the change of the photons' mean linear polarization along the
    laser field (P_y^2 - P_z^2) and mean circular polarization (P . k/|k|); the change of the
    electrons' mean spin vector.  Fields that no bin supports are None."""
    out = dict(bins=0, spectrum_max_rel=None, spectrum_mean_rel=None, spectrum_stat_1sigma=None,
               linear_pol_max_abs=None, circular_pol_max_abs=None,
               spin_mean_abs=round(float(np.abs(np.asarray(got["s_mean"]) - np.asarray(ref["s_mean"])).max()), 6)
               if len(ref["s_mean"]) else None,
               photons_ref=int(ref["k"].size), photons=int(got["k"].size))
    kr = ref["k"][ref["k"] > 0]
    if kr.size == 0 or got["k"].size == 0:
        return out
    lo, hi = np.log10(max(kr.min(), 1e-3)), np.log10(kr.max())
    edges = 10 ** np.arange(np.floor(lo * bins_per_decade) / bins_per_decade, hi + 1 / bins_per_decade,
                            1 / bins_per_decade)
    if edges.size < 2:
        return out
    nr, _ = np.histogram(ref["k"], edges)
    ng, _ = np.histogram(got["k"], edges)
    ok = nr >= min_count
    if not ok.any():
        return out
    rel = np.abs(ng[ok] / nr[ok] - 1)
    stat = 1 / np.sqrt(nr[ok])
    dlin, dcirc = [], []
    for a, b_ in zip(edges[:-1][ok], edges[1:][ok]):
        sr, sg = (ref["k"] >= a) & (ref["k"] < b_), (got["k"] >= a) & (got["k"] < b_)
        if sg.any():
            dlin.append(abs(got["lin"][sg].mean() - ref["lin"][sr].mean()))
            dcirc.append(abs(got["xi2"][sg].mean() - ref["xi2"][sr].mean()))
    out.update(bins=int(ok.sum()), spectrum_max_rel=round(float(rel.max()), 5),
               spectrum_mean_rel=round(float(rel.mean()), 5), spectrum_stat_1sigma=round(float(stat.max()), 5),
               max_rel_over_stat=round(float((rel / stat).max()), 2),
               linear_pol_max_abs=round(float(max(dlin)), 5) if dlin else None,
               circular_pol_max_abs=round(float(max(dcirc)), 5) if dcirc else None)
    return out


# ----------------------------------------------------------------------------- oracle leg
def oracle_leg(q, args, w, t32, cfg):
    """The benchmark's only contact with the oracle (test infrastructure): the oracle's own
    throughput on the host cores, and two figures measured against it -- the decision mismatch
    rate of the single-precision path at the peak of the pulse, and the table method error."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import oracle_run
    res = {}
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    nthreads = max(1, min(16, cores))
    host = dict(nproc=os.cpu_count(), affinity_cores=cores, cpu_model=_cpu_model())
    T = oracle.OracleTables(nthreads=nthreads)
    # all threads: the first n electrons of the collision, all 3000 steps
    wsub = synth.subsample(synth.c2(), np.arange(args.cpu_sample))
    t0 = time.perf_counter()
    r = oracle_run(T, wsub, COLLISION_STEPS, oracle.F_ALL, cap_e=wsub.n * 2 + 1000, cap_p=wsub.n + 1000,
                   cap_g=wsub.n * 80 + 10_000, nthreads=nthreads)
    dt = time.perf_counter() - t0
    c = r["ctr"]
    res["cpu_baseline"] = dict(
        value=round(work_of(c) / dt, 1), unit="particle-QED-steps/s", cores=nthreads, kind="oracle",
        sample=f"first {wsub.n} electrons of the same collision, all {COLLISION_STEPS} time steps, FP64 with the "
               f"tables, both channels ({c['n_lepton_steps']} lepton-steps + {c['n_photon_steps']} photon-steps "
               f"in {dt:.1f} s on {nthreads} OpenMP threads)", host=host)
    log(f"cpu baseline ({nthreads} threads): {res['cpu_baseline']['value']:.4g}/s")
    # one core
    w1 = synth.subsample(synth.c2(), np.arange(args.cpu_sample_1core))
    t0 = time.perf_counter()
    r1 = oracle_run(T, w1, COLLISION_STEPS, oracle.F_ALL, cap_e=w1.n * 2 + 1000, cap_p=w1.n + 1000,
                    cap_g=w1.n * 80 + 10_000, nthreads=1)
    dt1 = time.perf_counter() - t0
    res["cpu_baseline"]["one_core"] = dict(value=round(work_of(r1["ctr"]) / dt1, 1), electrons=w1.n,
                                           seconds=round(dt1, 2))
    log(f"cpu baseline (1 thread): {res['cpu_baseline']['one_core']['value']:.4g}/s")
    # decision mismatch of the single-precision path against the oracle at the peak of the pulse
    try:
        res["decision_mismatch"] = decision_mismatch(q, w, t32, cfg, T, nthreads)
        log(f"decision mismatch: {res['decision_mismatch']}")
    except Exception as e:               # reported, never fatal
        res["decision_mismatch"] = {"error": f"{type(e).__name__}: {e}"}
        traceback.print_exc()
    res["table_method_error"] = table_method_error()
    return res


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def decision_mismatch(q, w, t32, cfg, T, nthreads, k0=850):
    """FP32 run of the whole collision to time step k0 (the peak of the pulse), then one more step
    of every particle on the GPU and in the oracle from the same FP32 state (24-bit uniforms, photon
    retirement at birth off so every emission carries its parent's index).  Decision mismatches:
    leptons whose emit / no-emit decision differs, photons whose pair / no-pair decision differs;
    each is checked against the oracle's near-tie flag (draw within 1e-5 of the threshold)."""
    import torch
    from parity import decision_flips
    col = Collision(q, t32, w, cfg, steps=k0)
    col.run(1)
    torch.cuda.synchronize()
    st = col.sim.snapshot(device=False)
    col.close()
    res = decision_flips(q, t32, w, st, k0, T, nthreads)
    return res


def table_method_error():
    """The table grid's interpolation error against the exact inverse CDF and rates, as written by
    tests/golden/make_table_method_error.py (oracle only) for this grid."""
    path = os.path.join(ROOT, "tests", "golden", "table_method_error.json")
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError) as e:
        return {"error": f"{path}: {e}"}


# ----------------------------------------------------------------------------- extras
SURROGATE_JUDGE_BOUND = 0.01      # |dnu| above which a coarse cell falls back to the table inverse CDF


def extra_surrogate(q, args, w, t32, t64, cfg, out, v64):
    import torch
    t0 = time.perf_counter()
    sn, sb = q.Surrogate(t32, 0, seed=1), q.Surrogate(t32, 1, seed=2)
    ln, lb = sn.fit(), sb.fit()
    judged = [s.judge(SURROGATE_JUDGE_BOUND)[1] for s in (sn, sb)]
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    col = Collision(q, t32, w, cfg, surrogates=(sn, sb))
    wall, c = col.timed(args.extra_reps, 1)
    col.close()
    vs = work_of(c) / wall
    log(f"fp32 + learned inverse CDF: {vs:.4g}/s (training {t_train:.2f} s)")
    info = [s.info() for s in (sn, sb)]
    sp = t32.grid
    fine = [2 * sp["n_chi"][g] * sp["n_rho"] * 8 for g in (0, 1)]
    sur = {"value": round(vs, 1), "unit": "particle-QED-steps/s", "train_s": round(t_train, 3),
           "final_mse_y": [round(float(ln[-1]), 8), round(float(lb[-1]), 8)],
           "residual_scale": [round(i.out_s, 6) for i in info],
           "judge": {"bound_dnu": SURROGATE_JUDGE_BOUND, "points_per_cell": 64, "cells": [i.n_cells for i in info],
                     "marked": judged},
           "bytes": {"network_bf16": [i.bytes_network for i in info], "coarse_table_fp32": [i.bytes_base for i in info],
                     "mask": [i.bytes_mask for i in info], "fine_tables_fp64": fine}}
    if v64:
        sur["speedup_vs_fp64"] = round(vs / v64, 3)
    wsub = synth.subsample(w, np.arange(min(w.n, 100_000)))
    steps_e = 2000
    ref = spectra(q, t64, wsub, steps_e)
    out["fp32_error_vs_fp64"] = spectrum_error(ref, spectra(q, t32, wsub, steps_e))
    sur["error_vs_fp64"] = spectrum_error(ref, spectra(q, t32, wsub, steps_e, surrogates=(sn, sb)))
    out["error_workload"] = f"first {wsub.n} electrons of the same collision, {steps_e} steps, every photon kept"
    out["surrogate"] = sur
    log(f"error vs fp64: fp32 {out['fp32_error_vs_fp64']}; learned {sur['error_vs_fp64']}")
    del sn, sb
    torch.cuda.empty_cache()
    return ref, wsub, steps_e


def extra_flag_variant(q, args, w, t32, cfg, out, v64, key, flags, ref):
    col = Collision(q, t32, w, cfg, flags=flags)
    wall, c = col.timed(args.extra_reps, 1)
    col.close()
    v = work_of(c) / wall
    res = {"value": round(v, 1), "unit": "particle-QED-steps/s", "photons_emitted": c["n_emit"]}
    if v64:
        res["speedup_vs_fp64"] = round(v / v64, 3)
    if ref is not None:
        r, wsub, steps_e = ref
        got = spectra(q, t32, wsub, steps_e, flags=flags)
        res["error_vs_fp64"] = spectrum_error(r, got)
        res["mean_spin"] = [round(float(x), 6) for x in got["s_mean"]]
    out[key] = res
    log(f"{key}: {v:.4g}/s")


# Store sizes of an ensemble member, in slots per electron, from its initial chi0 = 2 gamma0 a0
# eps_r.  Members past chi0 ~ 6.5 cascade (pairs emit and make pairs) and emit some hundreds of
# photons per electron over the run; members with a0 near 200 need about 16 photon slots per
# electron between compactions even without.  Measured on the recipe at 5 % of its counts: no
# member overflows with these.  "compact50" is for compaction every 50 steps; "compact10" needs
# less room (fewer dead slots wait for the compaction), so the ensembles at full counts fit in
# FP64 (about 200 GB).
ENSEMBLE_SLOTS = {"compact50": ((6.5, 200, 4.0), (5.0, 60, 4.0), (0.0, 30, 1.5)),
                  "compact10": ((6.5, 100, 4.0), (5.0, 30, 4.0), (0.0, 20, 1.5))}


def ensemble_caps(x, rule):
    g0 = float(np.mean(np.sqrt(1.0 + (x.p ** 2).sum(0))))
    chi0 = 2.0 * g0 * x.a0 * synth.EPS_R
    pg, pp = next((g, p) for c, g, p in ENSEMBLE_SLOTS[rule] if chi0 >= c)
    return dict(cap_e=x.n + max(1000, int(pp * x.n)), cap_p=max(1000, int(pp * x.n)), cap_g=max(100_000, pg * x.n))


def extra_batched(q, args, t32, t64, out, scale=None, key="batched", every=COMPACT_EVERY):
    """The 64 batched ensembles (at `scale` of the recipe's particle counts) through one plan, FP32
    and FP64, each with its tuned launch shape; stores sized by ensemble_caps."""
    import torch
    from paper_2511_08929_amd import autotune
    from paper_2511_08929_amd.sim import Batch
    scale = args.batched_scale if scale is None else scale
    ws = synth.c5(scale=scale)
    steps_b = 2000

    def make(tab):
        rule = "compact10" if every <= 10 else "compact50"
        specs = [dict(**ensemble_caps(x, rule), track=x.track,
                      fields=dict(kind=x.field_kind, a0=x.a0, phase_len=x.phase_len), dt=x.dt,
                      eps_r=synth.EPS_R, seed=x.seed, flags=q.QED_ALL, k_retire=x.k_retire) for x in ws]
        b = Batch(tab, specs)
        for x, inst in zip(ws, b.inst):
            inst["e"].load(x.x, x.p, x.s)
        return b

    res = {}
    for label, tab in (("fp32", t32), ("fp64", t64)):
        b = make(tab)
        best, timings, cached = b.tune(300, every=every, log=log,
                                       space={k: v for k, v in autotune.SPACE.items() if k != "max_blocks_per_set"})
        g = b.capture(every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps_b // every):
            b.replay(g)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tot = {}
        for inst in b.inst:
            for k, v in q.counters_dict(inst["ctr"]).items():
                tot[k] = tot.get(k, 0) + v
        res[label] = {"value": round(work_of(tot) / wall, 1), "wall_s": round(wall, 3), "config": best,
                      "tuning_s_per_300_steps": timings, "capacity_overflow": tot["n_capacity_overflow"]}
        del g, b
        torch.cuda.empty_cache()
        log(f"batched {label}: {res[label]['value']:.4g}/s config {best}")
    out[key] = {"instances": len(ws), "electrons": int(sum(x.n for x in ws)), "steps": steps_b,
                      "unit": "particle-QED-steps/s",
                      "slots_per_electron": {"rule": "compact10" if every <= 10 else "compact50",
                                             "by_chi0": ENSEMBLE_SLOTS["compact10" if every <= 10 else "compact50"]},
                      "compact_every": every,
                      "recipe": f"64 head-on collisions, N ~ LogUniform[1e4, 1e7] x {scale}, "
                                "a0 ~ U[20, 200], gamma0 ~ U[500, 1e4], spin degree ~ U[0, 1]",
                      "value": res["fp32"]["value"], "fp64_value": res["fp64"]["value"],
                      "speedup_vs_fp64": round(res["fp32"]["value"] / res["fp64"]["value"], 3), **res}


def extra_cascade(q, args, t32, t64, cfg, out):
    wc = synth.c6(n=20_000, steps=3200)
    caps = (2_000_000, 2_000_000, 30_000_000)
    rc = {}
    for label, tab in (("fp32", t32), ("fp64", t64)):
        col = Collision(q, tab, wc, cfg, caps=caps, steps=wc.steps,
                        fields=q.make_fields(wc.field_kind, a0=wc.a0, phase_len=wc.phase_len))
        wall, c = col.timed(1, 0)
        rc[label] = dict(value=round(work_of(c) / wall, 1), wall_s=round(wall, 4), electrons=col.sim.e.n(),
                         positrons=col.sim.p.n(), photons=col.sim.g.n(), capacity_overflow=c["n_capacity_overflow"])
        col.close()
        log(f"cascade {label}: {rc[label]['value']:.4g}/s")
    out["cascade"] = dict(workload="seeded pair cascade, rotating E field a0 = 1000, 20000 electrons from rest, "
                                   "omega t = 16 (3200 steps of 0.005)", unit="particle-QED-steps/s",
                          speedup_fp32_vs_fp64=round(rc["fp32"]["value"] / rc["fp64"]["value"], 3), **rc)


def extra_grid(q, args, t32, cfg, out, n=1 << 24, steps=200):
    import torch
    wg = synth.c3(n=n, steps=steps)
    fg = q.make_fields(q.QED_FIELD_GRID2D, grid=torch.as_tensor(wg.extra["grid"], device="cuda"), dx=wg.extra["dx"],
                       dy=wg.extra["dy"])
    # pairs reach about 0.28 per electron in 200 steps: room for half an electron's worth
    col = Collision(q, t32, wg, cfg, fields=fg, steps=steps, caps=(n + n // 2, n // 2, 24 * n))
    wall, c = col.timed(1, 0)
    col.close()
    v = work_of(c) / wall
    log(f"grid workload: {v:.4g}/s, counters {c}")
    out["grid"] = {"workload": f"grid-interpolated fields (4096 x 1024 cells, a0 = 200 standing CP waves, 1 % noise), "
                               f"{n} electrons (16 per cell at 2^26), gamma ~ LogUniform(10, 1e4), {steps} steps, FP32",
                   "value": round(v, 1), "unit": "particle-QED-steps/s", "wall_s": round(wall, 4),
                   "photons_emitted": c["n_emit"], "pairs": c["n_pair"], "capacity_overflow": c["n_capacity_overflow"]}


def extra_subcycle(q, args, t64, out, n=100_000, steps=200, n_mixed=100_000):
    """Per-particle sub-cycling in the test-particle workload (W dt ~ 0.95 at the start) against the
    plain step at dt/16, and the throughput of both, per-species calls and merged step replayed
    from HIP graphs; then a mixed population (the head-on collision at a0 = 300, where few leptons
    need sub-steps), merged step with and without sub-cycling"""
    import torch
    from paper_2511_08929_amd.sim import Simulation
    w = synth.c1(n=n)
    base = q.QED_ALL & ~q.QED_PAIR
    g0 = w.extra["gamma0"]

    def run(dt, nsteps, flags, every, merged=False):
        sim = Simulation(t64, cap_e=n, cap_p=1, cap_g=24 * n, track=w.track,
                         fields=q.make_fields(w.field_kind, B0=w.B0), dt=dt, eps_r=synth.EPS_R, seed=w.seed,
                         flags=flags, k_retire=1e30, device_clock=True, merged=merged)
        sim.e.load(w.x, w.p, w.s)
        g = sim.capture(every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps // every):
            sim.replay(g)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        _, p, s = sim.e.arrays()
        gam = np.sqrt(1 + np.sum(p * p, axis=0))
        c = q.counters_dict(sim.ctr)
        del sim, g
        torch.cuda.empty_cache()
        return dict(loss=float(g0 - gam.mean()), s_beta=float(-s[2].mean()), wall=wall, emitted=c["n_emit"],
                    rate=n * nsteps / wall)

    ref = run(w.dt / 16, 16 * steps, base, 160, merged=True)
    plain = run(w.dt, steps, base, 10, merged=True)
    sub_ps = run(w.dt, steps, base | q.QED_SUBCYCLE, 10)
    sub = run(w.dt, steps, base | q.QED_SUBCYCLE, 10, merged=True)
    res = {"workload": f"test particle in a uniform B (chi = 1, gamma0 = 2000), {n} electrons, {steps} steps of "
                       "1/100 gyro period (W dt ~ 0.95), FP64",
           "unit": "lepton-steps/s", "value": round(sub["rate"], 1), "per_species_value": round(sub_ps["rate"], 1),
           "plain_value": round(plain["rate"], 1),
           "merged_equals_per_species": sub["loss"] == sub_ps["loss"] and sub["s_beta"] == sub_ps["s_beta"]}
    for key, r in (("reference_dt_over_16", ref), ("plain", plain), ("subcycled", sub)):
        res[key] = {"mean_energy_loss": round(r["loss"], 3), "mean_s_beta": round(r["s_beta"], 5),
                    "photons": r["emitted"]}
    for key, r in (("plain", plain), ("subcycled", sub)):
        res[key]["energy_loss_rel_error"] = round(abs(r["loss"] / ref["loss"] - 1), 5)
        res[key]["s_beta_abs_error"] = round(abs(r["s_beta"] - ref["s_beta"]), 5)
    # mixed population: merged step, sub-cycled against plain, whole collisions from HIP graphs
    wm = synth.subsample(synth.c2(a0=300.0), np.arange(n_mixed))
    mixed = {}
    for key, flags in (("plain", q.QED_ALL), ("subcycled", q.QED_ALL | q.QED_SUBCYCLE)):
        col = Collision(q, t64, wm, {}, flags=flags)
        wall, c = col.timed(1, 0)
        col.close()
        mixed[key] = {"value": round(work_of(c) / wall, 1), "emitted": c["n_emit"], "pairs": c["n_pair"]}
    mixed["slowdown"] = round(mixed["plain"]["value"] / mixed["subcycled"]["value"], 3)
    res["mixed"] = {"workload": f"head-on collision at a0 = 300, {n_mixed} electrons, {COLLISION_STEPS} steps, FP64, "
                                "merged step", "unit": "particle-QED-steps/s", **mixed}
    out["subcycle"] = res
    log(f"sub-cycling: {res}")


def extra_full_scale(q, args, t32, t64, cfg, out):
    """The two workloads at their stated sizes (opt-in, several minutes): the head-on collision at
    10^8 electrons (24 photon slots per electron, every photon kept) through the FP32 tables, the
    learned inverse CDF and the FP64 tables, in the launch shape tuned on 10^6 electrons; and the 64
    batched ensembles at full particle counts, FP32 and FP64."""
    import torch
    wb = synth.c2(n=args.full_n)
    log(f"full scale: head-on collision, {wb.n} electrons, {COLLISION_STEPS} steps")
    sn, sb = q.Surrogate(t32, 0, seed=1), q.Surrogate(t32, 1, seed=2)
    sn.fit(), sb.fit()
    for s_ in (sn, sb):
        s_.judge(SURROGATE_JUDGE_BOUND)
    res = {}
    for label, tab, sur in (("fp32", t32, (None, None)), ("surrogate", t32, (sn, sb)), ("fp64", t64, (None, None))):
        col = Collision(q, tab, wb, cfg, surrogates=sur, photons_per_electron=24)
        wall, c = col.timed(1, 0)
        col.close()
        res[label] = {"value": round(work_of(c) / wall, 1), "wall_s": round(wall, 3), "photons_emitted": c["n_emit"],
                      "pairs": c["n_pair"], "capacity_overflow": c["n_capacity_overflow"]}
        log(f"full scale {label}: {wall:.2f} s, {res[label]['value']:.4g}/s, counters {c}")
        torch.cuda.empty_cache()
    for label in ("fp32", "surrogate"):
        res[label]["speedup_vs_fp64"] = round(res[label]["value"] / res["fp64"]["value"], 3)
    out["full_scale_head_on"] = dict(electrons=wb.n, steps=COLLISION_STEPS, photon_slots_per_electron=24,
                                     config=cfg, **res)
    del sn, sb, wb
    torch.cuda.empty_cache()
    extra_batched(q, args, t32, t64, out, scale=1.0, key="full_scale_batched", every=args.full_compact_every)


def run_extra(out, name, budget_s, fn, *a):
    """run one extra unless the time budget is spent; a failure is recorded, never fatal"""
    el = time.perf_counter() - T_START
    if el > budget_s:
        out.setdefault("skipped", []).append(f"{name}: time budget ({el:.0f} s of {budget_s:.0f} s used)")
        log(f"skip {name}: budget")
        return None
    try:
        return fn(*a)
    except Exception as e:
        out.setdefault("errors", {})[name] = f"{type(e).__name__}: {e}"
        traceback.print_exc()
        try:
            import torch
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        except Exception:
            pass
        return None


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed benchmark steps, each a whole collision of 3000 time steps")
    ap.add_argument("--warmup", type=int, default=2, help="untimed whole collisions before the timed ones")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--budget-s", type=float, default=330.0,
                    help="extras that would start after this many seconds are skipped (reported)")
    ap.add_argument("--no-fp64", action="store_true", help="skip timing the FP64 path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=30000)
    ap.add_argument("--cpu-sample-1core", type=int, default=1500)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extra-reps", type=int, default=2, help="timed collisions of each extra variant")
    ap.add_argument("--batched-scale", type=float, default=0.05,
                    help="particle counts of the 64 batched ensembles relative to the full recipe")
    ap.add_argument("--ppb", type=int, default=0, help="fixed particles per block (0: autotuned)")
    ap.add_argument("--full-scale", action="store_true",
                    help="also run the head-on collision at 10^8 electrons (FP32 tables, learned inverse CDF, FP64) "
                         "and the 64 batched ensembles at full particle counts (several minutes)")
    ap.add_argument("--full-n", type=int, default=100_000_000, help="electrons of the --full-scale head-on run")
    ap.add_argument("--full-compact-every", type=int, default=10,
                    help="compaction interval of the --full-scale batched run (its stores are bounded by FP64 memory)")
    ap.add_argument("--probe", action="store_true",
                    help="profiler run: copy calibration + one eager FP32 collision, no JSON line")
    ap.add_argument("--probe-steps", type=int, default=COLLISION_STEPS)
    ap.add_argument("--probe-grid", action="store_true",
                    help="profiler run: the grid workload (2^24 electrons, 200 steps, FP32) once, eagerly, "
                         "no JSON line")
    return ap.parse_args(argv)


def probe(q, w, cfg, steps):
    """Counter-collection run: a plain elementwise kernel over 256 MiB in and 256 MiB out (the
    calibration of FETCH_SIZE / WRITE_SIZE), then the single-precision path eagerly."""
    import torch
    from paper_2511_08929_amd.sim import Simulation
    a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b
    cap_p = max(1000, w.n // 5)
    sim = Simulation(q.Tables(precision=q.QED_F32), cap_e=w.n + cap_p, cap_p=cap_p, cap_g=30 * w.n, track=w.track,
                     fields=q.make_fields(w.field_kind, a0=w.a0, phase_len=w.phase_len), dt=w.dt, eps_r=synth.EPS_R,
                     seed=w.seed, flags=q.QED_ALL, k_retire=w.k_retire, device_clock=True, merged=True,
                     particles_per_block=cfg["particles_per_block"], process_group=cfg["process_group"],
                     max_blocks_per_set=cfg["max_blocks_per_set"], photon_variant=cfg.get("photon_variant", 0))
    sim.e.load(w.x, w.p, w.s)
    t0 = time.perf_counter()
    for k in range(steps):
        sim.step()
        if (k + 1) % COMPACT_EVERY == 0:
            sim.compact()
    torch.cuda.synchronize()
    log(f"probe: {steps} steps in {time.perf_counter() - t0:.2f} s, counters {q.counters_dict(sim.ctr)}")


def probe_grid(q, n=1 << 24, steps=200):
    """Profiler run of the grid workload as the `grid` extra sizes it, stepped eagerly."""
    import torch
    from paper_2511_08929_amd import autotune
    wg = synth.c3(n=n, steps=steps)
    fg = q.make_fields(q.QED_FIELD_GRID2D, grid=torch.as_tensor(wg.extra["grid"], device="cuda"), dx=wg.extra["dx"],
                       dy=wg.extra["dy"])
    col = Collision(q, q.Tables(precision=q.QED_F32), wg, autotune.DEFAULT, fields=fg, steps=steps,
                    caps=(n + n // 2, n // 2, 24 * n))
    sim = col.sim
    t0 = time.perf_counter()
    for k in range(steps):
        sim.step()
        if (k + 1) % COMPACT_EVERY == 0:
            sim.compact()
    torch.cuda.synchronize()
    log(f"grid probe: {steps} steps in {time.perf_counter() - t0:.2f} s, counters {q.counters_dict(sim.ctr)}")
    col.close()


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; multi-GPU runs are out of scope (the path shards by "
              "particle index with no per-step exchange).", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2511_08929_amd as q
    from paper_2511_08929_amd import autotune
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    w = synth.c2(n=args.n)
    log(f"workload {w.name}: n={w.n}, {COLLISION_STEPS} time steps per collision; timed collisions {args.steps}, "
        f"warmup {args.warmup}")
    if args.probe:
        probe(q, w, dict(autotune.DEFAULT, **({"particles_per_block": args.ppb} if args.ppb else {})),
              args.probe_steps)
        return
    if args.probe_grid:
        probe_grid(q)
        return

    t32, t64 = q.Tables(precision=q.QED_F32), q.Tables(precision=q.QED_F64)
    col = Collision(q, t32, w, autotune.DEFAULT)
    # launch shape of the merged step, chosen by timing whole collisions of this workload
    if args.ppb:
        cfg, tune_t, cached = dict(autotune.DEFAULT, particles_per_block=args.ppb), {}, False
        col.set_config(cfg)
    else:
        cfg, tune_t, cached = col.sim.tune(COLLISION_STEPS, every=COMPACT_EVERY, log=log,
                                           workload_key=f"head_on_collision|n={w.n}|fp32")
        col.graph = None
    log(f"launch config {cfg}")
    wall, c = col.timed(args.steps, args.warmup)
    per = {k: v // args.steps for k, v in c.items()}
    value = work_of(c) / wall
    log(f"fp32: {args.steps} collisions in {wall:.3f} s, {value:.4g}/s, counters per collision {per}")
    col.close()

    kt, ck, kwall = profiled_collision(q, t32, w, cfg)
    if work_of(ck) != work_of(per):
        log(f"warning: profiled collision work {work_of(ck)} != timed {work_of(per)}")
    cg = copy_gbs()
    roof = roofline(kt, ck, cg)
    log(f"roofline {roof}")

    out = {"metric": METRIC, "value": round(value, 1), "unit": "particle-QED-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded head-on collision inputs)",
           "config": {"workload": "head_on_collision_lp_plane_wave", "electrons": w.n, "gamma0": "N(4000, 5%)",
                      "a0": w.a0, "pulse": "sin^2, 30 fs intensity FWHM", "dt": "lambda/(100 c)",
                      "time_steps": COLLISION_STEPS, "bench_step": "one whole collision (3000 time steps)",
                      "precision": "FP32 bulk + FP64 islands", "channels": "NLC + NBW, spin and polarization resolved"},
           "ms_per_time_step": round(1e3 * wall / (args.steps * COLLISION_STEPS), 5),
           "hip_graph": True, "roofline": roof,
           "tuning": {"config": cfg, "cached": cached, "seconds_per_collision": tune_t},
           "work_per_collision": {"lepton_steps": per["n_lepton_steps"], "photon_steps": per["n_photon_steps"],
                                  "photons_emitted": per["n_emit"], "pairs": per["n_pair"],
                                  "capacity_overflow": per["n_capacity_overflow"]}}

    v64 = None
    if not args.no_fp64:
        try:
            c64 = Collision(q, t64, w, cfg)
            wall64, cc = c64.timed(max(1, args.steps // 4), 1)
            c64.close()
            v64 = work_of(cc) / wall64
            out["fp64_value"] = round(v64, 1)
            out["speedup_fp32_vs_fp64"] = round(value / v64, 3)
            log(f"fp64: {v64:.4g}/s")
        except Exception as e:
            out.setdefault("errors", {})["fp64"] = f"{type(e).__name__}: {e}"
            traceback.print_exc()

    if not args.no_cpu_baseline:
        try:
            out.update(oracle_leg(q, args, w, t32, cfg))
        except Exception as e:
            out.setdefault("errors", {})["cpu_baseline"] = f"{type(e).__name__}: {e}"
            traceback.print_exc()

    if not args.no_extras:
        ref = run_extra(out, "surrogate", args.budget_s, extra_surrogate, q, args, w, t32, t64, cfg, out, v64)
        run_extra(out, "rejection", args.budget_s, extra_flag_variant, q, args, w, t32, cfg, out, v64, "rejection",
                  q.QED_ALL | q.QED_REJECTION, ref)
        run_extra(out, "g_chi", args.budget_s, extra_flag_variant, q, args, w, t32, cfg, out, v64, "g_chi",
                  q.QED_ALL | q.QED_G_CHI, ref)
        run_extra(out, "batched", args.budget_s, extra_batched, q, args, t32, t64, out)
        run_extra(out, "cascade", args.budget_s, extra_cascade, q, args, t32, t64, cfg, out)
        run_extra(out, "grid", args.budget_s, extra_grid, q, args, t32, cfg, out)
        run_extra(out, "subcycle", args.budget_s, extra_subcycle, q, args, t64, out)
    if args.full_scale:
        run_extra(out, "full_scale", float("inf"), extra_full_scale, q, args, t32, t64, cfg, out)
    out["bench_wall_s"] = round(time.perf_counter() - T_START, 1)
    print(json.dumps(out), flush=True)


import synth  # noqa: E402  (seeded workload recipes; holds no QED arithmetic)

if __name__ == "__main__":
    main()
