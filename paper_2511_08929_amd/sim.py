"""Time-step drivers over the C ABI.

``Simulation``: one instance; a step is qed_emit (push + NLC) for the electrons, then for the
positrons, then qed_pair (NBW) for the photons born in earlier steps; qed_compact on demand.
With ``merged=True`` the same step runs as one qed_plan_step (two launches for all three sets).
``Batch``: many independent instances stepped together by one plan.

All counts stay on the device; a step enqueues without host synchronization.  With a device
clock (``device_clock=True``, always on for plans) the step index and time come from a device
counter that the step itself advances, so the same sequence of launches is valid at every step
and can be captured once in a HIP graph and replayed (``capture`` / ``replay``).
"""
from __future__ import annotations

import math

from . import (ALPHA, QED_F32, QED_F64, QED_PAIR, LeptonBuffers, PhotonBuffers, Plan, Tables, make_fields, make_step,
               new_counters, new_workspace, qed_clock_advance, qed_compact, qed_compact_workspace_size, qed_emit,
               qed_pair, qed_workspace_size)


class Simulation:
    def __init__(self, tables: Tables, *, cap_e, cap_p, cap_g, track, fields, dt, eps_r, seed, flags,
                 k_retire=0.0, t0=0.0, a_e=ALPHA / (2 * math.pi), chi_e_min=1e-3, chi_e_max=1e2, chi_g_min=0.05,
                 chi_g_max=1e2, device="cuda", device_clock=False, merged=False, particles_per_block=0,
                 max_blocks_per_set=0, process_group=0, optical_depth=False, surrogates=(None, None),
                 photon_variant=0):
        import torch
        self.tables = tables
        self.dtype = torch.float64 if tables.precision == QED_F64 else torch.float32
        self.e = LeptonBuffers(0, cap_e, self.dtype, device, track, tau=optical_depth)
        self.p = LeptonBuffers(1, cap_p, self.dtype, device, track, tau=optical_depth)
        self.g = PhotonBuffers(cap_g, self.dtype, device, track)
        self.ctr = new_counters(device)
        nbytes = max(qed_workspace_size(max(cap_e, cap_p, cap_g)),
                     qed_compact_workspace_size(self.g, tables.precision))
        self.ws = new_workspace(nbytes, device)
        self.fields = fields if not isinstance(fields, dict) else make_fields(**fields)
        self.dt, self.eps_r, self.seed, self.flags = dt, eps_r, seed, flags
        self.k_retire, self.t0, self.a_e = k_retire, t0, a_e
        self.chi = (chi_e_min, chi_e_max, chi_g_min, chi_g_max)
        self.n = 0
        self._sp = None
        merged = merged or any(x is not None for x in surrogates)     # the learned inverse CDF runs in plans
        self.clock = torch.zeros(1, dtype=torch.int64, device=device) if (device_clock or merged) else None
        self.merged, self.ppb, self.maxb, self.group = merged, particles_per_block, max_blocks_per_set, process_group
        self.pvar = photon_variant
        self.surrogates = surrogates
        self.plan = None

    def step_params(self, n):
        return make_step(self.dt, self.eps_r, step=n, t=self.t0 + n * self.dt, seed=self.seed, flags=self.flags,
                         a_e=self.a_e, chi_e_min=self.chi[0], chi_e_max=self.chi[1], chi_g_min=self.chi[2],
                         chi_g_max=self.chi[3], k_retire=self.k_retire)

    def _params(self):
        sp = self._sp
        if sp is None:
            sp = self._sp = self.step_params(0)
        if self.clock is not None:
            # step = 0 + *clock, t = t0 + *clock dt on the device
            sp.step, sp.t, sp.d_clock = 0, self.t0, self.clock.data_ptr()
        else:
            sp.step, sp.t, sp.d_clock = self.n, self.t0 + self.n * self.dt, None
        sp.flags = self.flags
        return sp

    def _ensure_plan(self):
        if self.merged and self.plan is None:
            self.plan = Plan(self.tables, [(self.e, self.p, self.g, self.fields, self._params(), self.ctr)],
                             particles_per_block=self.ppb, max_blocks_per_set=self.maxb,
                             surrogates=self.surrogates, process_group=self.group, photon_variant=self.pvar)

    def set_launch_config(self, particles_per_block=0, process_group=0, max_blocks_per_set=0, photon_variant=0):
        """Launch shape of the merged step (0: the library's default).  The plan is rebuilt at the
        next step, so graphs captured before this call must not be replayed after it."""
        import torch
        if self.plan is not None:
            torch.cuda.synchronize()
            self.plan.close()
            self.plan = None
        self.ppb, self.group, self.maxb = particles_per_block, process_group, max_blocks_per_set
        self.pvar = photon_variant

    def _enqueue_step(self, stream=None):
        if self.merged:
            self._ensure_plan()
            self.plan.step(stream)
            return
        sp = self._params()
        qed_emit(self.tables, self.e, self.fields, sp, self.g, self.ctr, self.ws, stream)
        if self.flags & QED_PAIR:
            qed_emit(self.tables, self.p, self.fields, sp, self.g, self.ctr, self.ws, stream)
            qed_pair(self.tables, self.g, self.fields, sp, self.e, self.p, self.ctr, self.ws, stream)
        if self.clock is not None:
            qed_clock_advance(self.clock, stream)

    def step(self, stream=None):
        if self.clock is not None and self.n == 0:
            self.clock.fill_(0)
        self._enqueue_step(stream)
        self.n += 1

    def compact(self, stream=None):
        qed_compact(self.g, self.tables.precision, self.ws, stream)

    def capture(self, nsteps, compact_at_end=True):
        """Record `nsteps` steps (and a compaction) into a HIP graph; needs device_clock=True.
        The graph reads every count, the step and the time from device memory, so it can be
        replayed from any state."""
        import torch
        assert self.clock is not None, "graph capture needs the device clock"
        self._ensure_plan()
        torch.cuda.synchronize()
        self.clock.fill_(self.n)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        with torch.cuda.graph(graph, stream=side):
            for _ in range(nsteps):
                self._enqueue_step()
            if compact_at_end:
                self.compact()
        graph.steps = nsteps
        return graph

    def replay(self, graph):
        graph.replay()
        self.n += graph.steps

    # ---------------------------------------------------------------- state
    def snapshot(self, device=True):
        """The whole state: live slots of every set, counts, counters and the step index (device
        copies, or host numpy arrays with device=False).  Philox is counter-based, so a run
        restored from a snapshot continues bit for bit as the uninterrupted run."""
        return _snapshot(self.e, self.p, self.g, self.ctr, self.n, device)

    def restore(self, snap, counters=True):
        """Put a snapshot back (stream-ordered device copies; no host synchronization when the
        snapshot is device-resident).  counters=False keeps the accumulated counters."""
        _restore(snap, self.e, self.p, self.g, self.ctr if counters else None)
        self.n = snap["n"]
        if self.clock is not None:
            self.clock.fill_(self.n)

    def save(self, path):
        """Checkpoint to a .npz file (host copy of snapshot())."""
        _save(path, self.snapshot(device=False))

    def load_checkpoint(self, path):
        self.restore(_load(path))

    # ---------------------------------------------------------------- launch shape
    def workload_key(self, steps):
        f = self.fields
        return (f"sim|prec={self.tables.precision}|cap={self.e.capacity},{self.p.capacity},{self.g.capacity}|"
                f"n={self.e.n()},{self.p.n()},{self.g.n()}|flags={self.flags}|field={f.kind},{f.a0},{f.phase_len}|"
                f"dt={self.dt}|steps={steps}|sur={[s is not None for s in self.surrogates]}")

    def tune(self, steps, every=50, workload_key=None, space=None, cache_path=None, log=None):
        """Choose the merged step's launch shape (autotune.SPACE) by timing `steps` steps from the
        current state (graph replays of `every` steps and a compaction) for each candidate; the
        state is put back after every timing and at the end.  Returns (config, timings, cached)."""
        from . import autotune
        assert self.merged and steps % every == 0
        snap = self.snapshot()
        key = workload_key or self.workload_key(steps)
        space = dict(autotune.SPACE if space is None else space)
        if self.tables.precision != QED_F32:
            space.pop("photon_variant", None)      # the photon pass variants exist in single precision only

        def run(cfg):
            import time

            import torch
            self.set_launch_config(**cfg)
            self.restore(snap)
            g = self.capture(every)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps // every):
                self.replay(g)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            del g
            return wall

        best, timings, cached = autotune.tune(key, run, space, cache_path=cache_path, log=log)
        self.set_launch_config(**best)
        self.restore(snap)
        return best, timings, cached


class Batch:
    """Independent instances stepped by one plan.  ``specs`` is a list of dicts with keys
    cap_e, cap_p, cap_g, track, fields, dt, eps_r, seed, flags and optionally k_retire, t0, a_e."""

    def __init__(self, tables: Tables, specs, device="cuda", particles_per_block=0, max_blocks_per_set=0,
                 process_group=0, photon_variant=0):
        import torch
        self.tables = tables
        self.dtype = torch.float64 if tables.precision == QED_F64 else torch.float32
        self.inst = []
        for sp in specs:
            e = LeptonBuffers(0, sp["cap_e"], self.dtype, device, sp["track"])
            p = LeptonBuffers(1, sp["cap_p"], self.dtype, device, sp["track"])
            g = PhotonBuffers(sp["cap_g"], self.dtype, device, sp["track"])
            clock = torch.zeros(1, dtype=torch.int64, device=device)
            ctr = new_counters(device)
            f = sp["fields"] if not isinstance(sp["fields"], dict) else make_fields(**sp["fields"])
            step = make_step(sp["dt"], sp["eps_r"], step=0, t=sp.get("t0", 0.0), seed=sp["seed"], flags=sp["flags"],
                             a_e=sp.get("a_e", ALPHA / (2 * math.pi)), k_retire=sp.get("k_retire", 0.0))
            step.d_clock = clock.data_ptr()
            self.inst.append(dict(e=e, p=p, g=g, clock=clock, ctr=ctr, fields=f, step=step))
        self.ws = new_workspace(max(qed_compact_workspace_size(i["g"], tables.precision) for i in self.inst), device)
        self.ppb, self.maxb, self.group = particles_per_block, max_blocks_per_set, process_group
        self.pvar = photon_variant
        self.plan = None
        self.n = 0

    def _ensure_plan(self):
        if self.plan is None:
            self.plan = Plan(self.tables, [(i["e"], i["p"], i["g"], i["fields"], i["step"], i["ctr"]) for i in self.inst],
                             particles_per_block=self.ppb, max_blocks_per_set=self.maxb, process_group=self.group,
                             photon_variant=self.pvar)

    def set_launch_config(self, particles_per_block=0, process_group=0, max_blocks_per_set=0, photon_variant=0):
        """As Simulation.set_launch_config: the plan is rebuilt at the next step."""
        import torch
        if self.plan is not None:
            torch.cuda.synchronize()
            self.plan.close()
            self.plan = None
        self.ppb, self.group, self.maxb = particles_per_block, process_group, max_blocks_per_set
        self.pvar = photon_variant

    def snapshot(self, device=True):
        return [_snapshot(i["e"], i["p"], i["g"], i["ctr"], self.n, device) for i in self.inst]

    def restore(self, snaps, counters=True):
        for i, sn in zip(self.inst, snaps):
            _restore(sn, i["e"], i["p"], i["g"], i["ctr"] if counters else None)
            i["clock"].fill_(sn["n"])
        self.n = snaps[0]["n"]

    def workload_key(self, steps):
        sizes = ";".join(f'{i["e"].capacity},{i["p"].capacity},{i["g"].capacity},{i["step"].flags},'
                         f'{i["fields"].kind},{i["fields"].a0:.6g}' for i in self.inst)
        return f"batch|prec={self.tables.precision}|n={len(self.inst)}|{hashlib_hex(sizes)}|steps={steps}"

    def tune(self, steps, every=50, workload_key=None, space=None, cache_path=None, log=None):
        """As Simulation.tune, for all instances at once."""
        from . import autotune
        assert steps % every == 0
        snap = self.snapshot()
        key = workload_key or self.workload_key(steps)
        space = dict(autotune.SPACE if space is None else space)
        if self.tables.precision != QED_F32:
            space.pop("photon_variant", None)      # the photon pass variants exist in single precision only

        def run(cfg):
            import time

            import torch
            self.set_launch_config(**cfg)
            self.restore(snap)
            g = self.capture(every)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps // every):
                self.replay(g)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            del g
            return wall

        best, timings, cached = autotune.tune(key, run, space, cache_path=cache_path, log=log)
        self.set_launch_config(**best)
        self.restore(snap)
        return best, timings, cached

    def step(self, stream=None):
        self._ensure_plan()
        self.plan.step(stream)
        self.n += 1

    def compact(self, stream=None):
        for i in self.inst:
            qed_compact(i["g"], self.tables.precision, self.ws, stream)

    def capture(self, nsteps, compact_at_end=True):
        import torch
        self._ensure_plan()
        torch.cuda.synchronize()
        for i in self.inst:
            i["clock"].fill_(self.n)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        with torch.cuda.graph(graph, stream=side):
            for _ in range(nsteps):
                self.plan.step()
            if compact_at_end:
                self.compact()
        graph.steps = nsteps
        return graph

    def replay(self, graph):
        graph.replay()
        self.n += graph.steps


def hashlib_hex(text):
    import hashlib
    return hashlib.sha256(text.encode()).hexdigest()[:16]


# -------------------------------------------------------------------- snapshots
def _snapshot(e, p, g, ctr, n, device):
    import torch
    torch.cuda.synchronize()

    def cut(arrs, m):
        out = []
        for a in arrs:
            if a is None:
                out.append(None)
            else:
                v = a[:m].clone()
                out.append(v if device else v.cpu().numpy())
        return out

    snap = {"n": n, "ctr": ctr.clone() if device else ctr.cpu().numpy()}
    for name, L in (("e", e), ("p", p)):
        m = L.n()
        snap[name] = dict(count=m, x=cut(L.x, m), p=cut(L.p, m), s=cut(L.s, m),
                          tau=cut([L.tau, L.tau_target], m))
    m = g.n()
    snap["g"] = dict(count=m, count_prev=int(g.count_prev.item()), x=cut(g.x, m), k=cut(g.k, m), P=cut(g.P, m),
                     id=cut([g.id], m)[0])
    return snap


def _restore(snap, e, p, g, ctr):
    import torch

    def put(dst, src):
        for d, s in zip(dst, src):
            if d is not None and s is not None:
                d[:s.shape[0]].copy_(torch.as_tensor(s, device=d.device), non_blocking=True)

    for name, L in (("e", e), ("p", p)):
        st = snap[name]
        put(L.x, st["x"]); put(L.p, st["p"]); put(L.s, st["s"]); put([L.tau, L.tau_target], st["tau"])
        L.count.fill_(st["count"])
    st = snap["g"]
    put(g.x, st["x"]); put(g.k, st["k"]); put(g.P, st["P"]); put([g.id], [st["id"]])
    g.count.fill_(st["count"])
    g.count_prev.fill_(st["count_prev"])
    if ctr is not None:
        ctr.copy_(torch.as_tensor(snap["ctr"], device=ctr.device))


def _save(path, snap):
    import numpy as np
    flat = {"n": np.int64(snap["n"]), "ctr": snap["ctr"]}
    for name in ("e", "p", "g"):
        for key, val in snap[name].items():
            if isinstance(val, list):
                for j, a in enumerate(val):
                    if a is not None:
                        flat[f"{name}.{key}.{j}"] = a
            elif val is not None and not isinstance(val, int):
                flat[f"{name}.{key}"] = val
            else:
                flat[f"{name}.{key}"] = np.int64(val)
    np.savez(path, **flat)


def _load(path):
    import numpy as np
    z = np.load(path, allow_pickle=False)
    snap = {"n": int(z["n"]), "ctr": z["ctr"]}
    lists = {"e": ("x", "p", "s", "tau"), "p": ("x", "p", "s", "tau"), "g": ("x", "k", "P")}
    for name, keys in lists.items():
        st = {"count": int(z[f"{name}.count"])}
        for key in keys:
            width = 2 if key == "tau" else 3
            st[key] = [z[f"{name}.{key}.{j}"] if f"{name}.{key}.{j}" in z.files else None for j in range(width)]
        snap[name] = st
    snap["g"]["count_prev"] = int(z["g.count_prev"])
    snap["g"]["id"] = z["g.id"]
    return snap
