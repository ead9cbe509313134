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

from . import (ALPHA, QED_F64, QED_PAIR, LeptonBuffers, PhotonBuffers, Plan, Tables, make_fields, make_step,
               new_counters, new_workspace, qed_clock_advance, qed_compact, qed_compact_workspace_size, qed_emit,
               qed_pair, qed_workspace_size)


class Simulation:
    def __init__(self, tables: Tables, *, cap_e, cap_p, cap_g, track, fields, dt, eps_r, seed, flags,
                 k_retire=0.0, t0=0.0, a_e=ALPHA / (2 * math.pi), chi_e_min=1e-3, chi_e_max=1e2, chi_g_min=0.05,
                 chi_g_max=1e2, device="cuda", device_clock=False, merged=False, particles_per_block=0,
                 max_blocks_per_set=0, optical_depth=False, surrogates=(None, None)):
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
        self.merged, self.ppb, self.maxb = merged, particles_per_block, max_blocks_per_set
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
                             surrogates=self.surrogates)

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


class Batch:
    """Independent instances stepped by one plan.  ``specs`` is a list of dicts with keys
    cap_e, cap_p, cap_g, track, fields, dt, eps_r, seed, flags and optionally k_retire, t0, a_e."""

    def __init__(self, tables: Tables, specs, device="cuda", particles_per_block=0, max_blocks_per_set=0):
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
        self.ppb, self.maxb = particles_per_block, max_blocks_per_set
        self.plan = None
        self.n = 0

    def _ensure_plan(self):
        if self.plan is None:
            self.plan = Plan(self.tables, [(i["e"], i["p"], i["g"], i["fields"], i["step"], i["ctr"]) for i in self.inst],
                             particles_per_block=self.ppb, max_blocks_per_set=self.maxb)

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
