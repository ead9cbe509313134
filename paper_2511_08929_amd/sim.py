"""Time-step driver over the C ABI: one step = qed_emit (push + NLC) for electrons, then for
positrons, then qed_pair (NBW) for the photons born in earlier steps; qed_compact on demand.

All counts stay on the device; a step enqueues without host synchronization, so a sequence of
steps can be captured in a HIP graph.
"""
from __future__ import annotations

import math

from . import (ALPHA, QED_F32, QED_F64, QED_PAIR, LeptonBuffers, PhotonBuffers, Tables, make_fields, make_step,
               new_counters, new_workspace, qed_compact, qed_compact_workspace_size, qed_emit, qed_pair,
               qed_workspace_size)


class Simulation:
    def __init__(self, tables: Tables, *, cap_e, cap_p, cap_g, track, fields, dt, eps_r, seed, flags,
                 k_retire=0.0, t0=0.0, a_e=ALPHA / (2 * math.pi), chi_e_min=1e-3, chi_e_max=1e2, chi_g_min=0.05,
                 chi_g_max=1e2, device="cuda"):
        import torch
        self.tables = tables
        self.dtype = torch.float64 if tables.precision == QED_F64 else torch.float32
        self.e = LeptonBuffers(0, cap_e, self.dtype, device, track)
        self.p = LeptonBuffers(1, cap_p, self.dtype, device, track)
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

    def step_params(self, n):
        return make_step(self.dt, self.eps_r, step=n, t=self.t0 + n * self.dt, seed=self.seed, flags=self.flags,
                         a_e=self.a_e, chi_e_min=self.chi[0], chi_e_max=self.chi[1], chi_g_min=self.chi[2],
                         chi_g_max=self.chi[3], k_retire=self.k_retire)

    def step(self, stream=None):
        sp = self._sp
        if sp is None:
            sp = self._sp = self.step_params(self.n)
        sp.step, sp.t, sp.flags = self.n, self.t0 + self.n * self.dt, self.flags
        qed_emit(self.tables, self.e, self.fields, sp, self.g, self.ctr, self.ws, stream)
        if self.flags & QED_PAIR:
            qed_emit(self.tables, self.p, self.fields, sp, self.g, self.ctr, self.ws, stream)
            qed_pair(self.tables, self.g, self.fields, sp, self.e, self.p, self.ctr, self.ws, stream)
        self.n += 1

    def compact(self, stream=None):
        qed_compact(self.g, self.tables.precision, self.ws, stream)
