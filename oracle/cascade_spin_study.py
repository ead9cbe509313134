"""Study of the lepton spin ratio in the seeded pair cascade (polarized-cascade section), with the
oracle alone: the spins of pair-born leptons at birth and the ratio of the two spin populations
in the exponential phase, under three readings of pair production.

  r1      the photon basis of reading R1 (electron-line convention, as built)
  flip    the other orientation of the photon basis: e and b reversed.  The chi_gamma, the rates
          and the Stokes parameters are unchanged by it (xi1, xi3 involve twice the polarization
          angle, xi2 the k component); only the e and b components of the pair spins, sampled in
          that basis, reverse.  The run applies exactly that to every pair-born lepton at birth.
  nospin  pair spins not assigned (pair-born leptons unpolarized, s = 0)

"Down" is the radiatively favoured state (Sokolov-Ternov): spin against the rest-frame magnetic
field for electrons, along it for positrons, which is s.beta > 0 for both species in the R1
lepton basis.  Counts by the sign of s.beta and polarization-weighted, (1 +- <s.beta>)/2.

Test infrastructure, like the rest of oracle/.  Run from the repository root:
    python oracle/cascade_spin_study.py [seeds=300] [omega_t=14] [threads=8]
(about a minute and a half per reading on 8 threads)."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402


def lepton_sbeta(L, lo, hi, q, F, t):
    """s.beta of leptons lo..hi-1 in their own basis at time t (uniform fields: any position)"""
    E, B = oracle.fields_eval(F, np.zeros(3), t)
    out = np.empty(hi - lo)
    for j, i in enumerate(range(lo, hi)):
        p = np.array([L.p[a][i] for a in range(3)])
        s = np.array([L.s[a][i] for a in range(3)])
        _, e, b, k = oracle.basis(q, synth.EPS_R, E, B, p)
        out[j] = s @ b
    return out


def run(tables, mode, seeds=300, omega_t=14.0, threads=8):
    w = synth.c6(n=seeds)
    steps = int(round(omega_t / w.dt))
    flags = oracle.F_ALL if mode != "nospin" else oracle.F_ALL & ~oracle.F_PAIR_SPIN
    cap = 200 * seeds + 1000
    E = oracle.LeptonSet(0, cap, track=w.track)
    E.set(w.x, w.p, w.s)
    P = oracle.LeptonSet(1, cap, track=w.track)
    G = oracle.PhotonSet(2000 * seeds + 10000, track=w.track)
    F = oracle.make_fields(w.field_kind, a0=w.a0)
    ctr = oracle.Counters()
    births = {0: [], 1: []}
    for k in range(steps):
        t = k * w.dt
        prm = oracle.make_params(w.dt, synth.EPS_R, step=k, t=t, seed=w.seed, flags=flags, k_retire=w.k_retire)
        oracle.lepton_step(tables, prm, F, E, G, ctr, threads)
        oracle.lepton_step(tables, prm, F, P, G, ctr, threads)
        ne, npo = E.n, P.n
        oracle.photon_step(tables, prm, F, G, E, P, ctr, threads)
        if E.n > ne and mode == "flip":
            Ef, Bf = oracle.fields_eval(F, np.zeros(3), t + w.dt)
            for L, lo, hi in ((E, ne, E.n), (P, npo, P.n)):
                for i in range(lo, hi):
                    p = np.array([L.p[a][i] for a in range(3)])
                    s = np.array([L.s[a][i] for a in range(3)])
                    # the photon's basis: electron-line convention, momentum along the pair's
                    _, e, b, _ = oracle.basis(-1, synth.EPS_R, Ef, Bf, p)
                    s = s - 2 * (s @ e) * e - 2 * (s @ b) * b
                    for a in range(3):
                        L.s[a][i] = s[a]
        if E.n > ne:
            births[0].append(lepton_sbeta(E, ne, E.n, -1, F, t + w.dt))
            births[1].append(lepton_sbeta(P, npo, P.n, 1, F, t + w.dt))
        if (k + 1) % 50 == 0:
            oracle.compact(G)
    tf = steps * w.dt
    out = {"mode": mode, "omega_t": tf, "seeds": seeds}
    for name, L, q, sp in (("electrons", E, -1, 0), ("positrons", P, 1, 1)):
        sb = lepton_sbeta(L, 0, L.n, q, F, tf)
        b = np.concatenate(births[sp]) if births[sp] else np.zeros(0)
        out[name] = dict(n=int(L.n), down_up_sign=float((sb > 0).sum() / max(1, (sb < 0).sum())),
                         down_up_weighted=float((1 + sb.mean()) / (1 - sb.mean())),
                         pair_born=int(b.size), birth_sbeta_mean=float(b.mean()) if b.size else None)
    return out


if __name__ == "__main__":
    seeds = int(sys.argv[1]) if len(sys.argv) > 1 else 300
    omega_t = float(sys.argv[2]) if len(sys.argv) > 2 else 14.0
    threads = int(sys.argv[3]) if len(sys.argv) > 3 else 8
    tables = oracle.OracleTables(nthreads=threads)
    for mode in ("r1", "flip", "nospin"):
        r = run(tables, mode, seeds, omega_t, threads)
        print(r["mode"], "omega t", r["omega_t"], {k: r[k] for k in ("electrons", "positrons")}, flush=True)
