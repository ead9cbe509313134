"""Helpers of the GPU parity tests: run the oracle on the same seeded inputs with the same step
order as the HIP driver, and compare particle by particle.  Imports the oracle (test side only)."""
from __future__ import annotations

import numpy as np

import oracle


def oracle_run(tables, w, steps, flags, *, cap_e=None, cap_p=None, cap_g=None, u24=False, near_tol=1e-10,
               index=None, seed=None, k_retire=None, t0=0.0, nthreads=16, x=None, p=None, s=None,
               fields=None, step0=0, tau=False, round32=False):
    """Run the oracle for `steps` steps of workload `w` (optionally a subset with original indices
    `index`).  Returns dict of oracle sets, counters and accumulated near-tie flags.
    round32: round the stored particle state (x, p, s, k, P) to FP32 after every step, as the
    single-precision path stores it, so that a comparison measures one step's arithmetic."""
    x = w.x if x is None else x
    p = w.p if p is None else p
    s = w.s if s is None else s
    n = p.shape[1]
    cap_e = cap_e or n
    cap_p = cap_p or max(1, cap_e - n)
    cap_g = cap_g or 1
    E = oracle.LeptonSet(0, cap_e, track=w.track, tau=tau)
    E.set(x, p, s, index=index)
    P = oracle.LeptonSet(1, cap_p, track=w.track, tau=tau)
    G = oracle.PhotonSet(cap_g, track=w.track)
    F = fields or oracle.make_fields(w.field_kind, E0=w.E0, B0=w.B0, a0=w.a0, phase_len=w.phase_len)
    ctr = oracle.Counters()
    near_e = np.zeros(cap_e, dtype=bool)
    near_p = np.zeros(cap_p, dtype=bool)
    near_g = np.zeros(cap_g, dtype=bool)
    pair = bool(flags & oracle.F_PAIR)
    for k in range(step0, step0 + steps):
        prm = oracle.make_params(w.dt, oracle_eps(), step=k, t=t0 + k * w.dt,
                                 seed=w.seed if seed is None else seed, flags=flags,
                                 k_retire=w.k_retire if k_retire is None else k_retire, near_tol=near_tol, u24=u24)
        oracle.lepton_step(tables, prm, F, E, G, ctr, nthreads)
        near_e |= E.near.astype(bool)
        if pair:
            oracle.lepton_step(tables, prm, F, P, G, ctr, nthreads)
            near_p |= P.near.astype(bool)
            oracle.photon_step(tables, prm, F, G, E, P, ctr, nthreads)
            near_g |= G.near.astype(bool)
        if round32:
            for S_ in (E, P):
                for arr in list(S_.x) + list(S_.p) + list(S_.s):
                    if arr is not None:
                        arr[:] = arr.astype(np.float32)
            for arr in list(G.x) + list(G.k) + list(G.P):
                if arr is not None:
                    arr[:] = arr.astype(np.float32)
    return dict(E=E, P=P, G=G, ctr=ctr.as_dict(), near_e=near_e[:E.n], near_p=near_p[:P.n], near_g=near_g[:G.n])


def oracle_eps():
    import synth
    return synth.EPS_R


def rel_vec_err(a, b, floor=1e-300):
    """per-column |a - b| / max(|b|, floor) for (3, n) arrays"""
    return np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), floor)


def compare_leptons(gpu, orc, exclude, rtol_p, atol_s, rtol_x=None, what="", events=None, outlier_rate=1e-5):
    """events: number of spin collapses behind the compared spins (default: one per particle);
    the ill-conditioned collapse axis allows a fraction outlier_rate of them above atol_s (1e-5 in
    FP64; in FP32, whose rounding is 1e9 times larger, axes with conditioning above ~100 exceed
    1e-5, so single-precision checks pass 1e-2)."""
    xg, pg, sg = gpu
    xo, po, so = orc
    assert pg.shape == po.shape, f"{what}: count {pg.shape[1]} vs oracle {po.shape[1]}"
    keep = ~exclude
    ep = rel_vec_err(pg[:, keep], po[:, keep])
    es = np.linalg.norm(sg[:, keep] - so[:, keep], axis=0)
    worst = dict(p=float(ep.max(initial=0)), s=float(es.max(initial=0)),
                 p_median=float(np.median(ep)) if ep.size else 0.0, n=int(keep.sum()),
                 s_over_tol=int((es > atol_s).sum()))
    assert worst["p"] <= rtol_p, f"{what}: momentum rel err {worst['p']:.3e} (argmax {int(np.argmax(ep))})"
    # the spin axis g/|g| of the collapse has the same conditioning as the photon axis
    allowed = max(1, int((es.size if events is None else events) * outlier_rate))
    assert worst["s_over_tol"] <= allowed and worst["s"] <= 1e3 * atol_s, \
        f"{what}: spin err {worst['s']:.3e} (argmax {int(np.argmax(es))}, {worst['s_over_tol']} over tol)"
    if rtol_x is not None:
        ex = np.abs(xg[:, keep] - xo[:, keep]).max(axis=0) / np.maximum(np.abs(xo[:, keep]).max(axis=0), 1.0)
        worst["x"] = float(ex.max(initial=0))
        assert worst["x"] <= rtol_x, f"{what}: position err {worst['x']:.3e}"
    return worst


def director_err(Pa, Pb, k):
    """|Pa - Pb| with the transverse part of a P-vector taken as a director: P_perp and -P_perp
    encode the same photon state (the Stokes angle is twice the P angle)."""
    kh = k / np.linalg.norm(k, axis=0)
    Pb_flip = 2 * np.sum(Pb * kh, axis=0) * kh - Pb          # reflect the transverse part
    return np.minimum(np.linalg.norm(Pa - Pb, axis=0), np.linalg.norm(Pa - Pb_flip, axis=0))


def photon_parent(ids):
    ids = ids.astype(np.uint64)
    return ((ids >> np.uint64(61)) & np.uint64(3)).astype(np.int64), \
        ((ids >> np.uint64(24)) & np.uint64((1 << 33) - 1)).astype(np.int64)


def compare_photons(gpu, orc, excluded_parents, rtol_k, atol_P, what="", near_photons=None, outlier_rate=1e-5):
    """Match live photons by id; ids absent on one side must belong to excluded parents.
    outlier_rate: fraction of photons allowed above atol_P (ill-conditioned polarization axis)."""
    xg, kg, Pg, idg = gpu
    xo, ko, Po, ido = orc
    lg, lo = idg != 0, ido != 0
    ig, io = idg[lg], ido[lo]
    assert len(np.unique(ig)) == ig.size and len(np.unique(io)) == io.size, f"{what}: duplicate ids"
    common, cg, co = np.intersect1d(ig, io, return_indices=True)
    only = np.setxor1d(ig, io)
    if only.size:
        sp, pi = photon_parent(only)
        bad = [(int(a), int(b)) for a, b in zip(sp, pi) if (int(a), int(b)) not in excluded_parents]
        assert not bad, f"{what}: {only.size} unmatched photons, e.g. parents {bad[:5]}"
    sp, pi = photon_parent(common)
    keep = np.array([(int(a), int(b)) not in excluded_parents for a, b in zip(sp, pi)], dtype=bool)
    if near_photons is not None:
        keep &= ~np.isin(common, near_photons)
    kgs, kos = kg[:, lg][:, cg][:, keep], ko[:, lo][:, co][:, keep]
    Pgs, Pos = Pg[:, lg][:, cg][:, keep], Po[:, lo][:, co][:, keep]
    ek = rel_vec_err(kgs, kos)
    eP = director_err(Pgs, Pos, kos)
    worst = dict(k=float(ek.max(initial=0)), P=float(eP.max(initial=0)), matched=int(keep.sum()),
                 unmatched=int(only.size), P_over_tol=int((eP > atol_P).sum()),
                 P_median=float(np.median(eP)) if eP.size else 0.0,
                 P_90=float(np.quantile(eP, 0.9)) if eP.size else 0.0,
                 P_999999=float(np.quantile(eP, 0.999999)) if eP.size else 0.0)
    assert worst["k"] <= rtol_k, f"{what}: photon momentum rel err {worst['k']:.3e}"
    # The polarization axis F/|F| is ill-conditioned where the photon's polarization degree
    # |F|/F0 is small (axis error ~ eps F0/|F|): at most a fraction outlier_rate (default 1e-5)
    # of the photons may exceed atol_P, and none may exceed 1e3 atol_P.
    assert worst["P_over_tol"] <= max(1, int(eP.size * outlier_rate)) and worst["P"] <= 1e3 * atol_P, \
        f"{what}: photon P-vector err {worst['P']:.3e} ({worst['P_over_tol']} over {atol_P:.1e})"
    return worst


# ------------------------------------------------------------------ decision mismatches
def oracle_sets_from_snapshot(st, track, extra_e=0, extra_g=0):
    """Oracle particle sets holding a host snapshot (sim.Simulation.snapshot(device=False)): the
    FP32 or FP64 values of the GPU state, widened to FP64."""
    e, p, g = st["e"], st["p"], st["g"]
    ne, np_, ng = e["count"], p["count"], g["count"]

    def stack(arrs, n):
        return np.stack([(a.astype(np.float64) if a is not None else np.zeros(n)) for a in arrs])

    E = oracle.LeptonSet(0, ne + np_ + extra_e + 1, track=track)
    E.set(stack(e["x"], ne), stack(e["p"], ne), stack(e["s"], ne))
    P = oracle.LeptonSet(1, ne + np_ + extra_e + 1, track=track)
    P.set(stack(p["x"], np_), stack(p["p"], np_), stack(p["s"], np_))
    G = oracle.PhotonSet(ng + ne + np_ + extra_g + 1, track=track)
    for i in range(3):
        if G.x[i] is not None:
            G.x[i][:ng] = g["x"][i].astype(np.float64)
        G.k[i][:ng] = g["k"][i].astype(np.float64)
        G.P[i][:ng] = g["P"][i].astype(np.float64)
    G.id[:ng] = np.asarray(g["id"]).view(np.uint64)
    G.n, G.n_prev = ng, g["count_prev"]
    return E, P, G


def decision_flips(q, tab, w, st, k0, T, nthreads, u24=True, near_tol=1e-5, fields=None, flags=None):
    """One step of every particle of a host snapshot `st` (taken at time step k0 of workload w) on the
    GPU (merged step, tables `tab`) and in the oracle, photon retirement at birth off (k_retire = 0)
    so that every emitted photon carries its parent's index.  Counts the leptons whose emit / no-emit
    decision and the photons whose pair / no-pair decision differ, and how many of those the oracle
    flagged as near ties (its draw within near_tol of a threshold); emitters on both sides whose
    photon energies differ by more than 1e-3 (the spin-down / spin-up branch) are counted apart."""
    import torch

    from paper_2511_08929_amd.sim import Simulation
    flags = q.QED_ALL if flags is None else flags
    e, p, g = st["e"], st["p"], st["g"]
    ne, np_, ng, ngp = e["count"], p["count"], g["count"], g["count_prev"]
    f = fields or q.make_fields(w.field_kind, E0=w.E0, B0=w.B0, a0=w.a0, phase_len=w.phase_len)
    sim = Simulation(tab, cap_e=ne + np_ + ngp + 16, cap_p=ne + np_ + ngp + 16, cap_g=ng + ne + np_ + 16, track=w.track,
                     fields=f, dt=w.dt, eps_r=oracle_eps(), seed=w.seed, flags=flags, k_retire=0.0, device_clock=True,
                     merged=True)
    sim.restore(st, counters=False)
    sim.ctr.zero_()
    sim.step()
    torch.cuda.synchronize()
    gx, gk, gP, gid = sim.g.arrays()
    c_gpu = q.counters_dict(sim.ctr)
    del sim
    torch.cuda.empty_cache()
    E, P, G = oracle_sets_from_snapshot(st, w.track, extra_e=ngp, extra_g=ne + np_)
    F = oracle.make_fields(w.field_kind, E0=w.E0, B0=w.B0, a0=w.a0, phase_len=w.phase_len)
    prm = oracle.make_params(w.dt, oracle_eps(), step=k0, t=k0 * w.dt, seed=w.seed, flags=flags, k_retire=0.0,
                             near_tol=near_tol, u24=u24)
    ctr = oracle.Counters()
    oracle.lepton_step(T, prm, F, E, G, ctr, nthreads)
    near_e = E.near[:ne].astype(bool).copy()
    oracle.lepton_step(T, prm, F, P, G, ctr, nthreads)
    near_p = P.near[:np_].astype(bool).copy()
    oracle.photon_step(T, prm, F, G, E, P, ctr, nthreads)
    near_g = G.near[:ngp].astype(bool).copy()
    _, ok, _, oid = G.arrays()
    # emissions: photons appended this step, by parent (species, index)
    new_g, new_o = gid[ng:], oid[ng:]
    assert (new_g != 0).all() and (new_o != 0).all(), "an emitted photon without id (k_retire is 0)"
    par_g = dict(zip(map(tuple, np.stack(photon_parent(new_g), 1).tolist()), range(ng, ng + new_g.size)))
    par_o = dict(zip(map(tuple, np.stack(photon_parent(new_o), 1).tolist()), range(ng, ng + new_o.size)))
    flips = set(par_g) ^ set(par_o)
    near = {(0, int(i)) for i in np.nonzero(near_e)[0]} | {(1, int(i)) for i in np.nonzero(near_p)[0]}
    branch = 0
    for key in set(par_g) & set(par_o):
        a = np.linalg.norm(gk[:, par_g[key]])
        b = np.linalg.norm(ok[:, par_o[key]])
        if abs(a - b) > 1e-3 * b and key not in near:
            branch += 1
    # pair decisions of the photons stepped this step (alive before)
    alive0 = np.asarray(g["id"][:ngp]) != 0
    dead_g = gid[:ngp] == 0
    dead_o = oid[:ngp] == 0
    pflip = np.nonzero(alive0 & (dead_g != dead_o))[0]
    res = dict(leptons=int(ne + np_), photons=int(alive0.sum()), emissions_gpu=int(len(par_g)),
               emissions_oracle=int(len(par_o)), pairs_gpu=c_gpu["n_pair"], pairs_oracle=int(ctr.n_pair),
               lepton_near_ties=int(near_e.sum() + near_p.sum()), photon_near_ties=int(near_g[alive0].sum()),
               lepton_flips=len(flips), lepton_flips_not_near=len(flips - near),
               photon_flips=int(pflip.size), photon_flips_not_near=int((~near_g[pflip]).sum()),
               energy_mismatch_not_near=int(branch))
    res["flip_rate"] = (res["lepton_flips"] + res["photon_flips"]) / max(1, res["leptons"] + res["photons"])
    res["near_tie_rate"] = (res["lepton_near_ties"] + res["photon_near_ties"]) / max(1, res["leptons"] + res["photons"])
    return res
