"""Helpers of the GPU parity tests: run the oracle on the same seeded inputs with the same step
order as the HIP driver, and compare particle by particle.  Imports the oracle (test side only)."""
from __future__ import annotations

import numpy as np

import oracle


def oracle_run(tables, w, steps, flags, *, variant="", **kw):
    """Run the oracle for `steps` steps of workload `w` (see _oracle_run); variant "fma": on the
    oracle's build with contracted multiply-adds (same algorithm, other rounding)."""
    with oracle.use_variant(variant):
        return _oracle_run(tables, w, steps, flags, **kw)


_DECISION_COUNTERS = ("n_emit", "n_pair", "n_prob_clamped", "n_chi_clamped", "n_capacity_overflow", "n_retired",
                      "n_lepton_steps", "n_photon_steps")


def sensitivity_run(tables, w, steps, flags, ref, perturb32=False, **kw):
    """A second oracle run whose only difference from `ref` is rounding: on the oracle's
    multiply-add build (FP64 runs), or with perturb32 (single-precision runs, round32) the stored
    FP32 state nudged by one unit in the last place after every step, as an FP32 computation of it
    may land there.  Its particle-by-particle distance from `ref` is how far rounding alone moves
    each trajectory (strong rotation per step, fields whose direction turns with position).  The
    two runs must make the same decisions except at the near ties `ref` flagged."""
    if perturb32:
        alt = oracle_run(tables, w, steps, flags, perturb32=True, **kw)
    else:
        alt = oracle_run(tables, w, steps, flags, variant="fma", **kw)
    near = set()
    for sp, key in ((0, "near_e"), (1, "near_p")):
        near |= {(sp, int(i)) for i in np.nonzero(ref[key])[0]}
    ia, ir = alt["G"].id[:alt["G"].n], ref["G"].id[:ref["G"].n]
    diff = np.setxor1d(ia[ia != 0], ir[ir != 0])
    if diff.size:
        sp, par = photon_parent(diff)
        bad = [(int(a), int(b)) for a, b in zip(sp, par) if (int(a), int(b)) not in near]
        assert not bad, f"the rounding-sensitivity run decided differently away from near ties: {bad[:5]}"
    else:
        for c in _DECISION_COUNTERS:
            assert alt["ctr"][c] == ref["ctr"][c], f"rounding-sensitivity run: {c} {alt['ctr'][c]} vs {ref['ctr'][c]}"
    return alt


SENS_FACTOR = 10.0     # allowance over the distance between the two oracle builds


def _oracle_run(tables, w, steps, flags, *, cap_e=None, cap_p=None, cap_g=None, u24=False, near_tol=1e-10,
                index=None, seed=None, k_retire=None, t0=0.0, nthreads=16, x=None, p=None, s=None,
                fields=None, step0=0, tau=False, round32=False, perturb32=False):
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
        if round32 or perturb32:
            for S_ in (E, P):
                for arr in list(S_.x) + list(S_.p) + list(S_.s):
                    if arr is not None:
                        arr[:] = _round32(arr, perturb32)
            for arr in list(G.x) + list(G.k) + list(G.P):
                if arr is not None:
                    arr[:] = _round32(arr, perturb32)
    return dict(E=E, P=P, G=G, ctr=ctr.as_dict(), near_e=near_e[:E.n], near_p=near_p[:P.n], near_g=near_g[:G.n])


def _round32(a, nudge):
    """FP32 rounding of an FP64 array; with nudge, one unit in the last place away from zero"""
    r = a.astype(np.float32)
    if nudge:
        r = np.nextafter(r, np.copysign(np.float32(np.inf), r)).astype(np.float32)
        r[a == 0] = 0
    return r


def oracle_eps():
    import synth
    return synth.EPS_R


def rel_vec_err(a, b, floor=1e-300):
    """per-column |a - b| / max(|b|, floor) for (3, n) arrays"""
    return np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), floor)


def _cond_of(orc, cond, what):
    cond = cond if cond is not None else getattr(orc, "cond", None)
    assert cond is not None, f"{what}: the oracle's conditioning of the collapse axes is needed"
    return np.asarray(cond, dtype=np.float64)


def compare_leptons(gpu, orc, exclude, rtol_p, atol_s, rtol_x=None, what="", cond=None, sens=None):
    """Per particle: momentum within rtol_p (relative), position within rtol_x, and spin within
    atol_s max(1, kappa), kappa the conditioning of the collapse axes behind that spin as the oracle
    recorded it (orc.cond, or `cond`): a spin collapsed onto g/|g| (or a pair spin onto j/|j|) has
    its direction known to the unit roundoff times kappa, and no later part of the step amplifies
    that.  sens: the same oracle run on its multiply-add build (sensitivity_run); where rounding
    alone moves a particle's trajectory by d between the two builds (strong rotation per step),
    that particle is allowed SENS_FACTOR d.  No particle is let off."""
    xg, pg, sg = gpu
    xo, po, so = orc
    assert pg.shape == po.shape, f"{what}: count {pg.shape[1]} vs oracle {po.shape[1]}"
    kap = _cond_of(orc, cond, what)
    keep = ~exclude
    ep = rel_vec_err(pg[:, keep], po[:, keep])
    es = np.linalg.norm(sg[:, keep] - so[:, keep], axis=0)
    lim = atol_s * np.maximum(1.0, kap[keep])
    lim_p = np.full(ep.shape, rtol_p)
    if sens is not None:
        xa, pa, sa = sens
        lim_p = np.maximum(lim_p, SENS_FACTOR * rel_vec_err(pa[:, keep], po[:, keep]))
        lim = np.maximum(lim, SENS_FACTOR * np.linalg.norm(sa[:, keep] - so[:, keep], axis=0))
        ep = ep * (rtol_p / lim_p)            # measured against each particle's own allowance

    worst = dict(p=float(ep.max(initial=0)), s=float(es.max(initial=0)),
                 p_median=float(np.median(ep)) if ep.size else 0.0, n=int(keep.sum()),
                 s_over_tol=int((es > atol_s).sum()), s_worst_over_bound=float((es / lim).max(initial=0)),
                 kappa_max=float(kap[keep].max(initial=0)))
    assert worst["p"] <= rtol_p, f"{what}: momentum rel err {worst['p']:.3e} (argmax {int(np.argmax(ep))})"
    if (es > lim).any():
        j = int(np.argmax(es / lim))
        raise AssertionError(f"{what}: spin err {es[j]:.3e} at kept particle {j} with kappa {kap[keep][j]:.3g} "
                             f"({int((es > lim).sum())} over atol_s max(1, kappa))")
    if rtol_x is not None:
        scale = np.maximum(np.abs(xo[:, keep]).max(axis=0), 1.0)
        ex = np.abs(xg[:, keep] - xo[:, keep]).max(axis=0) / scale
        if sens is not None:
            lim_x = np.maximum(rtol_x, SENS_FACTOR * np.abs(sens[0][:, keep] - xo[:, keep]).max(axis=0) / scale)
            ex = ex * (rtol_x / lim_x)
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


def compare_photons(gpu, orc, excluded_parents, rtol_k, atol_P, what="", near_photons=None, cond=None, sens=None):
    """Match live photons by id; ids absent on one side must belong to excluded parents.  Per
    matched photon: momentum within rtol_k, P-vector within atol_P max(1, kappa), kappa the
    conditioning of its Stokes collapse as the oracle recorded it (orc.cond, or `cond`, aligned
    with the oracle's arrays): (F0 + w max(1, w/|g|))/|F|, the axis F/|F| being known to the
    rounding of F's terms over |F|, and F carrying the parent's spin-axis error."""
    xg, kg, Pg, idg = gpu
    xo, ko, Po, ido = orc
    kap = _cond_of(orc, cond, what)
    lg, lo = idg != 0, ido != 0
    ig, io = idg[lg], ido[lo]
    assert len(np.unique(ig)) == ig.size and len(np.unique(io)) == io.size, f"{what}: duplicate ids"
    common, cg, co = np.intersect1d(ig, io, return_indices=True)
    only = np.setxor1d(ig, io)
    if near_photons is not None and only.size:
        only = only[~np.isin(only, near_photons)]           # a near-tie pair decision may differ
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
    ks = kap[lo][co][keep]
    ek = rel_vec_err(kgs, kos)
    eP = director_err(Pgs, Pos, kos)
    lim = atol_P * np.maximum(1.0, ks)
    if sens is not None:                      # the multiply-add build's photons, matched by id
        _, ka, Pa, ida = sens
        pos = {int(v): j for j, v in enumerate(ida.tolist()) if v}
        ids = io[co][keep].tolist()
        have = np.array([int(v) in pos for v in ids], dtype=bool)       # absent: near-tie parents
        sel = np.array([pos.get(int(v), 0) for v in ids], dtype=np.int64)
        ka_, Pa_ = np.where(have, ka[:, sel], kos), np.where(have, Pa[:, sel], Pos)
        lim_k = np.maximum(rtol_k, SENS_FACTOR * rel_vec_err(ka_, kos))
        ek = ek * (rtol_k / lim_k)
        lim = np.maximum(lim, SENS_FACTOR * director_err(Pa_, Pos, kos))
    worst = dict(k=float(ek.max(initial=0)), P=float(eP.max(initial=0)), matched=int(keep.sum()),
                 unmatched=int(only.size), P_over_tol=int((eP > atol_P).sum()),
                 P_worst_over_bound=float((eP / lim).max(initial=0)), kappa_max=float(ks.max(initial=0)),
                 P_median=float(np.median(eP)) if eP.size else 0.0,
                 P_90=float(np.quantile(eP, 0.9)) if eP.size else 0.0)
    assert worst["k"] <= rtol_k, f"{what}: photon momentum rel err {worst['k']:.3e}"
    if (eP > lim).any():
        j = int(np.argmax(eP / lim))
        raise AssertionError(f"{what}: photon P-vector err {eP[j]:.3e} with kappa {ks[j]:.3g} "
                             f"({int((eP > lim).sum())} over atol_P max(1, kappa))")
    return worst


# ------------------------------------------------------------------ decision mismatches
def oracle_sets_from_snapshot(st, track, extra_e=0, extra_g=0, tau=False):
    """Oracle particle sets holding a host snapshot (sim.Simulation.snapshot(device=False)): the
    FP32 or FP64 values of the GPU state, widened to FP64 (with the optical depths if tau)."""
    e, p, g = st["e"], st["p"], st["g"]
    ne, np_, ng = e["count"], p["count"], g["count"]

    def stack(arrs, n):
        return np.stack([(a.astype(np.float64) if a is not None else np.zeros(n)) for a in arrs])

    E = oracle.LeptonSet(0, ne + np_ + extra_e + 1, track=track, tau=tau)
    E.set(stack(e["x"], ne), stack(e["p"], ne), stack(e["s"], ne))
    P = oracle.LeptonSet(1, ne + np_ + extra_e + 1, track=track, tau=tau)
    P.set(stack(p["x"], np_), stack(p["p"], np_), stack(p["s"], np_))
    if tau:
        for L, d, n in ((E, e, ne), (P, p, np_)):
            L.tau[:n], L.tau_target[:n] = d["tau"][0], d["tau"][1]
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


def oracle_advance(tables, w, E, P, G, steps, flags, step0, *, u24=False, near_tol=1e-10, round32=False,
                   nthreads=16, fields=None, k_retire=None, seed=None):
    """Advance oracle sets (for example from oracle_sets_from_snapshot) by `steps` time steps from
    step index step0 (t = step0 dt) in the HIP driver's order: electrons, positrons, then the
    photons stored before the step.  Returns the counters and the near-tie flags accumulated per
    particle (over the sets' final extents)."""
    F = fields or oracle.make_fields(w.field_kind, E0=w.E0, B0=w.B0, a0=w.a0, phase_len=w.phase_len)
    ctr = oracle.Counters()
    near_e = np.zeros(E.cap, dtype=bool)
    near_p = np.zeros(P.cap, dtype=bool)
    near_g = np.zeros(G.cap, dtype=bool)
    near_ids = []
    for k in range(step0, step0 + steps):
        prm = oracle.make_params(w.dt, oracle_eps(), step=k, t=k * w.dt, seed=w.seed if seed is None else seed,
                                 flags=flags, k_retire=w.k_retire if k_retire is None else k_retire,
                                 near_tol=near_tol, u24=u24)
        oracle.lepton_step(tables, prm, F, E, G, ctr, nthreads)
        near_e |= E.near.astype(bool)
        if flags & oracle.F_PAIR:
            oracle.lepton_step(tables, prm, F, P, G, ctr, nthreads)
            near_p |= P.near.astype(bool)
            m = G.n
            ids = G.id[:m].copy()
            oracle.photon_step(tables, prm, F, G, E, P, ctr, nthreads)
            fl = G.near[:m].astype(bool)
            near_g[:m] |= fl
            near_ids.append(ids[fl])
        if round32:
            for S_ in (E, P):
                for arr in list(S_.x) + list(S_.p) + list(S_.s):
                    if arr is not None:
                        arr[:] = arr.astype(np.float32)
            for arr in list(G.x) + list(G.k) + list(G.P):
                if arr is not None:
                    arr[:] = arr.astype(np.float32)
    return dict(ctr=ctr.as_dict(), near_e=near_e[:E.n], near_p=near_p[:P.n], near_g=near_g[:G.n],
                near_photon_ids=np.concatenate(near_ids) if near_ids else np.zeros(0, np.uint64))


def near_tie_outcomes(gpu_ids, orc_ids, near_e, near_p=None):
    """Of the leptons the oracle flagged as near ties, how many ended with a different set of
    emitted photons on the GPU (the decision that was a near tie actually came out the other way,
    or a later one followed from it).  Returns (near ties, flipped, flipped leptons that were not
    near ties)."""
    def by_parent(ids):
        ids = ids[ids != 0]
        sp, par = photon_parent(ids)
        d = {}
        for a, b, i in zip(sp.tolist(), par.tolist(), ids.tolist()):
            d.setdefault((a, b), set()).add(i)
        return d

    g, o = by_parent(np.asarray(gpu_ids)), by_parent(np.asarray(orc_ids))
    near = {(0, int(i)) for i in np.nonzero(near_e)[0]}
    if near_p is not None:
        near |= {(1, int(i)) for i in np.nonzero(near_p)[0]}
    differ = {k for k in set(g) | set(o) if g.get(k, set()) != o.get(k, set())}
    return len(near), len(differ & near), len(differ - near)
