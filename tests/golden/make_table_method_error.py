"""Write table_method_error.json: the interpolation error of the rate and inverse-CDF tables on
the table grid, measured by the oracle alone (its tables against its exact quadrature and root
finding).  The GPU tables equal the oracle's to 1e-12, so the figures hold for both.

Samples, per channel (NLC spin down / up, NBW xi3 = -1 / +1), with a fixed seed:
  inverse CDF: ln chi uniform over the table's range, rho = logit r with r uniform (the
               distribution the sampling draws); the error of nu = logit lambda, of lambda
               (relative) and of 1 - lambda (relative);
  rates:       ln chi uniform over the table's range; the error of ln int w dlambda.
Run from the repository root:  python tests/golden/make_table_method_error.py [n_per_channel]
"""
from __future__ import annotations

import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table_method_error.json")
_T = None


def _init(spec):
    global _T
    _T = oracle.OracleTables(spec=spec, nthreads=1)


def _icdf(args):
    ch, lnchi, rho = args
    return oracle.icdf_nu(ch, float(np.exp(lnchi)), rho), _T.nu(ch, lnchi, rho)


def _rate(args):
    ch, lnchi = args
    return np.log(oracle.rate_integral(ch, float(np.exp(lnchi)))), _T.lnrate(ch, lnchi)


def measure(spec=None, n=500, seed=20251108, procs=8):
    spec = spec or oracle.default_spec()
    oracle.OracleTables(spec=spec, nthreads=procs)           # build (or load) the cache once
    rng = np.random.default_rng(seed)
    pts, rpts = [], []
    for ch in range(4):
        g = 0 if ch < 2 else 1
        lo, h, m = spec["lnchi0"][g], spec["dlnchi"][g], spec["n_chi"][g]
        for _ in range(n):
            lnchi = rng.uniform(lo, lo + (m - 1) * h)
            r = rng.random()
            pts.append((ch, lnchi, float(np.log(r) - np.log1p(-r))))
            rpts.append((ch, rng.uniform(lo, lo + (m - 1) * h)))
    with Pool(procs, initializer=_init, initargs=(spec,)) as p:
        icdf = np.array(p.map(_icdf, pts, chunksize=4))
        rate = np.array(p.map(_rate, rpts, chunksize=4))
    chs = np.array([c for c, _, _ in pts])
    rch = np.array([c for c, _ in rpts])
    nx, nt = icdf[:, 0], icdf[:, 1]
    lam = lambda v: 1.0 / (1.0 + np.exp(-v))            # noqa: E731
    oml = lambda v: 1.0 / (1.0 + np.exp(v))             # noqa: E731
    rel_l = np.abs(lam(nt) - lam(nx)) / lam(nx)
    rel_o = np.abs(oml(nt) - oml(nx)) / oml(nx)
    dnu = np.abs(nt - nx)
    dr = np.abs(rate[:, 0] - rate[:, 1])
    names = ["nlc_spin_down", "nlc_spin_up", "nbw_xi3_minus", "nbw_xi3_plus"]
    per = {}
    for c in range(4):
        m, mr = chs == c, rch == c
        per[names[c]] = dict(max_abs_dnu=float(dnu[m].max()), p99_abs_dnu=float(np.quantile(dnu[m], 0.99)),
                             max_rel_lambda=float(rel_l[m].max()), p99_rel_lambda=float(np.quantile(rel_l[m], 0.99)),
                             max_rel_one_minus_lambda=float(rel_o[m].max()),
                             max_abs_dlnrate=float(dr[mr].max()))
    return dict(
        grid=dict(n_chi=list(spec["n_chi"]), chi_nodes_per_decade=round(float(np.log(10) / spec["dlnchi"][0]), 6),
                  n_rho=spec["n_rho"], rho_range=[spec["rho0"], spec["rho0"] + (spec["n_rho"] - 1) * spec["drho"]]),
        samples_per_channel=n, seed=seed,
        max_abs_dnu=float(dnu.max()), p99_abs_dnu=float(np.quantile(dnu, 0.99)),
        max_rel_lambda=float(rel_l.max()), p99_rel_lambda=float(np.quantile(rel_l, 0.99)),
        max_abs_dlnrate=float(dr.max()), per_channel=per,
        method="oracle tables (4 x 4 Lagrange in ln chi and rho) against the oracle's exact inverse CDF "
               "(root of the quadrature CDF) and rate integral; ln chi uniform, rho = logit of a uniform r",
        script="tests/golden/make_table_method_error.py")


if __name__ == "__main__":
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 500
    res = measure(n=n)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))
