"""Plain FP64 CPU oracle of the spin- and polarization-resolved strong-field QED step
of arXiv 2511.08929 (Qian, Seipt, Vranic, Grismayer, Ridgers, Thomas).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code with the
HIP library (``paper_2511_08929_amd``) and never imports it.

The numerical work lives in ``qed_oracle.c`` (plain C, IEEE double); this module only
compiles it with gcc, loads it with ctypes and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "qed_oracle.c"
HDR = HERE / "qed_oracle.h"
LIB = HERE / "liborc.so"
CACHE = HERE.parent / "_build" / "oracle_tables"

ALPHA = 7.2973525693e-3

# channels of the rate / inverse-CDF tables
NLC_DOWN, NLC_UP, NBW_MINUS, NBW_PLUS = 0, 1, 2, 3

# flags (same meaning as the C enum in qed_oracle.h)
F_PUSH, F_TBMT, F_EMIT, F_RECOIL = 1 << 0, 1 << 1, 1 << 2, 1 << 3
F_SPIN, F_NOEMIT, F_PHOTON_POL, F_MEAN = 1 << 4, 1 << 5, 1 << 6, 1 << 7
F_PAIR, F_NOPAIR, F_PAIR_SPIN = 1 << 8, 1 << 9, 1 << 10
F_TAU = 1 << 11
F_REJECT = 1 << 12
F_GCHI = 1 << 13
F_SUB = 1 << 14
SUB_ROUNDS, SUB_WDT = 16, 0.1
GF_N, GF_LNCHI0, GF_DLNCHI = 705, -16.11809565095832, 0.03597789207803197
F_ALL = (F_PUSH | F_TBMT | F_EMIT | F_RECOIL | F_SPIN | F_NOEMIT | F_PHOTON_POL
         | F_PAIR | F_NOPAIR | F_PAIR_SPIN)

FIELD_UNIFORM, FIELD_PLANE_LP, FIELD_GRID2D, FIELD_ROTATING_E = 0, 1, 2, 3


# A second build of the same source with fused multiply-adds wherever an expression allows
# (-mfma -ffp-contract=fast).  It is the same algorithm rounded differently: where the two builds
# disagree on a particle, rounding alone moves that particle's trajectory that far, which the
# parity tests use as the particle's sensitivity to rounding.
LIB_FMA = HERE / "liborc_fma.so"
_VARIANT_FLAGS = {"": [], "fma": ["-mfma", "-ffp-contract=fast"]}


def build(force: bool = False, variant: str = "") -> Path:
    """Compile the oracle with gcc (portable -O2, OpenMP, no fast-math); variant "fma": the build
    with contracted multiply-adds."""
    out = LIB if not variant else LIB_FMA
    if out.exists() and not force and out.stat().st_mtime > max(SRC.stat().st_mtime, HDR.stat().st_mtime):
        return out
    tmp = out.with_suffix(".so.tmp")
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", *_VARIANT_FLAGS[variant],
           "-Wall", "-Wno-unknown-pragmas", "-o", str(tmp), str(SRC), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None
_libs = {}
_active = ""


class use_variant:
    """Context manager: the oracle calls inside it run on the given build ("" or "fma").  Tables
    built or loaded by either build serve both (plain C structs and arrays)."""

    def __init__(self, variant):
        self.variant = variant

    def __enter__(self):
        global _active, _lib
        self.prev = _active
        _active = self.variant
        _lib = None
        return self

    def __exit__(self, *exc):
        global _active, _lib
        _active = self.prev
        _lib = None
        return False


class TableSpec(C.Structure):
    _fields_ = [("n_chi", C.c_int * 2), ("lnchi0", C.c_double * 2), ("dlnchi", C.c_double * 2),
                ("n_rho", C.c_int), ("rho0", C.c_double), ("drho", C.c_double)]


class Tables(C.Structure):
    _fields_ = [("spec", TableSpec), ("lnrate", C.POINTER(C.c_double)), ("nu", C.POINTER(C.c_double)),
                ("off_rate", C.c_int64 * 4), ("off_nu", C.c_int64 * 4), ("lngfac", C.POINTER(C.c_double))]


class Fields(C.Structure):
    _fields_ = [("kind", C.c_int), ("E0", C.c_double * 3), ("B0", C.c_double * 3),
                ("a0", C.c_double), ("phase_len", C.c_double), ("grid", C.POINTER(C.c_float) * 6),
                ("nx", C.c_int), ("ny", C.c_int), ("dx", C.c_double), ("dy", C.c_double), ("x0", C.c_double),
                ("y0", C.c_double)]


class Params(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("a_e", C.c_double), ("eps_r", C.c_double),
                ("chi_e_min", C.c_double), ("chi_e_max", C.c_double), ("chi_g_min", C.c_double),
                ("chi_g_max", C.c_double), ("k_retire", C.c_double), ("near_tol", C.c_double),
                ("step", C.c_int64), ("seed", C.c_uint64), ("flags", C.c_uint32), ("u24", C.c_int),
                ("sub_round", C.c_int)]


DP = C.POINTER(C.c_double)


class Leptons(C.Structure):
    _fields_ = [("n", C.c_int64), ("cap", C.c_int64), ("species", C.c_int),
                ("x", DP * 3), ("p", DP * 3), ("s", DP * 3), ("near", C.POINTER(C.c_uint8)),
                ("index", C.POINTER(C.c_int64)), ("tau", DP), ("tau_target", DP), ("cond", DP)]


class Photons(C.Structure):
    _fields_ = [("n", C.c_int64), ("cap", C.c_int64), ("n_prev", C.c_int64),
                ("x", DP * 3), ("k", DP * 3), ("P", DP * 3), ("id", C.POINTER(C.c_uint64)),
                ("near", C.POINTER(C.c_uint8)), ("cond", DP)]


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_emit", "n_pair", "n_prob_clamped", "n_chi_clamped",
                                         "n_norm_clamped", "n_capacity_overflow", "n_retired",
                                         "n_near_threshold", "n_lepton_steps", "n_photon_steps",
                                         "n_nonfinite")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def lib():
    global _lib
    if _lib is None and _active in _libs:
        _lib = _libs[_active]
    if _lib is None:
        L = C.CDLL(str(build(variant=_active)))
        d, i, u32, u64 = C.c_double, C.c_int, C.c_uint32, C.c_uint64
        L.orc_philox4x32_10.argtypes = [C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
        L.orc_u01_53.argtypes = [u32, u32]; L.orc_u01_53.restype = d
        L.orc_u01_24.argtypes = [u32]; L.orc_u01_24.restype = d
        L.orc_bessel3.argtypes = [d, DP]
        L.orc_nlc_w.argtypes = [d, d, d]; L.orc_nlc_w.restype = d
        L.orc_nlc_g.argtypes = [d, d, DP, DP]
        L.orc_nlc_F.argtypes = [d, d, DP, DP, DP]
        L.orc_nbw_G.argtypes = [d, d, DP, DP, DP]
        L.orc_nbw_j.argtypes = [d, d, DP, DP, DP, DP]
        L.orc_density_nu.argtypes = [i, d, d]; L.orc_density_nu.restype = d
        L.orc_rate_integral.argtypes = [i, d]; L.orc_rate_integral.restype = d
        L.orc_cdf.argtypes = [i, d, d]; L.orc_cdf.restype = d
        L.orc_ccdf.argtypes = [i, d, d]; L.orc_ccdf.restype = d
        L.orc_icdf_nu.argtypes = [i, d, d]; L.orc_icdf_nu.restype = d
        L.orc_tables_build.argtypes = [C.POINTER(Tables), C.POINTER(TableSpec), i]
        L.orc_tables_load.argtypes = [C.POINTER(Tables), C.POINTER(TableSpec), DP, DP, DP]
        L.orc_tables_free.argtypes = [C.POINTER(Tables)]
        L.orc_table_lnrate.argtypes = [C.POINTER(Tables), i, d]; L.orc_table_lnrate.restype = d
        L.orc_table_nu.argtypes = [C.POINTER(Tables), i, d, d]; L.orc_table_nu.restype = d
        L.orc_fields_eval.argtypes = [C.POINTER(Fields), DP, d, DP, DP]
        L.orc_push_one.argtypes = [i, d, DP, DP, d, u32, C.POINTER(Tables), d, DP, DP, DP]
        L.orc_scorer_gi.argtypes = [d]; L.orc_scorer_gi.restype = d
        L.orc_gfactor_ratio.argtypes = [d]; L.orc_gfactor_ratio.restype = d
        L.orc_table_gfac.argtypes = [C.POINTER(Tables), d]; L.orc_table_gfac.restype = d
        L.orc_lepton_step.argtypes = [C.POINTER(Tables), C.POINTER(Params), C.POINTER(Fields),
                                      C.POINTER(Leptons), C.POINTER(Photons), C.POINTER(Counters), i]
        L.orc_photon_step.argtypes = [C.POINTER(Tables), C.POINTER(Params), C.POINTER(Fields),
                                      C.POINTER(Photons), C.POINTER(Leptons), C.POINTER(Leptons),
                                      C.POINTER(Counters), i]
        L.orc_compact.argtypes = [C.POINTER(Photons)]
        L.orc_lepton_qed_one.argtypes = [C.POINTER(Tables), C.POINTER(Params), i, C.c_int64, DP, DP, DP,
                                         DP, DP, DP, DP, C.POINTER(u64), DP, C.POINTER(Counters)]
        L.orc_lepton_qed_one.restype = i
        L.orc_photon_qed_one.argtypes = [C.POINTER(Tables), C.POINTER(Params), u64, DP, DP, DP, DP,
                                         DP, DP, DP, DP, C.POINTER(Counters)]
        L.orc_photon_qed_one.restype = i
        L.orc_stokes_to_P.argtypes = [DP, DP, DP, DP, DP]
        L.orc_P_to_stokes.argtypes = [DP, DP, DP, DP, DP]
        L.orc_basis.argtypes = [i, d, DP, DP, DP, DP, DP, DP]; L.orc_basis.restype = d
        _libs[_active] = L
        _lib = L
    return _lib


def _v(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(DP)


# ---------------------------------------------------------------- scalar helpers
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u01_53(hi, lo):
    return lib().orc_u01_53(hi, lo)


def u01_24(hi):
    return lib().orc_u01_24(hi)


def bessel3(x):
    """(K_1/3(x), K_2/3(x), int_x^inf K_1/3) by the oracle's own quadrature / series."""
    o = (C.c_double * 3)()
    lib().orc_bessel3(float(x), o)
    return tuple(o)


def nlc_w(chi, lam, sb):
    return lib().orc_nlc_w(chi, lam, sb)


def nlc_g(chi, lam, si):
    si, psi = _v(si)
    g = np.zeros(3)
    lib().orc_nlc_g(chi, lam, psi, g.ctypes.data_as(DP))
    return g


def nlc_F(chi, lam, si, sf):
    si, a = _v(si)
    sf, b = _v(sf)
    F = np.zeros(4)
    lib().orc_nlc_F(chi, lam, a, b, F.ctypes.data_as(DP))
    return F


def nbw_G(chi, lam, se, sp):
    se, a = _v(se)
    sp, b = _v(sp)
    G = np.zeros(4)
    lib().orc_nbw_G(chi, lam, a, b, G.ctypes.data_as(DP))
    return G


def nbw_j(chi, lam, xi):
    xi, a = _v(xi)
    w0 = C.c_double()
    je, jp = np.zeros(3), np.zeros(3)
    lib().orc_nbw_j(chi, lam, a, C.byref(w0), je.ctypes.data_as(DP), jp.ctypes.data_as(DP))
    return w0.value, je, jp


def density_nu(ch, chi, nu):
    return lib().orc_density_nu(ch, chi, nu)


def rate_integral(ch, chi):
    return lib().orc_rate_integral(ch, chi)


def cdf(ch, chi, lam):
    return lib().orc_cdf(ch, chi, lam)


def ccdf(ch, chi, lam):
    return lib().orc_ccdf(ch, chi, lam)


def icdf_nu(ch, chi, rho):
    return lib().orc_icdf_nu(ch, chi, rho)


def basis(charge, eps_r, E, B, p):
    E, pE = _v(E); B, pB = _v(B); p, pp = _v(p)
    e, b, k = np.zeros(3), np.zeros(3), np.zeros(3)
    chi = lib().orc_basis(charge, eps_r, pE, pB, pp, e.ctypes.data_as(DP), b.ctypes.data_as(DP),
                          k.ctypes.data_as(DP))
    return chi, e, b, k


def stokes_to_P(xi, e, b, k):
    args = [_v(a) for a in (xi, e, b, k)]
    P = np.zeros(3)
    lib().orc_stokes_to_P(*[a[1] for a in args], P.ctypes.data_as(DP))
    return P


def P_to_stokes(P, e, b, k):
    args = [_v(a) for a in (P, e, b, k)]
    xi = np.zeros(3)
    lib().orc_P_to_stokes(*[a[1] for a in args], xi.ctypes.data_as(DP))
    return xi


def push_one(charge, a_e, E, B, dt, flags, p, s, x, tables=None, eps_r=0.0):
    """One push; with F_GCHI the anomalous moment a_e a(chi)/a(0) comes from `tables`
    (an OracleTables) at the mid-step chi (eps_r needed)."""
    E, pE = _v(E); B, pB = _v(B)
    p = np.array(p, dtype=np.float64); s = np.array(s, dtype=np.float64); x = np.array(x, dtype=np.float64)
    if (flags & F_GCHI) and tables is None:
        raise ValueError("F_GCHI needs the oracle tables")
    T = C.byref(tables.struct) if tables is not None else None
    lib().orc_push_one(charge, a_e, pE, pB, dt, flags, T, eps_r, p.ctypes.data_as(DP), s.ctypes.data_as(DP),
                       x.ctypes.data_as(DP))
    return p, s, x


def scorer_gi(z):
    """Scorer function Gi(z), z >= 0 (loop appendix)."""
    return lib().orc_scorer_gi(z)


def gfactor_ratio(chi):
    """a(chi)/a(0) of the field-dependent anomalous moment, by direct quadrature."""
    return lib().orc_gfactor_ratio(chi)


# ---------------------------------------------------------------- tables
def default_spec(n_chi_per_decade=32, n_rho=1024, rho_max=37.5,
                 nlc_range=(1e-3, 1e2), nbw_chi_min=0.05, nbw_decades=3.3125):
    """The table grid of the method contract: nodes uniform in ln chi and in rho = logit r."""
    h = np.log(10.0) / n_chi_per_decade
    n_nlc = int(round(np.log(nlc_range[1] / nlc_range[0]) / h)) + 1
    n_nbw = int(round(nbw_decades * n_chi_per_decade)) + 1
    return dict(n_chi=(n_nlc, n_nbw), lnchi0=(np.log(nlc_range[0]), np.log(nbw_chi_min)),
                dlnchi=(h, h), n_rho=n_rho, rho0=-rho_max, drho=2.0 * rho_max / (n_rho - 1))


def _spec_struct(spec):
    s = TableSpec()
    s.n_chi[0], s.n_chi[1] = spec["n_chi"]
    s.lnchi0[0], s.lnchi0[1] = spec["lnchi0"]
    s.dlnchi[0], s.dlnchi[1] = spec["dlnchi"]
    s.n_rho, s.rho0, s.drho = spec["n_rho"], spec["rho0"], spec["drho"]
    return s


class OracleTables:
    """Rate and inverse-CDF tables on the specified grid, built by the oracle's own
    quadrature (cached on disk by spec and oracle-source hash)."""

    def __init__(self, spec=None, nthreads=0, cache=True):
        self.spec = spec or default_spec()
        self.struct = Tables()
        key = hashlib.sha256((repr(sorted(self.spec.items())) + SRC.read_text()).encode()).hexdigest()[:16]
        path = CACHE / f"tables_{key}.npz"
        ss = _spec_struct(self.spec)
        if cache and path.exists():
            z = np.load(path)
            self._lnrate, self._nu, self._lngfac = z["lnrate"], z["nu"], z["lngfac"]
            lib().orc_tables_load(C.byref(self.struct), C.byref(ss), self._lnrate.ctypes.data_as(DP),
                                  self._nu.ctypes.data_as(DP), self._lngfac.ctypes.data_as(DP))
        else:
            lib().orc_tables_build(C.byref(self.struct), C.byref(ss), nthreads)
            nr = sum(self.n_chi(c) for c in range(4))
            nv = nr * self.spec["n_rho"]
            self._lnrate = np.ctypeslib.as_array(self.struct.lnrate, shape=(nr,)).copy()
            self._nu = np.ctypeslib.as_array(self.struct.nu, shape=(nv,)).copy()
            self._lngfac = np.ctypeslib.as_array(self.struct.lngfac, shape=(GF_N,)).copy()
            if cache:
                CACHE.mkdir(parents=True, exist_ok=True)
                tmp = path.with_suffix(".tmp.npz")
                np.savez(tmp, lnrate=self._lnrate, nu=self._nu, lngfac=self._lngfac)
                os.replace(tmp, path)

    def n_chi(self, ch):
        return self.spec["n_chi"][0 if ch < 2 else 1]

    def lnrate_nodes(self, ch):
        """the stored rate row: ln int w dlam at the nodes, + 8/(3 chi) in the pair rows (2, 3)"""
        o = self.struct.off_rate[ch]
        return self._lnrate[o:o + self.n_chi(ch)]

    def nu_nodes(self, ch):
        o = self.struct.off_nu[ch]
        return self._nu[o:o + self.n_chi(ch) * self.spec["n_rho"]].reshape(self.n_chi(ch), -1)

    def lnrate(self, ch, lnchi):
        return lib().orc_table_lnrate(C.byref(self.struct), ch, lnchi)

    def nu(self, ch, lnchi, rho):
        return lib().orc_table_nu(C.byref(self.struct), ch, lnchi, rho)

    def lngfac_nodes(self):
        """ln(a(chi)/a(0)) at ln chi = GF_LNCHI0 + i GF_DLNCHI, i < GF_N."""
        return self._lngfac

    def gfac(self, chi):
        """a(chi)/a(0) interpolated from the table."""
        return lib().orc_table_gfac(C.byref(self.struct), chi)

    def __del__(self):
        try:
            lib().orc_tables_free(C.byref(self.struct))
        except Exception:
            pass


# ---------------------------------------------------------------- particle sets
class SetArrays(tuple):
    """The arrays of a particle set; ``cond`` holds, per particle, the conditioning of the collapse
    axes behind its spin (leptons) or polarization (photons): how many times the rounding of the
    spectrum's terms the direction can be off (0 or 1 where no collapse was made)."""
    cond = None


def _set_arrays(vals, cond):
    t = SetArrays(vals)
    t.cond = cond
    return t


class LeptonSet:
    """SoA lepton storage (float64) with a capacity; x components may be absent."""

    def __init__(self, species, cap, track=(True, True, True), tau=False):
        self.species, self.cap, self.n = species, int(cap), 0
        self.x = [np.zeros(cap) if t else None for t in track]
        self.p = [np.zeros(cap) for _ in range(3)]
        self.s = [np.zeros(cap) for _ in range(3)]
        self.near = np.zeros(cap, dtype=np.uint8)
        self.index = None
        self.tau = np.zeros(cap) if tau else None           # optical depth and its target
        self.tau_target = np.zeros(cap) if tau else None
        self.cond = np.zeros(cap)

    def set(self, x, p, s, index=None):
        n = p.shape[1]
        assert n <= self.cap
        if index is not None:
            self.index = np.zeros(self.cap, dtype=np.int64)
            self.index[:n] = index
        for i in range(3):
            if self.x[i] is not None:
                self.x[i][:n] = x[i]
            self.p[i][:n] = p[i]
            self.s[i][:n] = s[i]
        self.n = n

    def struct(self):
        L = Leptons()
        L.n, L.cap, L.species = self.n, self.cap, self.species
        for i in range(3):
            L.x[i] = self.x[i].ctypes.data_as(DP) if self.x[i] is not None else DP()
            L.p[i] = self.p[i].ctypes.data_as(DP)
            L.s[i] = self.s[i].ctypes.data_as(DP)
        L.near = self.near.ctypes.data_as(C.POINTER(C.c_uint8))
        L.index = (self.index.ctypes.data_as(C.POINTER(C.c_int64)) if self.index is not None
                   else C.POINTER(C.c_int64)())
        L.tau = self.tau.ctypes.data_as(DP) if self.tau is not None else DP()
        L.tau_target = self.tau_target.ctypes.data_as(DP) if self.tau_target is not None else DP()
        L.cond = self.cond.ctypes.data_as(DP)
        return L

    def arrays(self):
        n = self.n
        x = np.stack([(a[:n] if a is not None else np.zeros(n)) for a in self.x])
        return _set_arrays((x, np.stack([a[:n] for a in self.p]), np.stack([a[:n] for a in self.s])),
                           self.cond[:n].copy())


class PhotonSet:
    def __init__(self, cap, track=(True, True, True)):
        self.cap, self.n, self.n_prev = int(cap), 0, 0
        self.x = [np.zeros(cap) if t else None for t in track]
        self.k = [np.zeros(cap) for _ in range(3)]
        self.P = [np.zeros(cap) for _ in range(3)]
        self.id = np.zeros(cap, dtype=np.uint64)
        self.near = np.zeros(cap, dtype=np.uint8)
        self.cond = np.zeros(cap)

    def struct(self):
        G = Photons()
        G.n, G.cap, G.n_prev = self.n, self.cap, self.n_prev
        for i in range(3):
            G.x[i] = self.x[i].ctypes.data_as(DP) if self.x[i] is not None else DP()
            G.k[i] = self.k[i].ctypes.data_as(DP)
            G.P[i] = self.P[i].ctypes.data_as(DP)
        G.id = self.id.ctypes.data_as(C.POINTER(C.c_uint64))
        G.near = self.near.ctypes.data_as(C.POINTER(C.c_uint8))
        G.cond = self.cond.ctypes.data_as(DP)
        return G

    def pull(self, G):
        self.n, self.n_prev = G.n, G.n_prev

    def arrays(self):
        n = self.n
        x = np.stack([(a[:n] if a is not None else np.zeros(n)) for a in self.x])
        return _set_arrays((x, np.stack([a[:n] for a in self.k]), np.stack([a[:n] for a in self.P]),
                            self.id[:n].copy()), self.cond[:n].copy())


def make_params(dt, eps_r, step=0, t=0.0, seed=1, flags=F_ALL, a_e=ALPHA / (2 * np.pi),
                chi_e_min=1e-3, chi_e_max=1e2, chi_g_min=0.05, chi_g_max=1e2, k_retire=0.0,
                near_tol=1e-9, u24=False):
    P = Params()
    P.t, P.dt, P.a_e, P.eps_r = t, dt, a_e, eps_r
    P.chi_e_min, P.chi_e_max, P.chi_g_min, P.chi_g_max = chi_e_min, chi_e_max, chi_g_min, chi_g_max
    P.k_retire, P.near_tol, P.step, P.seed, P.flags, P.u24 = k_retire, near_tol, step, seed, flags, int(u24)
    return P


def make_fields(kind=FIELD_UNIFORM, E0=(0, 0, 0), B0=(0, 0, 0), a0=0.0, phase_len=0.0, grid=None, dx=1.0, dy=1.0,
                x0=0.0, y0=0.0):
    """grid: float32 array (6, ny, nx) of Ex, Ey, Ez, Bx, By, Bz at the nodes (kind FIELD_GRID2D);
    the returned structure keeps a reference to it"""
    F = Fields()
    F.kind = kind
    for i in range(3):
        F.E0[i], F.B0[i] = E0[i], B0[i]
    F.a0, F.phase_len = a0, phase_len
    if grid is not None:
        g = np.ascontiguousarray(grid, dtype=np.float32)
        F._grid = g
        F.ny, F.nx = g.shape[1], g.shape[2]
        for c in range(6):
            F.grid[c] = g[c].ctypes.data_as(C.POINTER(C.c_float))
        F.dx, F.dy, F.x0, F.y0 = dx, dy, x0, y0
    return F


def fields_eval(F, x, t):
    x, px = _v(x)
    E, B = np.zeros(3), np.zeros(3)
    lib().orc_fields_eval(C.byref(F), px, t, E.ctypes.data_as(DP), B.ctypes.data_as(DP))
    return E, B


def lepton_step(tables, params, fields, L: LeptonSet, G: PhotonSet, ctr: Counters, nthreads=0):
    Ls, Gs = L.struct(), G.struct()
    lib().orc_lepton_step(C.byref(tables.struct), C.byref(params), C.byref(fields), C.byref(Ls),
                          C.byref(Gs), C.byref(ctr), nthreads)
    G.pull(Gs)


def photon_step(tables, params, fields, G: PhotonSet, Le: LeptonSet, Lp: LeptonSet, ctr: Counters,
                nthreads=0):
    Gs, Es, Ps = G.struct(), Le.struct(), Lp.struct()
    lib().orc_photon_step(C.byref(tables.struct), C.byref(params), C.byref(fields), C.byref(Gs),
                          C.byref(Es), C.byref(Ps), C.byref(ctr), nthreads)
    G.pull(Gs)
    Le.n, Lp.n = Es.n, Ps.n


def compact(G: PhotonSet):
    Gs = G.struct()
    lib().orc_compact(C.byref(Gs))
    G.pull(Gs)


def lepton_qed_one(tables, params, species, index, E, B, x, p, s, tau2=None):
    """tau2: optional [tau, tau*] (optical-depth decision), updated in place"""
    E, pE = _v(E); B, pB = _v(B); x, px = _v(x)
    p = np.array(p, dtype=np.float64); s = np.array(s, dtype=np.float64)
    k, P = np.zeros(3), np.zeros(3)
    pid = C.c_uint64()
    ctr = Counters()
    pt = tau2.ctypes.data_as(DP) if tau2 is not None else DP()
    r = lib().orc_lepton_qed_one(C.byref(tables.struct), C.byref(params), species, index, pE, pB, px,
                                 p.ctypes.data_as(DP), s.ctypes.data_as(DP), k.ctypes.data_as(DP),
                                 P.ctypes.data_as(DP), C.byref(pid), pt, C.byref(ctr))
    return r, p, s, k, P, pid.value, ctr.as_dict()


def photon_qed_one(tables, params, pid, E, B, k, P):
    E, pE = _v(E); B, pB = _v(B); k, pk = _v(k)
    P = np.array(P, dtype=np.float64)
    out = [np.zeros(3) for _ in range(4)]
    ctr = Counters()
    r = lib().orc_photon_qed_one(C.byref(tables.struct), C.byref(params), C.c_uint64(pid), pE, pB, pk,
                                 P.ctypes.data_as(DP), *[o.ctypes.data_as(DP) for o in out], C.byref(ctr))
    return (r, P, *out, ctr.as_dict())
