"""MI355X (gfx950) spin- and polarization-resolved strong-field QED particle step.

Thin Python binding of the C ABI in ``include/qedspin.h`` (``libqedspin.so``): argument
marshalling only.  Every step of the method runs in the HIP kernels of ``csrc/``; PyTorch
provides device memory and streams.  The product path has no CPU fallback: if the library
is not built, or no GPU is present, calls raise.

Names follow the C ABI: qed_init_tables, qed_free_tables, qed_tables_download,
qed_workspace_size, qed_push_spin, qed_emit, qed_pair, qed_compact_workspace_size,
qed_compact.  ``LeptonBuffers`` / ``PhotonBuffers`` hold SoA torch tensors and build the
ABI views; ``sim.Simulation`` strings the calls into time steps.
"""
from __future__ import annotations

import ctypes as C
import math
from pathlib import Path

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libqedspin.so"

ALPHA = 7.2973525693e-3

QED_OK, QED_ERR_INVALID, QED_ERR_HIP, QED_ERR_CAPACITY, QED_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
QED_F64, QED_F32 = 0, 1
QED_PUSH, QED_TBMT, QED_EMIT, QED_RECOIL = 1 << 0, 1 << 1, 1 << 2, 1 << 3
QED_SPIN, QED_NOEMIT, QED_PHOTON_POL, QED_MEAN = 1 << 4, 1 << 5, 1 << 6, 1 << 7
QED_PAIR, QED_NOPAIR, QED_PAIR_SPIN = 1 << 8, 1 << 9, 1 << 10
QED_OPTICAL_DEPTH = 1 << 11
QED_REJECTION = 1 << 12
QED_G_CHI = 1 << 13
QED_SUBCYCLE = 1 << 14
QED_ALL = (QED_PUSH | QED_TBMT | QED_EMIT | QED_RECOIL | QED_SPIN | QED_NOEMIT | QED_PHOTON_POL
           | QED_PAIR | QED_NOPAIR | QED_PAIR_SPIN)
QED_FIELD_UNIFORM, QED_FIELD_PLANE_LP, QED_FIELD_GRID2D, QED_FIELD_ROTATING_E = 0, 1, 2, 3

ABI_SYMBOLS = ("qed_init_tables", "qed_last_error", "qed_free_tables", "qed_tables_download",
               "qed_tables_download_gfac", "qed_workspace_size",
               "qed_push_spin", "qed_emit", "qed_emit_noalloc", "qed_pair", "qed_compact_workspace_size", "qed_compact",
               "qed_profile_start", "qed_profile_stop", "qed_clock_advance", "qed_plan_create", "qed_plan_step",
               "qed_plan_blocks", "qed_plan_destroy", "qed_surrogate_n_params", "qed_surrogate_create",
               "qed_surrogate_norm", "qed_surrogate_train", "qed_surrogate_gradient", "qed_surrogate_eval",
               "qed_surrogate_get_params", "qed_surrogate_set_params", "qed_surrogate_destroy",
               "qed_surrogate_judge", "qed_surrogate_get_info")


class QedError(RuntimeError):
    pass


# ------------------------------------------------------------------ ABI structs
class TableGrid(C.Structure):
    _fields_ = [("n_chi", C.c_int * 2), ("lnchi0", C.c_double * 2), ("dlnchi", C.c_double * 2),
                ("n_rho", C.c_int), ("rho0", C.c_double), ("drho", C.c_double)]


class TableParams(C.Structure):
    _fields_ = [("grid", TableGrid), ("precision", C.c_int)]


class Leptons(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("d_count", C.c_void_p), ("species", C.c_int),
                ("x", C.c_void_p * 3), ("p", C.c_void_p * 3), ("s", C.c_void_p * 3),
                ("tau", C.c_void_p), ("tau_target", C.c_void_p)]


class Photons(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("d_count", C.c_void_p), ("d_count_prev", C.c_void_p),
                ("x", C.c_void_p * 3), ("k", C.c_void_p * 3), ("P", C.c_void_p * 3), ("id", C.c_void_p)]


class Fields(C.Structure):
    _fields_ = [("kind", C.c_int), ("E0", C.c_double * 3), ("B0", C.c_double * 3),
                ("a0", C.c_double), ("phase_len", C.c_double), ("grid", C.c_void_p * 6), ("nx", C.c_int),
                ("ny", C.c_int), ("dx", C.c_double), ("dy", C.c_double), ("x0", C.c_double), ("y0", C.c_double)]


class StepParams(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("a_e", C.c_double), ("eps_r", C.c_double),
                ("chi_e_min", C.c_double), ("chi_e_max", C.c_double), ("chi_g_min", C.c_double),
                ("chi_g_max", C.c_double), ("k_retire", C.c_double), ("step", C.c_int64),
                ("seed", C.c_uint64), ("flags", C.c_uint32), ("d_clock", C.c_void_p)]


COUNTER_NAMES = ("n_emit", "n_pair", "n_prob_clamped", "n_chi_clamped", "n_norm_clamped",
                 "n_capacity_overflow", "n_retired", "n_lepton_steps", "n_photon_steps", "n_photon_qed",
                 "n_nonfinite")


class Instance(C.Structure):
    _fields_ = [("electrons", Leptons), ("positrons", Leptons), ("photons", Photons), ("fields", Fields),
                ("params", StepParams), ("d_counters", C.c_void_p)]


class PlanConfig(C.Structure):
    _fields_ = [("particles_per_block", C.c_int), ("max_blocks_per_set", C.c_int), ("icdf_nlc", C.c_void_p),
                ("icdf_nbw", C.c_void_p), ("process_group", C.c_int), ("photon_variant", C.c_int)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char_p), ("calls", C.c_longlong), ("total_ms", C.c_double)]

_lib = None


def lib():
    """Load libqedspin.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise QedError(f"{LIB_PATH} is missing: build it with paper_2511_08929_amd/build.py "
                           "(there is no CPU fallback)")
        # torch's HIP runtime must be the one resident in the process: it is loaded under the
        # same soname, so libqedspin.so then binds to it instead of a second copy
        import torch  # noqa: F401
        L = C.CDLL(str(LIB_PATH))
        P, vp, i64, sz = C.POINTER, C.c_void_p, C.c_int64, C.c_size_t
        L.qed_init_tables.argtypes = [P(TableParams), vp, P(vp)]
        L.qed_free_tables.argtypes = [vp]
        L.qed_last_error.argtypes = []
        L.qed_last_error.restype = C.c_char_p
        L.qed_tables_download.argtypes = [vp, vp, P(i64), vp, P(i64)]
        L.qed_tables_download_gfac.argtypes = [vp, vp, P(i64)]
        L.qed_workspace_size.argtypes = [i64]; L.qed_workspace_size.restype = sz
        L.qed_push_spin.argtypes = [P(Leptons), P(Fields), P(StepParams), vp, vp]
        L.qed_emit.argtypes = [vp, P(Leptons), P(Fields), P(StepParams), P(Photons), vp, vp, sz, vp]
        L.qed_emit_noalloc.argtypes = [vp, P(Leptons), P(Fields), P(StepParams), P(Photons), vp, vp]
        L.qed_pair.argtypes = [vp, P(Photons), P(Fields), P(StepParams), P(Leptons), P(Leptons), vp, vp, sz, vp]
        L.qed_compact_workspace_size.argtypes = [P(Photons), C.c_int]; L.qed_compact_workspace_size.restype = sz
        L.qed_compact.argtypes = [P(Photons), C.c_int, vp, sz, vp]
        L.qed_clock_advance.argtypes = [vp, vp]
        L.qed_plan_create.argtypes = [vp, C.c_int, P(Instance), P(PlanConfig), P(vp)]
        L.qed_plan_step.argtypes = [vp, vp]
        L.qed_plan_blocks.argtypes = [vp]; L.qed_plan_blocks.restype = i64
        L.qed_plan_destroy.argtypes = [vp]
        f = C.c_float
        L.qed_surrogate_n_params.argtypes = []; L.qed_surrogate_n_params.restype = i64
        L.qed_surrogate_create.argtypes = [vp, C.c_int, C.c_uint64, P(vp)]
        L.qed_surrogate_norm.argtypes = [vp, P(f)]
        L.qed_surrogate_train.argtypes = [vp, C.c_int, C.c_int, f, vp, vp]
        L.qed_surrogate_gradient.argtypes = [vp, vp, vp, i64, vp, vp]
        L.qed_surrogate_eval.argtypes = [vp, vp, i64, C.c_int, vp, vp]
        L.qed_surrogate_judge.argtypes = [vp, f, C.c_int, vp, P(i64), vp]
        L.qed_surrogate_get_info.argtypes = [vp, P(SurrogateInfo)]
        L.qed_surrogate_get_params.argtypes = [vp, vp, vp]
        L.qed_surrogate_set_params.argtypes = [vp, vp, vp]
        L.qed_surrogate_destroy.argtypes = [vp]
        L.qed_profile_start.argtypes = []
        L.qed_profile_stop.argtypes = [P(KernelTime), C.c_int, P(C.c_int)]
        for name in ABI_SYMBOLS:
            if name not in ("qed_workspace_size", "qed_compact_workspace_size", "qed_last_error", "qed_plan_blocks",
                            "qed_surrogate_n_params"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status, what):
    if status != QED_OK:
        detail = lib().qed_last_error().decode() if status in (QED_ERR_HIP, QED_ERR_CAPACITY) else ""
        raise QedError(f"{what} failed with status {status} {detail}")


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


# ------------------------------------------------------------------ table grid
def contract_grid(n_chi_per_decade=32, n_rho=1024, rho_max=37.5, nlc_range=(1e-3, 1e2),
                  nbw_chi_min=0.05, nbw_decades=3.3125):
    """The table grid of the method contract: nodes uniform in ln chi and in rho = logit r."""
    h = math.log(10.0) / n_chi_per_decade
    n_nlc = int(round(math.log(nlc_range[1] / nlc_range[0]) / h)) + 1
    n_nbw = int(round(nbw_decades * n_chi_per_decade)) + 1
    return dict(n_chi=(n_nlc, n_nbw), lnchi0=(math.log(nlc_range[0]), math.log(nbw_chi_min)),
                dlnchi=(h, h), n_rho=n_rho, rho0=-rho_max, drho=2.0 * rho_max / (n_rho - 1))


# ------------------------------------------------------------------ ABI wrappers
class Tables:
    """Owner of a qed_tables handle (qed_init_tables / qed_free_tables)."""

    def __init__(self, grid=None, precision=QED_F64, stream=None):
        g = grid or contract_grid()
        p = TableParams()
        p.grid.n_chi[0], p.grid.n_chi[1] = g["n_chi"]
        p.grid.lnchi0[0], p.grid.lnchi0[1] = g["lnchi0"]
        p.grid.dlnchi[0], p.grid.dlnchi[1] = g["dlnchi"]
        p.grid.n_rho, p.grid.rho0, p.grid.drho = g["n_rho"], g["rho0"], g["drho"]
        p.precision = precision
        self.grid, self.precision = g, precision
        h = C.c_void_p()
        _check(lib().qed_init_tables(C.byref(p), _stream_ptr(stream), C.byref(h)), "qed_init_tables")
        self.handle = h

    def download(self):
        import numpy as np
        nr, nv = C.c_int64(), C.c_int64()
        _check(lib().qed_tables_download(self.handle, None, C.byref(nr), None, C.byref(nv)), "qed_tables_download")
        lnrate, nu = np.zeros(nr.value), np.zeros(nv.value)
        _check(lib().qed_tables_download(self.handle, lnrate.ctypes.data, None, nu.ctypes.data, None),
               "qed_tables_download")
        return lnrate, nu

    def download_gfac(self):
        """ln(a(chi)/a(0)) nodes of the field-dependent anomalous moment (QED_G_CHI)."""
        import numpy as np
        n = C.c_int64()
        _check(lib().qed_tables_download_gfac(self.handle, None, C.byref(n)), "qed_tables_download_gfac")
        out = np.zeros(n.value)
        _check(lib().qed_tables_download_gfac(self.handle, out.ctypes.data, None), "qed_tables_download_gfac")
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().qed_free_tables(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qed_workspace_size(max_particles):
    return int(lib().qed_workspace_size(int(max_particles)))


class LeptonBuffers:
    """Device SoA storage for one lepton species (torch tensors) and its ABI view."""

    def __init__(self, species, capacity, dtype, device="cuda", track=(True, True, True), tau=False):
        import torch
        self.species, self.capacity, self.dtype = species, int(capacity), dtype
        self.x = [torch.zeros(capacity, dtype=dtype, device=device) if t else None for t in track]
        self.p = [torch.zeros(capacity, dtype=dtype, device=device) for _ in range(3)]
        self.s = [torch.zeros(capacity, dtype=dtype, device=device) for _ in range(3)]
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        # optical depth and its target (FP64 in both precisions), for QED_OPTICAL_DEPTH
        self.tau = torch.zeros(capacity, dtype=torch.float64, device=device) if tau else None
        self.tau_target = torch.zeros(capacity, dtype=torch.float64, device=device) if tau else None

    def load(self, x, p, s):
        import torch
        n = p.shape[1]
        assert n <= self.capacity
        for i in range(3):
            if self.x[i] is not None:
                self.x[i][:n] = torch.as_tensor(x[i], dtype=self.dtype)
            self.p[i][:n] = torch.as_tensor(p[i], dtype=self.dtype)
            self.s[i][:n] = torch.as_tensor(s[i], dtype=self.dtype)
        self.count.fill_(n)

    def view(self):
        if getattr(self, "_view", None) is not None and self._view.capacity == self.capacity:
            return self._view
        v = Leptons()
        v.capacity, v.d_count, v.species = self.capacity, self.count.data_ptr(), self.species
        for i in range(3):
            v.x[i] = self.x[i].data_ptr() if self.x[i] is not None else None
            v.p[i] = self.p[i].data_ptr()
            v.s[i] = self.s[i].data_ptr()
        v.tau = self.tau.data_ptr() if self.tau is not None else None
        v.tau_target = self.tau_target.data_ptr() if self.tau_target is not None else None
        self._view = v
        return v

    def n(self):
        return int(self.count.item())

    def arrays(self):
        import numpy as np
        n = self.n()
        x = np.stack([(a[:n].double().cpu().numpy() if a is not None else np.zeros(n)) for a in self.x])
        return (x, np.stack([a[:n].double().cpu().numpy() for a in self.p]),
                np.stack([a[:n].double().cpu().numpy() for a in self.s]))

    def tau_arrays(self):
        n = self.n()
        return self.tau[:n].cpu().numpy(), self.tau_target[:n].cpu().numpy()


class PhotonBuffers:
    def __init__(self, capacity, dtype, device="cuda", track=(True, True, True)):
        import torch
        self.capacity, self.dtype = int(capacity), dtype
        self.x = [torch.zeros(capacity, dtype=dtype, device=device) if t else None for t in track]
        self.k = [torch.zeros(capacity, dtype=dtype, device=device) for _ in range(3)]
        self.P = [torch.zeros(capacity, dtype=dtype, device=device) for _ in range(3)]
        self.id = torch.zeros(capacity, dtype=torch.int64, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.count_prev = torch.zeros(1, dtype=torch.int64, device=device)

    def load(self, x, k, P, ids, n_prev=None):
        """Store n photons (x: (3, n) or None, k, P: (3, n), ids: (n,) uint64) at slots [0, n);
        count = n, count_prev = n_prev (default n: every stored photon is stepped next)."""
        import numpy as np
        import torch
        n = k.shape[1]
        assert n <= self.capacity
        for i in range(3):
            if self.x[i] is not None:
                self.x[i][:n] = torch.as_tensor(x[i], dtype=self.dtype)
            self.k[i][:n] = torch.as_tensor(k[i], dtype=self.dtype)
            self.P[i][:n] = torch.as_tensor(P[i], dtype=self.dtype)
        self.id[:n] = torch.as_tensor(np.ascontiguousarray(ids, dtype=np.uint64).view(np.int64))
        self.count.fill_(n)
        self.count_prev.fill_(n if n_prev is None else n_prev)

    def view(self):
        if getattr(self, "_view", None) is not None and self._view.capacity == self.capacity:
            return self._view
        v = Photons()
        v.capacity, v.d_count, v.d_count_prev = self.capacity, self.count.data_ptr(), self.count_prev.data_ptr()
        for i in range(3):
            v.x[i] = self.x[i].data_ptr() if self.x[i] is not None else None
            v.k[i] = self.k[i].data_ptr()
            v.P[i] = self.P[i].data_ptr()
        v.id = self.id.data_ptr()
        self._view = v
        return v

    def n(self):
        return int(self.count.item())

    def arrays(self):
        import numpy as np
        n = self.n()
        x = np.stack([(a[:n].double().cpu().numpy() if a is not None else np.zeros(n)) for a in self.x])
        return (x, np.stack([a[:n].double().cpu().numpy() for a in self.k]),
                np.stack([a[:n].double().cpu().numpy() for a in self.P]),
                self.id[:n].cpu().numpy().view(np.uint64))


def make_fields(kind=QED_FIELD_UNIFORM, E0=(0, 0, 0), B0=(0, 0, 0), a0=0.0, phase_len=0.0, grid=None, dx=1.0, dy=1.0,
                x0=0.0, y0=0.0):
    """grid (QED_FIELD_GRID2D): float32 device tensor (6, ny, nx) of Ex, Ey, Ez, Bx, By, Bz at the
    nodes; the returned structure keeps a reference to it"""
    f = Fields()
    f.kind = kind
    for i in range(3):
        f.E0[i], f.B0[i] = E0[i], B0[i]
    f.a0, f.phase_len = a0, phase_len
    if grid is not None:
        import torch
        g = grid.contiguous()
        assert g.dtype == torch.float32 and g.dim() == 3 and g.shape[0] == 6 and g.is_cuda
        f._grid = g
        f.ny, f.nx = int(g.shape[1]), int(g.shape[2])
        for c in range(6):
            f.grid[c] = g[c].data_ptr()
        f.dx, f.dy, f.x0, f.y0 = dx, dy, x0, y0
    return f


def make_step(dt, eps_r, step=0, t=0.0, seed=1, flags=QED_ALL, a_e=ALPHA / (2 * math.pi), chi_e_min=1e-3,
              chi_e_max=1e2, chi_g_min=0.05, chi_g_max=1e2, k_retire=0.0):
    p = StepParams()
    p.t, p.dt, p.a_e, p.eps_r = t, dt, a_e, eps_r
    p.chi_e_min, p.chi_e_max, p.chi_g_min, p.chi_g_max, p.k_retire = chi_e_min, chi_e_max, chi_g_min, chi_g_max, k_retire
    p.step, p.seed, p.flags = step, seed, flags
    return p


def qed_push_spin(leptons: LeptonBuffers, fields, step, tables: Tables, stream=None):
    v = leptons.view()
    _check(lib().qed_push_spin(C.byref(v), C.byref(fields), C.byref(step), tables.handle, _stream_ptr(stream)),
           "qed_push_spin")


def qed_emit(tables: Tables, leptons: LeptonBuffers, fields, step, photons: PhotonBuffers, counters, workspace,
             stream=None):
    lv, pv = leptons.view(), photons.view()
    _check(lib().qed_emit(tables.handle, C.byref(lv), C.byref(fields), C.byref(step), C.byref(pv), _ptr(counters),
                          _ptr(workspace), workspace.numel() * workspace.element_size(), _stream_ptr(stream)),
           "qed_emit")


QED_NOALLOC_MAX_LEPTONS = 4194304


def qed_emit_noalloc(tables: Tables, leptons: LeptonBuffers, fields, step, photons: PhotonBuffers, counters,
                     stream=None):
    """qed_emit with the library's static per-device scratch instead of a workspace (no allocation);
    lepton capacity up to QED_NOALLOC_MAX_LEPTONS.  Calls that overlap on one GPU race."""
    lv, pv = leptons.view(), photons.view()
    _check(lib().qed_emit_noalloc(tables.handle, C.byref(lv), C.byref(fields), C.byref(step), C.byref(pv),
                                  _ptr(counters), _stream_ptr(stream)), "qed_emit_noalloc")


def qed_pair(tables: Tables, photons: PhotonBuffers, fields, step, electrons: LeptonBuffers,
             positrons: LeptonBuffers, counters, workspace, stream=None):
    gv, ev, pv = photons.view(), electrons.view(), positrons.view()
    _check(lib().qed_pair(tables.handle, C.byref(gv), C.byref(fields), C.byref(step), C.byref(ev), C.byref(pv),
                          _ptr(counters), _ptr(workspace), workspace.numel() * workspace.element_size(),
                          _stream_ptr(stream)), "qed_pair")


def qed_compact_workspace_size(photons: PhotonBuffers, precision):
    v = photons.view()
    return int(lib().qed_compact_workspace_size(C.byref(v), precision))


def qed_compact(photons: PhotonBuffers, precision, workspace, stream=None):
    v = photons.view()
    _check(lib().qed_compact(C.byref(v), precision, _ptr(workspace), workspace.numel() * workspace.element_size(),
                             _stream_ptr(stream)), "qed_compact")


def new_counters(device="cuda"):
    import torch
    return torch.zeros(len(COUNTER_NAMES), dtype=torch.int64, device=device)


def counters_dict(ctr):
    return {n: int(v) for n, v in zip(COUNTER_NAMES, ctr.cpu().tolist())}


def new_workspace(nbytes, device="cuda"):
    import torch
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def qed_profile_start():
    _check(lib().qed_profile_start(), "qed_profile_start")


def qed_profile_stop():
    """{kernel name: (calls, total ms)} of the launches since qed_profile_start."""
    buf = (KernelTime * 32)()
    n = C.c_int()
    _check(lib().qed_profile_stop(buf, 32, C.byref(n)), "qed_profile_stop")
    return {buf[i].name.decode(): (int(buf[i].calls), float(buf[i].total_ms)) for i in range(min(n.value, 32))}


def qed_clock_advance(clock, stream=None):
    _check(lib().qed_clock_advance(_ptr(clock), _stream_ptr(stream)), "qed_clock_advance")


class Plan:
    """qed_plan over instances given as (electrons, positrons, photons, fields, step params, counters).
    The buffers must stay alive (and unmoved) for the plan's lifetime; step params need d_clock."""

    def __init__(self, tables: Tables, instances, particles_per_block=0, max_blocks_per_set=0, surrogates=(None, None),
                 process_group=0, photon_variant=0):
        n = len(instances)
        arr = (Instance * n)()
        self._keep = []
        for j, (e, p, g, fields, step, ctr) in enumerate(instances):
            if not step.d_clock:
                raise QedError("a plan needs step params with d_clock")
            arr[j].electrons = e.view()
            arr[j].positrons = p.view()
            arr[j].photons = g.view()
            arr[j].fields = fields
            arr[j].params = step
            arr[j].d_counters = ctr.data_ptr()
            self._keep.append((e, p, g, ctr))
        cfg = PlanConfig(particles_per_block, max_blocks_per_set,
                         surrogates[0].handle if surrogates[0] is not None else None,
                         surrogates[1].handle if surrogates[1] is not None else None, process_group, photon_variant)
        self._keep.append(surrogates)
        h = C.c_void_p()
        _check(lib().qed_plan_create(tables.handle, n, arr, C.byref(cfg), C.byref(h)), "qed_plan_create")
        self.handle = h
        self.blocks = int(lib().qed_plan_blocks(h))

    def step(self, stream=None):
        _check(lib().qed_plan_step(self.handle, _stream_ptr(stream)), "qed_plan_step")

    def close(self):
        if self.handle:
            lib().qed_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SURROGATE_AS_USED, SURROGATE_NETWORK, SURROGATE_BASE = 0, 1, 2


class SurrogateInfo(C.Structure):
    _fields_ = [("process", C.c_int), ("n_params", C.c_int), ("in_m", C.c_float), ("in_h", C.c_float),
                ("rho_s", C.c_float), ("out_s", C.c_float), ("base_lnchi0", C.c_float), ("base_dlnchi", C.c_float),
                ("base_n_chi", C.c_int), ("base_rho0", C.c_float), ("base_drho", C.c_float), ("base_n_rho", C.c_int),
                ("n_cells", C.c_int64), ("n_masked", C.c_int64), ("bound", C.c_float),
                ("bytes_network", C.c_int64), ("bytes_base", C.c_int64), ("bytes_mask", C.c_int64)]


class Surrogate:
    """qed_surrogate: the learned inverse CDF of one process (0 = NLC, 1 = NBW): a coarse table
    plus a network for its residual, judged by the fine tables (table inverse CDF in the cells
    the judgement marks)."""

    def __init__(self, tables: Tables, process, seed=1):
        h = C.c_void_p()
        _check(lib().qed_surrogate_create(tables.handle, process, seed, C.byref(h)), "qed_surrogate_create")
        self.handle, self.tables, self.process = h, tables, process
        self.n_params = int(lib().qed_surrogate_n_params())

    def norm(self):
        out = (C.c_float * 4)()
        _check(lib().qed_surrogate_norm(self.handle, out), "qed_surrogate_norm")
        return tuple(float(v) for v in out)

    def train(self, steps, tiles_per_wave=2, lr=1e-3, stream=None):
        """run `steps` Adam steps; returns the per-step mean squared errors (device tensor)"""
        import torch
        loss = torch.zeros(max(steps, 1), dtype=torch.float32, device="cuda")
        _check(lib().qed_surrogate_train(self.handle, steps, tiles_per_wave, lr, _ptr(loss), _stream_ptr(stream)),
               "qed_surrogate_train")
        return loss[:steps]

    def fit(self, schedule=((2e-3, 3000), (5e-4, 3000), (1e-4, 2000)), tiles_per_wave=1, stream=None):
        """the standard training: Adam at piecewise-constant learning rates; returns the losses"""
        import torch
        return torch.cat([self.train(n, tiles_per_wave, lr, stream) for lr, n in schedule])

    def gradient(self, x, y, stream=None):
        """gradient of sum (y(x) - y)^2 over the samples (x: (n, 3) float32 device, y: (n,) targets
        of the network output); the returned tensor has n_params + 1 entries, the last one the sum
        of squares"""
        import torch
        g = torch.zeros(self.n_params + 1, dtype=torch.float32, device="cuda")
        _check(lib().qed_surrogate_gradient(self.handle, _ptr(x), _ptr(y), x.shape[0], _ptr(g), _stream_ptr(stream)),
               "qed_surrogate_gradient")
        return g

    def eval(self, x, mode=SURROGATE_AS_USED, stream=None):
        """nu at raw inputs x (n, 3) = (ln chi, rho, c): as the step uses it, the network without
        the fallback (SURROGATE_NETWORK) or the coarse table alone (SURROGATE_BASE)"""
        import torch
        nu = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().qed_surrogate_eval(self.handle, _ptr(x), x.shape[0], mode, _ptr(nu), _stream_ptr(stream)),
               "qed_surrogate_eval")
        return nu

    def judge(self, bound, points_per_axis=8, stream=None):
        """mark the coarse cells whose largest sampled error against the fine tables exceeds
        `bound`; returns (per-cell largest error as a numpy array, number marked)"""
        import numpy as np
        info = self.info()
        err = np.zeros(info.n_cells, dtype=np.float32)
        nm = C.c_int64(0)
        _check(lib().qed_surrogate_judge(self.handle, bound, points_per_axis, err.ctypes.data_as(C.c_void_p),
                                         C.byref(nm), _stream_ptr(stream)), "qed_surrogate_judge")
        return err, int(nm.value)

    def info(self):
        out = SurrogateInfo()
        _check(lib().qed_surrogate_get_info(self.handle, C.byref(out)), "qed_surrogate_get_info")
        return out

    def get_params(self, stream=None):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().qed_surrogate_get_params(self.handle, _ptr(p), _stream_ptr(stream)), "qed_surrogate_get_params")
        return p

    def set_params(self, p, stream=None):
        _check(lib().qed_surrogate_set_params(self.handle, _ptr(p), _stream_ptr(stream)), "qed_surrogate_set_params")

    def close(self):
        if self.handle:
            lib().qed_surrogate_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
