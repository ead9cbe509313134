"""Seeded synthetic workloads shaped like the laser-electron collisions of arXiv 2511.08929.

This module only draws initial particle states and states field / step parameters.  It
holds none of the QED method's arithmetic, and it is shared by the oracle tests, the GPU
parity tests and the benchmark.  All randomness comes from ``numpy.random.Generator``
(PCG64) seeded per workload.

Units: time in 1/omega_r, length in c/omega_r, momentum in m c, fields in m c omega_r / e,
with omega_r the angular frequency of a lambda = 0.8 um laser.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# physical constants (CODATA 2018)
HC_EV_NM = 1239.841984332
MEC2_EV = 510998.95
C_LIGHT = 299792458.0
LAMBDA_UM = 0.8
EPS_R = HC_EV_NM / (LAMBDA_UM * 1000.0) / MEC2_EV      # hbar omega_r / (m c^2)
OMEGA_R = 2.0 * math.pi * C_LIGHT / (LAMBDA_UM * 1e-6)  # rad/s

FIELD_UNIFORM, FIELD_PLANE_LP, FIELD_GRID2D, FIELD_ROTATING_E = 0, 1, 2, 3


@dataclass
class Workload:
    name: str
    n: int                      # primary electrons
    steps: int
    dt: float
    seed: int
    field_kind: int
    E0: tuple = (0.0, 0.0, 0.0)
    B0: tuple = (0.0, 0.0, 0.0)
    a0: float = 0.0
    phase_len: float = 0.0
    track: tuple = (True, True, True)   # which position components matter
    pair: bool = False
    k_retire: float = 0.0               # photon energy (m c^2) below which chi_gamma < chi_min always
    x: np.ndarray = field(default=None, repr=False)
    p: np.ndarray = field(default=None, repr=False)
    s: np.ndarray = field(default=None, repr=False)
    extra: dict = field(default_factory=dict)


def c1(n: int = 10_000, seed: int = 1, steps: int = 1000) -> Workload:
    """Test-particle case: gamma0 = 2000 along +x, spins +y, uniform B_z with chi_e = 1,
    no E, dt = 1/100 of the relativistic gyro period, no pair production."""
    gamma0 = 2000.0
    pmag = math.sqrt(gamma0 * gamma0 - 1.0)
    Bz = 1.0 / (EPS_R * pmag)                 # chi_e = eps_r |p x B| = 1
    period = 2.0 * math.pi * gamma0 / Bz      # omega_c = B / gamma in these units
    x = np.zeros((3, n))
    p = np.zeros((3, n)); p[0] = pmag
    s = np.zeros((3, n)); s[1] = 1.0
    return Workload("c1_test_particle_uniform_B", n, steps, 0.01 * period, seed, FIELD_UNIFORM,
                    B0=(0.0, 0.0, Bz), track=(False, False, False), pair=False, k_retire=0.0,
                    x=x, p=p, s=s, extra=dict(gamma0=gamma0, Bz=Bz, gyro_period=period))


def sin2_phase_len(fwhm_fs: float) -> float:
    """Total length (in laser phase) of a sin^2 field envelope whose intensity FWHM is fwhm_fs."""
    th = math.asin(2.0 ** -0.25)               # sin^4 = 1/2
    return OMEGA_R * fwhm_fs * 1e-15 / (1.0 - 2.0 * th / math.pi)


def c2(n: int = 1_000_000, seed: int = 2, steps: int = 3000, a0: float = 100.0,
       gamma_mean: float = 4000.0, gamma_spread: float = 0.05) -> Workload:
    """Head-on collision: gamma0 ~ N(4000, 5 %), 1 mrad Gaussian angular spread, spins +/-y
    with equal probability, LP plane wave along -x with a0 = 100, sin^2 envelope of 30 fs
    intensity FWHM, dt = lambda/(100 c), 3000 steps, both QED channels on."""
    rng = np.random.default_rng(seed)
    gam = rng.normal(gamma_mean, gamma_spread * gamma_mean, n)
    gam = np.maximum(gam, 2.0)
    ty = rng.normal(0.0, 1e-3, n)
    tz = rng.normal(0.0, 1e-3, n)
    d = np.stack([np.ones(n), ty, tz])
    d /= np.linalg.norm(d, axis=0)
    p = d * np.sqrt(gam * gam - 1.0)
    sgn = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    s = np.zeros((3, n)); s[1] = sgn
    x = np.zeros((3, n)); x[0] = rng.uniform(-2.0 * math.pi, 0.0, n)
    chi_g_min = 0.05
    return Workload("c2_head_on_lp_a0_100", n, steps, 2.0 * math.pi / 100.0, seed, FIELD_PLANE_LP,
                    a0=a0, phase_len=sin2_phase_len(30.0), track=(True, False, False), pair=True,
                    k_retire=chi_g_min / (2.0 * a0 * EPS_R), x=x, p=p, s=s)


def c3_grid(nx: int = 4096, ny: int = 1024, a0: float = 200.0, noise: float = 0.01, seed: int = 3):
    """Field snapshot of the grid workload: two counter-propagating circularly polarized waves along
    +x and -x, each of amplitude a0 (lambda = 0.8 um), at t = 0 on a periodic 2-D grid of cell
    size lambda/40, plus noise * a0 * N(0, 1) at every node and component.  Returns a float32
    array (6, ny, nx) of Ex, Ey, Ez, Bx, By, Bz and the cell size in c/omega_r."""
    rng = np.random.default_rng(seed)
    dx = 2.0 * math.pi / 40.0
    x = dx * np.arange(nx)
    c, s_ = np.cos(x), np.sin(x)
    # wave along +x: E = a0 (cos x, sin x) in (y, z), B = x^ x E; wave along -x: E = a0 (cos x, -sin x),
    # B = -x^ x E
    g = np.zeros((6, ny, nx), dtype=np.float32)
    Ey = a0 * (c + c)
    Ez = a0 * (s_ - s_)
    By = a0 * (-s_ - s_)
    Bz = a0 * (c - c)
    for k, row in ((1, Ey), (2, Ez), (4, By), (5, Bz)):
        g[k] = row[None, :]
    g += (noise * a0 * rng.standard_normal(g.shape)).astype(np.float32)
    return g, dx


def c3(n: int = 1 << 26, seed: int = 3, steps: int = 1000, nx: int = 4096, ny: int = 1024,
       grid_seed: int = 3) -> Workload:
    """Grid-interpolated fields: electrons seeded cell by cell over the periodic box of the c3_grid
    snapshot, as a PIC code creates them (electron i in cell floor(i nx ny / n) of the row-major
    order, uniform within it: 16 per cell at full size), gamma ~ LogUniform(10, 1e4), isotropic
    directions and unit spins, dt = dx/2, 1000 steps, both channels; photons below 21 m c^2 are
    retired (chi_gamma stays below 0.05 in fields up to about 2 a0 plus the noise).  The field
    array is in extra['grid']."""
    rng = np.random.default_rng(seed)
    grid, dx = c3_grid(nx, ny, seed=grid_seed)
    cell = (np.arange(n, dtype=np.int64) * (nx * ny)) // n
    x = np.zeros((3, n))
    x[0] = ((cell % nx) + rng.uniform(0.0, 1.0, n)) * dx
    x[1] = ((cell // nx) + rng.uniform(0.0, 1.0, n)) * dx
    gam = np.exp(rng.uniform(math.log(10.0), math.log(1e4), n))
    p = random_unit_vectors(rng, n) * np.sqrt(gam * gam - 1.0)
    s = random_unit_vectors(rng, n)
    k_retire = 0.05 / (2.0 * 2.0 * 200.0 * EPS_R) * 1.0
    return Workload("c3_grid_cp_standing_a0_200", n, steps, dx / 2.0, seed, FIELD_GRID2D, track=(True, True, False),
                    pair=True, k_retire=k_retire, x=x, p=p, s=s,
                    extra=dict(grid=grid, dx=dx, dy=dx, nx=nx, ny=ny))


def c5(n_instances: int = 64, seed: int = 5, steps: int = 2000, n_min: float = 1e4, n_max: float = 1e7,
       scale: float = 1.0) -> list:
    """Batched ensembles: independent head-on collisions shaped like c2, except per instance
    N ~ LogUniform[n_min, n_max] (times `scale`), a0 ~ U[20, 200], gamma0 ~ U[500, 1e4] with
    a 5 % spread, and spin polarization degree d ~ U[0, 1] along a random axis n perpendicular
    to x: every electron is pure, +n with probability (1 + d)/2, else -n.  2000 steps."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n_instances):
        n = max(1, int(round(scale * math.exp(rng.uniform(math.log(n_min), math.log(n_max))))))
        a0 = rng.uniform(20.0, 200.0)
        g0 = rng.uniform(500.0, 1e4)
        w = c2(n=n, seed=int(rng.integers(1 << 62)), steps=steps, a0=a0, gamma_mean=g0)
        r = np.random.default_rng(int(rng.integers(1 << 62)))
        ang = r.uniform(0.0, 2.0 * math.pi)
        axis = np.array([0.0, math.cos(ang), math.sin(ang)])
        d = r.uniform(0.0, 1.0)
        sgn = np.where(r.random(n) < 0.5 * (1.0 + d), 1.0, -1.0)
        w.s = axis[:, None] * sgn[None, :]
        w.name = f"c5_instance_{j}"
        w.extra = dict(a0=a0, gamma0=g0, pol_degree=d, pol_axis=axis)
        out.append(w)
    return out


def c6(n: int = 64, seed: int = 6, steps: int = 2000, a0: float = 1000.0, dt: float = 0.005) -> Workload:
    """Seeded pair cascade in a rotating electric field (polarized-cascade section): a uniform field
    of magnitude a0 = 1000 rotating in the (x, y) plane at the laser frequency (lambda = 0.8 um),
    n seed electrons at rest with isotropic unit spins (an unpolarized seed), both channels.
    dt = 0.005 / omega: electrons reach gamma ~ a0 and chi ~ 3, where W dt stays near 0.03.
    Photons are retired below k = chi_g_min / (a0 eps_r), under which chi_gamma cannot reach
    chi_g_min in a field of magnitude a0.  No position is tracked (0-D)."""
    rng = np.random.default_rng(seed)
    x = np.zeros((3, n))
    p = np.zeros((3, n))
    s = random_unit_vectors(rng, n)
    return Workload("c6_cascade_rotating_e_a0_1000", n, steps, dt, seed, FIELD_ROTATING_E, a0=a0,
                    track=(False, False, False), pair=True, k_retire=0.05 / (a0 * EPS_R), x=x, p=p, s=s)


def subsample(w: Workload, idx) -> Workload:
    """The same workload restricted to the given primary-electron indices (for oracle samples)."""
    import copy
    v = copy.copy(w)
    v.x, v.p, v.s = w.x[:, idx].copy(), w.p[:, idx].copy(), w.s[:, idx].copy()
    v.n = v.p.shape[1]
    return v


def random_unit_vectors(rng, n):
    v = rng.normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0)
