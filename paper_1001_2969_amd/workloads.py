"""Seeded synthetic workloads: mesh/physics presets, cross-section tables and
random particle states.

This module generates *inputs* only.  It holds none of the method's
arithmetic (no push, weighting, field solve or collision logic), so both the
GPU library and the CPU oracle can be fed from it without sharing code.

Physical parameters follow the benchmark problem of Sec. 3 of the paper
(argon at 300 K, n0 = 5e15 m^-3, dt = 5e-11 s, 13.56 MHz 200 V drive, square
cells).  The paper's argon cross sections (Phelps) are not available here; the
synthetic tables below stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Species parameters (inputs handed to both implementations).
E_CHARGE = 1.602176634e-19
M_ELECTRON = 9.1093837015e-31
AMU = 1.66053906660e-27
M_ARGON = 39.948 * AMU
K_BOLTZMANN = 1.380649e-23
TORR = 101325.0 / 760.0

ELECTRON, ION = 0, 1
SPECIES_Q = (-E_CHARGE, E_CHARGE)
SPECIES_M = (M_ELECTRON, M_ARGON)
MC_NONE, MC_ELECTRON, MC_ION = 0, 1, 2
P_ELASTIC, P_EXCITATION, P_IONIZATION = 0, 1, 2
W_ZR2, W_ZR = 0, 1
DAMP_D1, DAMP_FRIEDMAN = 0, 1
PUSH_LOCAL, PUSH_XYZ = 0, 1
RESIZE_SPLIT, RESIZE_ZERO_ORDER = 0, 1
FACE_AVG, FACE_MAX = 0, 1

# Uniform energy grid of the cross-section tables: 0 .. 200 eV step 0.02 eV.
XSEC_DE = 0.02
XSEC_NE = 10001
OPAL_B_ARGON = 10.0  # eV


@dataclasses.dataclass
class Workload:
    name: str
    nr: int
    nz: int
    R: float
    L: float
    n_per_species: int
    steps: int
    dt: float = 5e-11
    weighting: int = W_ZR2
    chi_face: int = FACE_AVG
    V_dc: float = 0.0
    V_rf: float = 0.0
    f_rf: float = 13.56e6
    seed: int = 0
    mg_tol: float = 1e-10
    mg_max_cycles: int = 100
    mg_fixed_cycles: int = 0
    resize_every: int = 0
    sort_every: int = 0
    tile_z: int = 16
    tile_r: int = 32
    n0: float = 5e15
    Te_eV: float = 2.0
    Ti_eV: float = 0.026
    pressure_mTorr: float = 100.0
    T_gas: float = 300.0
    xsec: str = "constant"
    precision: str = "fp64"
    circuit_C: float = 0.0  # > 0: blocking capacitor (F) in series with the rf source
    ion_subcycle: int = 0  # K >= 2: ions move every K-th step with K dt
    push_form: int = 0  # PUSH_LOCAL (Sec. 2.3 local X-Y push) or PUSH_XYZ (global X-Y-Z)
    resize_mode: int = 0  # RESIZE_SPLIT (weight-conserving) or RESIZE_ZERO_ORDER (particle-based)
    damping: int = 0  # DAMP_D1 (Sec. 2.1) or DAMP_FRIEDMAN (adjustable damping, parameter theta)
    theta: float = 1.0  # DAMP_FRIEDMAN: damping parameter in [0, 1] (0: leapfrog)

    @property
    def n_gas(self) -> float:
        return self.pressure_mTorr * 1e-3 * TORR / (K_BOLTZMANN * self.T_gas)

    @property
    def m_gas(self) -> float:
        return M_ARGON

    @property
    def wcoef(self) -> float:
        """Initial weight per unit radius, w = wcoef * r (uniform density)."""
        return 2.0 * math.pi * self.n0 * self.R * self.L / self.n_per_species

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def small_fp64() -> Workload:
    """33x33 mesh, R = L = 2 cm, 20k + 20k particles, 50 V DC, 10 steps."""
    return Workload(name="33x33_20k_fp64_dc50V", nr=33, nz=33, R=0.02, L=0.02,
                    n_per_species=20000, steps=10, V_dc=50.0)


def rf_129x65() -> Workload:
    """129x65 mesh, R = 4 cm, L = 2 cm, 2M per species, 200 V rf, 3 cycles/step."""
    return Workload(name="129x65_2M_rf200V", nr=129, nz=65, R=0.04, L=0.02,
                    n_per_species=2_000_000, steps=200, V_rf=200.0,
                    mg_fixed_cycles=3, precision="mixed")


def large_513x129() -> Workload:
    """513x129 mesh, R = 15 cm, L = 2.5 cm, 16M per species, resize active,
    particles sorted by 16 x 32-cell tile every 20 steps."""
    return Workload(name="513x129_16M_resize", nr=513, nz=129, R=0.15, L=0.025,
                    n_per_species=16_000_000, steps=1000, V_rf=200.0,
                    mg_fixed_cycles=3, resize_every=100, sort_every=20, pressure_mTorr=20.0,
                    xsec="powerlaw")


def adjoint_257x129() -> Workload:
    """Gradient window: 257x129 mesh (R = 8 cm, L = 4 cm, square 0.3125 mm
    cells), 4M particles per species, FP64, 200 V 13.56 MHz drive, converged
    solves, no collisions, particles sorted by 16 x 32-cell tile after the
    prologue and every 10 steps; 50 steps, checkpointed every 10."""
    return Workload(name="257x129_4M_adjoint", nr=257, nz=129, R=0.08, L=0.04,
                    n_per_species=4_000_000, steps=50, V_rf=200.0, mg_tol=1e-12,
                    mg_max_cycles=200, sort_every=10)


def batch_64(seed: int = 0, n: int = 64):
    """n independent discharges of uneven size: meshes drawn from 65x33,
    129x65 and 257x129 (square 0.3125 mm cells: R x L = 2 x 1, 4 x 2, 8 x 4
    cm), particles per species log-uniform in [1e5, 2e6], 200 V rf drive, 3
    V-cycles per step, mixed precision, tile sort every 20 steps; seeded."""
    rng = np.random.default_rng(seed)
    shapes = ((65, 33, 0.02, 0.01), (129, 65, 0.04, 0.02), (257, 129, 0.08, 0.04))
    out = []
    for k in range(n):
        nr, nz, R, L = shapes[int(rng.integers(0, len(shapes)))]
        npart = int(round(math.exp(rng.uniform(math.log(1e5), math.log(2e6)))))
        out.append(Workload(name=f"batch{k}_{nr}x{nz}_{npart}", nr=nr, nz=nz, R=R, L=L,
                            n_per_species=npart, steps=100, V_rf=200.0, mg_fixed_cycles=3,
                            sort_every=20, seed=seed * 1000 + k, precision="mixed"))
    return out


def xsec_tables(w: Workload):
    """Synthetic tables on eps_k = k * XSEC_DE.

    Returns {species: (kinds, thresholds, sigma[nproc, ne], ejB)}.
    constant: electrons elastic 1e-19 m^2 + ionization 2e-20 m^2 above 15.8 eV;
              ions elastic 1e-19 m^2.
    powerlaw: electrons elastic 1e-19 (eps/1 eV)^-1/2, excitation 1e-20 above
              11.5 eV, ionization 2e-20 above 15.8 eV; ions elastic
              1e-19 (eps/1 eV)^-1/2.  The eps = 0 entry repeats eps = XSEC_DE.
    """
    eps = np.arange(XSEC_NE, dtype=np.float64) * XSEC_DE

    def step_fn(value, thr):
        return np.where(eps >= thr, value, 0.0)

    def power(value):
        e = np.maximum(eps, XSEC_DE)
        return value * e ** -0.5

    if w.xsec == "constant":
        e_kind = [P_ELASTIC, P_IONIZATION]
        e_thr = [0.0, 15.8]
        e_sig = np.stack([np.full_like(eps, 1e-19), step_fn(2e-20, 15.8)])
        i_sig = np.stack([np.full_like(eps, 1e-19)])
    elif w.xsec == "powerlaw":
        e_kind = [P_ELASTIC, P_EXCITATION, P_IONIZATION]
        e_thr = [0.0, 11.5, 15.8]
        e_sig = np.stack([power(1e-19), step_fn(1e-20, 11.5), step_fn(2e-20, 15.8)])
        i_sig = np.stack([power(1e-19)])
    else:
        raise ValueError(w.xsec)
    return {
        ELECTRON: (np.array(e_kind, np.int32), np.array(e_thr), np.ascontiguousarray(e_sig),
                   OPAL_B_ARGON),
        ION: (np.array([P_ELASTIC], np.int32), np.array([0.0]), np.ascontiguousarray(i_sig),
              OPAL_B_ARGON),
    }


FIELDS = ("r", "z", "vr", "vt", "vz", "ar", "az", "w")


def random_particles(seed: int, n: int, w: Workload, species: int, *,
                     accel_scale: float = 1e4, id0: int = 0, shuffle_ids: bool = True,
                     near_axis_frac: float = 0.0, near_wall_frac: float = 0.0):
    """A seeded particle state inside (0,R) x (0,L): uniform positions,
    Maxwellian velocities at the workload's temperature, damped accelerations
    of magnitude ~ |q/m| * accel_scale (V/m), weights proportional to r.
    Optional fractions are placed within one cell of the axis / the wall so
    that the axis rule and absorption are exercised."""
    rng = np.random.default_rng(seed)
    R, L = w.R, w.L
    hr = R / (w.nr - 1)
    r = rng.uniform(0.0, R, n)
    z = rng.uniform(0.0, L, n)
    k_axis = int(n * near_axis_frac)
    k_wall = int(n * near_wall_frac)
    if k_axis:
        r[:k_axis] = rng.uniform(0.0, hr, k_axis)
    if k_wall:
        r[k_axis:k_axis + k_wall] = rng.uniform(R - hr, R, k_wall)
    z = np.clip(z, L * 1e-9, L * (1 - 1e-9))
    r = np.minimum(r, R * (1 - 1e-12))
    T = w.Te_eV if species == ELECTRON else w.Ti_eV
    m = SPECIES_M[species]
    vth = math.sqrt(T * E_CHARGE / m)
    v = rng.normal(0.0, vth, (3, n))
    qm = abs(SPECIES_Q[species] / m)
    a = rng.normal(0.0, qm * accel_scale, (2, n))
    ids = np.arange(id0, id0 + n, dtype=np.uint64)
    if shuffle_ids:
        ids = rng.permutation(ids)
    return {
        "r": r, "z": z, "vr": v[0], "vt": v[1], "vz": v[2], "ar": a[0], "az": a[1],
        "w": w.wcoef * np.maximum(r, 0.5 * hr), "id": ids,
    }, id0 + n


def smooth_chi(w: Workload, amp: float = 1.0):
    """A smooth positive susceptibility on the mesh, chi ~ amp (MG tests)."""
    r = np.linspace(0.0, w.R, w.nr)[None, :]
    z = np.linspace(0.0, w.L, w.nz)[:, None]
    return amp * (1.0 + 0.5 * np.cos(math.pi * r / w.R)) * np.sin(math.pi * z / w.L) ** 2 + \
        0.0 * r * z


def smooth_rho(w: Workload, seed: int = 0, amp: float = 1e-4):
    """A seeded smooth charge density (C/m^3) plus small noise (MG tests)."""
    rng = np.random.default_rng(seed)
    r = np.linspace(0.0, w.R, w.nr)[None, :]
    z = np.linspace(0.0, w.L, w.nz)[:, None]
    base = amp * np.cos(0.5 * math.pi * r / w.R) * np.sin(math.pi * z / w.L)
    return base + 0.05 * amp * rng.standard_normal((w.nz, w.nr))
