"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None
_LIB_OMP = None

G_PHI, G_RHO, G_CHI, G_ER, G_EZ, G_N0, G_N1, G_DENS0, G_DENS1, G_VOL = range(10)
G_PHI_P, G_PHI_L = 10, 11
FIELDS = ("r", "z", "vr", "vt", "vz", "ar", "az", "w")


class Config(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nz", C.c_int32),
        ("R", C.c_double), ("L", C.c_double), ("dt", C.c_double),
        ("weighting", C.c_int32), ("chi_face", C.c_int32),
        ("V_dc", C.c_double), ("V_rf", C.c_double), ("f_rf", C.c_double),
        ("seed", C.c_uint64),
        ("mg_tol", C.c_double),
        ("mg_max_cycles", C.c_int32), ("mg_fixed_cycles", C.c_int32),
        ("resize_every", C.c_int32), ("sort_every", C.c_int32),
        ("resize_wcoef", C.c_double),
        ("n_gas", C.c_double), ("T_gas", C.c_double), ("m_gas", C.c_double),
        ("tile_z", C.c_int32), ("tile_r", C.c_int32),
        ("circuit_C", C.c_double),
        ("ion_subcycle", C.c_int32), ("push_form", C.c_int32),
        ("resize_mode", C.c_int32), ("damping", C.c_int32), ("theta", C.c_double),
    ]


def lib(omp=False):
    """The serial oracle, or (omp=True) its OpenMP timing build, which has the
    same entry points plus rzo_omp_step."""
    global _LIB, _LIB_OMP
    if (_LIB_OMP if omp else _LIB) is None:
        # RZO_LIB selects another build of the same source (the sanitized
        # one of oracle/sanitize.py)
        path = _build.LIB_OMP if omp else (os.environ.get("RZO_LIB") or _build.LIB)
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        L.rzo_create.restype = P
        L.rzo_create.argtypes = [C.POINTER(Config)]
        L.rzo_destroy.argtypes = [P]
        L.rzo_constants.argtypes = [dp]
        L.rzo_set_species.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_int]
        L.rzo_set_particles.argtypes = [P, C.c_int, C.c_int64] + [dp] * 8 + [up, C.c_uint64]
        L.rzo_count.restype = C.c_int64
        L.rzo_count.argtypes = [P, C.c_int]
        L.rzo_next_id.restype = C.c_uint64
        L.rzo_next_id.argtypes = [P, C.c_int]
        L.rzo_get_particles.argtypes = [P, C.c_int] + [dp] * 8 + [up]
        L.rzo_get_events.argtypes = [P, C.c_int, np.ctypeslib.ndpointer(np.uint8), C.c_int64]
        L.rzo_set_xsec.argtypes = [P, C.c_int, C.c_int,
                                   np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"),
                                   dp, C.c_double, C.c_int32, dp, C.c_double]
        L.rzo_mc_consts.argtypes = [P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.rzo_init_particles.argtypes = [P, C.c_int, C.c_int64, C.c_double, C.c_double,
                                         C.c_uint64]
        for name in ("rzo_push_first", "rzo_push_final", "rzo_compact", "rzo_resize", "rzo_sort"):
            getattr(L, name).argtypes = [P, C.c_int]
        L.rzo_resize_step.argtypes = [P, C.c_int, C.c_int64]
        L.rzo_tile_key.restype = C.c_int32
        L.rzo_tile_key.argtypes = [P, C.c_double, C.c_double]
        L.rzo_collide.argtypes = [P, C.c_int, C.c_int64]
        L.rzo_deposit.argtypes = [P]
        L.rzo_efield.argtypes = [P]
        L.rzo_prologue.argtypes = [P]
        L.rzo_solve.argtypes = [P, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.rzo_step.argtypes = [P, C.c_int64, C.c_int]
        L.rzo_get_grid.argtypes = [P, C.c_int, dp]
        L.rzo_set_grid.argtypes = [P, C.c_int, dp]
        L.rzo_absorbed.argtypes = [P, C.c_int, dp]
        L.rzo_set_circuit.argtypes = [P, C.c_double, C.c_double, C.c_double]
        L.rzo_set_at.argtypes = [P, C.c_int, C.c_int64, dp]
        L.rzo_get_at.argtypes = [P, C.c_int, dp]
        L.rzo_circuit.argtypes = [P, dp]
        L.rzo_apply_op.argtypes = [P, dp, dp]
        L.rzo_thomas.argtypes = [C.c_int32, dp, dp, dp, dp, dp]
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.rzo_philox.argtypes = [u32p, u32p, u32p]
        L.rzo_uniform_pair.argtypes = [C.c_uint64, C.c_int, C.c_uint64, C.c_uint32,
                                       C.c_uint32, dp]
        L.rzo_xsec.restype = C.c_double
        L.rzo_xsec.argtypes = [P, C.c_int, C.c_int, C.c_double]
        if omp:
            L.rzo_omp_step.argtypes = [P, C.c_int64, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_int32)]
            L.rzo_omp_set_threads.argtypes = [C.c_int]
            L.rzo_omp_set_threads.restype = None
            L.rzo_omp_threads.restype = C.c_int
            _LIB_OMP = L
        else:
            _LIB = L
    return _LIB_OMP if omp else _LIB


def constants():
    out = np.zeros(6)
    lib().rzo_constants(out)
    return dict(zip(("e", "m_e", "amu", "eps0", "k_B", "two_pi"), out))


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().rzo_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def uniform_pair(seed, s, pid, step, blk):
    out = np.zeros(2)
    lib().rzo_uniform_pair(seed, s, pid, step, blk, out)
    return out


def thomas(d, b, e, g):
    n = len(b)
    x = np.zeros(n)
    arr = [np.ascontiguousarray(a, np.float64) for a in (d, b, e, g)]
    rc = lib().rzo_thomas(n, *arr, x)
    assert rc == 0
    return x


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One simulation state held by the C oracle."""

    def __init__(self, w, *, mg_tol=None, mg_fixed_cycles=None, mg_max_cycles=None,
                 species=(0, 1), q=None, m=None, mc=True, omp=False):
        from paper_1001_2969_amd import workloads as wl
        self.w = w
        self.L = lib(omp)
        self.omp = omp
        cfg = Config(nr=w.nr, nz=w.nz, R=w.R, L=w.L, dt=w.dt, weighting=w.weighting,
                     chi_face=w.chi_face, V_dc=w.V_dc, V_rf=w.V_rf, f_rf=w.f_rf,
                     seed=w.seed,
                     mg_tol=w.mg_tol if mg_tol is None else mg_tol,
                     mg_max_cycles=w.mg_max_cycles if mg_max_cycles is None else mg_max_cycles,
                     mg_fixed_cycles=(w.mg_fixed_cycles if mg_fixed_cycles is None
                                      else mg_fixed_cycles),
                     resize_every=w.resize_every, sort_every=w.sort_every,
                     resize_wcoef=w.wcoef, n_gas=w.n_gas, T_gas=w.T_gas, m_gas=w.m_gas,
                     tile_z=w.tile_z, tile_r=w.tile_r, circuit_C=w.circuit_C,
                     ion_subcycle=w.ion_subcycle, push_form=w.push_form,
                     resize_mode=w.resize_mode, damping=w.damping, theta=w.theta)
        self._cfg = cfg
        self.h = self.L.rzo_create(C.byref(cfg))
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        self.nn = w.nr * w.nz
        qs = wl.SPECIES_Q if q is None else q
        ms = wl.SPECIES_M if m is None else m
        models = (wl.MC_ELECTRON, wl.MC_ION) if mc else (wl.MC_NONE, wl.MC_NONE)
        for s in (0, 1):
            assert self.L.rzo_set_species(self.h, s, qs[s], ms[s], models[s]) == 0
        if mc:
            for s, (kind, thr, sig, ejb) in wl.xsec_tables(w).items():
                self.set_xsec(s, kind, thr, wl.XSEC_DE, sig, ejb)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.L.rzo_destroy(h)
            self.h = None

    # ---- species
    def set_xsec(self, s, kind, thr, de, sigma, ejb):
        sigma = _f64(sigma)
        rc = self.L.rzo_set_xsec(self.h, s, sigma.shape[0], np.ascontiguousarray(kind, np.int32),
                                _f64(thr), de, sigma.shape[1], sigma, ejb)
        assert rc == 0

    def mc_consts(self, s):
        a, b = C.c_double(), C.c_double()
        self.L.rzo_mc_consts(self.h, s, C.byref(a), C.byref(b))
        return a.value, b.value

    def set_particles(self, s, parts, next_id):
        n = len(parts["r"])
        arr = [_f64(parts[f]) for f in FIELDS]
        rc = self.L.rzo_set_particles(self.h, s, n, *arr,
                                     np.ascontiguousarray(parts["id"], np.uint64), next_id)
        assert rc == 0

    def count(self, s):
        return int(self.L.rzo_count(self.h, s))

    def next_id(self, s):
        return int(self.L.rzo_next_id(self.h, s))

    def particles(self, s):
        n = self.count(s)
        out = {f: np.zeros(n) for f in FIELDS}
        out["id"] = np.zeros(n, np.uint64)
        self.L.rzo_get_particles(self.h, s, *[out[f] for f in FIELDS], out["id"])
        return out

    def events(self, s, n):
        ev = np.zeros(n, np.uint8)
        assert self.L.rzo_get_events(self.h, s, ev, n) == 0
        return ev

    def init_particles(self, s, n, n0, T_eV, id0=0):
        assert self.L.rzo_init_particles(self.h, s, n, n0, T_eV, id0) == 0

    # ---- operations
    def push_first(self, s):
        self.L.rzo_push_first(self.h, s)

    def push_final(self, s):
        self.L.rzo_push_final(self.h, s)

    def collide(self, s, step):
        assert self.L.rzo_collide(self.h, s, step) == 0

    def compact(self, s):
        self.L.rzo_compact(self.h, s)

    def resize(self, s, step=None):
        if step is None:
            assert self.L.rzo_resize(self.h, s) == 0
        else:
            assert self.L.rzo_resize_step(self.h, s, step) == 0

    def sort(self, s):
        """Stable counting sort by tile; returns the number of tiles."""
        nt = self.L.rzo_sort(self.h, s)
        assert nt > 0
        return nt

    def tile_key(self, r, z):
        return self.L.rzo_tile_key(self.h, r, z)

    def deposit(self):
        self.L.rzo_deposit(self.h)

    def efield(self):
        self.L.rzo_efield(self.h)

    def prologue(self):
        self.L.rzo_prologue(self.h)

    def solve(self, t):
        cyc, rr = C.c_int32(), C.c_double()
        st = self.L.rzo_solve(self.h, t, C.byref(cyc), C.byref(rr))
        return st, cyc.value, rr.value

    def step(self, n, merged=True):
        return self.L.rzo_step(self.h, n, 1 if merged else 0)

    def step_omp(self, n, with_cycles=False):
        """OpenMP timing build only: a merged step with the particle loops on
        threads; returns (status, particle seconds, solve seconds) and, with
        with_cycles, the V-cycles of the solve."""
        tp, ts, cy = C.c_double(), C.c_double(), C.c_int32()
        st = self.L.rzo_omp_step(self.h, n, C.byref(tp), C.byref(ts), C.byref(cy))
        return (st, tp.value, ts.value, cy.value) if with_cycles else (st, tp.value, ts.value)

    @staticmethod
    def set_threads(n):
        lib(True).rzo_omp_set_threads(int(n))

    @staticmethod
    def threads():
        return int(lib(True).rzo_omp_threads())

    # ---- grids
    def grid(self, which):
        out = np.zeros(self.nn)
        assert self.L.rzo_get_grid(self.h, which, out) == 0
        return out.reshape(self.w.nz, self.w.nr)

    def set_grid(self, which, arr):
        assert self.L.rzo_set_grid(self.h, which, _f64(np.asarray(arr).reshape(-1))) == 0

    def set_at(self, s, at):
        """a_theta of the global X-Y-Z push for the first len(at) particles."""
        at = _f64(at)
        assert self.L.rzo_set_at(self.h, s, len(at), at) == 0

    def get_at(self, s):
        out = np.zeros(self.count(s))
        assert self.L.rzo_get_at(self.h, s, out) == 0
        return out

    def set_circuit(self, V, Q, Qc):
        assert self.L.rzo_set_circuit(self.h, V, Q, Qc) == 0

    def circuit(self):
        """{V, Q, Q_c, Q_conv, Q_P, Q_L} of the last solve (external circuit)."""
        out = np.zeros(6)
        assert self.L.rzo_circuit(self.h, out) == 0
        return dict(zip(("V", "Q", "Qc", "Qconv", "Qp", "Ql"), out))

    def absorbed(self, s):
        out = np.zeros(3)
        self.L.rzo_absorbed(self.h, s, out)
        return out

    def apply_op(self, u):
        y = np.zeros(self.nn)
        self.L.rzo_apply_op(self.h, _f64(np.asarray(u).reshape(-1)), y)
        return y.reshape(self.w.nz, self.w.nr)

    def xsec(self, s, k, eps):
        return self.L.rzo_xsec(self.h, s, k, eps)
