"""ctypes binding of librzpic.so (include/rzpic.h).

Argument marshalling only: torch supplies device memory and the stream, every
step of the method runs in the HIP library.  There is no fallback: without
the built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librzpic.so")

FP64, MIXED = 0, 1
G_PHI, G_RHO, G_CHI, G_ER, G_EZ, G_N0, G_N1, G_DENS0, G_DENS1, G_VOL = range(10)
G_PHI_P, G_PHI_L = 10, 11
FIELDS = ("r", "z", "vr", "vt", "vz", "ar", "az", "w")
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ECAPACITY", 5: "ENOTCONV",
          6: "ENUMERIC", 7: "ESTATE"}
EXPORTS = (
    "rzpic_create", "rzpic_destroy", "rzpic_set_stream", "rzpic_bind_species", "rzpic_set_count",
    "rzpic_get_count", "rzpic_set_xsec", "rzpic_get_mc_consts", "rzpic_init_particles",
    "rzpic_push_first", "rzpic_deposit", "rzpic_solve", "rzpic_efield", "rzpic_push_final",
    "rzpic_collide", "rzpic_compact", "rzpic_resize", "rzpic_prologue", "rzpic_step",
    "rzpic_grid_copy", "rzpic_get_diag", "rzpic_sync", "rzpic_last_error", "rzpic_constants",
    "rzpic_set_timing", "rzpic_get_timing", "rzpic_set_mg", "rzpic_sort",
    "rzpic_batch_create", "rzpic_batch_step", "rzpic_batch_stats", "rzpic_batch_destroy",
    "rzpic_batch_set_graph", "rzpic_set_voltage", "rzpic_adjoint_create",
    "rzpic_adjoint_forward", "rzpic_adjoint_backward", "rzpic_adjoint_destroy",
    "rzpic_set_circuit", "rzpic_get_circuit", "rzpic_set_pass_shape", "rzpic_autotune",
    "rzpic_deposit_noalloc", "rzpic_solve_dev", "rzpic_grid_view", "rzpic_set_grid_source",
    "rzpic_set_pass_form", "rzpic_set_tiles", "rzpic_get_pass_config", "rzpic_batch_autotune",
    "rzpic_set_step_graph",
    "rzpic_set_step_pipeline",
)
FORM_AUTO, FORM_LDS, FORM_TILED = 0, 1, 2


class RzpicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rzpic {STATUS.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nz", C.c_int32),
        ("R", C.c_double), ("L", C.c_double), ("dt", C.c_double),
        ("precision", C.c_int32), ("weighting", C.c_int32), ("chi_face", C.c_int32),
        ("fixed_point_bits", C.c_int32),
        ("V_dc", C.c_double), ("V_rf", C.c_double), ("f_rf", C.c_double),
        ("seed", C.c_uint64),
        ("mg_tol", C.c_double), ("mg_max_cycles", C.c_int32), ("mg_fixed_cycles", C.c_int32),
        ("resize_every", C.c_int32), ("sort_every", C.c_int32),
        ("resize_wcoef", C.c_double),
        ("n_gas", C.c_double), ("T_gas", C.c_double), ("m_gas", C.c_double),
        ("tile_z", C.c_int32), ("tile_r", C.c_int32),
        ("circuit_C", C.c_double),
        ("ion_subcycle", C.c_int32), ("push_form", C.c_int32),
        ("resize_mode", C.c_int32), ("damping", C.c_int32), ("theta", C.c_double),
    ]


class SpeciesView(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in FIELDS] + [
        ("id", C.c_void_p), ("mc_event", C.c_void_p), ("capacity", C.c_int64),
        ("q", C.c_double), ("m", C.c_double), ("w_ref", C.c_double),
        ("mc_model", C.c_int32), ("reserved0", C.c_int32), ("at", C.c_void_p),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("count", C.c_int64 * 2), ("next_id", C.c_uint64 * 2),
        ("absorbed", (C.c_double * 3) * 2), ("candidates", C.c_int64 * 2),
        ("events", (C.c_int64 * 4) * 2), ("last_cycles", C.c_int32), ("status", C.c_int32),
        ("last_relres", C.c_double), ("particle_steps", C.c_uint64 * 2),
    ]


class AdjointConfig(C.Structure):
    _fields_ = [
        ("n_steps", C.c_int32), ("checkpoint_every", C.c_int32),
        ("id_capacity", C.c_int64 * 2), ("delta", C.c_double), ("tol", C.c_double),
        ("max_cycles", C.c_int32), ("reserved", C.c_int32),
    ]


_lib = None


class GridView(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nz", C.c_int32),
        ("phi", C.c_void_p), ("rho", C.c_void_p), ("chi", C.c_void_p), ("er", C.c_void_p),
        ("ez", C.c_void_p), ("dens0", C.c_void_p), ("dens1", C.c_void_p), ("vol", C.c_void_p),
        ("phi_p", C.c_void_p), ("phi_l", C.c_void_p),
    ]


class _DeviceArray:
    """A device array the library owns, exposed through the CUDA array
    interface so that torch wraps it without a copy."""

    def __init__(self, ptr, shape):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": "<f8",
                                         "data": (int(ptr), False), "version": 3,
                                         "strides": None}


class DepositArgs(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nz", C.c_int32), ("R", C.c_double), ("L", C.c_double),
        ("precision", C.c_int32), ("weighting", C.c_int32),
        ("fixed_point_bits", C.c_int32), ("reserved", C.c_int32),
        ("w_ref", C.c_double), ("r", C.c_void_p), ("z", C.c_void_p), ("w", C.c_void_p),
        ("n", C.c_int64), ("out", C.c_void_p), ("status", C.c_void_p),
    ]


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1001_2969_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I, D = C.c_void_p, C.c_int32, C.c_double
        st = C.c_int
        sig = {
            "rzpic_create": [C.POINTER(Config), P, C.POINTER(P)],
            "rzpic_destroy": [P], "rzpic_set_stream": [P, P],
            "rzpic_bind_species": [P, I, C.POINTER(SpeciesView)],
            "rzpic_set_count": [P, I, C.c_int64, C.c_uint64],
            "rzpic_get_count": [P, I, C.POINTER(C.c_int64), C.POINTER(C.c_uint64)],
            "rzpic_set_xsec": [P, I, I, P, P, D, I, P, D],
            "rzpic_get_mc_consts": [P, I, C.POINTER(D), C.POINTER(D)],
            "rzpic_init_particles": [P, I, C.c_int64, D, D, C.c_uint64],
            "rzpic_push_first": [P, I], "rzpic_push_final": [P, I], "rzpic_compact": [P, I],
            "rzpic_resize": [P, I], "rzpic_sort": [P, I], "rzpic_collide": [P, I, C.c_int64],
            "rzpic_deposit": [P], "rzpic_efield": [P], "rzpic_prologue": [P],
            "rzpic_solve": [P, D, C.POINTER(I), C.POINTER(D)],
            "rzpic_step": [P, C.c_int64], "rzpic_grid_copy": [P, I, P, I],
            "rzpic_get_diag": [P, C.POINTER(Diag)], "rzpic_sync": [P],
            "rzpic_set_timing": [P, I], "rzpic_get_timing": [P, P],
            "rzpic_set_mg": [P, D, I, I],
            "rzpic_batch_create": [P, I, P, C.POINTER(P)],
            "rzpic_batch_step": [P, C.c_int64], "rzpic_batch_stats": [P, P],
            "rzpic_batch_destroy": [P], "rzpic_batch_set_graph": [P, I],
            "rzpic_set_voltage": [P, D, D, D],
            "rzpic_set_circuit": [P, D, D, D], "rzpic_get_circuit": [P, P],
            "rzpic_set_pass_shape": [P, I, I],
            "rzpic_autotune": [P, I, C.c_int64, P, P, C.POINTER(C.c_int64)],
            "rzpic_adjoint_create": [P, C.POINTER(AdjointConfig), C.POINTER(P)],
            "rzpic_adjoint_forward": [P, C.c_int64, C.POINTER(D)],
            "rzpic_adjoint_backward": [P, P, P, P, P], "rzpic_adjoint_destroy": [P],
            "rzpic_deposit_noalloc": [C.POINTER(DepositArgs), P],
            "rzpic_solve_dev": [P, D, P, P],
            "rzpic_grid_view": [P, C.POINTER(GridView)],
            "rzpic_set_grid_source": [P, P, P],
            "rzpic_set_pass_form": [P, I], "rzpic_set_tiles": [P, I, I],
            "rzpic_set_step_graph": [P, I],
            "rzpic_set_step_pipeline": [P, I],
            "rzpic_get_pass_config": [P, P],
            "rzpic_batch_autotune": [P, I, C.c_int64, P, I, C.POINTER(I), C.POINTER(C.c_int64)],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = st
        L.rzpic_last_error.restype = C.c_char_p
        L.rzpic_last_error.argtypes = []
        L.rzpic_constants.restype = None
        L.rzpic_constants.argtypes = [P]
        _lib = L
    return _lib


def constants():
    out = (C.c_double * 6)()
    lib().rzpic_constants(C.cast(out, C.c_void_p))
    return dict(zip(("e", "m_e", "amu", "eps0", "k_B", "two_pi"), list(out)))


def _check(code):
    if code != 0:
        raise RzpicError(code, lib().rzpic_last_error().decode())


def deposit_noalloc(nr, nz, R, L, r, z, w, out, status, *, n=None, precision=FP64,
                    weighting=0, fixed_point_bits=0, w_ref=1.0, stream=None):
    """rzpic_deposit_noalloc: N_ij of the particles (r, z, w: device tensors of
    one dtype, float64 for FP64 or float32 for MIXED) into `out` (device
    float64 tensor of nz*nr), allocating nothing; `status` is a device int32
    tensor that receives the overflow bit.  Asynchronous on `stream` (a
    torch.cuda.Stream; the current one if None)."""
    import torch

    if n is None:
        n = r.numel()
    if stream is None:
        stream = torch.cuda.current_stream()
    a = DepositArgs(nr=nr, nz=nz, R=R, L=L, precision=precision, weighting=weighting,
                    fixed_point_bits=fixed_point_bits, reserved=0, w_ref=w_ref,
                    r=r.data_ptr(), z=z.data_ptr(), w=w.data_ptr(), n=n,
                    out=out.data_ptr(), status=status.data_ptr())
    _check(lib().rzpic_deposit_noalloc(C.byref(a), C.c_void_p(stream.cuda_stream)))


class Context:
    """One discharge on one GPU: the library context plus torch-owned particle
    arrays of both species.  `w` is a workloads.Workload."""

    def __init__(self, w, *, precision=None, mg_tol=None, mg_fixed_cycles=None,
                 mg_max_cycles=None, fixed_point_bits=0, device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("rzpic needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.device = torch.device(device)
        self.w = w
        prec = w.precision if precision is None else precision
        self.precision = MIXED if prec in ("mixed", MIXED) else FP64
        self.dtype = torch.float32 if self.precision == MIXED else torch.float64
        cfg = Config(nr=w.nr, nz=w.nz, R=w.R, L=w.L, dt=w.dt, precision=self.precision,
                     weighting=w.weighting, chi_face=w.chi_face,
                     fixed_point_bits=fixed_point_bits, V_dc=w.V_dc, V_rf=w.V_rf, f_rf=w.f_rf,
                     seed=w.seed, mg_tol=w.mg_tol if mg_tol is None else mg_tol,
                     mg_max_cycles=w.mg_max_cycles if mg_max_cycles is None else mg_max_cycles,
                     mg_fixed_cycles=(w.mg_fixed_cycles if mg_fixed_cycles is None
                                      else mg_fixed_cycles),
                     resize_every=w.resize_every, sort_every=w.sort_every,
                     resize_wcoef=w.wcoef, n_gas=w.n_gas, T_gas=w.T_gas, m_gas=w.m_gas,
                     tile_z=w.tile_z, tile_r=w.tile_r, circuit_C=w.circuit_C,
                     ion_subcycle=w.ion_subcycle, push_form=w.push_form,
                     resize_mode=w.resize_mode, damping=w.damping, theta=w.theta)
        self._cfg = cfg
        self.xyz = w.push_form == 1
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            _check(lib().rzpic_create(C.byref(cfg), C.c_void_p(self.stream.cuda_stream),
                                      C.byref(h)))
        self.h = h
        self.nn = w.nr * w.nz
        self.arrays = {}
        self.events = {}
        self.capacity = {}

    def close(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().rzpic_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- species
    def bind(self, s, capacity, q, m, w_ref, mc_model, events=False):
        t = self.torch
        arr = {f: t.zeros(capacity, dtype=self.dtype, device=self.device) for f in FIELDS}
        arr["id"] = t.zeros(capacity, dtype=t.int64, device=self.device)
        if self.xyz:  # a_theta of the global X-Y-Z push
            arr["at"] = t.zeros(capacity, dtype=self.dtype, device=self.device)
        ev = t.zeros(capacity, dtype=t.uint8, device=self.device) if events else None
        v = SpeciesView(**{f: arr[f].data_ptr() for f in FIELDS}, id=arr["id"].data_ptr(),
                        mc_event=ev.data_ptr() if ev is not None else None,
                        capacity=capacity, q=q, m=m, w_ref=w_ref, mc_model=mc_model,
                        reserved0=0, at=arr["at"].data_ptr() if self.xyz else None)
        _check(lib().rzpic_bind_species(self.h, s, C.byref(v)))
        self.arrays[s] = arr
        self.events[s] = ev
        self.capacity[s] = capacity

    def set_xsec(self, s, kind, thr, de, sigma, ejb):
        kind = np.ascontiguousarray(kind, np.int32)
        thr = np.ascontiguousarray(thr, np.float64)
        sigma = np.ascontiguousarray(sigma, np.float64)
        _check(lib().rzpic_set_xsec(self.h, s, sigma.shape[0], kind.ctypes.data,
                                    thr.ctypes.data, de, sigma.shape[1], sigma.ctypes.data, ejb))

    def mc_consts(self, s):
        a, b = C.c_double(), C.c_double()
        _check(lib().rzpic_get_mc_consts(self.h, s, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_particles(self, s, parts, next_id):
        t = self.torch
        n = len(parts["r"])
        arr = self.arrays[s]
        for f in FIELDS:
            arr[f][:n].copy_(t.as_tensor(np.asarray(parts[f]), dtype=self.dtype))
        arr["id"][:n].copy_(t.as_tensor(np.asarray(parts["id"]).astype(np.int64)))
        if self.xyz:
            at = parts.get("at")
            if at is None:
                arr["at"][:n].zero_()
            else:
                arr["at"][:n].copy_(t.as_tensor(np.asarray(at), dtype=self.dtype))
        _check(lib().rzpic_set_count(self.h, s, n, next_id))

    def count(self, s):
        n, nid = C.c_int64(), C.c_uint64()
        _check(lib().rzpic_get_count(self.h, s, C.byref(n), C.byref(nid)))
        return n.value, nid.value

    def particles(self, s):
        n, _ = self.count(s)
        arr = self.arrays[s]
        out = {f: arr[f][:n].double().cpu().numpy() for f in FIELDS}
        out["id"] = arr["id"][:n].cpu().numpy().astype(np.uint64)
        if self.xyz:
            out["at"] = arr["at"][:n].double().cpu().numpy()
        return out

    def event_codes(self, s, n):
        return self.events[s][:n].cpu().numpy()

    def init_particles(self, s, n, n0, T_eV, id0=0):
        _check(lib().rzpic_init_particles(self.h, s, n, n0, T_eV, id0))

    # ---- operations
    def push_first(self, s):
        _check(lib().rzpic_push_first(self.h, s))

    def push_final(self, s):
        _check(lib().rzpic_push_final(self.h, s))

    def collide(self, s, step):
        _check(lib().rzpic_collide(self.h, s, step))

    def compact(self, s):
        _check(lib().rzpic_compact(self.h, s))

    def resize(self, s):
        _check(lib().rzpic_resize(self.h, s))

    def sort(self, s):
        _check(lib().rzpic_sort(self.h, s))

    def deposit(self):
        _check(lib().rzpic_deposit(self.h))

    def efield(self):
        _check(lib().rzpic_efield(self.h))

    def prologue(self):
        _check(lib().rzpic_prologue(self.h))

    def solve(self, t, want=True):
        if not want:
            _check(lib().rzpic_solve(self.h, t, None, None))
            return None
        cyc, rr = C.c_int32(), C.c_double()
        _check(lib().rzpic_solve(self.h, t, C.byref(cyc), C.byref(rr)))
        return cyc.value, rr.value

    def solve_dev(self, t, cycles=None, relres=None):
        """rzpic_solve_dev: cycles (int32) and relres (float64) device tensors of
        one element, either may be None; filled on the stream."""
        _check(lib().rzpic_solve_dev(self.h, t,
                                     None if cycles is None else C.c_void_p(cycles.data_ptr()),
                                     None if relres is None else C.c_void_p(relres.data_ptr())))

    def grid_view(self):
        """The context's grids as torch tensors of shape (nz, nr) sharing its
        memory (rzpic_grid_view): no copy.  phi is valid until the next solve
        or step."""
        v = GridView()
        _check(lib().rzpic_grid_view(self.h, C.byref(v)))
        out = {}
        for f in ("phi", "rho", "chi", "er", "ez", "dens0", "dens1", "vol", "phi_p", "phi_l"):
            ptr = getattr(v, f)
            if ptr:
                out[f] = self.torch.as_tensor(_DeviceArray(ptr, (v.nz, v.nr)),
                                              device=self.device)
        return out

    def set_grid_source(self, rho, chi):
        """rzpic_set_grid_source from device float64 tensors of nz*nr values."""
        _check(lib().rzpic_set_grid_source(self.h, C.c_void_p(rho.data_ptr()),
                                           C.c_void_p(chi.data_ptr())))

    def set_mg(self, tol=1e-10, max_cycles=100, fixed_cycles=0):
        _check(lib().rzpic_set_mg(self.h, tol, max_cycles, fixed_cycles))

    def step(self, n):
        _check(lib().rzpic_step(self.h, n))

    def set_voltage(self, V_dc, V_rf, f_rf=None):
        f = self.w.f_rf if f_rf is None else f_rf
        _check(lib().rzpic_set_voltage(self.h, V_dc, V_rf, f))

    def set_circuit(self, V, Q, Qc):
        _check(lib().rzpic_set_circuit(self.h, V, Q, Qc))

    def set_pass_shape(self, threads, parts_per_block):
        _check(lib().rzpic_set_pass_shape(self.h, threads, parts_per_block))

    def use_stream(self, stream):
        """Run the context's work on `stream` (a torch stream) from now on."""
        self.stream.synchronize()
        _check(lib().rzpic_set_stream(self.h, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def set_step_graph(self, on=True):
        """Steps captured and replayed as HIP graphs (rzpic_set_step_graph);
        needs a stream other than the null stream (use_stream)."""
        _check(lib().rzpic_set_step_graph(self.h, 1 if on else 0))

    def set_step_pipeline(self, on=True):
        """Each directly launched step prepares the next step's grid in its
        list maintenance launches (rzpic_set_step_pipeline)."""
        _check(lib().rzpic_set_step_pipeline(self.h, 1 if on else 0))

    def set_pass_form(self, form):
        _check(lib().rzpic_set_pass_form(self.h, form))

    def set_tiles(self, tile_z, tile_r):
        _check(lib().rzpic_set_tiles(self.h, tile_z, tile_r))

    def pass_config(self):
        """{threads, parts_per_block, form, tile_z, tile_r} in use."""
        out = (C.c_int32 * 5)()
        _check(lib().rzpic_get_pass_config(self.h, C.cast(out, C.c_void_p)))
        return dict(zip(("threads", "parts_per_block", "form", "tile_z", "tile_r"), list(out)))

    def autotune(self, steps, step0):
        """Times the fused pass's launch shapes over real steps from step0 and
        keeps the fastest; returns (best (threads, parts_per_block), table of
        (threads, parts_per_block, ms per step), next step index)."""
        table = (C.c_double * 48)()
        best = (C.c_int32 * 2)()
        nxt = C.c_int64()
        _check(lib().rzpic_autotune(self.h, steps, step0, C.cast(table, C.c_void_p),
                                    C.cast(best, C.c_void_p), C.byref(nxt)))
        rows = [(int(table[3 * k]), int(table[3 * k + 1]), table[3 * k + 2]) for k in range(16)]
        return (best[0], best[1]), rows, nxt.value

    def circuit(self):
        """{V, Q, Q_c, Q_conv, Q_P, Q_L} of the last solve (external circuit)."""
        out = (C.c_double * 6)()
        _check(lib().rzpic_get_circuit(self.h, C.cast(out, C.c_void_p)))
        return dict(zip(("V", "Q", "Qc", "Qconv", "Qp", "Ql"), list(out)))

    def sync(self):
        _check(lib().rzpic_sync(self.h))

    # ---- grids
    def grid(self, which):
        t = self.torch
        buf = t.empty(self.nn, dtype=t.float64, device=self.device)
        _check(lib().rzpic_grid_copy(self.h, which, C.c_void_p(buf.data_ptr()), 0))
        return buf.cpu().numpy().reshape(self.w.nz, self.w.nr)

    def set_grid(self, which, arr):
        t = self.torch
        buf = t.as_tensor(np.ascontiguousarray(arr, np.float64).reshape(-1)).to(self.device)
        _check(lib().rzpic_grid_copy(self.h, which, C.c_void_p(buf.data_ptr()), 1))
        self.stream.synchronize()

    def diag(self):
        d = Diag()
        code = lib().rzpic_get_diag(self.h, C.byref(d))
        out = {"count": list(d.count), "next_id": list(d.next_id),
               "absorbed": [list(d.absorbed[s]) for s in range(2)],
               "candidates": list(d.candidates), "events": [list(d.events[s]) for s in range(2)],
               "last_cycles": d.last_cycles, "last_relres": d.last_relres, "status": d.status,
               "particle_steps": list(d.particle_steps)}
        if code:
            _check(code)
        return out

    def set_timing(self, on=True):
        _check(lib().rzpic_set_timing(self.h, 1 if on else 0))

    def timing(self):
        """Averages per recorded step (see rzpic_get_timing)."""
        out = (C.c_double * 12)()
        _check(lib().rzpic_get_timing(self.h, C.cast(out, C.c_void_p)))
        keys = ("steps", "step_ms", "solve_ms", "vcycles", "pass_ms", "collide_ms",
                "grid_ms", "lists_ms", "n0", "n1", "resize_ms", "sort_ms")
        return dict(zip(keys, list(out)))


class Batch:
    """Contexts stepped together (rzpic_batch_*): bitwise the same as stepping
    each alone, with one launch per kernel for each group of same-shaped
    discharges."""

    def __init__(self, contexts, stream=None):
        import torch
        self.contexts = list(contexts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (C.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = C.c_void_p()
        _check(lib().rzpic_batch_create(C.cast(arr, C.c_void_p), len(self.contexts),
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def step(self, n):
        _check(lib().rzpic_batch_step(self.h, n))

    def set_graph(self, on=True):
        _check(lib().rzpic_batch_set_graph(self.h, 1 if on else 0))

    def autotune(self, steps, step0, max_rows=512):
        """Per group of like discharges, times pass configurations over real
        batched steps from step0 and keeps the fastest (rzpic_batch_autotune);
        returns (rows of {group, threads, parts_per_block, form, tile_z,
        tile_r, ms, chosen}, next step index)."""
        table = (C.c_double * (8 * max_rows))()
        rows = C.c_int32()
        nxt = C.c_int64()
        _check(lib().rzpic_batch_autotune(self.h, steps, step0, C.cast(table, C.c_void_p),
                                          max_rows, C.byref(rows), C.byref(nxt)))
        keys = ("group", "threads", "parts_per_block", "form", "tile_z", "tile_r", "ms", "chosen")
        out = []
        for k in range(min(rows.value, max_rows)):
            r = dict(zip(keys, table[8 * k:8 * k + 8]))
            for key in keys:
                if key != "ms":
                    r[key] = int(r[key])
            out.append(r)
        return out, nxt.value

    def stats(self):
        out = (C.c_int32 * 3)()
        _check(lib().rzpic_batch_stats(self.h, C.cast(out, C.c_void_p)))
        return {"groups": out[0], "launches": out[1], "batched": out[2]}

    def close(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().rzpic_batch_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_context(w, *, capacity_factor=1.6, events=False, with_xsec=True, **kw):
    """Context with both species bound (capacity = factor * initial count) and
    the workload's synthetic cross sections loaded."""
    from . import workloads as wl
    ctx = Context(w, **kw)
    hr = w.R / (w.nr - 1)
    for s in (0, 1):
        cap = max(1024, int(w.n_per_species * capacity_factor))
        w_ref = w.wcoef * w.R  # heaviest initial weight
        model = (wl.MC_ELECTRON, wl.MC_ION)[s] if with_xsec else wl.MC_NONE
        ctx.bind(s, cap, wl.SPECIES_Q[s], wl.SPECIES_M[s], w_ref, model, events=events)
    if with_xsec:
        for s, (kind, thr, sig, ejb) in wl.xsec_tables(w).items():
            ctx.set_xsec(s, kind, thr, wl.XSEC_DE, sig, ejb)
    del hr
    return ctx


class Adjoint:
    """Gradient of the smooth ion-flux objective of an N-step collision-free
    window (rzpic_adjoint_*) with respect to V_dc, V_rf and the particle
    weights at the start of the window (by identity)."""

    def __init__(self, ctx, n_steps, *, checkpoint_every=0, id_capacity=None, delta=0.0,
                 tol=0.0, max_cycles=0):
        self.ctx = ctx
        caps = id_capacity or (ctx.capacity[0], ctx.capacity[1])
        self.cfg = AdjointConfig(n_steps=n_steps, checkpoint_every=checkpoint_every,
                                 id_capacity=(C.c_int64 * 2)(*caps), delta=delta, tol=tol,
                                 max_cycles=max_cycles, reserved=0)
        self.id_capacity = tuple(caps)
        h = C.c_void_p()
        _check(lib().rzpic_adjoint_create(ctx.h, C.byref(self.cfg), C.byref(h)))
        self.h = h

    def forward(self, step0=0):
        J = C.c_double()
        _check(lib().rzpic_adjoint_forward(self.h, step0, C.byref(J)))
        return J.value

    def backward(self, density=False):
        """Returns (dJ/dV_dc, dJ/dV_rf, [dJ/dw by identity, per species]) and,
        with density=True, also dJ/dpsi on the nodes ([nz, nr] tensor) for a
        relative perturbation psi of the initial density."""
        t = self.ctx.torch
        gw = [t.zeros(self.id_capacity[s], dtype=t.float64, device=self.ctx.device)
              for s in (0, 1)]
        gd = t.zeros(self.ctx.nn, dtype=t.float64, device=self.ctx.device) if density else None
        gv = (C.c_double * 2)()
        _check(lib().rzpic_adjoint_backward(self.h, C.cast(gv, C.c_void_p),
                                            C.c_void_p(gw[0].data_ptr()),
                                            C.c_void_p(gw[1].data_ptr()),
                                            C.c_void_p(gd.data_ptr()) if density else None))
        if density:
            return gv[0], gv[1], gw, gd.view(self.ctx.w.nz, self.ctx.w.nr)
        return gv[0], gv[1], gw

    def close(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().rzpic_adjoint_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def window_objective(adj, step0, v_dc, v_rf, w_by_id):
    """J of the window as a differentiable torch function of the electrode
    voltage (0-d tensors v_dc, v_rf) and of the species weights at the start
    of the window, given by identity (w_by_id: two float64 device tensors of
    id_capacity[s] entries).  The context's particles take these weights and
    voltages before the forward window runs."""
    import torch

    class _Window(torch.autograd.Function):
        @staticmethod
        def forward(fctx, vdc, vrf, w0, w1):
            ctx = adj.ctx
            ctx.set_voltage(float(vdc), float(vrf))
            for s, wid in ((0, w0), (1, w1)):
                n, _ = ctx.count(s)
                arr = ctx.arrays[s]
                arr["w"][:n].copy_(wid[arr["id"][:n]])
            ctx.deposit()  # the window's first deposit, with these weights
            J = adj.forward(step0)
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(fctx, gJ):
            dvdc, dvrf, gw = adj.backward()
            g = float(gJ)
            return (torch.tensor(g * dvdc, dtype=torch.float64),
                    torch.tensor(g * dvrf, dtype=torch.float64), gw[0] * g, gw[1] * g)

    return _Window.apply(v_dc, v_rf, w_by_id[0], w_by_id[1])
