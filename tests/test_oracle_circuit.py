"""Pins of the oracle's external circuit (Sec. 2.5, the superposition of
Vahedi with a blocking capacitor):

- the electrode charge of the unit Laplace solution equals its discrete
  Dirichlet energy, eps0 times the sum over the faces of the
  finite-volume mesh of (face coefficient) x (potential jump)^2, written
  here from the mesh geometry (the discrete Green identity);
- in vacuum the electrode follows the capacitive divider C/(C + Q_L) of the
  source at every step;
- phi = phi_P + V phi_L equals a direct solve with the electrode held at the
  circuit's V;
- a very large capacitor reproduces the directly driven electrode;
- the charge balance Q^t - Q^{t-1} = (Q_c^t - Q_c^{t-1}) + Q_conv^t holds and
  Q_conv is the charge of the particles absorbed at z = 0 since the
  previous solve (the first solve: since the start, prologue included)."""
import math

import numpy as np

from oracle import rzo
from paper_1001_2969_amd import workloads as wl

EPS0 = rzo.constants()["eps0"]
C_F = 1e-12


def _vacuum(w):
    o = rzo.Oracle(w, mc=False)
    empty = {f: np.zeros(0) for f in rzo.FIELDS}
    empty["id"] = np.zeros(0, np.uint64)
    for s in (0, 1):
        o.set_particles(s, empty, 0)
    o.prologue()
    return o


def _w(**kw):
    base = wl.small_fp64().replace(V_dc=0.0, V_rf=200.0, mg_tol=1e-13, mg_max_cycles=400,
                                   circuit_C=C_F)
    return base.replace(**kw)


def _dirichlet_energy(w, u, eps):
    """eps0 sum over faces of k (u_P - u_Q)^2: z-faces of the columns r < R
    (area pi hr^2/4 on the axis, 2 pi r_j hr off it, distance hz), r-faces of
    the interior rows (area 2 pi r_{j+1/2} hz, distance hr), and the half-height
    side face between the electrode's outermost node and the wall node."""
    nr, nz = w.nr, w.nz
    hr, hz = w.R / (nr - 1), w.L / (nz - 1)
    u = u.reshape(nz, nr)
    e = eps.reshape(nz, nr)
    tot = 0.0
    for j in range(nr - 1):
        area = math.pi * hr * hr / 4 if j == 0 else 2 * math.pi * j * hr * hr
        for i in range(nz - 1):
            k = 0.5 * (e[i, j] + e[i + 1, j]) * area / hz
            tot += k * (u[i, j] - u[i + 1, j]) ** 2
    for i in range(1, nz - 1):
        for j in range(nr - 1):
            k = 0.5 * (e[i, j] + e[i, j + 1]) * 2 * math.pi * (j + 0.5) * hr * hz / hr
            tot += k * (u[i, j] - u[i, j + 1]) ** 2
    jw = nr - 2
    k = 0.5 * (e[0, jw] + e[0, jw + 1]) * math.pi * (jw + 0.5) * hr * hz / hr
    tot += k * (u[0, jw] - u[0, jw + 1]) ** 2
    return EPS0 * tot


def test_electrode_charge_is_the_dirichlet_energy():
    w = _w()
    o = _vacuum(w)
    assert o.step(0) == 0
    c = o.circuit()
    phiL = o.grid(rzo.G_PHI_L)
    eps = 1.0 + o.grid(rzo.G_CHI)
    assert np.all(phiL[0, :-1] == 1.0) and np.all(phiL[-1] == 0.0) and np.all(phiL[:, -1] == 0.0)
    energy = _dirichlet_energy(w, phiL, eps)
    assert c["Ql"] > 0
    assert abs(c["Ql"] - energy) <= 1e-9 * energy, (c["Ql"], energy)


def test_vacuum_capacitive_divider():
    w = _w()
    o = _vacuum(w)
    for n in range(5):
        assert o.step(n) == 0
        c = o.circuit()
        Vs = w.V_rf * math.sin(2 * math.pi * w.f_rf * (n + 1) * w.dt)
        want = Vs * C_F / (C_F + c["Ql"])
        assert c["Qp"] == 0.0 and c["Qconv"] == 0.0
        assert abs(c["V"] - want) <= 1e-12 * abs(Vs), (n, c["V"], want)
        assert abs(c["Q"] - c["Ql"] * c["V"]) <= 1e-12 * abs(c["Q"])
        assert abs(c["Qc"] - C_F * (Vs - c["V"])) <= 1e-12 * abs(c["Qc"])


def _loaded(w, seed=3, n=3000):
    o = rzo.Oracle(w, mc=False)
    for s in (0, 1):
        parts, nid = wl.random_particles(seed + s, n, w, s, near_wall_frac=0.05)
        # electrons and ions started near the powered electrode reach it
        parts["z"][: n // 10] = np.linspace(1e-6, 2e-5, n // 10)
        o.set_particles(s, parts, nid)
    o.prologue()
    return o


def test_superposition_equals_a_direct_solve():
    w = _w()
    o = _loaded(w)
    assert o.step(0) == 0
    V = o.circuit()["V"]
    d = _loaded(w.replace(circuit_C=0.0, V_rf=0.0, V_dc=V))
    assert d.step(0) == 0
    a, b = o.grid(rzo.G_PHI), d.grid(rzo.G_PHI)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()
    for s in (0, 1):
        pa, pb = o.particles(s), d.particles(s)
        np.testing.assert_array_equal(pa["id"], pb["id"])
        assert np.abs(pa["r"] - pb["r"]).max() <= 1e-12 * w.R


def test_large_capacitor_is_the_driven_electrode():
    w = _w(circuit_C=1e-3)
    o = _loaded(w)
    d = _loaded(w.replace(circuit_C=0.0))
    for n in range(3):
        assert o.step(n) == 0 and d.step(n) == 0
        Vs = w.V_rf * math.sin(2 * math.pi * w.f_rf * (n + 1) * w.dt)
        assert abs(o.circuit()["V"] - Vs) <= 1e-6 * abs(Vs)
    a, b = o.grid(rzo.G_PHI), d.grid(rzo.G_PHI)
    assert np.abs(a - b).max() <= 1e-6 * np.abs(b).max()


def test_charge_balance_and_collected_charge():
    w = _w()
    o = _loaded(w)
    prev = o.circuit()
    counted = [0.0, 0.0]  # z = 0 absorption the previous solve counted up to
    moved = 0.0
    for n in range(8):
        # the solve of step n counts what was absorbed before the step's pass
        before = [o.absorbed(s)[0] for s in (0, 1)]
        assert o.step(n) == 0
        c = o.circuit()
        qconv = sum(wl.SPECIES_Q[s] * (before[s] - counted[s]) for s in (0, 1))
        assert abs(c["Qconv"] - qconv) <= 1e-12 * max(abs(qconv), 1e-30), (n, c["Qconv"], qconv)
        lhs = c["Q"] - prev["Q"]
        rhs = (c["Qc"] - prev["Qc"]) + c["Qconv"]
        assert abs(lhs - rhs) <= 1e-12 * max(abs(c["Q"]), abs(c["Qc"])), (n, lhs, rhs)
        moved += abs(c["Qconv"])
        prev, counted = c, before
    assert moved > 0.0  # particles did reach the electrode
