"""External circuit of the powered electrode (config circuit_C > 0; Sec. 2.5
superposition with a blocking capacitor): FP64 steps against the oracle at
the 1e-10 bar (particles, phi, phi_P, phi_L and the circuit state), with
converged and with fixed-cycle solves and collisions on; the mixed form
within the mixed tolerances (electrode charges 1e-5, unit-solution charge
1e-6, electrode potential 1e-5 of (|Q_P| + |Q_c|) / (C + Q_L), the scale its
charge balance sets); the merged step against the single
operations bit for bit; a circuit discharge in a batch bit for bit; the
state setter and the rejected calls."""
import math

import numpy as np
import pytest

from gpu_helpers import compare_grid, compare_particles, load_state, pair, random_state
from oracle import rzo
from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl
from test_gpu_mixed import TOL_GRID, compare_mixed

pytestmark = pytest.mark.gpu

W = wl.small_fp64().replace(n_per_species=6000, V_dc=20.0, V_rf=200.0, circuit_C=1e-12,
                            mg_tol=1e-12, mg_max_cycles=400)
KEYS = ("V", "Q", "Qc", "Qconv", "Qp", "Ql")


def _state(w, seed):
    st = random_state(w, seed, near_axis_frac=0.05, near_wall_frac=0.05)
    for s in (0, 1):  # a tenth of each species starts next to the powered electrode
        z = st[s][0]["z"]
        z[: len(z) // 10] = np.linspace(1e-6, 3e-5, len(z) // 10)
    return st


def _compare_circuit(gc, oc, label):
    scale = max(abs(oc["Q"]), abs(oc["Qc"]), abs(oc["Qp"]), 1e-30)
    for k in KEYS:
        sc = {"V": max(abs(oc["V"]), 1.0), "Ql": abs(oc["Ql"])}.get(k, scale)
        assert abs(gc[k] - oc[k]) <= 1e-10 * sc, (label, k, gc[k], oc[k])


@pytest.mark.parametrize("cycles", [0, 3])
def test_circuit_steps_match_oracle(cycles):
    w = W.replace(mg_fixed_cycles=cycles)
    o, g = pair(w, capacity_factor=3.0)
    load_state(o, g, _state(w, 71))
    o.prologue()
    g.prologue()
    g.set_circuit(5.0, -2e-12, 1e-12)  # a charged start
    o.set_circuit(5.0, -2e-12, 1e-12)
    moved = 0.0
    for n in range(6):
        assert o.step(n) == 0
        g.step(n)
        for s in (0, 1):
            assert g.count(s) == (o.count(s), o.next_id(s))
            compare_particles(g.particles(s), o.particles(s), w, 1e-10, label=f"step {n} s={s}")
        compare_grid(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI), 1e-10, f"phi step {n}")
        compare_grid(g.grid(rzpic.G_PHI_P), o.grid(rzo.G_PHI_P), 1e-10, f"phi_P step {n}")
        compare_grid(g.grid(rzpic.G_PHI_L), o.grid(rzo.G_PHI_L), 1e-10, f"phi_L step {n}")
        gc, oc = g.circuit(), o.circuit()
        _compare_circuit(gc, oc, f"step {n}")
        moved += abs(oc["Qconv"])
    assert moved > 0.0
    print("circuit after 6 steps", g.circuit())


@pytest.mark.parametrize("cycles", [3, 0])
def test_circuit_mixed_form(cycles):
    """Fixed cycles and converged solves: the electrode potential's error is
    the same in both (about 2e-4 V here), so it comes from the FP32 particle
    charge near the electrode, not from the FP32 correction cycles."""
    w = W.replace(mg_fixed_cycles=cycles)
    o, g = pair(w, precision="mixed", capacity_factor=3.0)
    load_state(o, g, _state(w, 72))
    o.prologue()
    g.prologue()
    for n in range(4):
        assert o.step(n) == 0
        g.step(n)
    for s in (0, 1):
        compare_mixed(g.particles(s), o.particles(s), w, label=f"s={s}")
    compare_grid(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI), TOL_GRID, "phi")
    # The electrode charges carry the FP32 particle state's error (~1e-6
    # relative here, with converged solves as with three cycles).  V is a
    # difference of charges over C + Q_L: its error scales with
    # (|Q_P| + |Q_c|) / (C + Q_L), here hundreds of volts against |V| ~ 1.6 V.
    gc, oc = g.circuit(), o.circuit()
    print("mixed circuit", gc, "oracle", oc)
    vscale = max(abs(oc["V"]), (abs(oc["Qp"]) + abs(oc["Qc"])) / (w.circuit_C + oc["Ql"]))
    assert abs(gc["V"] - oc["V"]) <= 1e-5 * vscale, (gc["V"], oc["V"], vscale)
    for k in ("Qp", "Q"):
        assert abs(gc[k] - oc[k]) <= 1e-5 * abs(oc[k]), (k, gc[k], oc[k])
    assert abs(gc["Ql"] - oc["Ql"]) <= 1e-6 * oc["Ql"], (gc["Ql"], oc["Ql"])


def test_circuit_merged_step_equals_single_operations():
    w = W.replace(mg_fixed_cycles=3)
    st = _state(w, 73)
    res = []
    for merged in (True, False):
        g = rzpic.make_context(w, capacity_factor=3.0)
        for s, (p, nid) in st.items():
            g.set_particles(s, p, nid)
        g.prologue()
        for n in range(4):
            if merged:
                g.step(n)
            else:
                g.deposit()
                g.solve((n + 1) * w.dt, want=False)
                g.efield()
                for s in (0, 1):
                    g.push_final(s)
                for s in (0, 1):
                    g.collide(s, n)
                for s in (0, 1):
                    g.push_first(s)
                g.deposit()
                for s in (0, 1):
                    g.compact(s)
        res.append(({s: g.particles(s) for s in (0, 1)}, g.grid(rzpic.G_PHI), g.circuit()))
    (pa, phia, ca), (pb, phib, cb) = res
    for s in (0, 1):
        for f in rzpic.FIELDS + ("id",):
            np.testing.assert_array_equal(pa[s][f], pb[s][f], err_msg=f"s={s} {f}")
    np.testing.assert_array_equal(phia, phib)
    assert ca == cb


def test_circuit_discharge_in_a_batch():
    w = W.replace(mg_fixed_cycles=3)
    other = wl.rf_129x65().replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=20000)
    st = _state(w, 74)

    def make(wk, own):
        g = rzpic.make_context(wk, precision="fp64" if own else "mixed", capacity_factor=3.0)
        if own:
            for s, (p, nid) in st.items():
                g.set_particles(s, p, nid)
        else:
            for s, T in ((0, wk.Te_eV), (1, wk.Ti_eV)):
                g.init_particles(s, wk.n_per_species, wk.n0, T, 0)
        g.prologue()
        return g

    alone, batched = make(w, True), [make(w, True), make(other, False)]
    b = rzpic.Batch(batched)
    for n in range(4):
        alone.step(n)
        b.step(n)
    for s in (0, 1):
        pa, pb = alone.particles(s), batched[0].particles(s)
        for f in rzpic.FIELDS + ("id",):
            np.testing.assert_array_equal(pa[f], pb[f], err_msg=f"s={s} {f}")
    np.testing.assert_array_equal(alone.grid(rzpic.G_PHI), batched[0].grid(rzpic.G_PHI))
    assert alone.circuit() == batched[0].circuit()
    b.close()


def test_circuit_state_and_rejections():
    g = rzpic.make_context(W.replace(circuit_C=0.0), capacity_factor=2.0)
    with pytest.raises(rzpic.RzpicError):
        g.circuit()
    with pytest.raises(rzpic.RzpicError):
        g.set_circuit(0.0, 0.0, 0.0)
    with pytest.raises(rzpic.RzpicError):
        rzpic.make_context(W.replace(circuit_C=-1.0), capacity_factor=2.0)
    g = rzpic.make_context(W, capacity_factor=2.0)
    assert g.circuit() == dict.fromkeys(KEYS, 0.0)
    g.set_circuit(1.5, 2e-12, -3e-12)
    c = g.circuit()
    assert (c["V"], c["Q"], c["Qc"]) == (1.5, 2e-12, -3e-12)
    with pytest.raises(rzpic.RzpicError):
        g.set_circuit(math.nan, 0.0, 0.0)
    with pytest.raises(rzpic.RzpicError):
        rzpic.Adjoint(g, 2)
