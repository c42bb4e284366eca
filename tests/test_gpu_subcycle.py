"""Ion subcycling (config ion_subcycle = K; Sec. 2.7): FP64 steps against the
oracle at the 1e-10 bar with collisions on, on a mesh whose deposit grid
fits in LDS and on one where it does not; the mixed form within its
tolerances; K = 1 equal to the plain step and a subcycled discharge in a
batch equal to its own steps, bit for bit."""
import numpy as np
import pytest

from gpu_helpers import compare_grid, compare_particles, load_state, pair, random_state
from oracle import rzo
from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl
from test_gpu_mixed import TOL_GRID, compare_mixed

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mesh", ["33x33", "257x129"])
def test_subcycled_steps_match_oracle(mesh):
    w = wl.small_fp64().replace(n_per_species=6000, ion_subcycle=3, V_rf=200.0)
    if mesh == "257x129":  # deposit grid larger than LDS
        w = w.replace(nr=257, nz=129, R=0.08, L=0.04, n_per_species=20000)
    o, g = pair(w, capacity_factor=3.0)
    load_state(o, g, random_state(w, 81, near_axis_frac=0.05, near_wall_frac=0.05))
    o.prologue()
    g.prologue()
    for n in range(7):
        assert o.step(n) == 0
        g.step(n)
        for s in (0, 1):
            assert g.count(s) == (o.count(s), o.next_id(s)), (n, s)
            compare_particles(g.particles(s), o.particles(s), w, 1e-10, label=f"step {n} s={s}")
        compare_grid(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI), 1e-10, f"phi step {n}")
        compare_grid(g.grid(rzpic.G_CHI), o.grid(rzo.G_CHI), 1e-10, f"chi step {n}")
        compare_grid(g.grid(rzpic.G_N1), o.grid(rzo.G_N1), 1e-10, f"N1 step {n}")


def test_subcycled_mixed_form():
    w = wl.small_fp64().replace(n_per_species=6000, ion_subcycle=2, V_rf=200.0,
                                mg_fixed_cycles=3)
    o, g = pair(w, precision="mixed", capacity_factor=3.0)
    load_state(o, g, random_state(w, 82))
    o.prologue()
    g.prologue()
    for n in range(5):
        assert o.step(n) == 0
        g.step(n)
    for s in (0, 1):
        compare_mixed(g.particles(s), o.particles(s), w, label=f"s={s}")
    compare_grid(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI), TOL_GRID, "phi")


def _run(w, steps, st, batch_with=None):
    g = rzpic.make_context(w, capacity_factor=3.0)
    for s, (p, nid) in st.items():
        g.set_particles(s, p, nid)
    g.prologue()
    if batch_with is None:
        for n in range(steps):
            g.step(n)
        return g, None
    b = rzpic.Batch([g] + batch_with)
    for n in range(steps):
        b.step(n)
    return g, b


def _same(ga, gb):
    for s in (0, 1):
        pa, pb = ga.particles(s), gb.particles(s)
        for f in rzpic.FIELDS + ("id",):
            np.testing.assert_array_equal(pa[f], pb[f], err_msg=f"s={s} {f}")
    np.testing.assert_array_equal(ga.grid(rzpic.G_PHI), gb.grid(rzpic.G_PHI))


def test_k1_equals_the_plain_step_and_batch():
    w = wl.small_fp64().replace(n_per_species=5000, V_rf=200.0, mg_fixed_cycles=3)
    st = random_state(w, 83)
    a, _ = _run(w, 4, st)
    b, _ = _run(w.replace(ion_subcycle=1), 4, st)
    _same(a, b)
    ws = w.replace(ion_subcycle=3)
    alone, _ = _run(ws, 6, st)
    other = rzpic.make_context(wl.rf_129x65().replace(nr=65, nz=33, R=0.02, L=0.01,
                                                      n_per_species=20000),
                               precision="mixed", capacity_factor=2.0)
    for s, T in ((0, 2.0), (1, 0.026)):
        other.init_particles(s, 20000, 5e15, T, 0)
    other.prologue()
    batched, bt = _run(ws, 6, st, batch_with=[other])
    _same(alone, batched)
    bt.close()
