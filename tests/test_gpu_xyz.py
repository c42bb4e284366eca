"""The global X-Y-Z push (config push_form = XYZ; Sec. 2.3's Cartesian
alternative, carried in the particle's local frame with a_theta kept):
FP64 steps against the oracle at the 1e-10 bar, a_theta included, with
collisions on, on a mesh whose grid fits in LDS (unsorted) and on one where
it does not (tile-sorted, windows); the mixed form within its tolerances;
a step under the local push differs, and the local push is unchanged when
the a_theta array is passed."""
import numpy as np
import pytest

from gpu_helpers import compare_grid, compare_particles, load_state, pair, random_state
from oracle import rzo
from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl
from test_gpu_mixed import TOL_GRID, compare_mixed

pytestmark = pytest.mark.gpu


def _state(w, seed):
    st = random_state(w, seed, near_axis_frac=0.2, near_wall_frac=0.05)
    rng = np.random.default_rng(seed)
    for s in (0, 1):  # a_theta of the order of a_r
        p = st[s][0]
        p["at"] = rng.normal(0.0, 1.0, len(p["r"])) * np.abs(p["ar"]).mean()
    return st


def _load(o, g, st):
    load_state(o, g, st)
    for s, (p, _) in st.items():
        o.set_at(s, p["at"])


@pytest.mark.parametrize("mesh", ["33x33", "257x129"])
def test_xyz_steps_match_oracle(mesh):
    w = wl.small_fp64().replace(n_per_species=6000, push_form=wl.PUSH_XYZ, V_rf=200.0)
    if mesh == "257x129":  # deposit grid larger than LDS: sorted tiles and windows
        w = w.replace(nr=257, nz=129, R=0.08, L=0.04, n_per_species=20000, sort_every=2,
                      tile_z=16, tile_r=32)
    o, g = pair(w, capacity_factor=3.0)
    st = _state(w, 91)
    _load(o, g, st)
    o.prologue()
    g.prologue()
    if w.sort_every:
        for s in (0, 1):
            o.sort(s)
            g.sort(s)
    for n in range(6):
        assert o.step(n) == 0
        g.step(n)
        for s in (0, 1):
            assert g.count(s) == (o.count(s), o.next_id(s)), (n, s)
            gp, op = g.particles(s), o.particles(s)
            compare_particles(gp, op, w, 1e-10, label=f"step {n} s={s}")
            oat = o.get_at(s)
            sc = max(np.abs(oat).max(), 1e-300)
            assert np.abs(gp["at"] - oat).max() <= 1e-10 * sc, (n, s)
        compare_grid(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI), 1e-10, f"phi step {n}")


def test_xyz_mixed_form():
    w = wl.small_fp64().replace(n_per_species=6000, push_form=wl.PUSH_XYZ, V_rf=200.0,
                                mg_fixed_cycles=3)
    o, g = pair(w, precision="mixed", capacity_factor=3.0)
    _load(o, g, _state(w, 92))
    o.prologue()
    g.prologue()
    for n in range(4):
        assert o.step(n) == 0
        g.step(n)
    for s in (0, 1):
        compare_mixed(g.particles(s), o.particles(s), w, label=f"s={s}")
    compare_grid(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI), TOL_GRID, "phi")


def test_local_push_differs_and_ignores_a_theta():
    w = wl.small_fp64().replace(n_per_species=4000, V_rf=200.0, mg_fixed_cycles=3)
    st = _state(w, 93)
    res = {}
    for form in (wl.PUSH_LOCAL, wl.PUSH_XYZ):
        g = rzpic.make_context(w.replace(push_form=form), capacity_factor=3.0)
        for s, (p, nid) in st.items():
            g.set_particles(s, p, nid)
        g.prologue()
        for n in range(3):
            g.step(n)
        res[form] = g.particles(0)
    assert not np.array_equal(res[wl.PUSH_LOCAL]["vt"], res[wl.PUSH_XYZ]["vt"])
    # the local form against the oracle's local form (a_theta never read)
    o, g = pair(w, capacity_factor=3.0)
    load_state(o, g, st)
    o.prologue()
    g.prologue()
    for n in range(3):
        assert o.step(n) == 0
        g.step(n)
    for s in (0, 1):
        compare_particles(g.particles(s), o.particles(s), w, 1e-10, label=f"local s={s}")
