"""Autotuner of the fused pass's launch shape (rzpic_autotune,
rzpic_set_pass_shape): the shapes it times change nothing but the speed.
A tuned context ends bit for bit where an untuned one stepped as far ends
(whole-grid LDS deposit, collisions on); on a tile-sorted mesh, where a new
shape is re-planned by a sort, the particles agree by identity (no
collisions, so no identities depend on the order); bad shapes are
rejected."""
import numpy as np
import pytest

from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _ctx(w, with_xsec=True):
    g = rzpic.make_context(w, capacity_factor=1.5, with_xsec=with_xsec)
    for s, T in ((0, w.Te_eV), (1, w.Ti_eV)):
        g.init_particles(s, w.n_per_species, w.n0, T, 0)
    g.prologue()
    if w.sort_every:
        for s in (0, 1):
            g.sort(s)
    return g


def _by_id(p):
    o = np.argsort(p["id"])
    return {f: p[f][o] for f in p}


def test_tuned_run_equals_untuned_bitwise():
    w = wl.rf_129x65().replace(n_per_species=200_000)
    tuned, plain = _ctx(w), _ctx(w)
    best, table, nxt = tuned.autotune(2, 0)
    print("best", best, "table", table)
    assert best in [(t, p) for t, p, ms in table if ms > 0]
    assert nxt == 3 * sum(1 for _, _, ms in table if ms > 0)
    for n in range(nxt):
        plain.step(n)
    for n in range(nxt, nxt + 3):
        tuned.step(n)
        plain.step(n)
    for s in (0, 1):
        a, b = tuned.particles(s), plain.particles(s)
        for f in rzpic.FIELDS + ("id",):
            np.testing.assert_array_equal(a[f], b[f], err_msg=f"s={s} {f}")
    np.testing.assert_array_equal(tuned.grid(rzpic.G_PHI), plain.grid(rzpic.G_PHI))


def test_tuned_tiled_run_equals_untuned_by_identity():
    w = wl.rf_129x65().replace(nr=257, nz=129, R=0.08, L=0.04, n_per_species=60_000,
                               sort_every=4, mg_fixed_cycles=3)
    tuned, plain = _ctx(w, with_xsec=False), _ctx(w, with_xsec=False)
    best, table, nxt = tuned.autotune(1, 0)
    print("best", best, "table", table)
    for n in range(nxt):
        plain.step(n)
    for s in (0, 1):
        a, b = _by_id(tuned.particles(s)), _by_id(plain.particles(s))
        for f in rzpic.FIELDS + ("id",):
            np.testing.assert_array_equal(a[f], b[f], err_msg=f"s={s} {f}")
    np.testing.assert_array_equal(tuned.grid(rzpic.G_PHI), plain.grid(rzpic.G_PHI))


def test_bad_shapes_rejected():
    g = _ctx(wl.small_fp64().replace(n_per_species=2000))
    for t, p in ((128, 8192), (512, 16), (2048, 8192)):
        with pytest.raises(rzpic.RzpicError):
            g.set_pass_shape(t, p)
    g.set_pass_shape(256, 4096)
    g.step(0)
