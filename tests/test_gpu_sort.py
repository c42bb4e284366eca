"""Tile sort and the tiled particle pass against the oracle.

The sort (the paper orders particles by cell for the weighting, Sec. 2.7) is
a stable counting sort by tile: the GPU result equals the oracle's bit for
bit, in array order.  The tiled pass (blocks over contiguous ranges of the
sorted array, deposit into LDS windows, global atomics for the particles
outside them) changes no result: the tests force it on small meshes
(RZPIC_NO_LDS disables the whole-grid LDS deposit) and compare every step
with the oracle in array order, and with the whole-grid LDS form bit for bit."""
import numpy as np
import pytest

from gpu_helpers import compare_grid, compare_particles, load_state, pair, random_state
from oracle import rzo
from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _small(**kw):
    return wl.small_fp64().replace(**kw)


def _edge_state(w, seed, n):
    """Random particles, some near the axis and the wall, and the first ones
    exactly on cell and tile boundaries (z = L and r = R included)."""
    st = random_state(w, seed, n=n, near_axis_frac=0.05, near_wall_frac=0.05)
    hz, hr = w.L / (w.nz - 1), w.R / (w.nr - 1)
    for s in (0, 1):
        p = st[s][0]
        k = min(n, 2 * w.nz)
        p["z"][:k] = hz * (np.arange(k) % w.nz)
        p["r"][:k] = hr * (np.arange(k) % w.nr)
    return st


def _as_float32(st):
    out = {}
    for s, (p, nid) in st.items():
        q = dict(p)
        for f in rzo.FIELDS:
            q[f] = np.asarray(p[f], np.float32).astype(np.float64)
        out[s] = (q, nid)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tiles,n", [((4, 8), 20000), ((1, 1), 9000), ((32, 32), 5000),
                                     ((3, 5), 777), ((16, 32), 0)])
def test_sort_equals_oracle_bitwise(precision, tiles, n):
    w = _small(n_per_species=max(n, 1000), tile_z=tiles[0], tile_r=tiles[1])
    o, g = pair(w, precision=precision)
    st = _edge_state(w, 41, n)
    ost = _as_float32(st) if precision == "mixed" else st
    for s in (0, 1):
        o.set_particles(s, *ost[s])
        g.set_particles(s, *st[s])
    for rnd in range(2):  # the second sort finds the order already sorted
        for s in (0, 1):
            o.sort(s)
            g.sort(s)
        for s in (0, 1):
            gp, op = g.particles(s), o.particles(s)
            assert g.count(s) == (o.count(s), o.next_id(s))
            for f in rzo.FIELDS + ("id",):
                np.testing.assert_array_equal(gp[f], op[f], err_msg=f"round {rnd} s={s} {f}")


def _steps_in_order(o, g, w, nsteps, tol=TOL):
    for n in range(nsteps):
        assert o.step(n) == 0
        g.step(n)
        for s in (0, 1):
            assert g.count(s) == (o.count(s), o.next_id(s)), (n, s)
            compare_particles(g.particles(s), o.particles(s), w, tol, ordered=True,
                              label=f"step {n} s={s}")
        compare_grid(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI), tol, f"phi step {n}")
        for go, oo in ((rzpic.G_N0, rzo.G_N0), (rzpic.G_N1, rzo.G_N1)):
            compare_grid(g.grid(go), o.grid(oo), tol, f"N step {n}")


@pytest.mark.parametrize("sort_every,resize_every", [(0, 0), (1, 0), (3, 0), (2, 2)])
def test_tiled_pass_steps_match_oracle(sort_every, resize_every, monkeypatch):
    """Sorted after the prologue and every sort_every steps (windows go stale
    in between: particles drift, holes are filled from the end, children and
    clones are appended), with collisions and weight splits.  sort_every = 0:
    never sorted, so the tiled pass runs without a plan (no windows)."""
    monkeypatch.setenv("RZPIC_NO_LDS", "1")
    w = _small(n_per_species=20000, sort_every=sort_every, resize_every=resize_every,
               tile_z=4, tile_r=8, xsec="powerlaw")
    o, g = pair(w, capacity_factor=4.0)
    st = random_state(w, 42, near_axis_frac=0.05, near_wall_frac=0.05)
    load_state(o, g, st)
    o.prologue()
    g.prologue()
    if sort_every:
        for s in (0, 1):
            o.sort(s)
            g.sort(s)
    _steps_in_order(o, g, w, 6)


def test_tiled_and_whole_grid_deposits_agree_bitwise(monkeypatch):
    """The same sorted run with the whole-grid LDS deposit, with LDS windows,
    and with the single operations (whose deposit is tiled too)."""
    w = _small(n_per_species=15000, sort_every=2, tile_z=8, tile_r=8)
    st = random_state(w, 43)
    outs = []
    for no_lds, merged in ((False, True), (True, True), (True, False)):
        if no_lds:
            monkeypatch.setenv("RZPIC_NO_LDS", "1")
        else:
            monkeypatch.delenv("RZPIC_NO_LDS", raising=False)
        g = rzpic.make_context(w, capacity_factor=2.0)
        for s, (p, nid) in st.items():
            g.set_particles(s, p, nid)
        g.prologue()
        for s in (0, 1):
            g.sort(s)
        for n in range(5):
            if merged:
                g.step(n)
                continue
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
            if n % 2 == 1:
                for s in (0, 1):
                    g.sort(s)
        out = {s: g.particles(s) for s in (0, 1)}
        out["phi"] = g.grid(rzpic.G_PHI)
        out["N0"] = g.grid(rzpic.G_N0)
        outs.append(out)
    for b in outs[1:]:
        for s in (0, 1):
            for f in rzo.FIELDS + ("id",):
                np.testing.assert_array_equal(outs[0][s][f], b[s][f])
        np.testing.assert_array_equal(outs[0]["phi"], b["phi"])
    np.testing.assert_array_equal(outs[0]["N0"], outs[1]["N0"])


def test_sort_rejects_staged_children():
    w = _small(n_per_species=2000)
    g = rzpic.make_context(w)
    st = random_state(w, 44, n=2000)
    st[0][0]["vr"] *= 20  # hot electrons ionize
    for s, (p, nid) in st.items():
        g.set_particles(s, p, nid)
    g.prologue()
    for s in (0, 1):
        g.push_final(s)
    g.collide(0, 0)
    with pytest.raises(rzpic.RzpicError) as ei:
        g.sort(0)
    assert ei.value.code == 7
