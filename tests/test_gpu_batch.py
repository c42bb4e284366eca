"""Batched steps of independent discharges (rzpic_batch_*): every discharge
of a batch ends bit for bit where stepping its context alone ends, whatever
the mix of meshes, particle counts and precisions; and one small FP64
discharge of a batch against the oracle."""
import numpy as np
import pytest

from gpu_helpers import compare_grid, compare_particles, load_state, pair, random_state
from oracle import rzo
from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _discharges():
    """Uneven meshes and counts; two share a shape (one group), one is FP64,
    one sorts by tile every 2 steps, one splits weights every 3 steps."""
    base = wl.rf_129x65()
    return [
        (base.replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=30000, seed=1), "mixed"),
        (base.replace(n_per_species=50000, seed=2), "mixed"),
        (base.replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=12000, seed=3), "mixed"),
        (base.replace(nr=33, nz=33, R=0.02, L=0.02, n_per_species=8000, seed=4,
                      V_rf=0.0, V_dc=50.0), "fp64"),
        (base.replace(nr=129, nz=65, n_per_species=40000, seed=5, sort_every=2, tile_z=8,
                      tile_r=16, xsec="powerlaw"), "mixed"),
        (base.replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=20000, seed=6,
                      resize_every=3), "fp64"),
    ]


def _make(w, precision):
    g = rzpic.make_context(w, precision=precision, capacity_factor=3.0)
    for s, T in ((0, w.Te_eV), (1, w.Ti_eV)):
        g.init_particles(s, w.n_per_species, w.n0, T, 0)
    g.prologue()
    return g


def _state(g):
    out = {s: g.particles(s) for s in (0, 1)}
    out["phi"] = g.grid(rzpic.G_PHI)
    out["N0"] = g.grid(rzpic.G_N0)
    out["N1"] = g.grid(rzpic.G_N1)
    return out


def test_batch_equals_separate_steps_bitwise():
    ds = _discharges()
    alone = [_make(w, p) for w, p in ds]
    batched = [_make(w, p) for w, p in ds]
    b = rzpic.Batch(batched)
    for n in range(6):
        for g in alone:
            g.step(n)
        b.step(n)
    for k, (ga, gb) in enumerate(zip(alone, batched)):
        a, c = _state(ga), _state(gb)
        for s in (0, 1):
            assert ga.count(s) == gb.count(s), (k, s)
            for f in rzo.FIELDS + ("id",):
                np.testing.assert_array_equal(a[s][f], c[s][f], err_msg=f"discharge {k} s={s} {f}")
        for key in ("phi", "N0", "N1"):
            np.testing.assert_array_equal(a[key], c[key], err_msg=f"discharge {k} {key}")
        da, dc = ga.diag(), gb.diag()
        assert da["absorbed"] == dc["absorbed"] and da["events"] == dc["events"]
    st = b.stats()
    print("batch stats", st)
    assert st["groups"] == len(ds) - 1  # the two 65x33 mixed discharges with no options share one
    assert st["batched"] > 0
    b.close()


def test_batched_fp64_discharge_matches_oracle():
    w = wl.small_fp64().replace(n_per_species=6000, mg_fixed_cycles=4)
    other = wl.rf_129x65().replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=10000)
    o, g = pair(w, capacity_factor=3.0)
    st = random_state(w, 51, near_axis_frac=0.05, near_wall_frac=0.05)
    load_state(o, g, st)
    o.prologue()
    g.prologue()
    g2 = _make(other, "mixed")
    b = rzpic.Batch([g2, g])
    for n in range(4):
        assert o.step(n) == 0
        b.step(n)
        for s in (0, 1):
            assert g.count(s) == (o.count(s), o.next_id(s))
            compare_particles(g.particles(s), o.particles(s), w, 1e-10, label=f"step {n} s={s}")
        compare_grid(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI), 1e-10, f"phi step {n}")
    b.close()


def test_batch_rejects_what_it_cannot_record():
    w = wl.small_fp64().replace(n_per_species=1000)  # tolerance-mode multigrid
    g = _make(w, "fp64")
    with pytest.raises(rzpic.RzpicError) as ei:
        rzpic.Batch([g])
    assert ei.value.code == 1
    g2 = _make(w.replace(mg_fixed_cycles=2), "fp64")
    b = rzpic.Batch([g2])
    g2.set_timing(True)
    with pytest.raises(rzpic.RzpicError) as ei:
        b.step(0)
    assert ei.value.code == 1
    g2.set_timing(False)
    b.step(0)
    b.close()


def test_graph_replayed_batch_equals_separate_steps_every_step():
    """Batched steps replayed from captured graphs (two captures, one per
    staging buffer; a tile-sort step in between launches directly), compared
    with the contexts stepped alone after every step, with the host reading
    results between replays."""
    base = wl.rf_129x65()
    ds = [(base.replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=20000, seed=11, sort_every=4),
           "mixed"),
          (base.replace(n_per_species=30000, seed=12), "mixed"),
          (base.replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=15000, seed=13), "fp64")]
    alone = [_make(w, p) for w, p in ds]
    batched = [_make(w, p) for w, p in ds]
    import torch
    stream = torch.cuda.Stream()
    b = rzpic.Batch(batched, stream=stream)
    b.set_graph(True)
    for n in range(9):
        for g in alone:
            g.step(n)
        b.step(n)
        stream.synchronize()
        for k, (ga, gb) in enumerate(zip(alone, batched)):
            for s in (0, 1):
                pa, pb = ga.particles(s), gb.particles(s)
                for f in ("r", "z", "vr", "w", "id"):
                    np.testing.assert_array_equal(pa[f], pb[f], err_msg=f"step {n} discharge {k} {f}")
            np.testing.assert_array_equal(ga.grid(rzpic.G_PHI), gb.grid(rzpic.G_PHI))
    b.close()
