"""Pass configuration of the deposit (rzpic_set_pass_form, rzpic_set_tiles,
rzpic_get_pass_config) and the batch autotuner (rzpic_batch_autotune): the
deposit form and the tile shape change nothing but the speed and the
particle order after a sort.  Without collisions no identity depends on the
order, so runs in different configurations agree particle by particle when
matched by identity, and their potentials bit for bit."""
import numpy as np
import pytest

from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _ctx(w, precision="mixed"):
    g = rzpic.make_context(w, precision=precision, capacity_factor=1.5, with_xsec=False)
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


def _same_by_identity(a, b, what):
    for s in (0, 1):
        x, y = _by_id(a.particles(s)), _by_id(b.particles(s))
        for f in rzpic.FIELDS + ("id",):
            np.testing.assert_array_equal(x[f], y[f], err_msg=f"{what} s={s} {f}")
    np.testing.assert_array_equal(a.grid(rzpic.G_PHI), b.grid(rzpic.G_PHI), err_msg=what)
    for g in (rzpic.G_N0, rzpic.G_N1):
        np.testing.assert_array_equal(a.grid(g), b.grid(g), err_msg=what)


def test_tiled_form_and_tile_shapes_equal_lds_form_by_identity():
    w = wl.rf_129x65().replace(n_per_species=60_000, sort_every=3)
    lds, tiled = _ctx(w), _ctx(w)
    assert lds.pass_config()["form"] == rzpic.FORM_LDS
    tiled.set_pass_form(rzpic.FORM_TILED)
    assert tiled.pass_config()["form"] == rzpic.FORM_TILED
    for n in range(4):
        lds.step(n)
        tiled.step(n)
    _same_by_identity(lds, tiled, "tiled 16x32")
    # new tiles mid-run: the plan is made again at once
    tiled.set_tiles(8, 16)
    cfg = tiled.pass_config()
    assert (cfg["tile_z"], cfg["tile_r"]) == (8, 16)
    for n in range(4, 9):
        lds.step(n)
        tiled.step(n)
    _same_by_identity(lds, tiled, "tiled 8x16")
    tiled.set_tiles(32, 64)
    tiled.set_pass_form(rzpic.FORM_AUTO)
    assert tiled.pass_config()["form"] == rzpic.FORM_LDS
    for n in range(9, 11):
        lds.step(n)
        tiled.step(n)
    _same_by_identity(lds, tiled, "back to the LDS form")


def test_bad_forms_and_tiles_rejected():
    w = wl.rf_129x65().replace(nr=257, nz=129, R=0.08, L=0.04, n_per_species=4000,
                               sort_every=2)
    g = _ctx(w, precision="fp64")  # 257x129 in FP64 does not fit one workgroup's LDS
    assert g.pass_config()["form"] == rzpic.FORM_TILED
    with pytest.raises(rzpic.RzpicError):
        g.set_pass_form(rzpic.FORM_LDS)
    with pytest.raises(rzpic.RzpicError):
        g.set_pass_form(7)
    for tz, tr in ((0, 16), (16, 0), (1, 1)):  # 1x1: 32768 tiles
        with pytest.raises(rzpic.RzpicError):
            g.set_tiles(tz, tr)
    g.set_pass_form(rzpic.FORM_AUTO)
    assert g.pass_config()["form"] == rzpic.FORM_TILED
    g.step(0)
    g.sync()


def test_batch_autotune_groups_choose_once_and_change_no_result():
    base = wl.rf_129x65().replace(sort_every=4)
    ws = [base.replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=20_000, seed=1),
          base.replace(n_per_species=30_000, seed=2),
          base.replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=12_000, seed=3),
          base.replace(nr=257, nz=129, R=0.08, L=0.04, n_per_species=25_000, seed=4)]
    tuned = [_ctx(w) for w in ws]
    alone = [_ctx(w) for w in ws]
    import torch
    b = rzpic.Batch(tuned, stream=torch.cuda.Stream())
    b.set_graph(True)  # graphs are captured for every configuration tried
    b.step(0)
    rows, nxt = b.autotune(1, 1)
    for r in rows:
        print(r)
    groups = sorted({r["group"] for r in rows})
    assert groups == [0, 1, 2]  # 65x33, 129x65, 257x129
    for g in groups:
        mine = [r for r in rows if r["group"] == g]
        assert sum(r["chosen"] for r in mine) == 1
        assert all(r["ms"] > 0 for r in mine)
        # both forms where the grid fits LDS, and tile shapes (the steps sort)
        assert {r["form"] for r in mine} == {rzpic.FORM_LDS, rzpic.FORM_TILED}
        assert len({(r["tile_z"], r["tile_r"]) for r in mine}) >= 5
    # each group's contexts run its chosen configuration
    chosen = {r["group"]: r for r in rows if r["chosen"]}
    for k, g in enumerate(tuned):
        grp = {(65, 33): 0, (129, 65): 1, (257, 129): 2}[(ws[k].nr, ws[k].nz)]
        cfg, want = g.pass_config(), chosen[grp]
        for key in ("threads", "parts_per_block", "form", "tile_z", "tile_r"):
            assert cfg[key] == want[key], (k, key, cfg, want)
    for n in range(nxt, nxt + 3):
        b.step(n)
    b.close()
    for g in alone:
        for n in range(nxt + 3):
            g.step(n)
    for k, (a, t) in enumerate(zip(alone, tuned)):
        _same_by_identity(a, t, f"discharge {k}")
