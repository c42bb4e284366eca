"""The grid access and solve entry points of the C ABI:

- rzpic_grid_view: torch tensors over the context's own grids (no copy);
  their values are the grids rzpic_grid_copy returns, and rho/chi written
  through them are the sources of the next solve;
- rzpic_set_grid_source: the same as writing rho and chi by rzpic_grid_copy;
- rzpic_solve_dev: cycles and relative residual written on the device, equal
  to what rzpic_solve returns on the host;
- tolerance-mode solves, which synchronise once per batch of cycles: a solve
  that stops after k cycles equals exactly k fixed cycles from the same start,
  and k - 1 cycles do not meet the tolerance (the stop is the first cycle that
  does), also when a solve needs more cycles than the one before it."""
import numpy as np
import pytest
import torch

from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _w(nr=65, nz=33, **kw):
    return wl.Workload(name="t", nr=nr, nz=nz, R=0.02 * nr / 33, L=0.02 * (nz - 1) / 32,
                       n_per_species=1, steps=1, V_dc=35.0, **kw)


def _ctx(w, **kw):
    return rzpic.Context(w, **kw)


def _phi0(w, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-5.0, 5.0, (w.nz, w.nr))


def test_grid_view_is_the_context_memory():
    w = _w()
    g = _ctx(w, mg_fixed_cycles=2)
    chi = wl.smooth_chi(w, 1.0)
    rho = wl.smooth_rho(w, 3, 2e-4)
    v = g.grid_view()
    assert set(v) >= {"phi", "rho", "chi", "er", "ez", "dens0", "dens1", "vol"}
    assert "phi_p" not in v
    v["rho"].copy_(torch.as_tensor(rho, device=v["rho"].device))
    v["chi"].copy_(torch.as_tensor(chi, device=v["chi"].device))
    v["phi"].copy_(torch.as_tensor(_phi0(w, 1), device=v["phi"].device))
    np.testing.assert_array_equal(g.grid(rzpic.G_RHO), rho)
    np.testing.assert_array_equal(g.grid(rzpic.G_CHI), chi)
    g.solve(1e-9, want=False)
    g.efield()
    v = g.grid_view()  # phi may have moved to the other buffer
    g.sync()
    np.testing.assert_array_equal(v["phi"].cpu().numpy(), g.grid(rzpic.G_PHI))
    np.testing.assert_array_equal(v["er"].cpu().numpy(), g.grid(rzpic.G_ER))
    np.testing.assert_array_equal(v["vol"].cpu().numpy(), g.grid(rzpic.G_VOL))
    # the same solve with the sources set by copies
    h = _ctx(w, mg_fixed_cycles=2)
    h.set_grid(rzpic.G_RHO, rho)
    h.set_grid(rzpic.G_CHI, chi)
    h.set_grid(rzpic.G_PHI, _phi0(w, 1))
    h.solve(1e-9, want=False)
    np.testing.assert_array_equal(h.grid(rzpic.G_PHI), g.grid(rzpic.G_PHI))


def test_set_grid_source_equals_grid_copies():
    w = _w(nr=129, nz=65)
    chi = wl.smooth_chi(w, 0.7)
    rho = wl.smooth_rho(w, 4, 1e-4)
    a, b = _ctx(w, mg_tol=1e-10), _ctx(w, mg_tol=1e-10)
    a.set_grid_source(torch.as_tensor(rho.ravel(), device="cuda:0"),
                      torch.as_tensor(chi.ravel(), device="cuda:0"))
    b.set_grid(rzpic.G_RHO, rho)
    b.set_grid(rzpic.G_CHI, chi)
    ra, rb = a.solve(0.0), b.solve(0.0)
    assert ra == rb
    np.testing.assert_array_equal(a.grid(rzpic.G_PHI), b.grid(rzpic.G_PHI))


@pytest.mark.parametrize("fixed", [3, 0])
def test_solve_dev_matches_host_results(fixed):
    w = _w()
    chi = wl.smooth_chi(w, 1.0)
    rho = wl.smooth_rho(w, 6, 2e-4)
    kw = {"mg_fixed_cycles": fixed} if fixed else {"mg_tol": 1e-10}
    a, b = _ctx(w, **kw), _ctx(w, **kw)
    for c in (a, b):
        c.set_grid(rzpic.G_RHO, rho)
        c.set_grid(rzpic.G_CHI, chi)
        c.set_grid(rzpic.G_PHI, _phi0(w, 2))
    cyc = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    rr = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    a.solve_dev(0.0, cyc, rr)
    a.sync()
    hc, hr = b.solve(0.0)
    assert int(cyc.item()) == hc
    assert float(rr.item()) == hr
    np.testing.assert_array_equal(a.grid(rzpic.G_PHI), b.grid(rzpic.G_PHI))
    a.solve_dev(0.0)  # no outputs asked: nothing to write
    a.sync()


@pytest.mark.parametrize("mesh,path", [((65, 33), "block"), ((129, 65), "default"),
                                       ((513, 129), "multi"), ((257, 129), "long")])
def test_tolerance_stop_equals_fixed_cycles(mesh, path, monkeypatch):
    if path != "default":
        monkeypatch.setenv("RZPIC_MG_PATH", path)
    w = _w(*mesh)
    chi = wl.smooth_chi(w, 1.0)
    tol = 1e-10
    g = _ctx(w, mg_tol=tol, mg_max_cycles=80)
    g.set_grid(rzpic.G_CHI, chi)
    g.set_grid(rzpic.G_PHI, _phi0(w, 5))
    # a sequence of solves: warm starts need few cycles, then a new source
    # needs many more than the hint of the previous solve
    for step, amp in enumerate((2e-4, 2e-4, 5e-2, 5e-2)):
        rho = wl.smooth_rho(w, 10 + step, amp)
        g.set_grid(rzpic.G_RHO, rho)
        start = g.grid(rzpic.G_PHI)
        k, rr = g.solve(0.0)
        assert rr <= tol
        got = g.grid(rzpic.G_PHI)
        for kk in (k, k - 1):
            if kk < 1:
                continue
            f = _ctx(w, mg_fixed_cycles=kk)
            f.set_grid(rzpic.G_CHI, chi)
            f.set_grid(rzpic.G_RHO, rho)
            f.set_grid(rzpic.G_PHI, start)
            fk, frr = f.solve(0.0)
            if kk == k:
                np.testing.assert_array_equal(f.grid(rzpic.G_PHI), got)
                assert frr == rr
            else:
                assert frr > tol, (k, frr)
