"""Friedman damping (RZPIC_DAMP_FRIEDMAN) on the GPU against the oracle: the
merged steps of the 33x33 workload with collisions (FP64 at 1e-10 per field
and on phi and the deposits), the mixed form on the 129x65 workload's mesh
(mixed tolerances), the leapfrog limit theta = 0, and the checks of the
configuration (theta in [0, 1], local push, no gradient window)."""
import numpy as np
import pytest

from gpu_helpers import pair, rel_err
from oracle import rzo
from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl
from test_gpu_mixed import TOL_GRID, compare_mixed
from test_gpu_parity import _run_steps

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("theta", [0.6, 1.0, 0.0])
def test_friedman_ten_steps_fp64(theta):
    """33x33 mesh, 20k + 20k particles, 50 V DC, 10 merged steps from the
    seeded init, with collisions."""
    w = wl.small_fp64().replace(damping=wl.DAMP_FRIEDMAN, theta=theta)
    o, g, errs = _run_steps(w, w.steps, own_init=True)
    d = g.diag()
    for s in (0, 1):
        np.testing.assert_allclose(d["absorbed"][s], o.absorbed(s), rtol=1e-9, atol=1e-30)
        assert d["next_id"][s] == o.next_id(s)
    # the damped push changed the run: chi scaled, B carried
    if theta != 1.0:
        np.testing.assert_allclose(g.grid(rzpic.G_CHI), o.grid(rzo.G_CHI), rtol=1e-10,
                                   atol=1e-12 * np.abs(o.grid(rzo.G_CHI)).max())
    print("theta", theta, "worst per-step errors", errs[-1])


def test_friedman_mixed_two_steps():
    """The 129x65 mesh with 200k + 200k particles, theta = 0.5: two merged
    steps of the mixed form against the FP64 oracle (the mixed tolerances)."""
    w = wl.rf_129x65().replace(n_per_species=200_000, damping=wl.DAMP_FRIEDMAN, theta=0.5)
    o, g = pair(w, precision="mixed", capacity_factor=2.0)
    for s, T in ((0, w.Te_eV), (1, w.Ti_eV)):
        o.init_particles(s, w.n_per_species, w.n0, T, 0)
        g.init_particles(s, w.n_per_species, w.n0, T, 0)
    o.prologue()
    g.prologue()
    for n in range(2):
        assert o.step(n) == 0
        g.step(n)
        for s in (0, 1):
            _, frac, _ = compare_mixed(g.particles(s), o.particles(s), w, f"step {n} s={s}")
            assert frac <= 1e-4
        e = rel_err(g.grid(rzpic.G_PHI), o.grid(rzo.G_PHI))
        print(f"step {n}: phi error {e:.3e}")
        assert e <= TOL_GRID


def test_friedman_configuration_checks():
    for kw in ({"theta": 1.5}, {"theta": -0.25}, {"theta": 0.5, "push_form": wl.PUSH_XYZ}):
        w = wl.small_fp64().replace(damping=wl.DAMP_FRIEDMAN, **kw)
        with pytest.raises(rzpic.RzpicError):
            rzpic.Context(w)
    w = wl.small_fp64().replace(damping=3)
    with pytest.raises(rzpic.RzpicError):
        rzpic.Context(w)
    w = wl.small_fp64().replace(damping=wl.DAMP_FRIEDMAN, theta=0.5, mg_fixed_cycles=0,
                                mg_tol=1e-10, mg_max_cycles=100)
    g = rzpic.make_context(w, precision="fp64", with_xsec=False)
    with pytest.raises(rzpic.RzpicError):
        rzpic.Adjoint(g, 4)
    g.close()
