"""Pins of the adjoint tests' reference values, the central differences of
the oracle's collision-free window: they do not depend on the step over two
decades (the objective is smooth where no particle changes cell or meets a
wall), and for a one-step window
the rf and dc voltage derivatives differ by exactly the factor sin(2 pi f t_1)
through which V_rf enters the electrode value of the only solve."""
import math

import numpy as np

from adjoint_fd import Window, cell_weights, objective_of
from paper_1001_2969_amd import workloads as wl


def _window(n=500, seed=40):
    w = wl.small_fp64().replace(n_per_species=n, V_rf=200.0, V_dc=50.0)
    states = {s: wl.random_particles(seed + s, n, w, s, near_wall_frac=0.05) for s in (0, 1)}
    return w, Window(w, states, 1e-13)


def test_central_differences_do_not_depend_on_the_step():
    w, win = _window()
    delta = 2 * w.L / (w.nz - 1)
    d = np.array([win.central(1000, 4, delta, h, V_rf=200.0) for h in (0.2, 0.02, 0.002)])
    assert d[0] != 0.0
    assert np.ptp(d) <= 1e-7 * abs(d[0]), d


def test_one_step_voltage_derivatives_differ_by_the_rf_factor():
    w, win = _window()
    delta = 2 * w.L / (w.nz - 1)
    step0 = 1000
    dc = win.central(step0, 1, delta, 0.5, V_dc=50.0)
    rf = win.central(step0, 1, delta, 0.5, V_rf=200.0)
    s = math.sin(2 * math.pi * w.f_rf * (step0 + 1) * w.dt)
    assert dc != 0.0
    assert abs(rf - s * dc) <= 1e-6 * abs(dc), (rf, s * dc)


def test_objective_and_weights_by_hand():
    """The objective on two ions written out, and the node weights of a point
    in the r^2 weighting (fractions of the annulus areas) by hand."""
    w = wl.small_fp64()
    ions = {"w": np.array([2.0, 3.0]), "vz": np.array([-10.0, 5.0]),
            "z": np.array([0.001, 0.002])}
    delta = 0.001
    q = wl.SPECIES_Q[1]
    want = q * w.dt / delta * (2.0 * 10.0 * math.exp(-1.0) + 3.0 * (-5.0) * math.exp(-2.0))
    assert math.isclose(objective_of(ions, w, delta), want, rel_tol=1e-14)
    hr, hz = w.R / (w.nr - 1), w.L / (w.nz - 1)
    r, z = np.array([2.25 * hr]), np.array([3.5 * hz])
    nodes, ws = cell_weights(w, r, z)
    fr = (2.25 ** 2 - 4.0) / (9.0 - 4.0)  # share of the outer node in r^2
    assert list(nodes[:, 0]) == [3 * w.nr + 2, 3 * w.nr + 3, 4 * w.nr + 2, 4 * w.nr + 3]
    np.testing.assert_allclose(ws[:, 0], [0.5 * (1 - fr), 0.5 * fr, 0.5 * (1 - fr), 0.5 * fr],
                               rtol=1e-14)
