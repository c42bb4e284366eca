"""Graph replay of rzpic_step (rzpic_set_step_graph): a context whose steps
are captured and replayed as HIP graphs ends every step bit for bit where
the same context stepped directly ends, through every step variant (ions
moving or not under subcycling, weight splits, tile sorts), with the
program's own reads and synchronisations between the replays; with step
timing on it steps directly; it refuses the null stream and tolerance-mode
solves."""
import numpy as np
import pytest
import torch

from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _ctx(w, precision, graph):
    g = rzpic.make_context(w, precision=precision, capacity_factor=3.0)
    if graph:
        g.use_stream(torch.cuda.Stream())
        g.set_step_graph(True)
    for s, T in ((0, w.Te_eV), (1, w.Ti_eV)):
        g.init_particles(s, w.n_per_species, w.n0, T, 0)
    g.prologue()
    return g


def _same(a, b, what):
    for s in (0, 1):
        x, y = a.particles(s), b.particles(s)
        for f in rzpic.FIELDS + ("id",):
            np.testing.assert_array_equal(x[f], y[f], err_msg=f"{what} s={s} {f}")
    for gi in (rzpic.G_PHI, rzpic.G_N0, rzpic.G_N1, rzpic.G_CHI):
        np.testing.assert_array_equal(a.grid(gi), b.grid(gi), err_msg=f"{what} grid {gi}")
    da, db = a.diag(), b.diag()
    assert da["count"] == db["count"] and da["next_id"] == db["next_id"], what


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_graph_steps_equal_direct_steps_every_step(precision):
    """65x33 mesh, 30k + 30k particles, 200 V rf, collisions on; tile sort
    every 3 steps, weight split every 4, ions moved every 2nd step: the
    graph variants of every combination recur within the 12 steps."""
    w = wl.rf_129x65().replace(nr=65, nz=33, R=0.02, L=0.01, n_per_species=30_000,
                               sort_every=3, resize_every=4, ion_subcycle=2)
    direct, graph = _ctx(w, precision, False), _ctx(w, precision, True)
    for n in range(12):
        direct.step(n)
        graph.step(n)
        _same(direct, graph, f"{precision} step {n}")


def test_graph_steps_with_circuit_and_timing_fallback():
    """33x33 FP64 workload with the external circuit (two solves, the
    capacitor update), graph replay for 4 steps, then 2 steps with step
    timing on (direct), then graph replay again."""
    w = wl.small_fp64().replace(n_per_species=6000, V_dc=20.0, V_rf=200.0, circuit_C=1e-12,
                                mg_fixed_cycles=3)
    direct, graph = _ctx(w, "fp64", False), _ctx(w, "fp64", True)
    for n in range(8):
        if n == 4:
            graph.set_timing(True)
        if n == 6:
            graph.timing()
            graph.set_timing(False)
        direct.step(n)
        graph.step(n)
        _same(direct, graph, f"circuit step {n}")
    np.testing.assert_array_equal(np.asarray(list(direct.circuit().values())),
                                  np.asarray(list(graph.circuit().values())))


def test_step_graph_refusals():
    w = wl.small_fp64().replace(n_per_species=2000, mg_fixed_cycles=3)
    g = rzpic.make_context(w, precision="fp64")
    if g.stream.cuda_stream == 0:
        with pytest.raises(rzpic.RzpicError):
            g.set_step_graph(True)
    g.close()
    w = wl.small_fp64().replace(n_per_species=2000, mg_fixed_cycles=0, mg_tol=1e-10,
                                mg_max_cycles=100)
    g = rzpic.make_context(w, precision="fp64")
    g.use_stream(torch.cuda.Stream())
    with pytest.raises(rzpic.RzpicError):
        g.set_step_graph(True)
    g.close()
