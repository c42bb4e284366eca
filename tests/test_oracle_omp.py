"""The OpenMP timing build of the oracle (the benchmark's all-core CPU
baseline) against the serial oracle: the same merged steps with the particle
loops on threads agree to 1e-12 (only the deposit's summation order
differs), with collisions, ionization and a weight split, on one, two and four
threads; the particle and solve times it reports are positive."""
import numpy as np
import pytest

from oracle import rzo
from paper_1001_2969_amd import workloads as wl


def _pair(w):
    a, b = rzo.Oracle(w), rzo.Oracle(w, omp=True)
    for s in (0, 1):
        parts, nid = wl.random_particles(40 + s, w.n_per_species, w, s, near_axis_frac=0.05,
                                         near_wall_frac=0.05)
        a.set_particles(s, parts, nid)
        b.set_particles(s, parts, nid)
    a.prologue()
    b.prologue()
    return a, b


def _close(x, y, tol, what):
    scale = max(np.abs(x).max(), 1e-300)
    err = np.abs(x - y).max() / scale
    assert err <= tol, f"{what}: {err:.3e}"


@pytest.mark.parametrize("threads", [1, 2, 4])
def test_omp_steps_match_serial_oracle(threads):
    w = wl.small_fp64().replace(n_per_species=6000, steps=6, resize_every=3, Te_eV=8.0)
    rzo.Oracle.set_threads(threads)
    a, b = _pair(w)
    tp_sum = ts_sum = 0.0
    for n in range(w.steps):
        assert a.step(n) == 0
        st, tp, ts = b.step_omp(n)
        assert st == 0
        tp_sum += tp
        ts_sum += ts
    assert tp_sum > 0 and ts_sum > 0
    for s in (0, 1):
        pa, pb = a.particles(s), b.particles(s)
        np.testing.assert_array_equal(pa["id"], pb["id"])
        for f in rzo.FIELDS:
            _close(pa[f], pb[f], 1e-12, f"species {s} {f}")
        np.testing.assert_allclose(a.absorbed(s), b.absorbed(s), rtol=1e-12, atol=0)
    for G in (rzo.G_PHI, rzo.G_N0, rzo.G_N1):
        _close(a.grid(G), b.grid(G), 1e-12, f"grid {G}")
    # ionization happened, so identities of new particles were assigned
    assert b.next_id(0) > w.n_per_species
