"""The 32-bit LDS deposit of FP32 particles (deposit4_lds32): each block adds
its particles' int32 contributions into a 32-bit LDS copy of the grid; an add
that wraps is seen in the value it replaced and carries 2^32 quanta straight
to the 64-bit grid.  Every particle in one cell at 1.2 w_ref with the finest
quantum the mixed form allows (w_ref 2^-30) makes each block's accumulators
of that cell wrap dozens of times; the grid must still equal, bit for bit,
the deposit of the same particles by 64-bit global atomics
(rzpic_deposit_noalloc), and hold the particles' total weight."""
import numpy as np
import pytest

from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_lds32_carries_equal_global_64bit_deposit():
    import torch

    n = 200_000
    w = wl.rf_129x65().replace(n_per_species=n, precision="mixed")
    g = rzpic.make_context(w, capacity_factor=1.5, with_xsec=False, fixed_point_bits=30)
    w_ref = w.wcoef * w.R
    hr, hz = w.R / (w.nr - 1), w.L / (w.nz - 1)
    for s in (0, 1):
        parts, nid = wl.random_particles(40 + s, n, w, s)
        rng = np.random.default_rng(50 + s)
        parts["r"] = (64.3 + rng.uniform(0.0, 0.4, n)) * hr  # inside cell (32, 64)
        parts["z"] = (32.2 + rng.uniform(0.0, 0.5, n)) * hz
        parts["w"] = np.full(n, 1.2 * w_ref)
        g.set_particles(s, parts, nid)
    g.deposit()
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    for s, G in ((0, rzpic.G_N0), (1, rzpic.G_N1)):
        ref = g.grid(G)
        out = torch.full((w.nz * w.nr,), -7.0, dtype=torch.float64, device="cuda:0")
        arr = g.arrays[s]
        rzpic.deposit_noalloc(w.nr, w.nz, w.R, w.L, arr["r"], arr["z"], arr["w"], out, status,
                              n=n, precision=rzpic.MIXED, weighting=w.weighting, w_ref=w_ref,
                              fixed_point_bits=30)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(w.nz, w.nr)
        np.testing.assert_array_equal(ref, got, err_msg=f"species {s}")
        # four nodes of one cell, each far beyond 2^32 quanta
        assert np.count_nonzero(ref) == 4
        assert ref.max() / (w_ref * 2.0 ** -30) > 2.0 ** 40
        # total weight, to the FP32 rounding of the contributions
        assert abs(ref.sum() - n * 1.2 * w_ref) <= 1e-6 * n * 1.2 * w_ref
    assert int(status.item()) == 0
    g.close()
