"""Pins of the oracle's zero-order particle-based resizing (Sec. 2.2, after
Bird; resize_mode = ZERO_ORDER): a particle of weight w at radius r, whose
weight there should be w_r = c max(r, hr/2), is kept as floor(w/w_r) copies
plus one more with probability frac(w/w_r), each of weight w_r.

- Rates: populations with a fractional ratio keep the extra copy (or, below
  one, survive) at the binomial rate, and the expected weight is conserved.
- Decisions: each particle's copy count follows from the first uniform of
  draw block 6 of (seed, s, id, step), the stream pinned by the Philox
  known-answer test; duplicates copy the parent's record, take new ids in
  parent order, and the removed particles leave a compacted array."""
import math

import numpy as np

from oracle import rzo
from paper_1001_2969_amd import workloads as wl


def _oracle(seed=5):
    w = wl.small_fp64().replace(resize_mode=wl.RESIZE_ZERO_ORDER, resize_every=1, seed=seed)
    return w, rzo.Oracle(w, mc=False)


def _population(w, n, q, rng, s=1):
    hr = w.R / (w.nr - 1)
    r = rng.uniform(hr, 0.9 * w.R, n)
    parts = {f: np.zeros(n) for f in rzo.FIELDS}
    parts.update(r=r, z=rng.uniform(0.1 * w.L, 0.9 * w.L, n), vr=rng.normal(0, 1, n),
                 vt=rng.normal(0, 1, n), vz=rng.normal(0, 1, n), ar=rng.normal(0, 1, n),
                 az=rng.normal(0, 1, n))
    wr = w.wcoef * np.maximum(r, 0.5 * hr)
    parts["w"] = q * wr
    parts["id"] = rng.permutation(n).astype(np.uint64)
    return parts, wr


def test_rates_and_expected_weight():
    rng = np.random.default_rng(1)
    for q in (2.3, 0.4, 1.0):
        w, o = _oracle()
        n = 20000
        parts, wr = _population(w, n, q, rng)
        o.set_particles(1, parts, n)
        o.resize(1, step=7)
        after = o.particles(1)
        k, f = math.floor(q), q - math.floor(q)
        extra = len(after["w"]) - k * n  # copies beyond floor(q) each
        sigma = math.sqrt(n * f * (1 - f)) if 0 < f < 1 else 0.0
        assert abs(extra - f * n) <= 5 * sigma + 1, (q, extra, f * n)
        tot_before, tot_after = parts["w"].sum(), after["w"].sum()
        rel_sigma = sigma * wr.mean() / tot_before + 1e-12
        assert abs(tot_after - tot_before) <= 6 * rel_sigma * tot_before, (q, tot_after / tot_before)


def test_decisions_follow_the_keyed_draws():
    rng = np.random.default_rng(2)
    w, o = _oracle(seed=11)
    n = 3000
    q = rng.uniform(0.0, 3.5, n)
    parts, wr = _population(w, n, 1.0, rng)
    parts["w"] = q * wr
    o.set_particles(1, parts, n)
    step = 123
    o.resize(1, step=step)
    after = o.particles(1)
    # expected copies per parent, from the published rule and the pinned stream
    N = np.zeros(n, np.int64)
    for p in range(n):
        qq = parts["w"][p] / wr[p]
        u = rzo.uniform_pair(w.seed, 1, int(parts["id"][p]), step, 6)[0]
        N[p] = math.floor(qq) + (1 if u < qq - math.floor(qq) else 0)
    assert len(after["id"]) == N.sum()
    # survivors keep their ids; duplicates take n, n+1, ... in parent order
    survivors = set(int(i) for i in parts["id"][N > 0])
    old = after["id"] < n
    assert set(int(i) for i in after["id"][old]) == survivors
    parent_of_clone = np.repeat(np.arange(n), np.maximum(N - 1, 0))
    new_ids = np.sort(after["id"][~old])
    np.testing.assert_array_equal(new_ids, n + np.arange(len(parent_of_clone)))
    by_id = {int(i): k for k, i in enumerate(after["id"])}
    for c, p in enumerate(parent_of_clone):
        k = by_id[n + c]
        for f in rzo.FIELDS:
            want = wr[p] if f == "w" else parts[f][p]
            assert after[f][k] == want, (f, c, p)
    for p in np.flatnonzero(N > 0)[:200]:
        assert after["w"][by_id[int(parts["id"][p])]] == wr[p]
    assert o.next_id(1) == n + len(parent_of_clone)
