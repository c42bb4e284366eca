"""Pins of the oracle's ion subcycling (Sec. 2.7, the subcycling of Vahedi
et al., with the reading: ions move in every K-th step, n = K-1, 2K-1, ...,
with time step K dt; in the other steps their deposit is kept and they add
charge but no susceptibility):

- pushed with K dt, ions follow the closed-form D1 orbit in a uniform field
  with time step K dt;
- in the full step they are frozen between their steps and move on them,
  electrons every step;
- the susceptibility holds the ions' term, with (K dt)^2, only in their steps;
- K = 1 is the plain step, bit for bit; merged and unmerged forms agree."""
import numpy as np

from oracle import rzo
from paper_1001_2969_amd import workloads as wl

EPS0 = rzo.constants()["eps0"]


def _uniform_ez(o, w, V=37.0):
    zz = np.linspace(0.0, w.L, w.nz)[:, None] * np.ones((1, w.nr))
    o.set_grid(rzo.G_PHI, V * (1.0 - zz / w.L))
    o.efield()
    return V / w.L


def test_ions_follow_the_closed_form_with_k_dt():
    K = 4
    w = wl.Workload(name="t", nr=33, nz=33, R=0.02, L=0.02, n_per_species=1, steps=1,
                    ion_subcycle=K)
    o = rzo.Oracle(w, mc=False)
    E = _uniform_ez(o, w)
    a = wl.SPECIES_Q[1] / wl.SPECIES_M[1] * E
    rng = np.random.default_rng(4)
    n = 16
    parts = {f: np.zeros(n) for f in rzo.FIELDS}
    parts.update(r=rng.uniform(1e-3, 1.5e-2, n), z=rng.uniform(8e-3, 1.2e-2, n),
                 vz=rng.uniform(-50.0, 50.0, n), az=np.full(n, a), w=np.ones(n))
    parts["id"] = np.arange(n, dtype=np.uint64)
    o.set_particles(1, parts, n)
    dt, N = K * w.dt, 300
    for _ in range(N):
        o.push_first(1)
        o.push_final(1)
    p = o.particles(1)
    z_ex = parts["z"] + N * parts["vz"] * dt + a * dt * dt * N * (N + 1) / 2
    np.testing.assert_allclose(p["z"], z_ex, rtol=1e-13)
    np.testing.assert_allclose(p["vz"], parts["vz"] + N * a * dt, rtol=1e-11)


def _run(w, steps, merged=True, seed=9):
    o = rzo.Oracle(w)
    for s in (0, 1):
        parts, nid = wl.random_particles(seed + s, 3000, w, s)
        o.set_particles(s, parts, nid)
    o.prologue()
    hist = []
    for n in range(steps):
        assert o.step(n, merged=merged) == 0
        h = {s: o.particles(s) for s in (0, 1)}
        h.update(chi=o.grid(rzo.G_CHI), d0=o.grid(rzo.G_DENS0), d1=o.grid(rzo.G_DENS1))
        hist.append(h)
    return o, hist


def test_ions_frozen_between_their_steps():
    K = 3
    w = wl.small_fp64().replace(n_per_species=3000, ion_subcycle=K, V_rf=200.0)
    _, hist = _run(w, 7)
    for n in range(1, 7):
        prev, cur = hist[n - 1][1], hist[n][1]
        e_prev, e_cur = hist[n - 1][0], hist[n][0]
        assert not np.array_equal(e_prev["z"][:100], e_cur["z"][:100])  # electrons move
        keep = np.isin(cur["id"], prev["id"])
        ip = {int(i): k for k, i in enumerate(prev["id"])}
        idx = np.array([ip[int(i)] for i in cur["id"][keep]])
        if n % K == K - 1:
            assert not np.array_equal(prev["z"][idx[:100]], cur["z"][keep][:100])
        else:
            # surviving old ions are untouched; only children are new
            for f in rzo.FIELDS:
                np.testing.assert_array_equal(cur[f][keep], prev[f][idx], err_msg=f"{n} {f}")


def test_susceptibility_only_in_ion_steps():
    K = 3
    w = wl.small_fp64().replace(n_per_species=3000, ion_subcycle=K)
    _, hist = _run(w, 6)
    q0, q1 = wl.SPECIES_Q
    m0, m1 = wl.SPECIES_M
    for n in range(6):
        h = hist[n]
        want = q0 * q0 * h["d0"] * w.dt ** 2 / (2 * m0 * EPS0)
        if n % K == K - 1:
            want = want + q1 * q1 * h["d1"] * (K * w.dt) ** 2 / (2 * m1 * EPS0)
        np.testing.assert_allclose(h["chi"], want, rtol=1e-14, atol=0, err_msg=f"step {n}")


def test_k1_is_the_plain_step_and_forms_agree():
    w = wl.small_fp64().replace(n_per_species=3000)
    _, a = _run(w, 4)
    _, b = _run(w.replace(ion_subcycle=1), 4)
    for s in (0, 1):
        for f in rzo.FIELDS:
            np.testing.assert_array_equal(a[-1][s][f], b[-1][s][f])
    ws = w.replace(ion_subcycle=2)
    _, hm = _run(ws, 5, merged=True)
    _, hu = _run(ws, 5, merged=False)
    for s in (0, 1):
        pm, pu = hm[-1][s], hu[-1][s]
        im, iu = np.argsort(pm["id"]), np.argsort(pu["id"])
        np.testing.assert_array_equal(pm["id"][im], pu["id"][iu])
        for f in rzo.FIELDS:
            np.testing.assert_allclose(pm[f][im], pu[f][iu], rtol=1e-11, atol=0, err_msg=f)
