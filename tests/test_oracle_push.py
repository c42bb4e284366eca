"""Pins of the oracle's particle push (Sec. 2.1 D1 scheme, Sec. 2.3 local X-Y
push and rotation) against closed-form trajectories and invariants."""
import numpy as np
import pytest

from oracle import rzo
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore")


def _oracle(nr=33, nz=33, R=0.02, L=0.02):
    w = wl.Workload(name="t", nr=nr, nz=nz, R=R, L=L, n_per_species=1, steps=1)
    return w, rzo.Oracle(w, mc=False)


def _set(o, s, **kw):
    n = len(kw["r"])
    parts = {f: np.asarray(kw.get(f, np.zeros(n)), float) for f in rzo.FIELDS}
    parts["id"] = np.arange(n, dtype=np.uint64)
    o.set_particles(s, parts, n)


def test_field_free_orbit_is_a_straight_line():
    """E = 0, a = 0: the local X-Y push plus rotation must reproduce the exact
    straight 3-D line r(t) = |(r0 + vr0 t, vt0 t)|, including passes close to
    the axis, and keep r * v_theta constant."""
    w, o = _oracle()
    o.set_grid(rzo.G_PHI, np.zeros((w.nz, w.nr)))
    o.efield()
    rng = np.random.default_rng(1)
    n = 64
    r0 = rng.uniform(1e-5, 2e-4, n)
    vr0 = rng.uniform(-4e3, 4e3, n)
    vt0 = rng.uniform(-1e3, 1e3, n) * np.where(rng.random(n) < 0.3, 1e-3, 1.0)
    vz0 = rng.uniform(-1e3, 1e3, n)
    z0 = np.full(n, 0.01)
    _set(o, 1, r=r0, z=z0, vr=vr0, vt=vt0, vz=vz0, w=np.ones(n))
    dt = w.dt
    for k in range(1, 1001):
        o.push_first(1)
        o.push_final(1)
        if k % 100:
            continue
        p = o.particles(1)
        order = np.argsort(p["id"])
        X = r0 + vr0 * k * dt
        Y = vt0 * k * dt
        r_ex = np.hypot(X, Y)
        np.testing.assert_allclose(p["r"][order], r_ex, rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(p["z"][order], z0 + vz0 * k * dt, rtol=1e-13)
        vr_ex = (vr0 * X + vt0 * Y) / r_ex
        vt_ex = (vt0 * X - vr0 * Y) / r_ex
        vscale = np.hypot(vr0, vt0)
        np.testing.assert_allclose(p["vr"][order], vr_ex, rtol=0, atol=1e-11 * vscale.max())
        np.testing.assert_allclose(p["vt"][order], vt_ex, rtol=0, atol=1e-11 * vscale.max())
        L_ang = p["r"][order] * p["vt"][order]
        np.testing.assert_allclose(L_ang, r0 * vt0, rtol=1e-11, atol=1e-22)
    # nothing reached the axis rule or was absorbed
    assert o.count(1) == n


@pytest.mark.parametrize("preset", [True, False])
def test_uniform_ez_closed_form(preset):
    """Uniform E_z, E_r = 0.  With the damped acceleration preset to a = qE/m the
    D1 cycle is leapfrog: z_n = z0 + n v dt + a dt^2 n(n+1)/2.  With it started at
    zero, abar^k = a (1 - 2^-(k+1)) and
    z_n = z0 + n v dt + a dt^2 (n(n-1)/2 + 1 - 2^-n)."""
    w, o = _oracle()
    V = 37.0
    zz = np.linspace(0.0, w.L, w.nz)[:, None] * np.ones((1, w.nr))
    o.set_grid(rzo.G_PHI, V * (1.0 - zz / w.L))
    o.efield()
    Ez = o.grid(rzo.G_EZ)
    np.testing.assert_allclose(Ez, V / w.L, rtol=1e-12)
    assert np.all(o.grid(rzo.G_ER) == 0.0)
    q, m = wl.SPECIES_Q[1], wl.SPECIES_M[1]
    a = q / m * V / w.L
    n = 16
    rng = np.random.default_rng(2)
    r0 = rng.uniform(1e-3, 1.5e-2, n)
    z0 = rng.uniform(8e-3, 1.2e-2, n)
    v0 = rng.uniform(-50.0, 50.0, n)
    _set(o, 1, r=r0, z=z0, vz=v0, az=np.full(n, a if preset else 0.0), w=np.ones(n))
    dt = w.dt
    N = 1000
    for _ in range(N):
        o.push_first(1)
        o.push_final(1)
    p = o.particles(1)
    order = np.argsort(p["id"])
    if preset:
        z_ex = z0 + N * v0 * dt + a * dt * dt * N * (N + 1) / 2
        v_ex = v0 + N * a * dt
        a_ex = a
    else:
        z_ex = z0 + N * v0 * dt + a * dt * dt * (N * (N - 1) / 2 + 1 - 2.0 ** -N)
        v_ex = v0 + a * dt * (N - 1 + 2.0 ** -N)
        a_ex = a * (1 - 2.0 ** -N)
    np.testing.assert_allclose(p["z"][order], z_ex, rtol=1e-13)
    np.testing.assert_allclose(p["vz"][order], v_ex, rtol=1e-11)
    np.testing.assert_allclose(p["az"][order], a_ex, rtol=1e-13)
    np.testing.assert_array_equal(p["r"][order], r0)


def test_angular_momentum_conserved_without_er():
    """With E_r = 0 the first push, rotation and final push leave r * v_theta
    unchanged (to rounding) for any radial acceleration and axial field."""
    w, o = _oracle()
    rng = np.random.default_rng(3)
    o.set_grid(rzo.G_PHI, rng.normal(0, 5.0, (w.nz, 1)) * np.ones((1, w.nr)))
    o.efield()
    assert np.all(o.grid(rzo.G_ER) == 0.0)
    n = 200
    parts, _ = wl.random_particles(4, n, w, wl.ION, accel_scale=1e3)
    parts["z"] = rng.uniform(0.45 * w.L, 0.55 * w.L, n)
    parts["r"] = rng.uniform(1e-4, 0.9 * w.R, n)
    o.set_particles(1, parts, n)
    L0 = parts["r"] * parts["vt"]
    for _ in range(200):
        o.push_first(1)
        o.push_final(1)
    p = o.particles(1)
    idx = {int(i): k for k, i in enumerate(parts["id"])}
    sel = np.array([idx[int(i)] for i in p["id"]])
    np.testing.assert_allclose(p["r"] * p["vt"], L0[sel], rtol=1e-12, atol=1e-25)


def test_axis_rule_makes_radial_components_positive():
    """A final push that carries r below zero reflects r, v_r and a_r to their
    absolute values and leaves v_theta alone (Sec. 2.3)."""
    w, o = _oracle()
    hr = w.R / (w.nr - 1)
    jj = np.arange(w.nr)[None, :]
    # phi falling with r gives an outward E_r that pushes electrons onto the axis
    o.set_grid(rzo.G_PHI, -1e7 * (jj / (w.nr - 1.0)) ** 2 * np.ones((w.nz, 1)))
    o.efield()
    n = 8
    _set(o, 0, r=np.full(n, 0.3 * hr), z=np.full(n, 0.01), vr=np.full(n, -3.0),
         vt=np.linspace(-1, 1, n), ar=np.full(n, -1e9), w=np.ones(n))
    o.push_final(0)
    p = o.particles(0)
    assert np.all(p["r"] > 0)
    assert np.all(p["vr"] >= 0) and np.all(p["ar"] >= 0)
    np.testing.assert_array_equal(np.sort(p["vt"]), np.linspace(-1, 1, n))


def test_absorption_tallies_and_compaction_rule():
    """Particles leaving through z<=0, z>=L or r>=R are removed with their
    weight tallied per boundary; the holes are filled in increasing order by
    the live particles of the tail [n-D, n), also in increasing order."""
    w, o = _oracle()
    o.set_grid(rzo.G_PHI, np.zeros((w.nz, w.nr)))
    o.efield()
    rng = np.random.default_rng(5)
    n = 50
    r = rng.uniform(0.1 * w.R, 0.8 * w.R, n)
    z = rng.uniform(0.2 * w.L, 0.8 * w.L, n)
    vr = np.zeros(n)
    vz = np.zeros(n)
    dt = w.dt
    kill0 = [3, 17, 40]
    killL = [5, 48]
    killR = [0, 22, 49]
    vz[kill0] = -(z[kill0] + 1e-6) / dt
    vz[killL] = (w.L - z[killL] + 1e-6) / dt
    vr[killR] = (w.R - r[killR] + 1e-6) / dt
    wts = rng.uniform(1, 2, n)
    _set(o, 0, r=r, z=z, vr=vr, vz=vz, w=wts)
    o.push_first(0)
    o.compact(0)
    np.testing.assert_allclose(o.absorbed(0), [wts[kill0].sum(), wts[killL].sum(),
                                               wts[killR].sum()], rtol=1e-15)
    dead = set(kill0 + killL + killR)
    # brute-force statement of the rule
    order = list(range(n))
    keep = n - len(dead)
    tail_live = [p for p in range(keep, n) if p not in dead]
    holes = [h for h in range(keep) if h in dead]
    for h, src in zip(holes, tail_live):
        order[h] = src
    expect_ids = np.array(order[:keep], dtype=np.uint64)
    np.testing.assert_array_equal(o.particles(0)["id"], expect_ids)
