"""Pins of the oracle's Friedman damping (RZO_DAMP_FRIEDMAN): the time-
averaged acceleration abar_n = c a_{n+1} + (1-c)[(1-c) a_n + c abar_{n-1}],
c = theta/2, with the particle carrying the known part B of the next step.
Each pin is a property the scheme's definition fixes, not the recurrence
typed again:
- theta = 0 is leapfrog: in a harmonic well a = -w^2 (z - z0) the quantity
  w^2 (z_n - z0)^2 + v_{n+1/2} v_{n-1/2} is conserved exactly;
- in a uniform field a, from B = 0, the recurrence has the closed-form
  solution B_k = (1-c) a (1 - rho^k), rho = (1-c) c, and then
  v_N = v_0 + h a [N - (1-c)(1 - rho^N)/(1 - rho)],
  z_N = z_0 + N h v_0 + h^2 a [N(N+1)/2 - (1-c)/(1-rho) (N - rho (1 - rho^N)/(1 - rho))];
  preset at the fixed point B = (1-c) a it is the exact leapfrog parabola;
- theta > 0 damps the harmonic oscillation (that invariant decreases);
- chi is theta times the D1 chi (the implicit coefficient theta/2)."""
import numpy as np
import pytest

from oracle import rzo
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore")


def _oracle(theta, damping=wl.DAMP_FRIEDMAN):
    w = wl.Workload(name="t", nr=33, nz=33, R=0.02, L=0.02, n_per_species=1, steps=1,
                    damping=damping, theta=theta)
    return w, rzo.Oracle(w, mc=False)


def _set(o, s, **kw):
    n = len(kw["r"])
    parts = {f: np.asarray(kw.get(f, np.zeros(n)), float) for f in rzo.FIELDS}
    parts["id"] = np.arange(n, dtype=np.uint64)
    o.set_particles(s, parts, n)


def _well(o, w, omega_dt):
    """phi = (|K|/2)(z - z0)^2 about the mid-plane: for the ions
    a = -(q/m)|K| (z - z0), w^2 = (q/m)|K| (centred differences of a
    quadratic are exact, and the gather interpolates a linear field exactly)."""
    q, m = wl.SPECIES_Q[1], wl.SPECIES_M[1]
    om2 = (omega_dt / w.dt) ** 2
    K = om2 / (q / m)
    z0 = 0.5 * w.L
    zz = np.linspace(0.0, w.L, w.nz)[:, None] * np.ones((1, w.nr))
    o.set_grid(rzo.G_PHI, 0.5 * K * (zz - z0) ** 2)
    o.efield()
    assert np.all(o.grid(rzo.G_ER) == 0.0)
    return om2, z0


def _orbit(o, n_steps):
    zs, vs = [], []
    for _ in range(n_steps):
        o.push_first(1)
        p = o.particles(1)
        zs.append(p["z"].copy())
        vs.append(p["vz"].copy())
        o.push_final(1)
    return np.array(zs), np.array(vs)


def test_theta_zero_is_leapfrog():
    """After the k-th first push the particle holds z_k and v_{k+1/2}... read
    here as the pair the leapfrog invariant couples:
    I_k = w^2 (z_k - z0)^2 + v_{k+1/2} v_{k-1/2}."""
    w, o = _oracle(0.0)
    om2, z0 = _well(o, w, 0.3)
    n = 8
    rng = np.random.default_rng(5)
    z = z0 + rng.uniform(-4e-3, 4e-3, n)
    _set(o, 1, r=rng.uniform(2e-3, 1.5e-2, n), z=z, vz=rng.uniform(-2.0, 2.0, n), w=np.ones(n))
    zs, vs = _orbit(o, 2000)
    inv = om2 * (zs[:-1] - z0) ** 2 + vs[1:] * vs[:-1]
    np.testing.assert_allclose(inv, np.broadcast_to(inv[:1], inv.shape), rtol=1e-11)
    assert np.all(np.abs(zs - z0) < 5e-3)  # stayed inside the interior cells


@pytest.mark.parametrize("theta", [0.3, 0.7, 1.0])
@pytest.mark.parametrize("preset", [True, False])
def test_uniform_field_closed_form(theta, preset):
    w, o = _oracle(theta)
    V = 37.0
    zz = np.linspace(0.0, w.L, w.nz)[:, None] * np.ones((1, w.nr))
    o.set_grid(rzo.G_PHI, V * (1.0 - zz / w.L))
    o.efield()
    q, m = wl.SPECIES_Q[1], wl.SPECIES_M[1]
    a = q / m * V / w.L
    c = theta / 2
    rho = (1 - c) * c
    n = 16
    rng = np.random.default_rng(2)
    r0 = rng.uniform(1e-3, 1.5e-2, n)
    z0 = rng.uniform(8e-3, 1.2e-2, n)
    v0 = rng.uniform(-50.0, 50.0, n)
    _set(o, 1, r=r0, z=z0, vz=v0, az=np.full(n, (1 - c) * a if preset else 0.0), w=np.ones(n))
    h = w.dt
    N = 600
    for _ in range(N):
        o.push_first(1)
        o.push_final(1)
    p = o.particles(1)
    order = np.argsort(p["id"])
    if preset:
        z_ex = z0 + N * v0 * h + a * h * h * N * (N + 1) / 2
        v_ex = v0 + N * a * h
        b_ex = (1 - c) * a
    else:
        g = (1 - c) / (1 - rho)
        z_ex = z0 + N * v0 * h + a * h * h * (N * (N + 1) / 2 -
                                              g * (N - rho * (1 - rho ** N) / (1 - rho)))
        v_ex = v0 + a * h * (N - g * (1 - rho ** N))
        b_ex = (1 - c) * a * (1 - rho ** N)
    np.testing.assert_allclose(p["z"][order], z_ex, rtol=1e-13)
    np.testing.assert_allclose(p["vz"][order], v_ex, rtol=1e-11)
    np.testing.assert_allclose(p["az"][order], b_ex, rtol=1e-12)
    np.testing.assert_array_equal(p["r"][order], r0)


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_positive_theta_damps_the_oscillation(theta):
    """The leapfrog invariant (conserved at theta = 0) decays for theta > 0,
    faster for the larger theta, and the oscillation keeps its frequency
    close to w (zero crossings)."""
    w, o = _oracle(theta)
    om2, z0 = _well(o, w, 0.3)
    _set(o, 1, r=np.array([5e-3]), z=np.array([z0 + 4e-3]), vz=np.zeros(1), w=np.ones(1))
    steps = 600  # about 29 periods, far above rounding at the strongest damping
    zs, vs = _orbit(o, steps)
    inv = (om2 * (zs[:-1] - z0) ** 2 + vs[1:] * vs[:-1])[:, 0]
    per = int(round(2 * np.pi / 0.3))
    env = inv[: (len(inv) // per) * per].reshape(-1, per).max(axis=1)
    assert np.all(np.diff(env) < 0.0)
    assert env[-1] < 0.9 * env[0]
    crossings = np.count_nonzero(np.diff(np.sign(zs[:, 0] - z0)) != 0)
    assert abs(crossings - steps * 0.3 / np.pi) <= 0.1 * steps * 0.3 / np.pi
    return env[-1] / env[0]


def test_damping_grows_with_theta():
    a = test_positive_theta_damps_the_oscillation(0.5)
    b = test_positive_theta_damps_the_oscillation(1.0)
    assert b < a


@pytest.mark.parametrize("theta", [1.0, 0.5, 0.0])
def test_chi_is_theta_times_the_d1_chi(theta):
    w = wl.small_fp64().replace(n_per_species=4000)
    states = {s: wl.random_particles(7 + s, 4000, w, s) for s in (0, 1)}
    chis = []
    for damping, th in ((wl.DAMP_D1, 1.0), (wl.DAMP_FRIEDMAN, theta)):
        o = rzo.Oracle(w.replace(damping=damping, theta=th), mc=False)
        for s, (parts, nid) in states.items():
            o.set_particles(s, parts, nid)
        o.deposit()
        chis.append(o.grid(rzo.G_CHI))
    assert chis[0].max() > 0
    np.testing.assert_allclose(chis[1], theta * chis[0], rtol=1e-15, atol=0)


def test_friedman_needs_the_local_push_and_theta_in_range():
    for kw in ({"theta": 1.5}, {"theta": -0.1}, {"theta": 0.5, "push_form": wl.PUSH_XYZ}):
        w = wl.small_fp64().replace(damping=wl.DAMP_FRIEDMAN, **kw)
        with pytest.raises(ValueError):
            rzo.Oracle(w, mc=False)
