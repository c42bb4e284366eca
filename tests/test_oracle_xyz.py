"""Pins of the oracle's global X-Y-Z push (Sec. 2.3, the paper's alternative
push: Cartesian particles in the 2-D field, E_x = E_r cos(theta),
E_y = E_r sin(theta) with cos = 1, sin = 0 on the axis).  The oracle carries it
in the particle's local frame (one extra stored component, a_theta); these
tests run the paper's Cartesian equations directly, in numpy, on the same
node field with the same weights, and compare trajectories, including
passes through the axis in both pushes."""
import numpy as np

from adjoint_fd import cell_weights
from oracle import rzo
from paper_1001_2969_amd import workloads as wl


def _field(o, w, V=40.0, A=-30.0):
    """phi = V (1 - z/L) + A (r/R)^2: E_z = V/L, E_r = -2 A r / R^2 (A < 0 pushes
    positive ions towards the axis)."""
    rr = np.linspace(0.0, w.R, w.nr)[None, :]
    zz = np.linspace(0.0, w.L, w.nz)[:, None]
    o.set_grid(rzo.G_PHI, V * (1.0 - zz / w.L) + A * (rr / w.R) ** 2 + 0.0 * zz)
    o.efield()
    return o.grid(rzo.G_ER).reshape(-1), o.grid(rzo.G_EZ).reshape(-1)


def _gather(w, er, ez, r, z):
    nodes, ws = cell_weights(w, r, z)
    return np.sum(ws * er[nodes], axis=0), np.sum(ws * ez[nodes], axis=0)


def test_xyz_push_matches_the_cartesian_equations():
    """Electrons in a focusing field E_r = k r (exact on the nodes for the
    quadratic potential and, with the z-r weights, between them) strong enough
    that a final push moves a particle by 1.2 times its radius: every final
    push carries it through the axis (the local frame turns by pi); thermal
    velocities move it azimuthally (a_theta builds up)."""
    dt = 1e-10
    w = wl.Workload(name="t", nr=33, nz=33, R=0.02, L=0.02, n_per_species=1, steps=1,
                    dt=dt, push_form=wl.PUSH_XYZ, weighting=wl.W_ZR)
    o = rzo.Oracle(w, mc=False)
    qm0 = abs(wl.SPECIES_Q[0] / wl.SPECIES_M[0])
    A = -1.2 * w.R ** 2 / (qm0 * dt * dt)
    er, ez = _field(o, w, V=40.0, A=A)
    s = 0
    qm = wl.SPECIES_Q[s] / wl.SPECIES_M[s]
    rng = np.random.default_rng(11)
    n = 48
    phi0 = rng.uniform(0, 2 * np.pi, n)
    r0 = rng.uniform(1e-5, 3e-3, n)
    x, y = r0 * np.cos(phi0), r0 * np.sin(phi0)
    z = rng.uniform(0.008, 0.012, n)
    v = rng.normal(0, 2e4, (3, n))
    a = rng.normal(0, 1e17, (3, n)) * np.array([[1.0], [1.0], [1e-7]])
    # the same state in the particle's local frame (r_hat, theta_hat, z)
    ch, sh = np.cos(phi0), np.sin(phi0)
    parts = {"r": r0, "z": z.copy(), "vr": v[0] * ch + v[1] * sh, "vt": -v[0] * sh + v[1] * ch,
             "vz": v[2].copy(), "ar": a[0] * ch + a[1] * sh, "az": a[2].copy(), "w": np.ones(n),
             "id": np.arange(n, dtype=np.uint64)}
    o.set_particles(s, parts, n)
    o.set_at(s, -a[0] * sh + a[1] * ch)
    crossings = 0
    for k in range(1, 21):
        # Cartesian first push
        v = v + 0.5 * a * dt
        x, y, z = x + v[0] * dt, y + v[1] * dt, z + v[2] * dt
        o.push_first(s)
        # Cartesian final push with E gathered at r = |(x, y)|
        r = np.hypot(x, y)
        Er, Ez = _gather(w, er, ez, r, z)
        c = np.where(r > 0, x / np.where(r > 0, r, 1.0), 1.0)
        sn = np.where(r > 0, y / np.where(r > 0, r, 1.0), 0.0)
        E = np.stack([Er * c, Er * sn, Ez])
        xb, yb = x, y
        x = x + 0.5 * qm * E[0] * dt * dt
        y = y + 0.5 * qm * E[1] * dt * dt
        z = z + 0.5 * qm * E[2] * dt * dt
        crossings += int(np.sum((xb * x + yb * y) < 0))
        v = v + 0.5 * qm * E * dt
        a = 0.5 * (qm * E + a)
        o.push_final(s)
        if k in (2, 20):  # a_theta still large after two steps, damped by 20
            _compare(o, s, x, y, z, v, a, f"step {k}")
    assert o.count(s) == n
    assert crossings == 20 * n, crossings  # every final push crosses the axis


def _compare(o, s, x, y, z, v, a, label):
    p = o.particles(s)
    at = o.get_at(s)
    order = np.argsort(p["id"])
    r = np.hypot(x, y)
    rh = np.stack([x / r, y / r])
    th = np.stack([-y / r, x / r])
    np.testing.assert_allclose(p["r"][order], r, rtol=1e-9, atol=1e-18, err_msg=label)
    np.testing.assert_allclose(p["z"][order], z, rtol=1e-12, err_msg=label)
    vs = np.abs(v).max()
    for f, want in (("vr", v[0] * rh[0] + v[1] * rh[1]), ("vt", v[0] * th[0] + v[1] * th[1]),
                    ("vz", v[2])):
        np.testing.assert_allclose(p[f][order], want, rtol=0, atol=1e-9 * vs, err_msg=f"{label} {f}")
    as_ = np.abs(a).max()
    at_want = a[0] * th[0] + a[1] * th[1]
    np.testing.assert_allclose(p["ar"][order], a[0] * rh[0] + a[1] * rh[1], rtol=0,
                               atol=1e-9 * as_, err_msg=label)
    np.testing.assert_allclose(at[order], at_want, rtol=0, atol=1e-9 * as_, err_msg=label)
    np.testing.assert_allclose(p["az"][order], a[2], rtol=0, atol=1e-9 * as_, err_msg=label)
    return np.abs(at_want).max() / as_


def test_local_and_xyz_forms_differ_only_through_a_theta():
    """With a_theta = 0 and no azimuthal motion (v_theta = 0) the orbits stay in
    their meridian plane and never cross the axis: both forms agree exactly."""
    w = wl.Workload(name="t", nr=33, nz=33, R=0.02, L=0.02, n_per_species=1, steps=1)
    out = []
    for form in (wl.PUSH_LOCAL, wl.PUSH_XYZ):
        o = rzo.Oracle(w.replace(push_form=form), mc=False)
        _field(o, w, A=20.0)  # outward radial field: no axis crossing
        rng = np.random.default_rng(3)
        n = 32
        parts = {"r": rng.uniform(2e-3, 8e-3, n), "z": rng.uniform(0.008, 0.012, n),
                 "vr": rng.normal(0, 100, n), "vt": np.zeros(n), "vz": rng.normal(0, 100, n),
                 "ar": np.zeros(n), "az": np.zeros(n), "w": np.ones(n),
                 "id": np.arange(n, dtype=np.uint64)}
        o.set_particles(1, parts, n)
        for _ in range(50):
            o.push_first(1)
            o.push_final(1)
        out.append(o.particles(1))
    for f in rzo.FIELDS:
        np.testing.assert_array_equal(out[0][f], out[1][f], err_msg=f)
