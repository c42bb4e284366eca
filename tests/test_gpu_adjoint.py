"""Adjoint of the collision-free window (rzpic_adjoint_*): the objective
against the oracle's, and every gradient (electrode dc and rf amplitudes,
starting weights along a direction and one by one, the initial density field
along a direction) against central differences of the oracle's window; the
one-step voltage identity, independence of the checkpoint spacing, the
context left at the window's end, the torch.autograd wrapper, the rejected
configurations, and a larger window against central differences of the HIP
forward itself."""
import math

import numpy as np
import pytest

from adjoint_fd import Window, cell_weights
from gpu_helpers import random_state
from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

pytestmark = pytest.mark.gpu

W = wl.small_fp64().replace(n_per_species=4000, V_rf=200.0, V_dc=50.0, mg_tol=1e-13,
                            mg_max_cycles=400)
STEP0, N, K = 1000, 12, 5  # segments of 5, 5 and 2 steps
DELTA = 2 * W.L / (W.nz - 1)
# Central differences with a relative step of 1e-6 agree with the adjoint to
# ~1e-9 here; larger steps can move a particle across a cell face (the
# weights are only piecewise smooth) and err by ~1e-6.
H = 1e-6
RTOL = 1e-7


def _states(w, seed):
    return random_state(w, seed, near_axis_frac=0.05, near_wall_frac=0.05)


def _context(w, states):
    g = rzpic.make_context(w, precision="fp64", with_xsec=False, capacity_factor=2.0)
    for s, (parts, nid) in states.items():
        g.set_particles(s, parts, nid)
    g.prologue()
    return g


@pytest.fixture(scope="module")
def case():
    states = _states(W, 61)
    g = _context(W, states)
    adj = rzpic.Adjoint(g, N, checkpoint_every=K, delta=DELTA)
    J = adj.forward(STEP0)
    dvdc, dvrf, gw, gd = adj.backward(density=True)
    win = Window(W, states, W.mg_tol)
    out = dict(J=J, dvdc=dvdc, dvrf=dvrf, gw=[x.cpu().numpy() for x in gw],
               gd=gd.cpu().numpy(), win=win, states=states)
    adj.close()
    return out


def _close(a, b, rtol, label):
    assert abs(a - b) <= rtol * abs(b), f"{label}: adjoint {a!r} vs differences {b!r}"


def test_window_objective_matches_oracle(case):
    J_o, _ = case["win"].run(STEP0, N, DELTA)
    assert J_o != 0.0
    assert abs(case["J"] - J_o) <= 1e-10 * abs(J_o), (case["J"], J_o)


def test_voltage_gradients_match_oracle_differences(case):
    win = case["win"]
    fd_rf = win.central(STEP0, N, DELTA, H * W.V_rf, V_rf=W.V_rf)
    fd_dc = win.central(STEP0, N, DELTA, H * W.V_dc, V_dc=W.V_dc)
    print("dJ/dV_rf", case["dvrf"], fd_rf, "dJ/dV_dc", case["dvdc"], fd_dc)
    _close(case["dvrf"], fd_rf, RTOL, "dJ/dV_rf")
    _close(case["dvdc"], fd_dc, RTOL, "dJ/dV_dc")


def test_weight_gradient_along_a_direction(case):
    win, gw = case["win"], case["gw"]
    rng = np.random.default_rng(7)
    u = [rng.normal(size=len(gw[s])) for s in (0, 1)]
    fd = win.central(STEP0, N, DELTA, H, dir=lambda s, p: u[s][p["id"].astype(np.int64)])
    ad = 0.0
    for s in (0, 1):
        p = win.start[s][0]
        ids = p["id"].astype(np.int64)
        ad += float(np.sum(gw[s][ids] * p["w"] * u[s][ids]))
    print("directional dJ/dw", ad, fd)
    _close(ad, fd, RTOL, "dJ/dw along u")


def test_weight_gradient_one_by_one_and_absent_identities(case):
    win, gw = case["win"], case["gw"]
    for s in (0, 1):
        p = win.start[s][0]
        ids = p["id"].astype(np.int64)
        present = np.zeros(len(gw[s]), bool)
        present[ids] = True
        assert np.all(gw[s][~present] == 0.0), "identities absent at the start have no gradient"
        # the particles with the largest gradients, and one with an ordinary one
        order = np.argsort(-np.abs(gw[s][ids] * p["w"]))
        for k in (order[0], order[1], order[len(order) // 2]):
            pid = ids[k]
            fd = win.central(STEP0, N, DELTA, 1e-3,
                             dir=lambda ss, pp, pid=pid, s=s: (
                                 (pp["id"].astype(np.int64) == pid) & (ss == s)).astype(float))
            ad = float(gw[s][pid] * p["w"][k])
            if fd == 0.0 and ad == 0.0:
                continue
            _close(ad, fd, 1e-5, f"dJ/dw species {s} id {pid}")


def test_density_gradient_along_a_direction(case):
    win, gd = case["win"], case["gd"]
    rr = np.linspace(0.0, W.R, W.nr)[None, :]
    zz = np.linspace(0.0, W.L, W.nz)[:, None]
    psi = (np.cos(2.0 * rr / W.R) * np.sin(3.0 * zz / W.L) + 0.3).reshape(-1)

    def factor(s, p):
        nodes, ws = cell_weights(W, p["r"], p["z"])
        return np.sum(ws * psi[nodes], axis=0)

    fd = win.central(STEP0, N, DELTA, H, dir=factor)
    ad = float(np.sum(gd.reshape(-1) * psi))
    print("directional dJ/dpsi", ad, fd)
    _close(ad, fd, RTOL, "dJ/dpsi along psi")


def test_one_step_voltage_identity():
    states = _states(W, 62)
    g = _context(W, states)
    adj = rzpic.Adjoint(g, 1, delta=DELTA)
    adj.forward(STEP0)
    dvdc, dvrf, _ = adj.backward()
    s = math.sin(2 * math.pi * W.f_rf * (STEP0 + 1) * W.dt)
    assert dvdc != 0.0
    assert abs(dvrf - s * dvdc) <= 1e-12 * abs(dvdc), (dvrf, s * dvdc)


def test_checkpoint_spacing_does_not_change_the_gradient():
    states = _states(W, 63)
    res = []
    for k in (1, 4, N):
        g = _context(W, states)
        adj = rzpic.Adjoint(g, N, checkpoint_every=k, delta=DELTA)
        J = adj.forward(STEP0)
        dvdc, dvrf, gw = adj.backward()
        res.append((J, dvdc, dvrf, [x.cpu().numpy() for x in gw]))
        adj.close()
    for J, dvdc, dvrf, gw in res[1:]:
        assert J == res[0][0]  # the forward window is the same launches
        assert abs(dvrf - res[0][2]) <= 1e-12 * abs(res[0][2])
        assert abs(dvdc - res[0][1]) <= 1e-12 * abs(res[0][1])
        for s in (0, 1):
            sc = np.abs(res[0][3][s]).max()
            assert np.abs(gw[s] - res[0][3][s]).max() <= 1e-12 * sc


def test_sorted_particles_give_the_same_gradient():
    """Tile-sorted particles (sort after the prologue and every 3 steps; the
    reverse pass then sums dJ/dE in LDS windows) against the unsorted run."""
    states = _states(W, 67)
    res = []
    for sort_every in (0, 3):
        w = W.replace(sort_every=sort_every, tile_z=8, tile_r=8)
        g = _context(w, states)
        if sort_every:
            for s in (0, 1):
                g.sort(s)
        adj = rzpic.Adjoint(g, N, checkpoint_every=K, delta=DELTA)
        J = adj.forward(STEP0)
        dvdc, dvrf, gw, gd = adj.backward(density=True)
        res.append((J, dvdc, dvrf, [x.cpu().numpy() for x in gw], gd.cpu().numpy()))
        adj.close()
    (J0, dc0, rf0, gw0, gd0), (J1, dc1, rf1, gw1, gd1) = res
    assert abs(J1 - J0) <= 1e-13 * abs(J0)
    assert abs(rf1 - rf0) <= 1e-11 * abs(rf0) and abs(dc1 - dc0) <= 1e-11 * abs(dc0)
    for s in (0, 1):
        assert np.abs(gw1[s] - gw0[s]).max() <= 1e-11 * np.abs(gw0[s]).max()
    assert np.abs(gd1 - gd0).max() <= 1e-11 * np.abs(gd0).max()


def test_context_is_left_at_the_end_of_the_window():
    states = _states(W, 64)
    g = _context(W, states)
    adj = rzpic.Adjoint(g, 7, checkpoint_every=3, delta=DELTA)
    adj.forward(STEP0)
    after = {s: g.particles(s) for s in (0, 1)}
    phi, n0 = g.grid(rzpic.G_PHI), g.grid(rzpic.G_N0)
    adj.backward()
    for s in (0, 1):
        p = g.particles(s)
        for f in rzpic.FIELDS + ("id",):
            np.testing.assert_array_equal(p[f], after[s][f], err_msg=f"s={s} {f}")
    np.testing.assert_array_equal(g.grid(rzpic.G_PHI), phi)
    np.testing.assert_array_equal(g.grid(rzpic.G_N0), n0)
    g.step(STEP0 + 7)  # and it steps on from there


def test_autograd_wrapper():
    import torch
    states = _states(W, 65)
    g = _context(W, states)
    adj = rzpic.Adjoint(g, 5, checkpoint_every=2, delta=DELTA)
    w_by_id = []
    for s in (0, 1):
        n, _ = g.count(s)
        t = torch.zeros(adj.id_capacity[s], dtype=torch.float64, device=g.device)
        t[g.arrays[s]["id"][:n]] = g.arrays[s]["w"][:n]
        w_by_id.append(t.requires_grad_())
    vdc = torch.tensor(W.V_dc, dtype=torch.float64, requires_grad=True)
    vrf = torch.tensor(W.V_rf, dtype=torch.float64, requires_grad=True)
    J = rzpic.window_objective(adj, STEP0, vdc, vrf, w_by_id)
    (2.0 * J).backward()
    # the same window through the plain calls
    g2 = _context(W, states)
    adj2 = rzpic.Adjoint(g2, 5, checkpoint_every=2, delta=DELTA)
    J2 = adj2.forward(STEP0)
    dvdc, dvrf, gw = adj2.backward()
    assert float(J.detach()) == J2
    assert abs(float(vrf.grad) - 2.0 * dvrf) <= 1e-12 * abs(dvrf)
    assert abs(float(vdc.grad) - 2.0 * dvdc) <= 1e-12 * abs(dvdc)
    for s in (0, 1):
        a, b = w_by_id[s].grad.cpu().numpy(), 2.0 * gw[s].cpu().numpy()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_rejected_configurations():
    states = _states(W, 66)
    for bad in (dict(mg_fixed_cycles=3), dict(resize_every=5), dict(chi_face=wl.FACE_MAX)):
        g = _context(W.replace(**bad), states)
        with pytest.raises(rzpic.RzpicError) as ei:
            rzpic.Adjoint(g, 3)
        assert ei.value.code == 1, bad
    g = rzpic.make_context(W, precision="fp64", with_xsec=True, capacity_factor=2.0)
    with pytest.raises(rzpic.RzpicError):  # collisions on
        rzpic.Adjoint(g, 3)
    gm = rzpic.make_context(W, precision="mixed", with_xsec=False, capacity_factor=2.0)
    with pytest.raises(rzpic.RzpicError):
        rzpic.Adjoint(gm, 3)
    g = _context(W, states)
    adj = rzpic.Adjoint(g, 3, delta=DELTA)
    with pytest.raises(rzpic.RzpicError) as ei:
        adj.backward()  # no forward window yet
    assert ei.value.code == 7
    small = rzpic.Adjoint(g, 2, id_capacity=(10, 10), delta=DELTA)
    small.forward(STEP0)
    with pytest.raises(rzpic.RzpicError) as ei:
        small.backward()  # identities up to 3999
    assert ei.value.code == 1


def test_larger_window_against_differences_of_the_hip_forward():
    """129x65, 200k particles per species, 10 steps in segments of 4, tile
    sort after the prologue and every 4 steps: the adjoint's dJ/dV_rf against
    the central difference of the HIP forward window (fresh contexts from the
    same seeded start)."""
    w = wl.rf_129x65().replace(n_per_species=200_000, mg_fixed_cycles=0, mg_tol=1e-13,
                               mg_max_cycles=400, precision="fp64", V_dc=20.0, sort_every=4)
    delta = 2 * w.L / (w.nz - 1)

    def start():
        g = rzpic.make_context(w, precision="fp64", with_xsec=False, capacity_factor=1.5)
        for s, T in ((0, w.Te_eV), (1, w.Ti_eV)):
            g.init_particles(s, w.n_per_species, w.n0, T, 0)
        g.prologue()
        for s in (0, 1):
            g.sort(s)
        return g

    g = start()
    adj = rzpic.Adjoint(g, 10, checkpoint_every=4, delta=delta)
    adj.forward(STEP0)
    _, dvrf, _ = adj.backward()
    h = H * w.V_rf
    Js, counts = [], []
    for v in (w.V_rf + h, w.V_rf - h):
        gg = start()
        gg.set_voltage(w.V_dc, v)
        a = rzpic.Adjoint(gg, 10, checkpoint_every=4, delta=delta)
        Js.append(a.forward(STEP0))
        counts.append((gg.count(0)[0], gg.count(1)[0]))
        a.close()
    assert counts[0] == counts[1]
    fd = (Js[0] - Js[1]) / (2 * h)
    print("129x65 dJ/dV_rf", dvrf, fd)
    _close(dvrf, fd, 1e-5, "dJ/dV_rf 129x65")
