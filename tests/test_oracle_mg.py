"""Pins of the oracle's field solver (Sec. 2.5): the finite-volume operator's
structure, the multigrid solution against a direct sparse solve, second-order
convergence on a Bessel-J0 x sine manufactured solution and on the Laplace
series solution, the convergence rates the paper quotes, and the line solve
against a banded LAPACK solve."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.special as ss

from oracle import rzo
from paper_1001_2969_amd import workloads as wl

J01 = ss.jn_zeros(0, 1)[0]
# the right-hand side is rho / eps0 with the oracle's own eps0 (CODATA 2018)
epsilon_0 = rzo.constants()["eps0"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_mg_convergence.txt")


def _w(nr, nz, R=0.02, L=0.02, **kw):
    return wl.Workload(name="t", nr=nr, nz=nz, R=R, L=L, n_per_species=1, steps=1, **kw)


def _assemble(o, w):
    """Matrix of A on the unknowns (interior rows, j < nr-1) column by column."""
    nz, nr = w.nz, w.nr
    unk = [(i, j) for i in range(1, nz - 1) for j in range(nr - 1)]
    A = np.zeros((len(unk), len(unk)))
    for c, (i, j) in enumerate(unk):
        u = np.zeros((nz, nr))
        u[i, j] = 1.0
        y = o.apply_op(u)
        A[:, c] = [y[a, b] for a, b in unk]
    return A, unk


@pytest.mark.parametrize("face", [wl.FACE_AVG, wl.FACE_MAX])
def test_fv_operator_structure(face):
    """Positive coefficients with b = a + c + d + e (A annihilates constants),
    symmetric and positive definite in the control-volume inner product."""
    w = _w(9, 9, chi_face=face)
    o = rzo.Oracle(w, mc=False)
    rng = np.random.default_rng(0)
    o.set_grid(rzo.G_CHI, rng.uniform(0.0, 3.0, (w.nz, w.nr)))
    ones = o.apply_op(np.ones((w.nz, w.nr)))
    assert np.abs(ones[1:-1, :-1]).max() < 1e-9 * (w.nr / w.R) ** 2
    A, unk = _assemble(o, w)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0.0) and np.all(np.diag(A) > 0)
    hr, hz = w.R / (w.nr - 1), w.L / (w.nz - 1)
    vol = np.array([math.pi * (hr / 2) ** 2 * hz if j == 0 else 2 * math.pi * j * hr * hr * hz
                    for (_, j) in unk])
    VA = vol[:, None] * A
    np.testing.assert_allclose(VA, VA.T, rtol=1e-12, atol=1e-12 * np.abs(VA).max())
    assert np.linalg.eigvalsh(0.5 * (VA + VA.T)).min() > 0


def test_multigrid_equals_direct_sparse_solve():
    w = _w(17, 33, R=0.03, L=0.02, V_dc=40.0, mg_tol=1e-13, chi_face=wl.FACE_MAX)
    o = rzo.Oracle(w, mc=False)
    rng = np.random.default_rng(1)
    chi = wl.smooth_chi(w, 1.0) + 0.2 * rng.random((w.nz, w.nr))
    rho = wl.smooth_rho(w, 2, 3e-4)
    o.set_grid(rzo.G_CHI, chi)
    o.set_grid(rzo.G_RHO, rho)
    st, cyc, rr = o.solve(0.0)
    assert st == 0 and rr <= 1e-13
    phi = o.grid(rzo.G_PHI)
    A, unk = _assemble(o, w)
    ubc = np.zeros((w.nz, w.nr))
    ubc[0, :-1] = w.V_dc
    bterm = -o.apply_op(ubc)
    f = np.array([rho[i, j] / epsilon_0 + bterm[i, j] for i, j in unk])
    x = spla.spsolve(sp.csr_matrix(A), f)
    got = np.array([phi[i, j] for i, j in unk])
    np.testing.assert_allclose(got, x, rtol=0, atol=1e-11 * np.abs(x).max())
    # boundary data honoured
    assert np.all(phi[0, :-1] == w.V_dc) and np.all(phi[-1] == 0) and np.all(phi[:, -1] == 0)


def _mms(nr, nz, variable_eps):
    """phi = J0(j01 r/R) sin(pi z/L); with eps = 1 + chi0 exp(-(r/R)^2)(1 + z/L)/2
    the right-hand side is -div(eps grad phi) = -eps lap(phi) - grad eps . grad phi."""
    R = L = 0.02
    w = _w(nr, nz, R=R, L=L, mg_tol=1e-12)
    r = np.linspace(0, R, nr)[None, :]
    z = np.linspace(0, L, nz)[:, None]
    kr, kz = J01 / R, math.pi / L
    J0, J1 = ss.j0(kr * r), ss.j1(kr * r)
    S, Cz = np.sin(kz * z), np.cos(kz * z)
    phi = J0 * S
    lap = -(kr ** 2 + kz ** 2) * phi
    if variable_eps:
        chi0 = 1.5
        g = np.exp(-(r / R) ** 2)
        eps = 1.0 + chi0 * g * (1 + z / L) / 2
        deps_dr = chi0 * (1 + z / L) / 2 * g * (-2 * r / R ** 2)
        deps_dz = chi0 * g / (2 * L) + 0 * z
        dphi_dr = -kr * J1 * S
        dphi_dz = kz * J0 * Cz
        f = -(eps * lap + deps_dr * dphi_dr + deps_dz * dphi_dz)
    else:
        eps = np.ones_like(phi)
        f = -lap
    o = rzo.Oracle(w, mc=False)
    o.set_grid(rzo.G_CHI, eps - 1.0)
    o.set_grid(rzo.G_RHO, epsilon_0 * f)
    st, cyc, rr = o.solve(0.0)
    assert st == 0
    return np.abs(o.grid(rzo.G_PHI) - phi).max()


@pytest.mark.parametrize("variable_eps", [False, True])
def test_manufactured_bessel_solution_second_order(variable_eps):
    errs = [_mms(n, n, variable_eps) for n in (17, 33, 65)]
    assert errs[-1] < 2e-3
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4, errs


def test_laplace_bessel_series_with_powered_electrode():
    """eps = 1, rho = 0, V on z = 0:
    phi = sum_n 2V / (j_n J1(j_n)) J0(j_n r/R) sinh(j_n (L-z)/R) / sinh(j_n L/R).
    The corner (R, 0) is a jump in the boundary data, so compare on the half
    of the domain away from it; the error still falls at second order."""
    V = 100.0
    jn = ss.jn_zeros(0, 400)
    errs = []
    for n in (17, 33, 65):
        R = L = 0.02
        w = _w(n, n, R=R, L=L, V_dc=V, mg_tol=1e-12)
        o = rzo.Oracle(w, mc=False)
        o.set_grid(rzo.G_CHI, np.zeros((n, n)))
        o.set_grid(rzo.G_RHO, np.zeros((n, n)))
        assert o.solve(0.0)[0] == 0
        phi = o.grid(rzo.G_PHI)
        r = np.linspace(0, R, n)
        z = np.linspace(0, L, n)
        sel_i = (z >= 0.25 * L) & (z <= 0.75 * L)
        sel_j = r <= 0.5 * R
        Rg, Zg = np.meshgrid(r[sel_j], z[sel_i])
        ex = np.zeros_like(Rg)
        for j in jn:
            ex += 2 * V / (j * ss.j1(j)) * ss.j0(j * Rg / R) * (
                np.exp(-j * Zg / R) - np.exp(-j * (2 * L - Zg) / R)) / (1 - np.exp(-2 * j * L / R))
        errs.append(np.abs(phi[np.ix_(sel_i, sel_j)] - ex).max())
    assert errs[-1] < 5e-3 * V
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs


def _cycles(w, chi_amp, seed=3):
    o = rzo.Oracle(w.replace(mg_tol=1e-10, mg_max_cycles=60), mc=False)
    o.set_grid(rzo.G_CHI, wl.smooth_chi(w, chi_amp))
    o.set_grid(rzo.G_RHO, wl.smooth_rho(w, seed, 1e-4))
    st, cyc, rr = o.solve(0.0)
    assert st == 0 and rr <= 1e-10
    return cyc


def test_convergence_rates_quoted_by_the_paper():
    golden = dict(line.split() for line in open(GOLDEN) if line.strip() and line[0] != "#")
    bound = int(golden["accepted_upper_bound"])
    meshes = [_w(33, 33), _w(65, 65), _w(129, 65, R=0.04), _w(257, 129, R=0.075, L=0.025)]
    free = [_cycles(w, 0.0) for w in meshes]
    # chi = 0: cycle count independent of the grid size
    assert max(free) - min(free) <= 2, free
    smooth = [_cycles(w, 1.0) for w in meshes]
    assert max(smooth) <= bound, smooth


def test_line_solve_matches_banded_lapack():
    rng = np.random.default_rng(4)
    n = 200
    d = rng.uniform(0.1, 1.0, n)
    e = rng.uniform(0.1, 1.0, n)
    d[0] = 0.0
    e[-1] = 0.0
    b = d + e + rng.uniform(0.0, 0.5, n)
    g = rng.normal(size=n)
    x = rzo.thomas(d, b, e, g)
    ab = np.zeros((3, n))
    ab[0, 1:] = -e[:-1]
    ab[1] = b
    ab[2, :-1] = -d[1:]
    ref = sla.solve_banded((1, 1), ab, g)
    np.testing.assert_allclose(x, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
