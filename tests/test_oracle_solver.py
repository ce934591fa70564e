"""Pins of the oracle's iterative solver components (CPU only)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, mesh, solver
from synthetic import channel_obstacle


def test_gmres_solves_random_nonsymmetric_system():
    rng = np.random.default_rng(0)
    n = 60
    A = sp.csr_matrix(np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3)
    b = rng.standard_normal(n)
    x, it, hist = solver.gmres(A, b, lambda v: v, rtol=1e-12, restart=20, maxit=200)
    np.testing.assert_allclose(A @ x, b, atol=1e-10)
    assert it > 20          # restarts happened


def test_gmres_residual_estimate_is_true_residual():
    rng = np.random.default_rng(1)
    n = 40
    A = sp.csr_matrix(np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.4)
    b = rng.standard_normal(n)
    x, it, hist = solver.gmres(A, b, lambda v: 0.5 * v, rtol=1e-3, restart=40, maxit=40)
    assert abs(np.linalg.norm(b - A @ x) - hist[-1]) < 1e-10 * np.linalg.norm(b)


def test_vanka_block_extraction_is_exact():
    m = channel_obstacle(0)
    L = mesh.hierarchy(m, 1)[-1]
    prob = fem.Problem(nu=m.nu, dt=0.01)
    x = np.random.default_rng(0).uniform(-1, 1, 3 * L.n_nodes)
    J = fem.jacobian(L, prob, x)
    B = solver.cell_blocks(J, L.cells)
    Jd = J.toarray()
    d = solver.cell_dofs(L.cells)
    for c in (0, 17, L.n_cells - 1):
        np.testing.assert_array_equal(B[c], Jd[np.ix_(d[c], d[c])])


def test_vanka_on_block_diagonal_system_is_exact():
    """If the operator does not couple different cells' unknowns and every
    node lies in one cell, one additive Vanka sweep with omega = 1 is an exact
    solve (special case that reduces to block Jacobi)."""
    rng = np.random.default_rng(2)
    C = 5
    cells = np.arange(4 * C).reshape(C, 4)
    blocks = rng.standard_normal((C, 12, 12)) + 6 * np.eye(12)
    J = sp.block_diag(list(blocks)).tocsr()
    b = rng.standard_normal(12 * C)
    x = solver.vanka_sweep(J, solver.cell_blocks(J, cells), cells, np.zeros(12 * C), b, 1.0)
    np.testing.assert_allclose(J @ x, b, atol=1e-12)


@pytest.mark.slow
def test_gmres_multigrid_iterations_bounded_across_levels():
    """h-independence of the multigrid preconditioner: GMRES iterations per
    Newton step stay bounded as the finest level grows."""
    m = channel_obstacle(0)
    lev = mesh.hierarchy(m, 4)
    prob = fem.Problem(nu=m.nu, dt=0.01)
    counts = {}
    xf = np.zeros(3 * lev[4].n_nodes)
    xf = solver.newton_step(lev[4], prob, xf, 0.3, tol=1e-12)
    for fine in (2, 3, 4):
        levs = lev[:fine + 1]
        xl = xf[:3 * levs[-1].n_nodes]
        _, st = solver.newton_step_mg(levs, prob, xl, 0.31, tol=1e-11)
        counts[fine] = max(st["gmres"])
    assert max(counts.values()) <= 20, counts
    assert counts[4] <= 2 * counts[2] + 2, counts


def test_mg_newton_matches_direct_newton():
    m = channel_obstacle(1)
    lev = mesh.hierarchy(m, 2)
    prob = fem.Problem(nu=m.nu, dt=0.01)
    x0 = np.zeros(3 * lev[-1].n_nodes)
    xd = solver.newton_step(lev[-1], prob, x0, 0.2, tol=1e-13)
    xm, _ = solver.newton_step_mg(lev, prob, x0, 0.2, tol=1e-13)
    assert np.linalg.norm(xm - xd) <= 1e-10 * np.linalg.norm(xd)
