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


# ---- coloured multiplicative Vanka (reading N17)

def test_cell_colouring_is_valid_and_greedy():
    m = channel_obstacle(0)
    for L in mesh.hierarchy(m, 3)[1:]:
        col = solver.cell_colours(L.cells)
        # no two cells of one colour share a node
        for k in range(col.max() + 1):
            nodes = L.cells[col == k].reshape(-1)
            assert np.unique(nodes).size == nodes.size
        # greedy in cell order: every colour k > 0 of a cell is taken by an
        # earlier neighbour for each smaller colour
        node_cells = {}
        for c, cell in enumerate(L.cells):
            for v in cell:
                node_cells.setdefault(int(v), []).append(c)
        for c in range(0, L.n_cells, 7):
            earlier = {int(col[o]) for v in L.cells[c] for o in node_cells[int(v)] if o < c}
            assert all(k in earlier for k in range(col[c]))
        assert 4 <= col.max() + 1 <= 8            # a quad mesh needs at least 4


def test_coloured_sweep_on_one_cell_is_exact():
    """A single cell: the sweep solves its 12x12 system (special case)."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((12, 12)) + 5 * np.eye(12)
    J = sp.csr_matrix(A)
    cells = np.array([[0, 1, 2, 3]])
    b = rng.standard_normal(12)
    x = solver.vanka_sweep_coloured(J, solver.cell_blocks(J, cells), cells, solver.cell_colours(cells),
                                    np.zeros(12), b, 1.0)
    np.testing.assert_allclose(A @ x, b, atol=1e-12)


def test_coloured_sweep_is_multiplicative():
    """Two cells sharing an edge take two colours; with omega = 1 the sweep is
    block Gauss-Seidel: after it the residual vanishes on the unknowns of the
    second cell (the additive sweep leaves a residual there)."""
    rng = np.random.default_rng(8)
    cells = np.array([[0, 1, 4, 3], [1, 2, 5, 4]])
    n = 18
    A = rng.standard_normal((n, n)) * 0.3 + 4 * np.eye(n)
    d = solver.cell_dofs(cells)
    mask = np.zeros((n, n), dtype=bool)
    for c in range(2):
        mask[np.ix_(d[c], d[c])] = True
    A = np.where(mask, A, 0.0)                   # couplings only inside a cell
    J = sp.csr_matrix(A)
    col = solver.cell_colours(cells)
    assert list(col) == [0, 1]
    b = rng.standard_normal(n)
    blocks = solver.cell_blocks(J, cells)
    x = solver.vanka_sweep_coloured(J, blocks, cells, col, np.zeros(n), b, 1.0)
    r = b - A @ x
    assert np.abs(r[d[1]]).max() < 1e-12
    xa = solver.vanka_sweep(J, blocks, cells, np.zeros(n), b, 1.0)
    assert np.abs((b - A @ xa)[d[1]]).max() > 1e-3


def test_mg_newton_with_coloured_smoother_matches_direct_newton():
    m = channel_obstacle(1)
    lev = mesh.hierarchy(m, 2)
    prob = fem.Problem(nu=m.nu, dt=0.01)
    x0 = np.zeros(3 * lev[-1].n_nodes)
    xd = solver.newton_step(lev[-1], prob, x0, 0.2, tol=1e-13)
    xm, st = solver.newton_step_mg(lev, prob, x0, 0.2, tol=1e-13, smoother="coloured", omega=0.6)
    np.testing.assert_allclose(xm, xd, rtol=0, atol=1e-10 * np.abs(xd).max())
    # the multiplicative sweep is the stronger smoother: fewer Krylov steps
    _, sa = solver.newton_step_mg(lev, prob, x0, 0.2, tol=1e-13, smoother="additive", omega=0.6)
    assert sum(st["gmres"]) < sum(sa["gmres"]), (st["gmres"], sa["gmres"])


def test_coarse_sweep_count_changes_only_the_lower_levels():
    """nu_coarse acts below the level a cycle is called on: a cycle called
    on level 1 (whose only lower level is the direct solve) is unchanged, a
    cycle on level 2 changes; MG-Newton with it still reaches the direct
    Newton solution."""
    m = channel_obstacle(1)
    lev = mesh.hierarchy(m, 2)
    prob = fem.Problem(nu=m.nu, dt=0.01)
    x = np.random.default_rng(3).uniform(-0.3, 0.3, 3 * lev[2].n_nodes)
    a = solver.MGHierarchy(lev, prob, x)
    c = solver.MGHierarchy(lev, prob, x, nu_coarse=1)
    b1 = np.random.default_rng(4).standard_normal(3 * lev[1].n_nodes)
    np.testing.assert_array_equal(a.vcycle(1, b1), c.vcycle(1, b1))
    b2 = np.random.default_rng(5).standard_normal(3 * lev[2].n_nodes)
    assert np.abs(a.vcycle(2, b2) - c.vcycle(2, b2)).max() > 1e-8
    x0 = np.zeros(3 * lev[-1].n_nodes)
    xd = solver.newton_step(lev[-1], prob, x0, 0.2, tol=1e-13)
    xm, _ = solver.newton_step_mg(lev, prob, x0, 0.2, tol=1e-13, nu_coarse=1)
    np.testing.assert_allclose(xm, xd, rtol=0, atol=1e-10 * np.abs(xd).max())


def test_direct_solve_on_a_finer_coarse_level():
    """With the direct solve on level c, a cycle called on level c is the
    exact solve of J_c x = b, a cycle on a finer level changes against the
    level-0 hierarchy, a cycle below c is refused, and MG-Newton still
    reaches the direct Newton solution."""
    m = channel_obstacle(1)
    lev = mesh.hierarchy(m, 2)
    prob = fem.Problem(nu=m.nu, dt=0.01)
    x = np.random.default_rng(13).uniform(-0.3, 0.3, 3 * lev[2].n_nodes)
    a = solver.MGHierarchy(lev, prob, x)
    c = solver.MGHierarchy(lev, prob, x, coarse=1)
    b1 = np.random.default_rng(14).standard_normal(3 * lev[1].n_nodes)
    x1 = c.vcycle(1, b1)
    assert np.linalg.norm(c.J[1] @ x1 - b1) <= 1e-11 * np.linalg.norm(b1)
    # the level-0 hierarchy's cycle on level 1 is only an approximate solve
    assert np.linalg.norm(a.J[1] @ a.vcycle(1, b1) - b1) > 1e-6 * np.linalg.norm(b1)
    b2 = np.random.default_rng(15).standard_normal(3 * lev[2].n_nodes)
    assert np.abs(a.vcycle(2, b2) - c.vcycle(2, b2)).max() > 1e-8
    with pytest.raises(ValueError):
        c.vcycle(0, b1[:3 * lev[0].n_nodes])
    x0 = np.zeros(3 * lev[-1].n_nodes)
    xd = solver.newton_step(lev[-1], prob, x0, 0.2, tol=1e-13)
    xm, _ = solver.newton_step_mg(lev, prob, x0, 0.2, tol=1e-13, coarse=1)
    np.testing.assert_allclose(xm, xd, rtol=0, atol=1e-10 * np.abs(xd).max())
