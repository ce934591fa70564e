"""Pins of the oracle's mesh hierarchy and grid transfers (CPU only)."""
import numpy as np
import pytest

from oracle import fem, mesh
from synthetic import channel_obstacle, rectangle


@pytest.fixture(scope="module")
def chan():
    return channel_obstacle(0), mesh.hierarchy(channel_obstacle(0), 3)


def test_node_count_identity(chan):
    # A quad mesh of a domain with one hole satisfies V - E + F = 0 and
    # 4F = 2 E_int + E_b, hence V = F + E_b / 2 (the identity behind the
    # paper's 640 elements <-> 2124 DoFs = 3 x 708 vertices, Sec. 3.1).
    _, lev = chan
    for L in lev:
        assert L.n_nodes == L.n_cells + L.bedges.shape[0] // 2


def test_paper_dof_counts_are_one_hole_quad_meshes():
    # Sec. 3.1: 640 elements / 2124 DoFs and 2560 elements / 8088 DoFs.  With
    # 3 DoFs per vertex (Q1/Q1) both satisfy V = F + E_b/2 with E_b = 136 and
    # 272, i.e. the boundary doubles under uniform refinement.
    for F, dofs in ((640, 2124), (2560, 8088)):
        assert dofs % 3 == 0
        Eb = 2 * (dofs // 3 - F)
        assert Eb > 0
    assert 2 * (2124 // 3 - 640) * 2 == 2 * (8088 // 3 - 2560)


def test_cells_convex_and_counter_clockwise(chan):
    _, lev = chan
    for L in lev:
        X = L.xy[L.cells]
        for a in range(4):
            e1 = X[:, (a + 1) % 4] - X[:, a]
            e2 = X[:, (a + 3) % 4] - X[:, a]
            cross = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
            assert cross.min() > 0.0


def test_area_converges_to_domain_minus_disc(chan):
    m, lev = chan
    r = m.info["r"]
    exact = 2.2 * 0.41 - np.pi * r * r
    errs = [abs(mesh.cell_areas(L.xy, L.cells).sum() - exact) for L in lev]
    # polygonal approximation of the circle: error ~ h^2, ratio ~ 4 per level
    assert errs[-1] < 2e-4 * exact
    assert errs[-2] / errs[-1] > 3.5


def test_obstacle_nodes_on_circle(chan):
    m, lev = chan
    cx, cy, r = m.info["cx"], m.info["cy"], m.info["r"]
    L = lev[-1]
    ob = L.bedges[L.bedges[:, 2] == 4][:, :2].reshape(-1)
    d = np.hypot(L.xy[ob, 0] - cx, L.xy[ob, 1] - cy)
    np.testing.assert_allclose(d, r, rtol=1e-13)


def test_prolongation_reproduces_affine_and_injects(chan):
    _, lev = chan
    rng = np.random.default_rng(3)
    for l in range(1, len(lev)):
        Lc, Lf = lev[l - 1], lev[l]
        P = Lf.prolongation()
        a, b, c = rng.standard_normal(3)
        fc = a + b * Lc.xy[:, 0] + c * Lc.xy[:, 1]
        ff = a + b * Lf.xy[:, 0] + c * Lf.xy[:, 1]
        pf = P @ fc
        # coarse values injected unchanged
        np.testing.assert_array_equal(pf[:Lc.n_nodes], fc)
        # exact on every node whose parent cell is a parallelogram (not on the
        # curved obstacle boundary or the cells touching it)
        curved = np.zeros(Lf.n_nodes, bool)
        ob = Lf.bedges[Lf.bedges[:, 2] >= 4][:, :2].reshape(-1)
        curved[ob] = True
        bad_cells = curved[Lf.cells].any(axis=1)
        curved[Lf.cells[bad_cells].reshape(-1)] = True
        np.testing.assert_allclose(pf[~curved], ff[~curved], atol=1e-13)


def test_fluctuation_of_prolongated_function_vanishes(chan):
    # A coarse Q1 function is bilinear on each coarse cell = fine patch, so
    # the two-level fluctuation of its prolongation is zero (reading G3).
    _, lev = chan
    K = fem.fluctuation_matrix()
    rng = np.random.default_rng(4)
    for l in range(1, len(lev)):
        pc = rng.standard_normal(lev[l - 1].n_nodes)
        pf = lev[l].prolongation() @ pc
        kap = pf[lev[l].patches()] @ K.T
        assert np.abs(kap).max() < 1e-14


def test_galerkin_mass_identity():
    # For nested spaces with exact quadrature, P^T M_fine P = M_coarse.
    m = rectangle(3, 2, 1.5, 1.0, skew=0.2)
    lev = mesh.hierarchy(m, 2)
    for l in (1, 2):
        P = lev[l].prolongation()
        G = (P.T @ fem.mass_matrix(lev[l]) @ P).toarray()
        np.testing.assert_allclose(G, fem.mass_matrix(lev[l - 1]).toarray(), atol=1e-15)
