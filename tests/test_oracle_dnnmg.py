"""Pins of the oracle's DNN-MG correction (CPU only)."""
import numpy as np
import pytest

from oracle import dnnmg, fem, gru, mesh, solver
from synthetic import channel_obstacle, gru_weights, rectangle


def _parallelogram_mesh():
    m = rectangle(4, 2, 1.6, 0.41, nu=0.01)
    m.xy = m.xy.copy()
    m.xy[:, 0] += 0.35 * m.xy[:, 1]          # every cell a parallelogram
    return m


def _zero_net(D, hidden=8, layers=2):
    w = np.zeros(gru.n_params(D.n_in, hidden, layers, D.n_out))
    return dnnmg.NetSpec(weights=w, hidden=hidden, layers=layers, mu=np.zeros(10),
                         sigma=np.ones(10), out_scale=np.ones(2))


def test_patch_grid_is_lexicographic_in_parent_frame():
    m = rectangle(3, 2, 1.5, 1.0)
    lev = mesh.hierarchy(m, 3)
    D = dnnmg.DnnmgOracle(lev, fem.Problem(nu=0.01, dt=0.01), L=1, m=2)
    S = D.S
    assert S == 9 and D.n_in == 490 and D.n_out == 162
    assert D.n_patches == lev[0].n_cells
    xy = lev[3].xy[D.grid].reshape(-1, S, S, 2)
    assert np.all(np.diff(xy[..., 0], axis=2) > 0)       # i runs along +x
    assert np.all(np.diff(xy[..., 1], axis=1) > 0)       # j runs along +y


def test_patches_tile_the_fine_mesh():
    m = channel_obstacle(0)
    lev = mesh.hierarchy(m, 3)
    D = dnnmg.DnnmgOracle(lev, fem.Problem(nu=m.nu, dt=0.01), L=2, m=1)
    # every fine cell lies in exactly one patch: (S-1)^2 cells per patch
    assert D.n_patches * (D.S - 1) ** 2 == lev[3].n_cells
    assert set(np.unique(D.count)) <= {1.0, 2.0, 3.0, 4.0, 5.0, 6.0}
    assert D.count.min() == 1.0


def test_scatter_of_constant_prediction_is_constant():
    m = channel_obstacle(0)
    lev = mesh.hierarchy(m, 3)
    D = dnnmg.DnnmgOracle(lev, fem.Problem(nu=m.nu, dt=0.01), L=1, m=2)
    net = _zero_net(D)
    net.out_scale = np.array([0.7, -0.2])
    Y = np.ones((D.n_patches, D.n_out))
    d = D.scatter(Y, net)
    free = ~D.dir_f
    np.testing.assert_allclose(d[free, 0], 0.7, rtol=1e-15)
    np.testing.assert_allclose(d[free, 1], -0.2, rtol=1e-15)
    assert np.all(d[D.dir_f] == 0.0)


def test_zero_network_restricted_rhs_equals_coarse_rhs_on_parallelograms():
    """(P^m)^T Rhs^F(P^m v) = Rhs^L(v) when every cell is a parallelogram:
    nested Q1 spaces and exact 2x2 Gauss quadrature for every term."""
    m = _parallelogram_mesh()
    lev = mesh.hierarchy(m, 3)
    prob = fem.Problem(nu=0.01, dt=0.02)
    rng = np.random.default_rng(0)
    for (L, mm) in ((1, 2), (2, 1)):
        D = dnnmg.DnnmgOracle(lev, prob, L=L, m=mm)
        v = rng.uniform(-1, 1, 3 * lev[L].n_nodes)
        bL = D.restrict(D.rhs(D.prolong(v)))
        ref = np.zeros((lev[L].n_nodes, 3))
        ref[:, :2] = dnnmg.rhs_rows(lev[L], prob, v)
        np.testing.assert_allclose(bL.reshape(-1, 3), ref, rtol=1e-12, atol=1e-13)


def test_zero_network_dnnmg_step_equals_plain_coarse_step():
    m = _parallelogram_mesh()
    lev = mesh.hierarchy(m, 3)
    prob = fem.Problem(nu=0.01, dt=0.02)
    L, mm = 1, 2
    D = dnnmg.DnnmgOracle(lev, prob, L=L, m=mm)
    net = _zero_net(D)
    x = np.zeros(3 * lev[L].n_nodes)
    x_plain = x.copy()
    vprev = D.prolong(x)
    h = np.zeros((net.layers, D.n_patches, net.hidden))
    bL = None
    for n in range(1, 4):
        t = n * prob.dt
        x = dnnmg.dnnmg_newton(lev, prob, L, x, bL, t, tol=1e-13)
        x_plain = solver.newton_step(lev[L], prob, x_plain, t, tol=1e-13)
        np.testing.assert_allclose(x, x_plain, rtol=1e-9, atol=1e-12)
        bL, vprev, h, _ = D.correct(x, vprev, h, net, t)


def test_dnnmg_residual_with_plain_rhs_equals_plain_residual():
    """R = b - A_impl(x) with b = f(x_old) reproduces R = f(x_old) - A(x)."""
    m = channel_obstacle(2)
    lev = mesh.hierarchy(m, 2)
    prob = fem.Problem(nu=m.nu, dt=0.01)
    rng = np.random.default_rng(3)
    L = lev[2]
    x = rng.uniform(-1, 1, 3 * L.n_nodes)
    xo = rng.uniform(-1, 1, 3 * L.n_nodes)
    b = np.zeros((L.n_nodes, 3))
    b[:, :2] = dnnmg.rhs_rows(L, prob, xo)
    R1 = dnnmg.dnnmg_residual(lev, prob, 2, x, xo, b.reshape(-1), 0.4)
    R2 = fem.residual(L, prob, x, xo, 0.4)
    np.testing.assert_allclose(R1, R2, rtol=1e-12, atol=1e-13)


# ---- cell patches (one level-L element, the patch of the paper's experiments)

def test_cell_patches_are_the_level_L_cells():
    m = channel_obstacle(0)
    lev = mesh.hierarchy(m, 3)
    D = dnnmg.DnnmgOracle(lev, fem.Problem(nu=m.nu, dt=0.01), L=2, m=1, kind=dnnmg.PATCH_CELL)
    assert (D.S, D.n_in, D.n_out, D.n_stats) == (3, 51, 18, 11)      # Table 1's I and O
    assert D.n_patches == lev[2].n_cells
    g = D.grid
    # corners in the cell's own vertex order (c00, c10, c11, c01)
    np.testing.assert_array_equal(g[:, [0, 2, 8, 6]], lev[2].cells)
    # the nine nodes are the vertices of the cell's four children
    for c in range(0, lev[2].n_cells, 37):
        assert set(g[c].tolist()) == set(lev[3].cells[4 * c:4 * c + 4].reshape(-1).tolist())
    # the patches tile the fine mesh
    assert D.n_patches * (D.S - 1) ** 2 == lev[3].n_cells
    # m = 2: 5 x 5 nodes whose corners are still the level-L cell's vertices
    D2 = dnnmg.DnnmgOracle(lev, fem.Problem(nu=m.nu, dt=0.01), L=1, m=2, kind=dnnmg.PATCH_CELL)
    assert (D2.S, D2.n_in, D2.n_out) == (5, 131, 50)
    np.testing.assert_array_equal(D2.grid[:, [0, 4, 24, 20]], lev[1].cells)


def test_cell_patch_grid_is_lexicographic_and_orientation_feature():
    base = rectangle(3, 2, 1.5, 1.0)
    lev = mesh.hierarchy(base, 2)
    D = dnnmg.DnnmgOracle(lev, fem.Problem(nu=0.01, dt=0.01), L=1, m=1, kind=dnnmg.PATCH_CELL)
    xy = lev[2].xy[D.grid].reshape(-1, 3, 3, 2)
    assert np.all(np.diff(xy[..., 0], axis=2) > 0) and np.all(np.diff(xy[..., 1], axis=1) > 0)
    np.testing.assert_allclose(D.c2, 1.0, atol=1e-15)
    np.testing.assert_allclose(D.s2, 0.0, atol=1e-15)
    # the same mesh rotated by theta: the mid-line turns by theta
    th = 0.3
    rot = rectangle(3, 2, 1.5, 1.0)
    rot.xy = base.xy @ np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]])
    levr = mesh.hierarchy(rot, 2)
    Dr = dnnmg.DnnmgOracle(levr, fem.Problem(nu=0.01, dt=0.01), L=1, m=1, kind=dnnmg.PATCH_CELL)
    np.testing.assert_allclose(Dr.c2, np.cos(2 * th), atol=1e-13)
    np.testing.assert_allclose(Dr.s2, np.sin(2 * th), atol=1e-13)
    np.testing.assert_allclose(Dr.aspect, D.aspect, rtol=1e-13)


def test_cell_patch_inputs_channels_and_peclet():
    """Channels [u, v, r_u, r_v, r_p] (no pressure) and, for a uniform flow
    (1, 0), the Peclet feature h_P / nu."""
    base = rectangle(3, 2, 1.5, 1.0)
    lev = mesh.hierarchy(base, 2)
    prob = fem.Problem(nu=0.01, dt=0.01)
    D = dnnmg.DnnmgOracle(lev, prob, L=1, m=1, kind=dnnmg.PATCH_CELL)
    N = lev[2].n_nodes
    rng = np.random.default_rng(4)
    x = np.zeros((N, 3))
    x[:, 0] = 1.0
    x[:, 2] = rng.uniform(-1, 1, N)             # pressure must not appear as a channel
    X, r = D.inputs(x.reshape(-1), x.reshape(-1), 0.5)
    n = 9
    np.testing.assert_array_equal(X[:, :n], 1.0)
    np.testing.assert_array_equal(X[:, n:2 * n], 0.0)
    for k, f in enumerate((0, 1, 2)):
        np.testing.assert_array_equal(X[:, (2 + k) * n:(3 + k) * n], r[D.grid, f])
    np.testing.assert_allclose(X[:, 5 * n + 3], D.h / prob.nu, rtol=1e-14)
    assert X.shape[1] == 5 * n + 6 == 51


def test_static_features_of_known_quadrilaterals():
    """Aspect ratio, mid-line skew |cos| and h_P (reading N5) on patches whose
    values are known by hand: a parallelogram with sides a and sqrt(s^2 + b^2)
    (mid-lines (a, 0) and (s, b), area a b) and a symmetric trapezoid with
    parallel sides 4 and 2 and height 2 (mid-lines (3, 0) and (0, 2), area 6).
    Patch nodes are lexicographic in an S x S grid; only the corners enter."""
    S = 3
    a, s, b = 2.0, 0.5, 1.0
    para = {0: (0.0, 0.0), 2: (a, 0.0), 6: (s, b), 8: (a + s, b)}
    trap = {0: (0.0, 0.0), 2: (4.0, 0.0), 6: (1.0, 2.0), 8: (3.0, 2.0)}
    xy = np.zeros((2 * S * S, 2))
    for k, (px, py) in para.items():
        xy[k] = (px, py)
    for k, (px, py) in trap.items():
        xy[S * S + k] = (px, py)
    grid = np.arange(2 * S * S).reshape(2, S * S)
    aspect, skew, h = dnnmg.static_features(xy, grid, S)
    side2 = np.hypot(s, b)
    np.testing.assert_allclose(aspect, [a / side2, 4.0 / 2.0], rtol=1e-15)
    np.testing.assert_allclose(skew, [s / side2, 0.0], atol=1e-15)
    np.testing.assert_allclose(h, [np.sqrt(a * b), np.sqrt(6.0)], rtol=1e-15)
    # a rotated and scaled copy keeps aspect and skew, scales h
    c, sn = np.cos(0.7), np.sin(0.7)
    xr = 3.0 * xy @ np.array([[c, sn], [-sn, c]])
    a2, s2, h2 = dnnmg.static_features(xr, grid, S)
    np.testing.assert_allclose(a2, aspect, rtol=1e-13)
    np.testing.assert_allclose(s2, skew, atol=1e-13)
    np.testing.assert_allclose(h2, 3.0 * h, rtol=1e-13)
