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
