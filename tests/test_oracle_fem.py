"""Pins of the oracle's Q1/Q1-LPS discretisation (CPU only).

Each test checks the oracle against something other than itself: textbook
element matrices, a manufactured solution with its O(h^2) convergence, the
exact Poiseuille solution, exact discrete mass balance, and finite
differences of the residual.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy as sy

from oracle import fem, mesh, solver
from synthetic import channel_obstacle, rectangle


def test_textbook_q1_element_matrices():
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    cells = np.array([[0, 1, 2, 3]])
    det, grad = fem.geometry(xy, cells)
    M = np.einsum('cq,qa,qb->cab', det, fem.NQ, fem.NQ)[0]
    S = np.einsum('cq,cqad,cqbd->cab', det, grad, grad)[0]
    M_ref = np.array([[4, 2, 1, 2], [2, 4, 2, 1], [1, 2, 4, 2], [2, 1, 2, 4]]) / 36.0
    S_ref = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    np.testing.assert_allclose(M, M_ref, atol=1e-15)
    np.testing.assert_allclose(S, S_ref, atol=1e-15)


def test_fluctuation_matrix_kills_bilinears():
    K = fem.fluctuation_matrix()
    i, j = np.meshgrid(np.arange(3), np.arange(3), indexing="xy")
    xi, eta = i.reshape(-1) / 2.0, j.reshape(-1) / 2.0
    for f in (np.ones(9), xi, eta, xi * eta):
        np.testing.assert_allclose(K @ f, 0.0, atol=1e-15)
    assert np.linalg.matrix_rank(K) == 5          # 9 nodes - 4 bilinears


def _mms(nu):
    x, y = sy.symbols("x y")
    A = sy.sin(sy.pi * y) ** 2
    psi = A * sy.sin(sy.pi * x)
    u = sy.diff(psi, y)
    v = -sy.diff(psi, x)
    # do-nothing outflow at x = 1: nu du/dx = p and dv/dx = 0 there
    p = -nu * sy.pi * sy.diff(A, y) * x
    fx = u * sy.diff(u, x) + v * sy.diff(u, y) - nu * (sy.diff(u, x, 2) + sy.diff(u, y, 2)) + sy.diff(p, x)
    fy = u * sy.diff(v, x) + v * sy.diff(v, y) - nu * (sy.diff(v, x, 2) + sy.diff(v, y, 2)) + sy.diff(p, y)
    lam = lambda e: sy.lambdify((x, y), e, "numpy")
    return lam(u), lam(v), lam(p), lam(fx), lam(fy)


@pytest.mark.slow
def test_manufactured_solution_second_order_velocity():
    """Steady problem (1/k = 0, theta = 1) with a manufactured divergence-free
    velocity that satisfies the do-nothing condition on x = 1: the velocity
    error in L2 must fall as O(h^2) (manufactured-solution pin)."""
    nu = 0.1
    u, v, p, fx, fy = _mms(nu)
    bc = lambda X, Y, t: (u(X, Y) + 0 * X, v(X, Y) + 0 * X)
    force = lambda X, Y, t: (fx(X, Y) + 0 * X, fy(X, Y) + 0 * X)
    m = rectangle(2, 2, 1.0, 1.0, nu=nu)
    lev = mesh.hierarchy(m, 4)
    prob = fem.Problem(nu=nu, dt=np.inf, theta=1.0, force=force, dirichlet=bc)
    errs, perrs = [], []
    for L in lev[1:]:
        X, Y = L.xy[:, 0], L.xy[:, 1]
        xe = np.stack([u(X, Y) + 0 * X, v(X, Y) + 0 * X, p(X, Y) + 0 * X], 1).reshape(-1)
        xh = solver.newton_step(L, prob, xe, 0.0, tol=1e-11)
        M = fem.mass_matrix(L)
        d = (xh - xe).reshape(-1, 3)
        errs.append(np.sqrt(sum(d[:, f] @ (M @ d[:, f]) for f in range(2))))
        perrs.append(np.sqrt(d[:, 2] @ (M @ d[:, 2])))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    prates = np.log2(np.array(perrs[:-1]) / np.array(perrs[1:]))
    assert rates[-1] >= 1.9, (errs, rates)
    assert prates[-1] >= 1.0, (perrs, prates)


def _poiseuille(nu, U, H, Lx, wiggle, finest):
    m = rectangle(4, 2, Lx, H, nu=nu)
    # move the interior macro vertices of the middle row up and down so that
    # fine node rows are no longer horizontal
    mid = np.isclose(m.xy[:, 1], H / 2) & (m.xy[:, 0] > 0) & (m.xy[:, 0] < Lx)
    m.xy[mid, 1] += wiggle * H * (-1.0) ** np.arange(mid.sum())
    lev = mesh.hierarchy(m, finest)
    bc = lambda X, Y, t: (4 * U * Y * (H - Y) / H ** 2, 0 * X)
    prob = fem.Problem(nu=nu, dt=np.inf, theta=1.0, dirichlet=bc)
    return lev, prob


def test_poiseuille_nodally_exact_on_uniform_grid():
    """On a uniform rectangular grid the nodal interpolant of the exact
    Poiseuille solution u = 4 U y (H - y) / H^2, p = 8 nu U (L - x) / H^2
    (do-nothing outflow) is the discrete solution: tensor-product Q1 is
    nodally exact for this 1D profile and kappa(p) = 0 for linear p."""
    nu, U, H, Lx = 0.01, 0.3, 0.41, 2.2
    lev, prob = _poiseuille(nu, U, H, Lx, 0.0, 2)
    for L in lev:
        X, Y = L.xy[:, 0], L.xy[:, 1]
        xe = np.stack([4 * U * Y * (H - Y) / H ** 2, 0 * X, 8 * nu * U * (Lx - X) / H ** 2], 1).reshape(-1)
        R = fem.residual(L, prob, xe, xe, 0.0)
        assert np.abs(R).max() < 1e-14


def test_poiseuille_second_order_on_distorted_grid():
    nu, U, H, Lx = 0.01, 0.3, 0.41, 2.2
    lev, prob = _poiseuille(nu, U, H, Lx, 0.15, 3)
    errs = []
    for L in lev[1:]:
        X, Y = L.xy[:, 0], L.xy[:, 1]
        xe = np.stack([4 * U * Y * (H - Y) / H ** 2, 0 * X, 8 * nu * U * (Lx - X) / H ** 2], 1).reshape(-1)
        xh = solver.newton_step(L, prob, xe, 0.0, tol=1e-12).reshape(-1, 3)
        d = xh - xe.reshape(-1, 3)
        M = fem.mass_matrix(L)
        errs.append(np.sqrt(d[:, 0] @ (M @ d[:, 0]) + d[:, 1] @ (M @ d[:, 1])))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] > 0 and rates[-1] >= 1.8, (errs, rates)


def _boundary_flux(L, xh, tag):
    """Integral of u over the boundary edges with the given tag (u is linear
    along each edge, so the trapezoidal rule is exact)."""
    be = L.bedges[L.bedges[:, 2] == tag]
    u = xh.reshape(-1, 3)[:, 0]
    ln = np.hypot(*(L.xy[be[:, 1]] - L.xy[be[:, 0]]).T)
    return float(np.sum(0.5 * (u[be[:, 0]] + u[be[:, 1]]) * ln))


def test_discrete_mass_balance_channel():
    """Pressure test functions sum to one and the fluctuation of a constant
    is zero, so the converged pressure rows give (div v_h, 1) = 0, i.e. the
    inflow flux equals the outflow flux (walls and obstacle have v = 0)."""
    m = channel_obstacle(1)
    lev = mesh.hierarchy(m, 2)
    L = lev[-1]
    prob = fem.Problem(nu=m.nu, dt=0.05)
    x = np.zeros(3 * L.n_nodes)
    for n in range(1, 4):
        x = solver.newton_step(L, prob, x, 0.3 * n, tol=1e-13)
    fin = _boundary_flux(L, x, 1)
    fout = _boundary_flux(L, x, 3)
    assert fin > 0.05
    assert abs(fin - fout) < 1e-11 * fin * 1e2


def test_jacobian_matches_finite_differences():
    m = channel_obstacle(2)
    L = mesh.hierarchy(m, 1)[-1]
    prob = fem.Problem(nu=m.nu, dt=0.01)
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, 3 * L.n_nodes)
    xo = rng.uniform(-1, 1, 3 * L.n_nodes)
    w = rng.uniform(-1, 1, 3 * L.n_nodes)
    dn = L.dirichlet_nodes()
    w.reshape(-1, 3)[dn, :2] = 0.0
    J = fem.jacobian(L, prob, x)
    eps = 1e-6
    fd = -(fem.residual(L, prob, x + eps * w, xo, 0.3) - fem.residual(L, prob, x - eps * w, xo, 0.3)) / (2 * eps)
    free = np.ones(3 * L.n_nodes, bool)
    free.reshape(-1, 3)[dn, :2] = False
    Jw = J @ w
    assert np.linalg.norm(Jw[free] - fd[free]) <= 1e-8 * np.linalg.norm(Jw[free])


def test_newton_converges_quadratically():
    m = channel_obstacle(0)
    L = mesh.hierarchy(m, 2)[-1]
    prob = fem.Problem(nu=m.nu, dt=0.01)
    x = np.zeros(3 * L.n_nodes)
    x = solver.newton_step(L, prob, x, 0.5, tol=1e-12)
    # the rounding floor of ||R|| is ~1.6e-14 on this mesh (the paper's LPS
    # parameter makes the pressure rows' entries larger than the bounded one)
    _, hist = solver.newton_step(L, prob, x, 0.51, tol=5e-14, return_history=True)
    # e_{k+1} <= C e_k^2: the third residual is far below the square-law bound
    assert hist[2] < 1e3 * hist[1] ** 2 / hist[0] + 1e-15
    assert len(hist) <= 5


def test_dense_direct_solve_agrees_with_sparse():
    m = channel_obstacle(3)
    L = mesh.hierarchy(m, 1)[-1]
    prob = fem.Problem(nu=m.nu, dt=0.01)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, 3 * L.n_nodes)
    J = fem.jacobian(L, prob, x)
    b = rng.standard_normal(J.shape[0])
    xs = spla.spsolve(J.tocsc(), b)
    xd = np.linalg.solve(J.toarray(), b)
    np.testing.assert_allclose(xs, xd, rtol=1e-10, atol=1e-12 * np.abs(xd).max())


def _mms_unsteady(nu):
    """The manufactured field of _mms scaled by g(t) = 1 + sin(2 pi t) / 2:
    v = g v*, p = g p*, with the forcing f = g' v* + g^2 (v*.grad) v*
    - g nu lap v* + g grad p* of the unsteady Navier-Stokes equations (the
    do-nothing condition at x = 1 holds for every t since it is linear)."""
    x, y, t = sy.symbols("x y t")
    A = sy.sin(sy.pi * y) ** 2
    psi = A * sy.sin(sy.pi * x)
    u, v = sy.diff(psi, y), -sy.diff(psi, x)
    p = -nu * sy.pi * sy.diff(A, y) * x
    g = 1 + sy.sin(2 * sy.pi * t) / 2
    U, V, Pp = g * u, g * v, g * p
    fx = sy.diff(U, t) + U * sy.diff(U, x) + V * sy.diff(U, y) - nu * (sy.diff(U, x, 2) + sy.diff(U, y, 2)) \
        + sy.diff(Pp, x)
    fy = sy.diff(V, t) + U * sy.diff(V, x) + V * sy.diff(V, y) - nu * (sy.diff(V, x, 2) + sy.diff(V, y, 2)) \
        + sy.diff(Pp, y)
    lam = lambda e: sy.lambdify((x, y, t), e, "numpy")
    return lam(U), lam(V), lam(Pp), lam(fx), lam(fy)


def _unsteady_run(L, nu, theta, dt, T):
    u, v, p, fx, fy = _mms_unsteady(nu)
    bc = lambda X, Y, t: (u(X, Y, t) + 0 * X, v(X, Y, t) + 0 * X)
    force = lambda X, Y, t: (fx(X, Y, t) + 0 * X, fy(X, Y, t) + 0 * X)
    prob = fem.Problem(nu=nu, dt=dt, theta=theta, force=force, dirichlet=bc)
    X, Y = L.xy[:, 0], L.xy[:, 1]
    exact = lambda t: np.stack([u(X, Y, t) + 0 * X, v(X, Y, t) + 0 * X, p(X, Y, t) + 0 * X], 1).reshape(-1)
    x = exact(0.0)
    n = int(round(T / dt))
    for k in range(1, n + 1):
        x = solver.newton_step(L, prob, x, k * dt, tol=1e-11)
    return x, exact(n * dt)


def _vel_norm(L, d):
    M = fem.mass_matrix(L)
    d = d.reshape(-1, 3)
    return float(np.sqrt(d[:, 0] @ (M @ d[:, 0]) + d[:, 1] @ (M @ d[:, 1])))


@pytest.mark.slow
def test_unsteady_manufactured_solution_temporal_order():
    """Pins the time discretisation of eq. varformv: every (1 - theta) old-state
    term (mass, convection, viscosity, forcing) and the 1/k mass term.
    (i) At fixed h, successive differences of the velocity at T = 0.5 over
    dt = 0.1 .. 0.0125 fall as O(dt^2) for theta = 1/2 (Crank-Nicolson) and
    O(dt) for theta = 1 (backward Euler).  (ii) The limit is the PDE's:
    with the smallest dt the error against the exact velocity falls as O(h^2)
    from one level to the next, as in the steady manufactured-solution pin
    (a wrong sign or weight in an old-state term changes the limit ODE and
    leaves an O(1) error)."""
    nu, T = 0.1, 0.5
    lev = mesh.hierarchy(rectangle(2, 2, 1.0, 1.0, nu=nu), 3)
    L = lev[3]
    for theta, lo, hi in ((0.5, 1.9, 2.2), (1.0, 0.9, 1.15)):
        xs = [_unsteady_run(L, nu, theta, dt, T)[0] for dt in (0.1, 0.05, 0.025, 0.0125)]
        diffs = [_vel_norm(L, xs[k] - xs[k + 1]) for k in range(3)]
        rates = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
        assert lo <= rates[-1] <= hi, (theta, diffs, rates)
    errs = []
    for lvl in (2, 3):
        xh, xe = _unsteady_run(lev[lvl], nu, 0.5, 0.01, T)
        errs.append(_vel_norm(lev[lvl], xh - xe))
    assert np.log2(errs[0] / errs[1]) >= 1.8, errs


def _uniform_level(nx, ny, Lx, Ly, level):
    return mesh.hierarchy(rectangle(nx, ny, Lx, Ly, nu=0.01), level)[level]


def test_convective_stabilisation_closed_form_on_uniform_grid():
    """Quadratic form of the convective term for u = x y on a uniform grid of
    hx x hy cells (Q1 holds x y exactly): with b = (1, 0) the streamline
    derivative is y, its fluctuation y - y_c, so u^T S u = sum_T delta_T
    hx hy^3 / 12; with b = (0, 1) it is delta_T hx^3 hy / 12 (2x2 Gauss is
    exact for these quadratics), delta_T = delta0 / (nu / h_T^2 + |b| / h_T)."""
    L = _uniform_level(3, 2, 1.5, 0.8, 2)              # level 0 = macro refined once: 24 x 16 cells
    hx, hy = 1.5 / 24, 0.8 / 16
    assert L.n_cells == 24 * 16
    nu, d0 = 0.01, 0.7
    prob = fem.Problem(nu=nu, dt=np.inf, delta0=d0)
    X, Y = L.xy[:, 0], L.xy[:, 1]
    u = X * Y
    area = hx * hy
    for bvec, form in (((1.0, 0.0), hx * hy ** 3 / 12), ((0.0, 1.0), hx ** 3 * hy / 12),
                       ((0.6, 0.8), None)):
        xo = np.zeros((L.n_nodes, 3))
        xo[:, 0], xo[:, 1] = bvec
        Sc = fem.convective_matrices(L, prob, xo.reshape(-1))
        q = float(np.einsum('ca,cab,cb->', u[L.cells], Sc, u[L.cells]))
        delta = d0 / (nu / area + 1.0 / np.sqrt(area))
        if form is None:   # b = (0.6, 0.8): fluctuation 0.6 (y - y_c) + 0.8 (x - x_c)
            form = (0.36 * hx * hy ** 3 + 0.64 * hx ** 3 * hy) / 12
        assert abs(q - L.n_cells * delta * form) <= 1e-12 * q, (bvec, q, L.n_cells * delta * form)


def test_convective_stabilisation_vanishes_on_linear_fields_of_parallelograms():
    """On parallelogram cells a linear velocity has a constant gradient, so
    b . grad v is constant per cell and its fluctuation vanishes: the
    residual with delta0 > 0 equals the one without, for any old state."""
    m = rectangle(4, 2, 1.6, 0.41, nu=0.01)
    m.xy = m.xy.copy()
    m.xy[:, 0] += 0.35 * m.xy[:, 1]
    L = mesh.hierarchy(m, 2)[2]
    X, Y = L.xy[:, 0], L.xy[:, 1]
    x = np.stack([0.3 + 0.5 * X - 0.2 * Y, -0.1 + 0.4 * X + 0.7 * Y, np.sin(3 * X)], 1).reshape(-1)
    xo = np.random.default_rng(3).uniform(-1, 1, 3 * L.n_nodes)
    r0 = fem.residual(L, fem.Problem(nu=0.01, dt=0.02), x, xo, 0.3)
    r1 = fem.residual(L, fem.Problem(nu=0.01, dt=0.02, delta0=0.9), x, xo, 0.3)
    assert np.abs(r1 - r0).max() <= 1e-13 * np.abs(r0).max()
    # and it does not vanish for a bilinear field
    x2 = x.reshape(-1, 3).copy()
    x2[:, 0] += 2.0 * X * Y
    r2a = fem.residual(L, fem.Problem(nu=0.01, dt=0.02), x2.reshape(-1), xo, 0.3)
    r2b = fem.residual(L, fem.Problem(nu=0.01, dt=0.02, delta0=0.9), x2.reshape(-1), xo, 0.3)
    assert np.abs(r2b - r2a).max() > 1e-6


def test_convective_stabilisation_jacobian_matches_finite_differences():
    m = channel_obstacle(2)
    L = mesh.hierarchy(m, 1)[-1]
    prob = fem.Problem(nu=m.nu, dt=0.01, delta0=0.5)
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, 3 * L.n_nodes)
    xo = rng.uniform(-1, 1, 3 * L.n_nodes)
    w = rng.uniform(-1, 1, 3 * L.n_nodes)
    dn = L.dirichlet_nodes()
    w.reshape(-1, 3)[dn, :2] = 0.0
    J = fem.jacobian(L, prob, x, xo)
    eps = 1e-6
    fd = -(fem.residual(L, prob, x + eps * w, xo, 0.3) - fem.residual(L, prob, x - eps * w, xo, 0.3)) / (2 * eps)
    free = np.ones(3 * L.n_nodes, bool)
    free.reshape(-1, 3)[dn, :2] = False
    Jw = J @ w
    assert np.linalg.norm(Jw[free] - fd[free]) <= 1e-8 * np.linalg.norm(Jw[free])
    # the term is present: the Jacobian differs from the one without it
    J0 = fem.jacobian(L, fem.Problem(nu=m.nu, dt=0.01), x, xo)
    assert np.linalg.norm((J - J0) @ w) > 1e-3 * np.linalg.norm(Jw)


@pytest.mark.slow
def test_convective_stabilisation_keeps_manufactured_solution_convergence():
    """The manufactured solution of the steady pin with the convective term
    on (delta0 = 0.5, frozen field = the exact velocity): the velocity error
    still falls at second order (the term is consistent to higher order than
    the discretisation)."""
    nu = 0.1
    u, v, p, fx, fy = _mms(nu)
    bc = lambda X, Y, t: (u(X, Y) + 0 * X, v(X, Y) + 0 * X)
    force = lambda X, Y, t: (fx(X, Y) + 0 * X, fy(X, Y) + 0 * X)
    lev = mesh.hierarchy(rectangle(2, 2, 1.0, 1.0, nu=nu), 4)
    prob = fem.Problem(nu=nu, dt=np.inf, theta=1.0, force=force, dirichlet=bc, delta0=0.5)
    errs = []
    for L in lev[1:]:
        X, Y = L.xy[:, 0], L.xy[:, 1]
        xe = np.stack([u(X, Y) + 0 * X, v(X, Y) + 0 * X, p(X, Y) + 0 * X], 1).reshape(-1)
        xh = solver.newton_step(L, prob, xe, 0.0, tol=1e-11)
        M = fem.mass_matrix(L)
        d = (xh - xe).reshape(-1, 3)
        errs.append(np.sqrt(sum(d[:, f] @ (M @ d[:, f]) for f in range(2))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= 1.9, (errs, rates)
