"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances: FP64 mode, single operations 1e-12 relative (rounding order
only); time steps 1e-10 relative L2 per field (the FP64 parity bar); mixed mode
1e-5 relative L2 per step.  Inputs are seeded (synthetic.*) on the channel
configuration of the FP64 parity workload (level 3, ~5.5k nodes: 87 SELL
slices, the last one ragged).
"""
import numpy as np
import pytest

from oracle import fem, mesh, solver
from synthetic import channel_obstacle, random_state, rectangle

pytestmark = pytest.mark.gpu

DT = 0.01


def _ctx(precision, **kw):
    import paper_2106_07687_amd as P
    return P.Context(precision=precision, **kw)


@pytest.fixture(scope="module")
def c1():
    macro = channel_obstacle(0)
    lev = mesh.hierarchy(macro, 3)
    ctx = _ctx(0, nu=macro.nu)
    ctx.setup_mesh(macro, 3)
    prob = fem.Problem(nu=macro.nu, dt=DT)
    print(f"[c1] seed 0 level 3 nodes={lev[3].n_nodes}", flush=True)
    return macro, lev, ctx, prob


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_mesh_hierarchy_matches_oracle(c1):
    macro, lev, ctx, _ = c1
    for l, L in enumerate(lev):
        n, c, p = ctx.level_info(l)
        assert (n, c, p) == (L.n_nodes, L.n_cells, L.n_cells // 4)
        np.testing.assert_array_equal(ctx.level_cells(l), L.cells)
        np.testing.assert_allclose(ctx.level_coords(l), L.xy, rtol=0, atol=1e-15)


def test_residual_parity(c1):
    macro, lev, ctx, prob = c1
    for l in range(4):
        L = lev[l]
        x = random_state(L.n_nodes, 10 + l)
        xo = random_state(L.n_nodes, 20 + l)
        for t in (0.37, 1.5):
            r_gpu = ctx.residual(l, x, xo, t, DT)
            r_ref = fem.residual(L, prob, x, xo, t)
            assert rel(r_gpu, r_ref) < 1e-13, (l, t, rel(r_gpu, r_ref))


def test_residual_of_rest_state_is_zero(c1):
    # degenerate case: fluid at rest with zero inflow at t = 0
    macro, lev, ctx, prob = c1
    z = np.zeros(3 * lev[3].n_nodes)
    assert np.abs(ctx.residual(3, z, z, 0.0, DT)).max() == 0.0


def test_jacobian_parity_all_levels(c1):
    macro, lev, ctx, prob = c1
    x = random_state(lev[3].n_nodes, 5)
    st = ctx.state(3)
    st.set(x, 0.0)
    ctx.linearize(st, 3, DT)
    for l in range(4):
        L = lev[l]
        # level 3 carries the problem's own LPS parameter, the coarser levels
        # of its preconditioner the bounded one (reading G4)
        pl = prob if l == 3 else fem.coarse_operator_problem(prob)
        J = fem.jacobian(L, pl, x[:3 * L.n_nodes])
        w = random_state(L.n_nodes, 30 + l)
        y = ctx.jacobian_apply(l, w)
        assert rel(y, J @ w) < 1e-13, (l, rel(y, J @ w))
    st.close()


def test_transfer_parity(c1):
    macro, lev, ctx, prob = c1
    for l in range(1, 4):
        P = lev[l].prolongation()
        ec = random_state(lev[l - 1].n_nodes, 40 + l)
        rf = random_state(lev[l].n_nodes, 50 + l)
        pf = ctx.prolong(l, ec)
        np.testing.assert_allclose(pf, (P @ ec.reshape(-1, 3)).reshape(-1), rtol=0, atol=1e-15)
        rc = ctx.restrict(l, rf)
        ref = (P.T @ rf.reshape(-1, 3))
        ref[lev[l - 1].dirichlet_nodes(), :2] = 0.0
        np.testing.assert_allclose(rc, ref.reshape(-1), rtol=1e-14, atol=1e-14)


def _oracle_mg(lev, prob, x):
    return solver.MGHierarchy(lev, prob, x)


def test_vanka_and_vcycle_parity(c1):
    macro, lev, ctx, prob = c1
    x = random_state(lev[3].n_nodes, 6) * 0.3
    st = ctx.state(3)
    st.set(x, 0.0)
    ctx.linearize(st, 3, DT)
    mg = _oracle_mg(lev, prob, x)
    b = random_state(lev[3].n_nodes, 7)
    b.reshape(-1, 3)[lev[3].dirichlet_nodes(), :2] = 0.0
    x0 = random_state(lev[3].n_nodes, 8) * 0.1
    x0.reshape(-1, 3)[lev[3].dirichlet_nodes(), :2] = 0.0
    xs_gpu = ctx.vanka_sweep(3, x0, b)
    xs_ref = solver.vanka_sweep(mg.J[3], mg.blocks[3], lev[3].cells, x0, b, 0.6)
    assert rel(xs_gpu, xs_ref) < 1e-11, rel(xs_gpu, xs_ref)
    for l in (1, 2, 3):
        bl = b[:3 * lev[l].n_nodes].copy()
        bl.reshape(-1, 3)[lev[l].dirichlet_nodes(), :2] = 0.0
        v_gpu = ctx.vcycle(l, bl)
        v_ref = mg.vcycle(l, bl)
        assert rel(v_gpu, v_ref) < 1e-10, (l, rel(v_gpu, v_ref))
    st.close()


def test_gmres_solve_reduces_residual(c1):
    macro, lev, ctx, prob = c1
    x = random_state(lev[3].n_nodes, 9) * 0.3
    st = ctx.state(3)
    st.set(x, 0.0)
    ctx.linearize(st, 3, DT)
    J = fem.jacobian(lev[3], prob, x)
    b = random_state(lev[3].n_nodes, 11)
    b.reshape(-1, 3)[lev[3].dirichlet_nodes(), :2] = 0.0
    ctx.set_params(gmres_rtol=1e-8, gmres_max=200)
    try:
        w, info = ctx.solve(3, b)
    finally:
        ctx.set_params(gmres_rtol=1e-2, gmres_max=100)
    assert np.linalg.norm(b - J @ w) <= 1.1e-8 * np.linalg.norm(b), info
    st.close()


def test_fp64_time_steps_match_oracle(c1):
    """Ten Crank-Nicolson steps from rest (FP64 parity workload): the GPU
    Newton-GMRES-multigrid solution equals the oracle's Newton-direct
    solution within 1e-10 relative L2 per field at every step."""
    macro, lev, ctx, prob = c1
    L = lev[3]
    # parity runs: tolerances well below the 1e-10 relative bar (the velocity
    # is O(1e-4) during the first steps of the inflow ramp); the oracle's
    # Newton stops at 5e-15, above its rounding floor (up to 2.1e-15 over these
    # ten steps)
    ctx.set_params(newton_tol=1e-14)
    st = ctx.state(3)
    x_ref = np.zeros(3 * L.n_nodes)
    worst = 0.0
    try:
        for n in range(1, 11):
            info = ctx.step(st, DT)
            x_ref = solver.newton_step(L, prob, x_ref, n * DT, tol=5e-15)
            xg, t = st.get()
            assert abs(t - n * DT) < 1e-15
            for f in range(3):
                e = rel(xg.reshape(-1, 3)[:, f], x_ref.reshape(-1, 3)[:, f])
                worst = max(worst, e)
                assert e < 1e-10, (n, f, e, info)
    finally:
        ctx.set_params(newton_tol=1e-10)
        st.close()
    print(f"[c1] fp64 worst relative L2 over 10 steps: {worst:.3e}")


def test_mixed_precision_steps_match_oracle():
    macro = channel_obstacle(1)
    lev = mesh.hierarchy(macro, 3)
    L = lev[3]
    prob = fem.Problem(nu=macro.nu, dt=DT)
    ctx = _ctx(1, nu=macro.nu)
    ctx.setup_mesh(macro, 3)
    st = ctx.state(3)
    x_ref = np.zeros(3 * L.n_nodes)
    errs = []
    for n in range(1, 6):
        ctx.step(st, DT)
        x_ref = solver.newton_step(L, prob, x_ref, n * DT, tol=1e-13)
        xg, _ = st.get()
        e = max(rel(xg.reshape(-1, 3)[:, f], x_ref.reshape(-1, 3)[:, f]) for f in range(3))
        errs.append(e)
        # restart both from the oracle state: per-step error
        st.set(x_ref, n * DT)
    print(f"[c1-mixed] per-step relative L2: {['%.2e' % e for e in errs]}")
    assert max(errs) < 1e-5, errs


def test_rectangle_without_obstacle():
    # degenerate geometry: no curved boundary, a single macro cell row
    macro = rectangle(3, 1, 1.2, 0.41, nu=0.01)
    lev = mesh.hierarchy(macro, 2)
    ctx = _ctx(0, nu=0.01, newton_tol=1e-14)
    ctx.setup_mesh(macro, 2)
    prob = fem.Problem(nu=0.01, dt=DT)
    x = random_state(lev[2].n_nodes, 3)
    r = ctx.residual(2, x, x, 0.5, DT)
    assert rel(r, fem.residual(lev[2], prob, x, x, 0.5)) < 1e-13
    st = ctx.state(2)
    ctx.step(st, DT)
    xg, _ = st.get()
    xr = solver.newton_step(lev[2], prob, np.zeros(3 * lev[2].n_nodes), DT, tol=1e-15)
    e = float(rel(xg, xr))
    assert e < 1e-10, e


def test_coloured_vanka_and_vcycle_parity(c1):
    """The coloured multiplicative sweep (smoother = 1) and V-cycles built on
    it against the oracle's (same greedy colouring, FP64): 1e-11 / 1e-10."""
    macro, lev, ctx, prob = c1
    x = random_state(lev[3].n_nodes, 16) * 0.3
    st = ctx.state(3)
    st.set(x, 0.0)
    ctx.set_params(smoother=1)
    try:
        ctx.linearize(st, 3, DT)
        mg = solver.MGHierarchy(lev, prob, x, smoother="coloured")
        b = random_state(lev[3].n_nodes, 17)
        b.reshape(-1, 3)[lev[3].dirichlet_nodes(), :2] = 0.0
        x0 = random_state(lev[3].n_nodes, 18) * 0.1
        x0.reshape(-1, 3)[lev[3].dirichlet_nodes(), :2] = 0.0
        xs_gpu = ctx.vanka_sweep(3, x0, b)
        xs_ref = solver.vanka_sweep_coloured(mg.J[3], mg.blocks[3], lev[3].cells, mg.colours[3], x0, b, 0.6)
        print(f"[coloured] {mg.colours[3].max() + 1} colours on level 3; sweep {rel(xs_gpu, xs_ref):.2e}",
              flush=True)
        assert rel(xs_gpu, xs_ref) < 1e-11, rel(xs_gpu, xs_ref)
        for l in (1, 2, 3):
            bl = b[:3 * lev[l].n_nodes].copy()
            bl.reshape(-1, 3)[lev[l].dirichlet_nodes(), :2] = 0.0
            v_gpu = ctx.vcycle(l, bl)
            v_ref = mg.vcycle(l, bl)
            assert rel(v_gpu, v_ref) < 1e-10, (l, rel(v_gpu, v_ref))
    finally:
        ctx.set_params(smoother=0)
        st.close()


@pytest.mark.parametrize("precision,bar", [(0, 1e-10), (1, 1e-5)])
def test_coloured_smoother_steps_match_oracle(precision, bar):
    """Time steps with the coloured smoother reach the oracle's x_n (FP64
    1e-10 at Newton 5e-15; mixed 1e-5 per step).  In the first ramp steps the
    velocity is O(1e-4), so the 1e-10 relative bar needs the FP64 residual
    below ~1e-14 (the rounding floor of these three steps is below 1e-15)."""
    macro = channel_obstacle(0)
    lev = mesh.hierarchy(macro, 3)
    L = lev[3]
    prob = fem.Problem(nu=macro.nu, dt=DT)
    ctx = _ctx(precision, nu=macro.nu, smoother=1, newton_tol=5e-15 if precision == 0 else 1e-10)
    ctx.setup_mesh(macro, 3)
    st = ctx.state(3)
    x_ref = np.zeros(3 * L.n_nodes)
    for n in range(1, 4):
        info = ctx.step(st, DT)
        x_ref = solver.newton_step(L, prob, x_ref, n * DT, tol=5e-15)
        xg, _ = st.get()
        e = max(rel(xg.reshape(-1, 3)[:, f], x_ref.reshape(-1, 3)[:, f]) for f in range(3))
        print(f"[coloured] precision {precision} step {n}: {e:.2e}, gmres {info['gmres_iters']}", flush=True)
        assert e < bar, (n, e)
        if precision == 1:
            st.set(x_ref, n * DT)               # per-step error
    st.close()
    ctx.close()


def test_coarse_sweep_count_parity(c1):
    """nu_coarse = 1: V-cycles called on levels 3 and 2 take one sweep before
    and after on the levels below (oracle to 1e-10, FP64); FP64 time steps
    still reach the oracle's x_n (1e-10)."""
    macro, lev, ctx, prob = c1
    x = random_state(lev[3].n_nodes, 26) * 0.3
    st = ctx.state(3)
    st.set(x, 0.0)
    ctx.set_params(nu_coarse=1)
    try:
        ctx.linearize(st, 3, DT)
        mg = solver.MGHierarchy(lev, prob, x, nu_coarse=1)
        b = random_state(lev[3].n_nodes, 27)
        b.reshape(-1, 3)[lev[3].dirichlet_nodes(), :2] = 0.0
        for l in (3, 2, 1):
            bl = b[:3 * lev[l].n_nodes].copy()
            bl.reshape(-1, 3)[lev[l].dirichlet_nodes(), :2] = 0.0
            for rep in range(2):                   # captured, then replayed
                v_gpu = ctx.vcycle(l, bl)
                v_ref = mg.vcycle(l, bl)
                assert rel(v_gpu, v_ref) < 1e-10, (l, rep, rel(v_gpu, v_ref))
        ctx.set_params(newton_tol=1e-14)
        s2 = ctx.state(3)
        x_ref = np.zeros(3 * lev[3].n_nodes)
        for n in range(1, 3):
            ctx.step(s2, DT)
            x_ref = solver.newton_step(lev[3], prob, x_ref, n * DT, tol=5e-15)
            e = rel(s2.get()[0], x_ref)
            print(f"[nu_coarse] step {n}: {e:.2e}", flush=True)
            assert e < 1e-10
        s2.close()
    finally:
        ctx.set_params(nu_coarse=0, newton_tol=1e-10)
        st.close()


@pytest.mark.gpu
@pytest.mark.parametrize("coarse", [1, 2])
def test_coarse_level_direct_solve_parity(coarse):
    """coarse_level = c: the FP64 dense inverse sits on level c (level 1: one
    block of 1140 unknowns, the blocked Gauss-Jordan with two rows per panel
    thread; level 2: more than 1536 unknowns, one pivot and one elimination
    launch per column); V-cycles called on levels 3 .. c match the oracle's hierarchy
    with its direct solve on level c (1e-10, FP64; on level c the exact
    solve), a cycle below c is refused, and FP64 time steps reach the
    oracle's x_n (1e-10)."""
    import paper_2106_07687_amd as P
    macro = channel_obstacle(0)
    lev = mesh.hierarchy(macro, 3)
    prob = fem.Problem(nu=macro.nu, dt=DT)
    ctx = _ctx(0, nu=macro.nu, coarse_level=coarse)
    ctx.setup_mesh(macro, 3)
    print(f"[coarse_level {coarse}] level {coarse} unknowns {3 * lev[coarse].n_nodes}", flush=True)
    x = random_state(lev[3].n_nodes, 60 + coarse) * 0.3
    st = ctx.state(3)
    st.set(x, 0.0)
    ctx.linearize(st, 3, DT)
    mg = solver.MGHierarchy(lev, prob, x, coarse=coarse)
    b = random_state(lev[3].n_nodes, 70 + coarse)
    for l in range(3, coarse - 1, -1):
        bl = b[:3 * lev[l].n_nodes].copy()
        bl.reshape(-1, 3)[lev[l].dirichlet_nodes(), :2] = 0.0
        for rep in range(2):                       # captured, then replayed
            v_gpu = ctx.vcycle(l, bl)
            v_ref = mg.vcycle(l, bl)
            assert rel(v_gpu, v_ref) < 1e-10, (l, rep, rel(v_gpu, v_ref))
    with pytest.raises(P.DnnmgError):
        ctx.vcycle(coarse - 1, b[:3 * lev[coarse - 1].n_nodes].copy())
    with pytest.raises(P.DnnmgError):
        ctx.set_params(coarse_level=0)
    ctx.set_params(newton_tol=1e-14)
    s2 = ctx.state(3)
    x_ref = np.zeros(3 * lev[3].n_nodes)
    for n in range(1, 3):
        info = ctx.step(s2, DT)
        x_ref = solver.newton_step(lev[3], prob, x_ref, n * DT, tol=5e-15)
        e = rel(s2.get()[0], x_ref)
        print(f"[coarse_level {coarse}] step {n}: {e:.2e}, gmres {info['gmres_iters']}", flush=True)
        assert e < 1e-10
    s2.close()
    st.close()
    ctx.close()


def test_convective_stabilisation_parity(c1):
    """The optional convective stabilisation (delta0 = 0.5; frozen field b
    from the old state, or from the state itself in dnnmg_linearize) against
    the oracle: residual on levels 1 and 3 and the Jacobian action on every
    level at 1e-13 (FP64), and three FP64 time steps against the oracle's
    direct Newton at 1e-10."""
    macro, lev, _, _ = c1
    ctx = _ctx(0, nu=macro.nu, delta0=0.5, newton_tol=5e-15)
    ctx.setup_mesh(macro, 3)
    prob = fem.Problem(nu=macro.nu, dt=DT, delta0=0.5)
    plain = fem.Problem(nu=macro.nu, dt=DT)
    for l in (1, 3):
        L = lev[l]
        x = random_state(L.n_nodes, 60 + l)
        xo = random_state(L.n_nodes, 70 + l)
        r_gpu = ctx.residual(l, x, xo, 0.37, DT)
        r_ref = fem.residual(L, prob, x, xo, 0.37)
        assert rel(r_gpu, r_ref) < 1e-13, (l, rel(r_gpu, r_ref))
        assert rel(r_ref, fem.residual(L, plain, x, xo, 0.37)) > 1e-6     # the term is there
    x = random_state(lev[3].n_nodes, 75) * 0.5
    st = ctx.state(3)
    st.set(x, 0.0)
    ctx.linearize(st, 3, DT)
    for l in range(4):
        L = lev[l]
        pl = prob if l == 3 else fem.coarse_operator_problem(prob)
        xl = x[:3 * L.n_nodes]
        J = fem.jacobian(L, pl, xl, xl)
        w = random_state(L.n_nodes, 80 + l)
        assert rel(ctx.jacobian_apply(l, w), J @ w) < 1e-13, l
    st.close()
    st = ctx.state(3)
    x_ref = np.zeros(3 * lev[3].n_nodes)
    for n in range(1, 4):
        info = ctx.step(st, DT)
        x_ref = solver.newton_step(lev[3], prob, x_ref, n * DT, tol=5e-15)
        e = max(rel(st.get()[0].reshape(-1, 3)[:, f], x_ref.reshape(-1, 3)[:, f]) for f in range(3))
        print(f"[conv] step {n}: rel {e:.2e} ({info})", flush=True)
        assert e < 1e-10, (n, e)
    st.close()
    ctx.close()
