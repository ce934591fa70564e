"""Parity of the HIP flow functionals (J_div, drag, lift) with the oracle (GPU).

FP64 on both sides, same quadrature (2x2 Gauss per cell, 2-point Gauss per
obstacle edge): relative 1e-12.  States: seeded random nodal fields and a
flow state after a few time steps; meshes with one and with three obstacles.
"""
import numpy as np
import pytest

from oracle import functionals as F
from oracle import mesh
from synthetic import channel_obstacle, channel_obstacles, random_state

pytestmark = pytest.mark.gpu


def _close(a, b, tol=1e-12):
    a, b = np.atleast_1d(a), np.atleast_1d(b)
    return np.all(np.abs(a - b) <= tol * max(1.0, np.abs(b).max()))


@pytest.mark.parametrize("gen,seed,level", [(channel_obstacle, 0, 3), (channel_obstacles, 100, 2)])
def test_functionals_match_oracle(gen, seed, level):
    import paper_2106_07687_amd as P
    macro = gen(seed)
    k = len(macro.curves)
    ctx = P.Context(precision=0, nu=macro.nu)
    ctx.setup_mesh(macro, level)
    L = mesh.hierarchy(macro, level)[level]
    for s in (1, 2):
        x = random_state(L.n_nodes, s)
        jg, dg, lg = ctx.functionals(level, x, k)
        jo = F.j_div(L, x)
        do, lo = F.drag_lift(L, x, macro.nu, k)
        print(f"[functionals] {gen.__name__}({seed}) L{level}: J_div {jg:.6e}/{jo:.6e} "
              f"drag {dg} / {do} lift {lg} / {lo}", flush=True)
        assert _close(jg, jo) and _close(dg, do) and _close(lg, lo)
    # a flow state after three steps, through the state entry point
    st = ctx.state(level)
    for _ in range(3):
        ctx.step(st, 0.01)
    x, _ = st.get()
    jg, dg, lg = st.functionals(k)
    do, lo = F.drag_lift(L, x, macro.nu, k)
    assert _close(jg, F.j_div(L, x)) and _close(dg, do) and _close(lg, lo)
    with pytest.raises(P.DnnmgError):
        ctx.functionals(level, x, k + 1)
    st.close()
    ctx.close()


def test_velocity_error_matches_oracle_mass_norm():
    """dnnmg_velocity_error (Sec. 3.4 velocity errors, reading N13): the
    mass-weighted squared L2 norms of P^m v_a - v_b and of v_b equal the
    oracle's v^T M v with the level's Q1 mass matrix (2x2 Gauss), the nodal
    sums equal numpy's; FP64, 1e-12.  A field against itself has error 0, and
    the net's corrected fine velocity equals the correction's own output."""
    import paper_2106_07687_amd as P
    from oracle import fem
    macro = channel_obstacle(0)
    lev = mesh.hierarchy(macro, 3)
    ctx = P.Context(precision=0, nu=macro.nu)
    ctx.setup_mesh(macro, 3)
    a, b = ctx.state(1), ctx.state(3)
    xa = random_state(lev[1].n_nodes, 1)
    xb = random_state(lev[3].n_nodes, 2)
    a.set(xa, 0.0)
    b.set(xb, 0.0)
    out = ctx.velocity_error(1, a.device_ptr(), 3, b.device_ptr())
    xp = lev[3].prolongation() @ (lev[2].prolongation() @ xa.reshape(-1, 3))
    d = xp - xb.reshape(-1, 3)
    M = fem.mass_matrix(lev[3])
    vb = xb.reshape(-1, 3)
    ref = {"l2_err2": sum(d[:, f] @ (M @ d[:, f]) for f in range(2)),
           "l2_ref2": sum(vb[:, f] @ (M @ vb[:, f]) for f in range(2)),
           "nodal_err2": float(np.sum(d[:, :2] ** 2)), "nodal_ref2": float(np.sum(vb[:, :2] ** 2))}
    for k, v in ref.items():
        assert abs(out[k] - v) <= 1e-12 * abs(v), (k, out[k], v)
    same = ctx.velocity_error(3, b.device_ptr(), 3, b.device_ptr())
    assert same["l2_err2"] == 0.0 and same["nodal_err2"] == 0.0
    # the net's corrected fine velocity: x~ + d of the last correction
    net = P.Net(ctx, 1, 2, hidden=32, layers=1)
    net.set_weights(out_scale=np.array([1e-2, 1e-2], dtype=np.float32))
    net.reset(a)
    dbg = net.correct(a, 0.01, debug=True)
    vc = (lev[3].prolongation() @ (lev[2].prolongation() @ xa.reshape(-1, 3))).copy()
    vc[:, :2] += dbg["correction"]
    vc[:, 2] = 0.0
    c = ctx.state(3)
    c.set(vc.reshape(-1), 0.0)
    e = ctx.velocity_error(3, net.fine_velocity_ptr(), 3, c.device_ptr())
    assert e["nodal_err2"] <= 1e-24 * e["nodal_ref2"], e
    for s in (a, b, c):
        s.close()
    net.close()
    ctx.close()
