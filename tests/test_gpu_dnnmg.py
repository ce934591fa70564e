"""Parity of the HIP DNN-MG correction (Algorithm 1, the correction after the coarse step) with the oracle.

The network runs in BF16 (weights, inputs and the GEMM copy of the hidden
state) with FP32 accumulation and gates.  Bars: against a BF16-emulating
numpy model of the same arithmetic, relative L2 <= 1e-2 per output; against
the FP64 oracle, relative L2 <= 3e-2 with cosine >= 0.999.  Everything
downstream of the network output (scatter, rhs, restriction) is FP64 and is
compared with the oracle fed the GPU's own network output at 1e-12.
"""
import numpy as np
import pytest

from oracle import dnnmg, fem, gru, mesh, solver
from synthetic import channel_obstacle, gru_weights, random_state, rectangle

pytestmark = pytest.mark.gpu

DT = 0.01


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def bf16(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_gru_forward(flat, X, dims, h):
    """numpy model of the GPU arithmetic: BF16 operands, wide accumulation,
    FP32-like gates, BF16 copy of h for the next GEMM."""
    n_in, H, layers, n_out = dims
    Ws, wout = gru.unpack(flat, *dims)
    inp = bf16(X)
    h = h.copy()
    for l, (wih, whh) in enumerate(Ws):
        gi = inp @ bf16(wih).T
        gh = bf16(h[l]) @ bf16(whh).T
        r = 1 / (1 + np.exp(-(gi[:, :H] + gh[:, :H])))
        z = 1 / (1 + np.exp(-(gi[:, H:2 * H] + gh[:, H:2 * H])))
        n = np.tanh(gi[:, 2 * H:] + r * gh[:, 2 * H:])
        h[l] = (1 - z) * n + z * h[l]
        inp = bf16(h[l])
    return inp @ bf16(wout).T, h


@pytest.fixture(scope="module")
def setup():
    import paper_2106_07687_amd as P
    macro = channel_obstacle(0)
    lev = mesh.hierarchy(macro, 3)
    ctx = P.Context(precision=0, nu=macro.nu, newton_tol=1e-13)
    ctx.setup_mesh(macro, 3)
    prob = fem.Problem(nu=macro.nu, dt=DT)
    print(f"[dnnmg] seed 0, L=1, m=2, F=3, patches={lev[0].n_cells}", flush=True)
    return P, macro, lev, ctx, prob


def test_gru_forward_matches_bf16_model_and_oracle(setup):
    P, macro, lev, ctx, prob = setup
    net = P.Net(ctx, 1, 2, hidden=64, layers=2)
    dims = (net.n_in, 64, 2, net.n_out)
    assert (net.n_in, net.n_out, net.n_patches) == (490, 162, lev[0].n_cells)
    assert net.n_params == gru.n_params(490, 64, 2, 162)
    w = gru_weights(*dims, seed=7).astype(np.float32).astype(np.float64)
    net.set_weights(w)
    np.testing.assert_array_equal(net.get_weights(), w.astype(np.float32))
    rng = np.random.default_rng(1)
    h_model = np.zeros((2, net.n_patches, 64))
    h_ref = np.zeros_like(h_model)
    for step in range(3):                  # hidden state carried across calls
        X = rng.standard_normal((net.n_patches, net.n_in)).astype(np.float32)
        Y = net.forward(X)
        Ym, h_model = bf16_gru_forward(w, X.astype(np.float64), dims, h_model)
        Yr, h_ref = gru.forward(w, X.astype(np.float64)[None], dims, h0=h_ref)
        Yr = Yr[0]
        e_model, e_ref = rel(Y, Ym), rel(Y, Yr)
        cos = float(np.sum(Y * Yr) / (np.linalg.norm(Y) * np.linalg.norm(Yr)))
        print(f"[gru] step {step}: vs bf16 model {e_model:.2e}, vs fp64 oracle {e_ref:.2e}, cos {cos:.6f}")
        assert e_model < 1e-2 and e_ref < 3e-2 and cos > 0.999
    net.close()


def _net_spec(w, hidden, layers, mu, sg, osc):
    return dnnmg.NetSpec(weights=w, hidden=hidden, layers=layers, mu=mu, sigma=sg, out_scale=osc)


# (mu, sigma) per patch kind: nodal channels, then features
_STATS = {
    "block": ([0.3, 0.0, 0.1, 0.0, 0.0, 0.0, 1.5, 0.3, 1.0, 5.0],
              [0.5, 0.3, 0.4, 1.0, 1.0, 2.0, 1.0, 0.3, 0.5, 10.0]),
    "cell": ([0.3, 0.0, 0.0, 0.0, 0.0, 1.5, 0.3, 1.0, 5.0, 0.1, -0.2],
             [0.5, 0.3, 1.0, 1.0, 2.0, 1.0, 0.3, 0.5, 10.0, 0.7, 0.9]),
}


@pytest.mark.parametrize("L,m,patch", [(1, 2, "block"), (2, 1, "cell"), (1, 2, "cell")])
def test_correct_matches_oracle(setup, L, m, patch):
    P, macro, lev, ctx, prob = setup
    kind = dnnmg.PATCH_BLOCK if patch == "block" else dnnmg.PATCH_CELL
    D = dnnmg.DnnmgOracle(lev, prob, L, m, kind)
    net = P.Net(ctx, L, m, hidden=32, layers=2, patch=patch)
    assert (net.n_in, net.n_out, net.n_patches, net.n_stats) == (D.n_in, D.n_out, D.n_patches, D.n_stats)
    print(f"[correct] {patch} patches L={L} m={m}: I={net.n_in} O={net.n_out} B={net.n_patches}",
          flush=True)
    dims = (net.n_in, 32, 2, net.n_out)
    w = gru_weights(*dims, seed=3, scale=0.5).astype(np.float32).astype(np.float64)
    mu = np.array(_STATS[patch][0], dtype=np.float32)
    sg = np.array(_STATS[patch][1], dtype=np.float32)
    osc = np.array([1e-3, 5e-4], dtype=np.float32)
    net.set_weights(w, mu, sg, osc)
    spec = _net_spec(w, 32, 2, mu.astype(np.float64), sg.astype(np.float64), osc.astype(np.float64))
    st = ctx.state(L)
    xL = random_state(lev[L].n_nodes, 4) * 0.5
    xL0 = random_state(lev[L].n_nodes, 5) * 0.5
    st.set(xL0, 0.0)
    net.reset(st)
    st.set(xL, 0.3)
    out = net.correct(st, DT, debug=True)
    vprev = D.prolong(xL0)
    h0 = np.zeros((2, D.n_patches, 32))
    bL, vc, h1, ex = D.correct(xL, vprev, h0, spec, 0.3)
    # inputs (FP32 on the GPU)
    assert rel(out["inputs"], ex["Xn"]) < 1e-6, rel(out["inputs"], ex["Xn"])
    # network output
    e_out = rel(out["outputs"], ex["Y"])
    print(f"[correct] network output vs fp64 oracle: {e_out:.2e}")
    assert e_out < 3e-2
    # downstream of the network, fed the GPU output: FP64 parity
    d_ref = D.scatter(out["outputs"].astype(np.float64), spec)
    assert rel(out["correction"], d_ref) < 1e-12
    vc_g = ex["xt"].reshape(-1, 3).copy()
    vc_g[:, :2] += d_ref
    vc_g[:, 2] = 0.0
    bL_ref = D.restrict(D.rhs(vc_g.reshape(-1))).reshape(-1, 3)
    bL_g = out["rhs_coarse"].reshape(-1, 3)
    free = ~lev[L].dirichlet_nodes()
    assert rel(bL_g[free], bL_ref[free]) < 1e-12
    np.testing.assert_array_equal(bL_g[:, 2], 0.0)
    st.close()
    net.close()


def test_cell_patch_networks_have_table1_sizes(setup):
    """The six shapes of Table 1 on cell patches at m = 1 (I = 51, O = 18)."""
    import os
    P, macro, lev, ctx, prob = setup
    gold = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "table1_params.txt"),
                      dtype=np.int64)
    for hidden, layers, count in gold:
        net = P.Net(ctx, 2, 1, hidden=int(hidden), layers=int(layers), patch="cell")
        assert (net.n_in, net.n_out, net.n_params) == (51, 18, count)
        net.close()


def test_zero_network_dnnmg_equals_plain_on_parallelograms():
    """With W = 0 the correction is d = 0; on an all-parallelogram mesh the
    restricted fine right-hand side equals the coarse one, so DNN-MG steps
    reproduce plain coarse steps (GPU against GPU and against the oracle)."""
    import paper_2106_07687_amd as P
    mac = rectangle(4, 2, 1.6, 0.41, nu=0.01)
    mac.xy = mac.xy.copy()
    mac.xy[:, 0] += 0.35 * mac.xy[:, 1]
    lev = mesh.hierarchy(mac, 3)
    prob = fem.Problem(nu=0.01, dt=0.02)
    ctx = P.Context(precision=0, nu=0.01, newton_tol=1e-13)
    ctx.setup_mesh(mac, 3)
    L = 1
    net = P.Net(ctx, L, 2, hidden=32, layers=2)
    a, b = ctx.state(L), ctx.state(L)
    net.reset(a)
    x_ref = np.zeros(3 * lev[L].n_nodes)
    for n in range(1, 4):
        ia = ctx.step(a, 0.02)
        net.correct(a, 0.02)
        ctx.step(b, 0.02)
        xa, _ = a.get()
        xb, _ = b.get()
        x_ref = solver.newton_step(lev[L], prob, x_ref, n * 0.02, tol=1e-14)
        assert rel(xa, xb) < 1e-10, (n, rel(xa, xb), ia)
        assert rel(xa, x_ref) < 1e-10, (n, rel(xa, x_ref))
    for s in (a, b):
        s.close()
    net.close()


def test_dnnmg_trajectory_matches_oracle(setup):
    """Three DNN-MG steps (Newton on level 1 with the corrected rhs, network on
    level 3) with a small random network: the coarse solution tracks the
    oracle's within the BF16 network tolerance."""
    P, macro, lev, ctx, prob = setup
    L, m = 1, 2
    D = dnnmg.DnnmgOracle(lev, prob, L, m)
    net = P.Net(ctx, L, m, hidden=32, layers=2)
    dims = (net.n_in, 32, 2, net.n_out)
    w = gru_weights(*dims, seed=11, scale=0.5).astype(np.float32).astype(np.float64)
    mu = np.zeros(10, dtype=np.float32)
    sg = np.array([1, 1, 1, 10, 10, 10, 1, 1, 1, 100], dtype=np.float32)
    osc = np.array([2e-3, 2e-3], dtype=np.float32)
    net.set_weights(w, mu, sg, osc)
    spec = _net_spec(w, 32, 2, mu.astype(np.float64), sg.astype(np.float64), osc.astype(np.float64))
    st = ctx.state(L)
    net.reset(st)
    x = np.zeros(3 * lev[L].n_nodes)
    vprev = D.prolong(x)
    h = np.zeros((2, D.n_patches, 32))
    bL = None
    for n in range(1, 4):
        t = n * DT
        info = ctx.step(st, DT)
        net.correct(st, DT)
        x = dnnmg.dnnmg_newton(lev, prob, L, x, bL, t, tol=1e-14)
        bL, vprev, h, _ = D.correct(x, vprev, h, spec, t)
        xg, _ = st.get()
        e = rel(xg, x)
        print(f"[dnnmg] step {n}: rel L2 vs oracle {e:.2e} ({info})")
        assert info["converged"] == 1 and info["fallback"] == 0
        assert e < 1e-3
    st.close()
    net.close()


@pytest.mark.parametrize("L,m,patch,hidden,layers,T,B", [(1, 2, "block", 64, 2, 16, 64), (1, 2, "block", 128, 2, 32, 64),
                                                          (1, 2, "block", 256, 2, 16, 64), (2, 1, "cell", 32, 3, 16, 64),
                                                          (2, 1, "cell", 64, 1, 16, 64),
                                                          (1, 2, "block", 128, 2, 8, 2048)])
def test_bptt_gradient_matches_oracle(setup, L, m, patch, hidden, layers, T, B):
    """Hand-written BPTT (BF16 MFMA GEMMs, FP32 gates, checkpoints every 8
    steps) against the FP64 oracle gradient: relative L2 <= 3e-2 and cosine
    >= 0.999 (BF16 bar); the loss to 1e-2.  Shapes: the block-patch nets of
    the training workload (H = 64, 128 at its 32-step sequences, 256) and two
    of Table 1's cell-patch nets (I = 51, O = 18) on 64 sequences; H = 128 on
    2,048 sequences, whose input projections (8 x 2,048 rows, 384 gate
    columns) take the 128 x 128 tile GEMM (the 64 x 64 one with checkpoints
    every 4 steps)."""
    P, macro, lev, ctx, prob = setup
    net = P.Net(ctx, L, m, hidden=hidden, layers=layers, patch=patch)
    dims = (net.n_in, hidden, layers, net.n_out)
    print(f"[bptt] {patch} I={net.n_in} H={hidden} layers={layers} O={net.n_out}", flush=True)
    w = gru_weights(*dims, seed=21).astype(np.float32).astype(np.float64)
    net.set_weights(w)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((T, B, net.n_in)).astype(np.float32)
    Dt = (0.3 * rng.standard_normal((T, B, net.n_out))).astype(np.float32)
    loss_g, g_gpu = net.gradient(X, Dt, ckpt=8)
    loss_r, g_ref = gru.loss_and_grad_checkpointed(w, X.astype(np.float64), Dt.astype(np.float64), dims, seg=8)
    e = rel(g_gpu, g_ref)
    cos = float(np.dot(g_gpu, g_ref) / (np.linalg.norm(g_gpu) * np.linalg.norm(g_ref)))
    print(f"[bptt] loss gpu {loss_g:.6f} oracle {loss_r:.6f}; grad rel L2 {e:.2e}, cos {cos:.6f}")
    assert abs(loss_g - loss_r) <= 1e-2 * loss_r
    assert e < 3e-2 and cos > 0.999
    # checkpoint length does not change the gradient beyond rounding
    _, g4 = net.gradient(X, Dt, ckpt=4)
    assert rel(g4, g_gpu) < 1e-6
    net.close()


def test_adam_first_step_and_training_reduces_loss(setup):
    """First Adam step equals -lr g / (|g| + eps) with the GPU's own gradient
    (FP32 masters); repeated steps on a learnable target reduce the loss."""
    P, macro, lev, ctx, prob = setup
    net = P.Net(ctx, 1, 2, hidden=32, layers=2)
    dims = (net.n_in, 32, 2, net.n_out)
    w0 = gru_weights(*dims, seed=2).astype(np.float32)
    net.set_weights(w0)
    rng = np.random.default_rng(6)
    T, B = 8, 128
    X = rng.standard_normal((T, B, net.n_in)).astype(np.float32)
    Dt = np.full((T, B, net.n_out), 0.5, dtype=np.float32)
    _, g = net.gradient(X, Dt, ckpt=4)
    lr = 1e-3
    net.train_step(X, Dt, lr=lr, ckpt=4)
    w1 = net.get_weights()
    expect = w0 - lr * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(w1, expect, rtol=1e-5, atol=2e-7)
    losses = [net.train_step(X, Dt, lr=3e-3, ckpt=4) for _ in range(80)]
    print(f"[adam] loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.2 * losses[0]
    net.close()


def test_switch_off_redoes_slow_steps_with_the_plain_rhs(setup):
    """Sec. 3.3 switch-off: with switch_off_newton = 1 a step whose Newton
    iteration on the network's right-hand side needs more than one iteration
    is redone with the plain right-hand side (fallback = 1), and lands on the
    plain step's x_n; with 0 the same step keeps the network's right-hand side."""
    P, macro, lev, ctx, prob = setup
    L, m = 1, 2
    net = P.Net(ctx, L, m, hidden=32, layers=2)
    w = gru_weights(net.n_in, 32, 2, net.n_out, seed=5, scale=0.5)
    net.set_weights(w, out_scale=np.array([1e-2, 1e-2], dtype=np.float32))
    results = {}
    for off in (0, 1, None):
        ctx.set_params(switch_off_newton=off or 0)
        st = ctx.state(L)
        net.reset(st)
        for _ in range(2):
            ctx.step(st, DT)
        if off is not None:
            net.correct(st, DT)                  # a pending network right-hand side
        stats = ctx.step(st, DT)
        results[off] = (stats, st.get()[0])
        st.close()
    ctx.set_params(switch_off_newton=0)
    print(f"[switch-off] newton with network rhs {results[0][0]['newton_iters']}, "
          f"fallback {results[0][0]['fallback']} / {results[1][0]['fallback']}", flush=True)
    assert results[0][0]["newton_iters"] >= 2 and results[0][0]["fallback"] == 0
    assert results[1][0]["fallback"] == 1 and results[None][0]["fallback"] == 0
    assert rel(results[1][1], results[None][1]) < 1e-10
    assert rel(results[0][1], results[None][1]) > 1e-8     # the network's step differs
    net.close()


@pytest.mark.parametrize("L,m,patch", [(1, 2, "block"), (2, 1, "cell")])
def test_training_targets_and_teacher_forced_rhs_match_oracle(setup, L, m, patch):
    """Training data of Sec. 3.1 (eq. loss), through the C-ABI: the targets
    d* = v_F - P^m x^L at every patch node in the network's output layout,
    divided by the output scales (dnnmg_net_targets, FP32 output), and the
    teacher-forced right-hand side b^L = (P^m)^T Rhs(v_F)
    (dnnmg_rhs_from_fine), checked through the coarse Newton step it drives
    against the oracle's direct Newton with that right-hand side (FP64)."""
    P, macro, lev, ctx, prob = setup
    kind = dnnmg.PATCH_BLOCK if patch == "block" else dnnmg.PATCH_CELL
    D = dnnmg.DnnmgOracle(lev, prob, L, m, kind)
    net = P.Net(ctx, L, m, hidden=32, layers=1, patch=patch)
    osc = np.array([2e-3, 5e-4], dtype=np.float32)
    net.set_weights(out_scale=osc)
    print(f"[targets] {patch} L={L} m={m} patches={net.n_patches}", flush=True)
    st = ctx.state(L)
    xL = random_state(lev[L].n_nodes, 14) * 0.2
    t0 = 0.2
    st.set(xL, t0)
    vF = random_state(lev[D.F].n_nodes, 15) * 0.2
    Dg = net.targets(st, vF)
    xt = D.prolong(xL).reshape(-1, 3)
    vf3 = vF.reshape(-1, 3)
    Dref = np.concatenate([(vf3[D.grid, f] - xt[D.grid, f]) / float(osc[f]) for f in range(2)], axis=1)
    assert Dg.shape == Dref.shape
    assert rel(Dg, Dref) < 1e-6, rel(Dg, Dref)
    # teacher forcing as in training-data generation: the coarse state is the
    # fine solution at t_{n-1} injected to level L, its right-hand side is
    # restricted from that fine velocity
    sf = ctx.state(D.F)
    for _ in range(5):
        ctx.step(sf, DT)
    xf, tf = sf.get()
    sf.close()
    xL = xf[:3 * lev[L].n_nodes].copy()
    st.set(xL, tf)
    net.rhs_from_fine(st, xf, DT)
    info = ctx.step(st, DT)
    bL = D.restrict(D.rhs(xf))
    x_ref = dnnmg.dnnmg_newton(lev, prob, L, xL, bL, tf + DT, tol=1e-14)
    e = rel(st.get()[0], x_ref)
    print(f"[targets] teacher-forced step vs oracle {e:.2e} ({info})", flush=True)
    assert e < 1e-10
    st.close()
    net.close()
