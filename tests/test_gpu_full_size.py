"""Full-size checks of the plain method (GPU) at the size of the at-scale
workload: seeded channel with one obstacle, level 7 (1.38M nodes, 4.1M
DoFs), Re 100, dt 0.005, in the launch configuration the benchmark times
(autotuned launches, graphs, Jacobian reuse, Newton predictor).

* Mixed precision against the GPU's FP64 mode, step by step from rest:
  relative L2 per field <= 1e-5 (the mixed-precision bar).
* The oracle's own FP64 residual (eqs. varform, varformv; code that shares
  nothing with the GPU path) of the mixed-precision state: its l2 norm stays
  within 1e-11, i.e. the GPU state solves the oracle's discrete system at full
  size (Newton stops at 1e-13 on the GPU's residual; the rest is rounding).
* The same on level 5, the mesh on which the oracle solves in the at-scale
  comparison.
"""
import numpy as np
import pytest

from oracle import fem, mesh
from synthetic import channel_obstacle

pytestmark = pytest.mark.gpu

DT = 0.005
STEPS = 4


def _fields(a, b):
    a, b = a.reshape(-1, 3), b.reshape(-1, 3)
    return max(np.linalg.norm(a[:, f] - b[:, f]) / max(np.linalg.norm(b[:, f]), 1e-300) for f in range(3))


@pytest.mark.parametrize("level", [5, 7])
def test_mixed_precision_at_full_size(level):
    import paper_2106_07687_amd as P
    macro = channel_obstacle(0)
    # Newton to 1e-13: during the first steps of the inflow ramp the solution
    # is O(1e-4), and on 4.1M DoFs an absolute tolerance of 1e-10 leaves about
    # 1e-4 of relative freedom to either mode; the comparison is of the
    # precision modes, not of two points inside the tolerance ball
    common = dict(nu=macro.nu, autotune=1, use_graphs=1, jacobian_reuse=1, newton_predictor=1, newton_tol=1e-13)
    c32 = P.Context(precision=1, **common)
    c64 = P.Context(precision=0, **common)
    for c in (c32, c64):
        c.setup_mesh(macro, level)
    s32, s64 = c32.state(level), c64.state(level)
    print(f"[full] level {level}: {c32.level_info(level)[0]} nodes", flush=True)
    for k in range(STEPS):
        r32, r64 = c32.step(s32, DT), c64.step(s64, DT)
        assert r32["converged"] == 1 and r64["converged"] == 1
        err = _fields(s32.get()[0], s64.get()[0])
        print(f"[full] level {level} step {k}: mixed vs fp64 {err:.2e}, newton {r32['newton_iters']}/"
              f"{r64['newton_iters']}, builds {r32['jacobian_builds']}/{r64['jacobian_builds']}", flush=True)
        assert err <= 1e-5, (k, err)
    x, t = s32.get()
    L = mesh.hierarchy(macro, level)[level]
    assert L.n_nodes * 3 == x.size
    s32.close()
    s64.close()
    # one more step from a saved state, so that x_old is known exactly
    st = c32.state(level)
    st.set(x, t)
    c32.step(st, DT)
    x_new, t_new = st.get()
    prob = fem.Problem(nu=macro.nu, dt=DT)
    R = fem.residual(L, prob, x_new, x, t_new)
    nr = float(np.linalg.norm(R))
    print(f"[full] level {level}: oracle residual of the mixed-precision step {nr:.2e}", flush=True)
    assert nr <= 1e-11, nr
    st.close()
    c32.close()
    c64.close()
