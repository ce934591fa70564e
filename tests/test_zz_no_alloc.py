"""The allocation-free entry point (GPU): dnnmg_velocity_error_noalloc, called
through the C-ABI, against the allocating dnnmg_velocity_error on the same
inputs, on two calls in a row (the second on a smaller level).  Same kernels
and launch shape on both sides, so the sums must be bitwise equal."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_velocity_error_matches_allocating_entry_point():
    import torch

    import paper_2106_07687_amd as P
    from synthetic import channel_obstacle, random_state
    macro = channel_obstacle(0)
    ctx = P.Context(precision=0, nu=macro.nu)
    ctx.setup_mesh(macro, 3)
    out = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
    keys = ("l2_err2", "l2_ref2", "nodal_err2", "nodal_ref2")
    for level, seed in ((3, 1), (2, 2)):          # second call: smaller input
        n = ctx.level_info(level)[0]
        print(f"[noalloc] level {level}, {n} nodes", flush=True)
        a, b = ctx.state(level), ctx.state(level)
        a.set(random_state(n, seed), 0.0)
        b.set(random_state(n, seed + 10), 0.0)
        ref = ctx.velocity_error(level, a.device_ptr(), level, b.device_ptr())
        torch.cuda.synchronize()
        ctx.velocity_error_noalloc(level, a.device_ptr(), b.device_ptr(), out.data_ptr())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, np.array([ref[k] for k in keys])), (level, got, ref)
        a.close()
        b.close()
    with pytest.raises(P.DnnmgError):
        ctx.velocity_error_noalloc(4, out.data_ptr(), out.data_ptr(), out.data_ptr())   # no level 4
    ctx.close()
