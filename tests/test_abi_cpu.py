"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/dnnmg.h, and rejects bad arguments before any device work."""
import ctypes as C

import numpy as np
import pytest

import paper_2106_07687_amd as P
from paper_2106_07687_amd import _lib
from synthetic import channel_obstacle


def test_library_exports_every_declared_symbol():
    lib = P.load()
    syms = P.header_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_defaults_and_invalid_params():
    lib = P.load()
    p = _lib.Params()
    assert lib.dnnmg_params_default(C.byref(p)) == 0
    assert (p.theta, p.alpha0, p.nu_pre, p.nu_post, p.gmres_restart) == (0.5, 0.5, 2, 2, 30)
    h = C.c_void_p()
    assert (p.jacobian_reuse, p.reuse_contraction, p.smoother, p.switch_off_newton) == (0, 0.1, 0, 0)
    assert p.coarse_level == 0
    for field, bad in (("nu", -1.0), ("theta", 0.0), ("gmres_restart", 65), ("precision", 2),
                       ("vanka_omega", 0.0), ("gmres_rtol", 1.5), ("jacobian_reuse", 2),
                       ("reuse_contraction", 0.0), ("reuse_contraction", 1.0), ("smoother", 2),
                       ("switch_off_newton", -1), ("autotune", 4), ("newton_predictor", 3),
                       ("coarse_level", -1), ("coarse_level", 3)):
        q = _lib.Params()
        lib.dnnmg_params_default(C.byref(q))
        setattr(q, field, bad)
        assert lib.dnnmg_create(C.byref(q), C.byref(h)) == _lib.EINVAL, field
    assert lib.dnnmg_create(None, C.byref(h)) == _lib.EINVAL
    ctx = P.Context(precision=1, coarse_level=1)   # fixed at creation
    with pytest.raises(P.DnnmgError) as e:
        ctx.set_params(coarse_level=2)
    assert e.value.code == _lib.EINVAL
    ctx.set_params(coarse_level=1, nu_pre=1)
    ctx.close()


def test_calls_out_of_order_and_bad_mesh_are_rejected_without_device_work():
    ctx = P.Context(precision=0)
    with pytest.raises(P.DnnmgError) as e:
        ctx.level_info(0)
    assert e.value.code == _lib.ESTATE
    m = channel_obstacle(0)
    with pytest.raises(P.DnnmgError) as e:
        ctx.setup_mesh(m, 12)            # finest level out of range
    assert e.value.code == _lib.EINVAL
    bad = channel_obstacle(0)
    bad.quads = bad.quads.copy()
    bad.quads[0, 0] = 10_000             # vertex id out of range
    with pytest.raises(P.DnnmgError) as e:
        ctx.setup_mesh(bad, 1)
    assert e.value.code == _lib.EINVAL
    assert "out of range" in str(e.value)
    bad2 = channel_obstacle(0)
    bad2.bedges = bad2.bedges.copy()
    bad2.bedges[0, 2] = 9                # obstacle tag without a curve
    with pytest.raises(P.DnnmgError):
        ctx.setup_mesh(bad2, 1)
    ctx.close()


def test_oscillation_entry_point_matches_oracle():
    """dnnmg_oscillation is host code: callable without a GPU."""
    from oracle import functionals as F
    rng = np.random.default_rng(11)
    t = 9.0 + 0.005 * np.arange(400)
    y = 0.2 + np.sin(2 * np.pi * 3.3 * t + 0.4) + 1e-3 * rng.standard_normal(t.size)
    got = P.oscillation(y, 9.0, 0.005)
    ref = F.oscillation(y, 9.0, 0.005)
    assert got[2] == ref[2] and got[2] >= 6
    assert abs(got[0] - ref[0]) < 1e-12 and abs(got[1] - ref[1]) < 1e-12
    flat = P.oscillation(np.zeros(10), 0.0, 0.1)
    assert flat[2] == 0 and np.isnan(flat[0]) and np.isnan(flat[1])
    for bad in (dict(f=np.zeros(2), dt=0.1), dict(f=np.zeros(5), dt=0.0),
                dict(f=np.array([0.0, np.nan, 1.0, 0.0]), dt=0.1)):
        with pytest.raises(P.DnnmgError):
            P.oscillation(bad["f"], 0.0, bad["dt"])


def test_unknown_parameter_names_are_rejected():
    """A misspelt solver parameter must not be silently ignored."""
    with pytest.raises(TypeError):
        P.Context(precision=1, jacobain_reuse=1)
