"""ctypes binding of include/dnnmg.h (argument marshalling only).

Every numerical step runs in the HIP kernels of libdnnmg.so; this module only
converts numpy arrays / torch device pointers to C arguments and status codes
to exceptions.  If the library has not been built the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdnnmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dnnmg.h")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ESTATE = 0, -1, -2, -3, -4, -5
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOCONV: "ENOCONV",
          ESTATE: "ESTATE"}


class DnnmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("nu", C.c_double), ("alpha0", C.c_double), ("theta", C.c_double),
                ("u_mean", C.c_double), ("channel_h", C.c_double),
                ("newton_tol", C.c_double), ("newton_max", C.c_int),
                ("gmres_rtol", C.c_double), ("gmres_restart", C.c_int), ("gmres_max", C.c_int),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("vanka_omega", C.c_double),
                ("precision", C.c_int), ("use_graphs", C.c_int), ("autotune", C.c_int),
                ("newton_predictor", C.c_int), ("jacobian_reuse", C.c_int),
                ("reuse_contraction", C.c_double), ("switch_off_newton", C.c_int),
                ("nu_coarse", C.c_int), ("smoother", C.c_int), ("coarse_level", C.c_int),
                ("stream", C.c_void_p), ("delta0", C.c_double)]


class CoarseMesh(C.Structure):
    _fields_ = [("n_vert", C.c_int), ("xy", C.POINTER(C.c_double)),
                ("n_cell", C.c_int), ("quad", C.POINTER(C.c_int)),
                ("n_bedge", C.c_int), ("bedge", C.POINTER(C.c_int)),
                ("n_curve", C.c_int), ("curve", C.POINTER(C.c_double))]


class SimDesc(C.Structure):
    _fields_ = [("mesh", C.POINTER(CoarseMesh)), ("nu", C.c_double), ("depth", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("newton_iters", C.c_int), ("gmres_iters", C.c_int),
                ("gmres_iters_max", C.c_int), ("res_initial", C.c_double),
                ("res_final", C.c_double), ("converged", C.c_int), ("fallback", C.c_int),
                ("jacobian_builds", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("res0", C.c_double), ("res", C.c_double)]


_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int)
_FP = C.POINTER(C.c_float)


class CorrectOut(C.Structure):
    _fields_ = [("inputs", _FP), ("outputs", _FP), ("correction", _DP), ("rhs_coarse", _DP)]
_SIGS = {
    "dnnmg_params_default": (C.c_int, [C.POINTER(Params)]),
    "dnnmg_create": (C.c_int, [C.POINTER(Params), C.POINTER(_P)]),
    "dnnmg_destroy": (C.c_int, [_P]),
    "dnnmg_last_error": (C.c_char_p, [_P]),
    "dnnmg_set_params": (C.c_int, [_P, C.POINTER(Params)]),
    "dnnmg_setup_mesh": (C.c_int, [_P, C.POINTER(CoarseMesh), C.c_int]),
    "dnnmg_level_info": (C.c_int, [_P, C.c_int, _IP, _IP, _IP]),
    "dnnmg_level_coords": (C.c_int, [_P, C.c_int, _DP]),
    "dnnmg_level_cells": (C.c_int, [_P, C.c_int, _IP]),
    "dnnmg_state_create": (C.c_int, [_P, C.c_int, C.POINTER(_P)]),
    "dnnmg_state_destroy": (C.c_int, [_P]),
    "dnnmg_state_set": (C.c_int, [_P, _DP, C.c_double]),
    "dnnmg_state_get": (C.c_int, [_P, _DP, _DP]),
    "dnnmg_state_device_ptr": (C.c_int, [_P, C.POINTER(_P)]),
    "dnnmg_state_get_dev": (C.c_int, [_P, _P]),
    "dnnmg_step": (C.c_int, [_P, _P, C.c_double, C.POINTER(StepStats)]),
    "dnnmg_linearize": (C.c_int, [_P, _P, C.c_int, C.c_double]),
    "dnnmg_solve": (C.c_int, [_P, C.c_int, _DP, _DP, C.POINTER(SolveStats)]),
    "dnnmg_residual": (C.c_int, [_P, C.c_int, _DP, _DP, C.c_double, C.c_double, _DP]),
    "dnnmg_jacobian_apply": (C.c_int, [_P, C.c_int, _DP, _DP]),
    "dnnmg_vanka_sweep": (C.c_int, [_P, C.c_int, _DP, _DP, _DP]),
    "dnnmg_vcycle": (C.c_int, [_P, C.c_int, _DP, _DP]),
    "dnnmg_prolong": (C.c_int, [_P, C.c_int, _DP, _DP]),
    "dnnmg_restrict": (C.c_int, [_P, C.c_int, _DP, _DP]),
    "dnnmg_net_create": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(_P)]),
    "dnnmg_net_create_patch": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.POINTER(_P)]),
    "dnnmg_net_patch_info": (C.c_int, [_P, _IP, _IP, _IP]),
    "dnnmg_net_destroy": (C.c_int, [_P]),
    "dnnmg_oscillation": (C.c_int, [_DP, C.c_int, C.c_double, C.c_double, _DP, _DP, _IP]),
    "dnnmg_net_info": (C.c_int, [_P, _IP, _IP, _IP, C.POINTER(C.c_longlong)]),
    "dnnmg_net_set_weights": (C.c_int, [_P, _FP, _FP, _FP, _FP]),
    "dnnmg_net_get_weights": (C.c_int, [_P, _FP]),
    "dnnmg_net_reset": (C.c_int, [_P, _P]),
    "dnnmg_net_forward": (C.c_int, [_P, _FP, _FP]),
    "dnnmg_correct": (C.c_int, [_P, _P, _P, C.c_double, C.POINTER(CorrectOut)]),
    "dnnmg_rhs_from_fine": (C.c_int, [_P, _P, _P, _DP, C.c_double]),
    "dnnmg_net_targets": (C.c_int, [_P, _P, _P, _DP, _FP]),
    "dnnmg_net_gradient": (C.c_int, [_P, _FP, _FP, C.c_int, C.c_int, C.c_int, _FP, _FP]),
    "dnnmg_train_step": (C.c_int, [_P, _FP, _FP, C.c_int, C.c_int, C.c_int, C.c_float, _FP]),
    "dnnmg_train_step_dev": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_int, C.c_float, _FP]),
    "dnnmg_profile_enable": (C.c_int, [_P, C.c_int]),
    "dnnmg_profile_select": (C.c_int, [_P, C.c_char_p]),
    "dnnmg_launch_config": (C.c_int, [_P, C.c_int, _IP]),
    "dnnmg_functionals": (C.c_int, [_P, _P, _DP, _DP, _DP, C.c_int]),
    "dnnmg_functionals_host": (C.c_int, [_P, C.c_int, _DP, _DP, _DP, _DP, C.c_int]),
    "dnnmg_velocity_error": (C.c_int, [_P, C.c_int, _P, C.c_int, _P, _DP]),
    "dnnmg_net_fine_velocity": (C.c_int, [_P, C.POINTER(_P)]),
    "dnnmg_velocity_error_noalloc": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "dnnmg_profile_report": (C.c_int, [_P, C.c_char_p, C.c_size_t]),
    "dnnmg_level_stats": (C.c_int, [_P, C.c_int, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong),
                                    C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]),
    "dnnmg_batch_create": (C.c_int, [C.POINTER(Params), C.POINTER(SimDesc), C.c_int, C.POINTER(_P)]),
    "dnnmg_batch_destroy": (C.c_int, [_P]),
    "dnnmg_batch_last_error": (C.c_char_p, [_P]),
    "dnnmg_batch_groups": (C.c_int, [_P, _IP]),
    "dnnmg_batch_group_info": (C.c_int, [_P, C.c_int, _IP, _IP, _IP]),
    "dnnmg_batch_info": (C.c_int, [_P, C.c_int, _IP, _IP]),
    "dnnmg_batch_set": (C.c_int, [_P, C.c_int, _DP, C.c_double]),
    "dnnmg_batch_get": (C.c_int, [_P, C.c_int, _DP, C.POINTER(C.c_double)]),
    "dnnmg_batch_step": (C.c_int, [_P, C.c_double, C.POINTER(StepStats)]),
}

_lib = None


def load():
    """Loads libdnnmg.so and declares the signatures (no device work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                           "`python -m paper_2106_07687_amd.build` first")
    # One HIP runtime per process: torch ships its own copy of the runtime.
    # Loaded first, it satisfies the library's libamdhip64.so.7 dependency;
    # loaded after the library, it would add a second runtime, which then
    # may not see the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_symbols():
    """Names of all functions declared in include/dnnmg.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(dnnmg_[a-z_0-9]+)\s*\(", txt)))


def _dp(a):
    return a.ctypes.data_as(_DP)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _coarse_mesh(macro):
    """CoarseMesh struct of a synthetic macro mesh, plus the arrays it points to."""
    xy = _f64(macro.xy).reshape(-1)
    q = np.ascontiguousarray(macro.quads, dtype=np.int32).reshape(-1)
    be = np.ascontiguousarray(macro.bedges, dtype=np.int32).reshape(-1)
    cv = _f64(macro.curves).reshape(-1)
    if cv.size == 0:
        cv = np.zeros(5)
    m = CoarseMesh(macro.n_vert, _dp(xy), macro.n_cell, q.ctypes.data_as(_IP),
                   be.size // 3, be.ctypes.data_as(_IP), macro.curves.shape[0], _dp(cv))
    return m, (xy, q, be, cv)


def _params(precision, kw):
    lib = load()
    p = Params()
    lib.dnnmg_params_default(C.byref(p))
    p.precision = precision
    _set_fields(p, kw)
    return p


def _set_fields(p, kw):
    names = {k for k, _ in p._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solver parameter {k!r}")
        setattr(p, k, v)


def oscillation(f, t0, dt):
    """(time of the first maximum, mean period, number of maxima) of the
    sampled functional f[i] = J(t0 + i dt) (dnnmg_oscillation)."""
    lib = load()
    f = _f64(f)
    a, b, n = C.c_double(), C.c_double(), C.c_int()
    rc = lib.dnnmg_oscillation(_dp(f), f.size, t0, dt, C.byref(a), C.byref(b), C.byref(n))
    if rc != OK:
        raise DnnmgError(rc, "dnnmg_oscillation: invalid series")
    return a.value, b.value, n.value


class Context:
    """Owner of one dnnmg_ctx (the calls are the C calls of the same names)."""

    def __init__(self, precision=1, stream=None, **kw):
        self.lib = load()
        p = Params()
        self.lib.dnnmg_params_default(C.byref(p))
        p.precision = precision
        _set_fields(p, kw)
        if stream is not None:
            p.stream = stream
        self.params = p
        h = _P()
        self._check(self.lib.dnnmg_create(C.byref(p), C.byref(h)), ctx=None)
        self.h = h
        self.finest = -1

    def _check(self, rc, ctx="self"):
        if rc != OK:
            msg = self.lib.dnnmg_last_error(self.h if ctx == "self" else None)
            raise DnnmgError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.dnnmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw):
        p = Params()
        C.pointer(p)[0] = self.params          # copy: kept only if the library accepts it
        _set_fields(p, kw)
        self._check(self.lib.dnnmg_set_params(self.h, C.byref(p)))
        self.params = p

    def setup_mesh(self, macro, finest_level):
        m, keep = _coarse_mesh(macro)
        self._check(self.lib.dnnmg_setup_mesh(self.h, C.byref(m), finest_level))
        self.finest = finest_level

    def level_info(self, level):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        self._check(self.lib.dnnmg_level_info(self.h, level, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def level_coords(self, level):
        n = self.level_info(level)[0]
        out = np.empty(2 * n)
        self._check(self.lib.dnnmg_level_coords(self.h, level, _dp(out)))
        return out.reshape(n, 2)

    def level_cells(self, level):
        c = self.level_info(level)[1]
        out = np.empty(4 * c, dtype=np.int32)
        self._check(self.lib.dnnmg_level_cells(self.h, level, out.ctypes.data_as(_IP)))
        return out.reshape(c, 4)

    def state(self, level):
        return State(self, level)

    def profile_enable(self, on=True):
        self._check(self.lib.dnnmg_profile_enable(self.h, 1 if on else 0))

    def profile_select(self, keys=None):
        """Time only the given "kernel@Llevel" keys (None: all)."""
        arg = None if not keys else ",".join(keys).encode()
        self._check(self.lib.dnnmg_profile_select(self.h, arg))

    def profile_report(self):
        """{key: (launches, total_ms)} of the profiled kernel launches."""
        buf = C.create_string_buffer(1 << 16)
        self._check(self.lib.dnnmg_profile_report(self.h, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            k, n, ms = line.split()
            out[k] = (int(n), float(ms))
        return out

    def functionals(self, level, uvp, n_obstacles):
        """(J_div, drag[k], lift[k]) of a host state vector on `level`."""
        uvp = _f64(uvp)
        j = np.zeros(1)
        d, l = np.zeros(max(n_obstacles, 1)), np.zeros(max(n_obstacles, 1))
        self._check(self.lib.dnnmg_functionals_host(self.h, level, _dp(uvp), _dp(j), _dp(d), _dp(l),
                                                    n_obstacles))
        return float(j[0]), d[:n_obstacles], l[:n_obstacles]

    def velocity_error(self, level, x_ptr, ref_level, ref_ptr):
        """Squared velocity norms {"l2_err2", "l2_ref2", "nodal_err2",
        "nodal_ref2"} of the device field at x_ptr on `level` (prolongated to
        ref_level) against the device field at ref_ptr (mass-weighted L2 and
        nodal sums)."""
        out = np.zeros(4)
        self._check(self.lib.dnnmg_velocity_error(self.h, level, x_ptr, ref_level, ref_ptr, _dp(out)))
        return dict(zip(("l2_err2", "l2_ref2", "nodal_err2", "nodal_ref2"), (float(v) for v in out)))

    def velocity_error_noalloc(self, level, x_ptr, ref_ptr, out_ptr):
        """dnnmg_velocity_error_noalloc: the four sums of velocity_error for
        device fields on `level`, written to the device pointer out_ptr
        (4 doubles), enqueued without synchronisation."""
        self._check(self.lib.dnnmg_velocity_error_noalloc(self.h, level, x_ptr, ref_ptr, out_ptr))

    def launch_config(self, level):
        """Workgroup sizes {spmv, vanka_apply, vanka_update, restrict, prolong,
        vanka_smooth, vcycle_small, restrict_residual, spmv4} (vanka_smooth 0:
        residual and apply run separately; vcycle_small 1024: the level runs
        inside the single-workgroup bottom cycle; restrict_residual 0: the
        residual is stored, then restricted; spmv4 0: one thread per SpMV
        row; smooth_lanes: lanes per cell of the fused kernel, 0 if not
        fused; update_prolong: the next coarser level's last update fused into
        the prolongation, 0 if separate; vanka_apply4: FP32 apply with four
        cells per thread, 0 if one; update_ordered: the Vanka update over the
        nodes in cell order, 0 if in node order)."""
        out = np.zeros(13, dtype=np.int32)
        self._check(self.lib.dnnmg_launch_config(self.h, level, out.ctypes.data_as(_IP)))
        return dict(zip(("spmv", "vanka_apply", "vanka_update", "restrict", "prolong", "vanka_smooth",
                         "vcycle_small", "restrict_residual", "spmv4", "smooth_lanes", "update_prolong",
                         "vanka_apply4", "update_ordered"),
                        out.tolist()))

    def level_stats(self, level):
        v = [C.c_longlong() for _ in range(4)]
        self._check(self.lib.dnnmg_level_stats(self.h, level, *[C.byref(x) for x in v]))
        return dict(zip(("q_blocks", "x_entries", "q_slots", "x_slots"), (x.value for x in v)))

    def step(self, state, dt):
        st = StepStats()
        rc = self.lib.dnnmg_step(self.h, state.h, dt, C.byref(st))
        self._check(rc)
        return st.as_dict()

    def linearize(self, state, level, dt):
        self._check(self.lib.dnnmg_linearize(self.h, state.h, level, dt))

    def _nodes(self, level):
        return self.level_info(level)[0]

    def solve(self, level, rhs):
        rhs = _f64(rhs)
        out = np.empty(3 * self._nodes(level))
        st = SolveStats()
        self._check(self.lib.dnnmg_solve(self.h, level, _dp(rhs), _dp(out), C.byref(st)))
        return out, dict(iters=st.iters, res0=st.res0, res=st.res)

    def residual(self, level, x, x_old, t_new, dt):
        x, xo = _f64(x), _f64(x_old)
        out = np.empty(3 * self._nodes(level))
        self._check(self.lib.dnnmg_residual(self.h, level, _dp(x), _dp(xo), t_new, dt, _dp(out)))
        return out

    def jacobian_apply(self, level, w):
        w = _f64(w)
        out = np.empty(3 * self._nodes(level))
        self._check(self.lib.dnnmg_jacobian_apply(self.h, level, _dp(w), _dp(out)))
        return out

    def vanka_sweep(self, level, x, b):
        x, b = _f64(x), _f64(b)
        out = np.empty(3 * self._nodes(level))
        self._check(self.lib.dnnmg_vanka_sweep(self.h, level, _dp(x), _dp(b), _dp(out)))
        return out

    def vcycle(self, level, b):
        b = _f64(b)
        out = np.empty(3 * self._nodes(level))
        self._check(self.lib.dnnmg_vcycle(self.h, level, _dp(b), _dp(out)))
        return out

    def prolong(self, level, coarse):
        coarse = _f64(coarse)
        out = np.empty(3 * self._nodes(level))
        self._check(self.lib.dnnmg_prolong(self.h, level, _dp(coarse), _dp(out)))
        return out

    def restrict(self, level, fine):
        fine = _f64(fine)
        out = np.empty(3 * self._nodes(level - 1))
        self._check(self.lib.dnnmg_restrict(self.h, level, _dp(fine), _dp(out)))
        return out


def _fp(a):
    return None if a is None else a.ctypes.data_as(_FP)


class Net:
    """Owner of one dnnmg_net (patch GRU network of one simulation)."""

    PATCH = {"block": 0, "cell": 1}

    def __init__(self, ctx: Context, coarse_level: int, m_levels: int, hidden: int, layers: int,
                 patch: str = "block"):
        self.ctx = ctx
        h = _P()
        ctx._check(ctx.lib.dnnmg_net_create_patch(ctx.h, coarse_level, m_levels, hidden, layers,
                                                  self.PATCH[patch], C.byref(h)))
        self.h = h
        a, b, c, d = C.c_int(), C.c_int(), C.c_int(), C.c_longlong()
        ctx._check(ctx.lib.dnnmg_net_info(h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        self.n_in, self.n_out, self.n_patches, self.n_params = a.value, b.value, c.value, d.value
        ctx._check(ctx.lib.dnnmg_net_patch_info(h, None, C.byref(a), C.byref(b)))
        self.patch, self.nodes_per_side, self.n_stats = patch, a.value, b.value
        self.hidden, self.layers = hidden, layers
        self.coarse_level, self.m_levels = coarse_level, m_levels

    def set_weights(self, w=None, mu=None, sigma=None, out_scale=None):
        cv = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
        w, mu, sigma, out_scale = cv(w), cv(mu), cv(sigma), cv(out_scale)
        if w is not None and w.size != self.n_params:
            raise ValueError(f"expected {self.n_params} weights, got {w.size}")
        self.ctx._check(self.ctx.lib.dnnmg_net_set_weights(self.h, _fp(w), _fp(mu), _fp(sigma),
                                                           _fp(out_scale)))

    def get_weights(self):
        w = np.empty(self.n_params, dtype=np.float32)
        self.ctx._check(self.ctx.lib.dnnmg_net_get_weights(self.h, _fp(w)))
        return w

    def reset(self, state):
        self.ctx._check(self.ctx.lib.dnnmg_net_reset(self.h, state.h))

    def forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.empty((self.n_patches, self.n_out), dtype=np.float32)
        self.ctx._check(self.ctx.lib.dnnmg_net_forward(self.h, _fp(X), _fp(Y)))
        return Y

    def fine_velocity_ptr(self):
        """Device address of the fine state the next correction starts from
        (the corrected velocity after correct())."""
        p = _P()
        self.ctx._check(self.ctx.lib.dnnmg_net_fine_velocity(self.h, C.byref(p)))
        return p.value

    def rhs_from_fine(self, state, v_fine, dt):
        v = _f64(v_fine)
        self.ctx._check(self.ctx.lib.dnnmg_rhs_from_fine(self.ctx.h, state.h, self.h, _dp(v), dt))

    def targets(self, state, v_fine):
        """Scaled correction targets (n_patches, n_out) for the coarse state."""
        v = _f64(v_fine)
        D = np.empty((self.n_patches, self.n_out), dtype=np.float32)
        self.ctx._check(self.ctx.lib.dnnmg_net_targets(self.ctx.h, state.h, self.h, _dp(v), _fp(D)))
        return D

    def gradient(self, X, D, ckpt=8):
        """X: (T, B, n_in), D: (T, B, n_out) host arrays -> (loss, grad)."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        D = np.ascontiguousarray(D, dtype=np.float32)
        T, B = X.shape[:2]
        g = np.empty(self.n_params, dtype=np.float32)
        loss = C.c_float()
        self.ctx._check(self.ctx.lib.dnnmg_net_gradient(self.h, _fp(X), _fp(D), T, B, ckpt, _fp(g),
                                                        C.byref(loss)))
        return loss.value, g

    def train_step(self, X, D, lr=1e-3, ckpt=8):
        X = np.ascontiguousarray(X, dtype=np.float32)
        D = np.ascontiguousarray(D, dtype=np.float32)
        T, B = X.shape[:2]
        loss = C.c_float()
        self.ctx._check(self.ctx.lib.dnnmg_train_step(self.h, _fp(X), _fp(D), T, B, ckpt, lr,
                                                      C.byref(loss)))
        return loss.value

    def train_step_dev(self, X_ptr, D_ptr, T, B, lr=1e-3, ckpt=8):
        """Device-pointer variant (e.g. torch tensors' data_ptr())."""
        loss = C.c_float()
        self.ctx._check(self.ctx.lib.dnnmg_train_step_dev(self.h, X_ptr, D_ptr, T, B, ckpt, lr,
                                                          C.byref(loss)))
        return loss.value

    def correct(self, state, dt, debug=False):
        if not debug:
            self.ctx._check(self.ctx.lib.dnnmg_correct(self.ctx.h, state.h, self.h, dt, None))
            return None
        nf = self.ctx._nodes(self.coarse_level + self.m_levels)
        nl = self.ctx._nodes(self.coarse_level)
        out = dict(inputs=np.empty((self.n_patches, self.n_in), dtype=np.float32),
                   outputs=np.empty((self.n_patches, self.n_out), dtype=np.float32),
                   correction=np.empty((nf, 2)), rhs_coarse=np.empty(3 * nl))
        d = CorrectOut(_fp(out["inputs"]), _fp(out["outputs"]), _dp(out["correction"]),
                       _dp(out["rhs_coarse"]))
        self.ctx._check(self.ctx.lib.dnnmg_correct(self.ctx.h, state.h, self.h, dt, C.byref(d)))
        return out

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.dnnmg_net_destroy(self.h)
        self.h = None


class State:
    def __init__(self, ctx: Context, level: int):
        self.ctx = ctx
        self.level = level
        h = _P()
        ctx._check(ctx.lib.dnnmg_state_create(ctx.h, level, C.byref(h)))
        self.h = h

    def set(self, uvp, t):
        uvp = _f64(uvp)
        self.ctx._check(self.ctx.lib.dnnmg_state_set(self.h, _dp(uvp), t))

    def get(self):
        n = self.ctx._nodes(self.level)
        out = np.empty(3 * n)
        t = C.c_double()
        self.ctx._check(self.ctx.lib.dnnmg_state_get(self.h, _dp(out), C.byref(t)))
        return out, t.value

    def functionals(self, n_obstacles):
        """(J_div, drag[k], lift[k]) of the state."""
        j = np.zeros(1)
        d, l = np.zeros(max(n_obstacles, 1)), np.zeros(max(n_obstacles, 1))
        self.ctx._check(self.ctx.lib.dnnmg_functionals(self.ctx.h, self.h, _dp(j), _dp(d), _dp(l),
                                                       n_obstacles))
        return float(j[0]), d[:n_obstacles], l[:n_obstacles]

    def get_dev(self, dst_ptr):
        """Device-to-device copy of the state vector to dst_ptr (e.g. a torch
        tensor's data_ptr()), ordered on the context's stream."""
        self.ctx._check(self.ctx.lib.dnnmg_state_get_dev(self.h, dst_ptr))

    def device_ptr(self):
        p = _P()
        self.ctx._check(self.ctx.lib.dnnmg_state_device_ptr(self.h, C.byref(p)))
        return p.value

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.dnnmg_state_destroy(self.h)
        self.h = None


class Batch:
    """Owner of one dnnmg_batch: `sims` is a list of (macro mesh, nu, depth)."""

    def __init__(self, sims, precision=1, **kw):
        self.lib = load()
        self.params = _params(precision, kw)
        keep, descs = [], (SimDesc * len(sims))()
        meshes = []
        for k, (macro, nu, depth) in enumerate(sims):
            m, arrs = _coarse_mesh(macro)
            meshes.append(m)
            keep.append(arrs)
            descs[k].mesh = C.pointer(meshes[-1])
            descs[k].nu = nu
            descs[k].depth = depth
        h = _P()
        rc = self.lib.dnnmg_batch_create(C.byref(self.params), descs, len(sims), C.byref(h))
        if rc != OK:
            raise DnnmgError(rc, "dnnmg_batch_create failed")
        self.h = h
        self.n_sims = len(sims)

    def _check(self, rc):
        if rc != OK:
            msg = self.lib.dnnmg_batch_last_error(self.h)
            raise DnnmgError(rc, msg.decode() if msg else "")

    def n_groups(self):
        n = C.c_int()
        self._check(self.lib.dnnmg_batch_groups(self.h, C.byref(n)))
        return n.value

    def group_info(self, g):
        d, n, nn = C.c_int(), C.c_int(), C.c_int()
        self._check(self.lib.dnnmg_batch_group_info(self.h, g, C.byref(d), C.byref(n), C.byref(nn)))
        return dict(depth=d.value, n_sims=n.value, n_nodes=nn.value)

    def info(self, sim):
        g, n = C.c_int(), C.c_int()
        self._check(self.lib.dnnmg_batch_info(self.h, sim, C.byref(g), C.byref(n)))
        return g.value, n.value

    def set(self, sim, uvp, t):
        uvp = _f64(uvp)
        self._check(self.lib.dnnmg_batch_set(self.h, sim, _dp(uvp), t))

    def get(self, sim):
        out = np.empty(3 * self.info(sim)[1])
        t = C.c_double()
        self._check(self.lib.dnnmg_batch_get(self.h, sim, _dp(out), C.byref(t)))
        return out, t.value

    def step(self, dt):
        """One time step of every simulation; per-group stats dicts."""
        st = (StepStats * self.n_groups())()
        self._check(self.lib.dnnmg_batch_step(self.h, dt, st))
        return [x.as_dict() for x in st]

    def close(self):
        if getattr(self, "h", None):
            self.lib.dnnmg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
