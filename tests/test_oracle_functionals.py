"""Pins of the oracle flow functionals (J_div, drag, lift).

* J_div of linear fields is exact: v = (x, y) gives 4 |Omega_h|, the
  divergence-free (x, -y) gives 0; for v = (x^2, 0) it converges to the exact
  integral of 4 x^2 over the channel minus the disc.
* Drag and lift of a linear pressure p = c0 + c1 x + c2 y (v = 0) are
  -c1 |O_h| and -c2 |O_h| (divergence theorem on the polygonal obstacle
  O_h, whose area is the channel's minus the mesh's): this fixes the sign
  convention (normal into the obstacle) and the pressure term.
* The viscous term of a smooth divergence-free field converges to
  nu * int_O Laplace(u) dA (divergence theorem on the exact disc, evaluated by
  polar quadrature).
"""
import numpy as np

from oracle import functionals as F
from oracle import mesh
from synthetic import channel_obstacle, channel_obstacles
from synthetic.channel import CHANNEL_H, CHANNEL_L


def _area(L):
    x, y = L.xy[L.cells, 0], L.xy[L.cells, 1]
    return 0.5 * np.sum(x * np.roll(y, -1, axis=1) - np.roll(x, -1, axis=1) * y)


def _state(L, u, v, p):
    x = np.zeros((L.n_nodes, 3))
    X, Y = L.xy[:, 0], L.xy[:, 1]
    x[:, 0], x[:, 1], x[:, 2] = u(X, Y), v(X, Y), p(X, Y)
    return x.reshape(-1)


def test_jdiv_exact_on_linear_fields():
    L = mesh.hierarchy(channel_obstacle(0), 2)[2]
    x = _state(L, lambda X, Y: X, lambda X, Y: Y, lambda X, Y: 0 * X)
    assert abs(F.j_div(L, x) - 4.0 * _area(L)) < 1e-12
    x = _state(L, lambda X, Y: X, lambda X, Y: -Y, lambda X, Y: 0 * X)
    assert F.j_div(L, x) < 1e-24


def test_jdiv_converges_for_quadratic_field():
    m = channel_obstacle(0)
    cx, cy, r = m.info["cx"], m.info["cy"], m.info["r"]
    exact = 4 * (CHANNEL_L ** 3 / 3 * CHANNEL_H) - 4 * (np.pi * r ** 2 * cx ** 2 + np.pi * r ** 4 / 4)
    lev = mesh.hierarchy(m, 4)
    errs = [abs(F.j_div(lev[l], _state(lev[l], lambda X, Y: X ** 2, lambda X, Y: 0 * X,
                                        lambda X, Y: 0 * X)) - exact) for l in (2, 3, 4)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[2] > 3.0, errs


def test_pressure_drag_lift_equal_obstacle_area_moments():
    for macro, lvl in ((channel_obstacle(1), 2), (channel_obstacles(100), 1)):
        L = mesh.hierarchy(macro, lvl)[lvl]
        k = len(macro.curves)
        hole = CHANNEL_L * CHANNEL_H - _area(L)
        c0, c1, c2 = 0.7, -1.3, 2.1
        x = _state(L, lambda X, Y: 0 * X, lambda X, Y: 0 * X, lambda X, Y: c0 + c1 * X + c2 * Y)
        d, lft = F.drag_lift(L, x, 1e-3, k)
        assert abs(d.sum() + c1 * hole) < 1e-12 * max(1.0, abs(c1 * hole)), (d, hole)
        assert abs(lft.sum() + c2 * hole) < 1e-12 * max(1.0, abs(c2 * hole))
        x = _state(L, lambda X, Y: 0 * X, lambda X, Y: 0 * X, lambda X, Y: 1.0 + 0 * X)
        d, lft = F.drag_lift(L, x, 1e-3, k)
        assert np.abs(d).max() < 1e-14 and np.abs(lft).max() < 1e-14


def test_viscous_drag_converges_to_divergence_theorem_value():
    m = channel_obstacle(2)
    cx, cy, r = m.info["cx"], m.info["cy"], m.info["r"]
    u = lambda X, Y: np.sin(np.pi * X) * np.cos(np.pi * Y)
    v = lambda X, Y: -np.cos(np.pi * X) * np.sin(np.pi * Y)
    # nu * int_disc Laplace(u) = -2 pi^2 nu int_disc u  (polar Gauss-Legendre)
    nr, nt = 40, 160
    gr, wr = np.polynomial.legendre.leggauss(nr)
    rr = 0.5 * r * (gr + 1)
    th = 2 * np.pi * np.arange(nt) / nt
    R, T = np.meshgrid(rr, th, indexing="ij")
    W = (0.5 * r * wr)[:, None] * (2 * np.pi / nt) * R
    nu = 0.01
    exact_drag = -2 * np.pi ** 2 * nu * np.sum(W * u(cx + R * np.cos(T), cy + R * np.sin(T)))
    exact_lift = -2 * np.pi ** 2 * nu * np.sum(W * v(cx + R * np.cos(T), cy + R * np.sin(T)))
    lev = mesh.hierarchy(m, 5)
    errs = []
    for l in (3, 4, 5):
        x = _state(lev[l], u, v, lambda X, Y: 0 * X)
        d, lft = F.drag_lift(lev[l], x, nu, 1)
        errs.append(max(abs(d[0] - exact_drag), abs(lft[0] - exact_lift)))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[1] / errs[2] > 1.6, errs


# ---- oscillation diagnostics (reading F3)

def _wave(f0, phase, t0, dt, n, offset=0.3, harmonic=0.0):
    t = t0 + dt * np.arange(n)
    return offset + np.sin(2 * np.pi * f0 * t + phase) + harmonic * np.sin(4 * np.pi * f0 * t)


def test_oscillation_of_a_sinusoid():
    """Maxima of sin(2 pi f t + phase) sit at t = (1/4 - phase / 2 pi + k) / f;
    the parabola locates them to O((omega dt)^2 dt)."""
    f0, phase, t0, dt = 3.1, -1.0, 9.0, 0.005       # three whole excursions in [9, 10]
    y = _wave(f0, phase, t0, dt, 201)
    t1, per, cnt = F.oscillation(y, t0, dt)
    k = np.ceil((t0 - (0.25 - phase / (2 * np.pi)) / f0) * f0)
    exact = (0.25 - phase / (2 * np.pi) + k) / f0
    assert cnt == 3
    assert abs(t1 - exact) < 1e-5
    assert abs(per - 1 / f0) < 1e-6


def test_oscillation_phase_shift_and_degenerate_series():
    f0, dt = 2.0, 0.01
    a = F.oscillation(_wave(f0, 0.0, 0.0, dt, 300), 0.0, dt)
    b = F.oscillation(_wave(f0, -0.5, 0.0, dt, 300), 0.0, dt)
    assert abs((b[0] - a[0]) - 0.5 / (2 * np.pi * f0)) < 1e-5      # a lag of phase / omega
    # a harmonic that does not create extra maxima above the mean
    h = F.oscillation(_wave(f0, 0.0, 0.0, dt, 300, harmonic=0.1), 0.0, dt)
    assert h[2] == a[2] and abs(h[1] - a[1]) < 1e-3
    t1, per, cnt = F.oscillation(np.full(50, 0.4), 0.0, dt)      # no maxima
    assert cnt == 0 and np.isnan(t1) and np.isnan(per)
    t1, per, cnt = F.oscillation(np.sin(np.linspace(-np.pi / 2, 3 * np.pi / 2, 41)), 0.0, 0.1)
    assert cnt == 1 and abs(t1 - 2.0) < 1e-12 and np.isnan(per)           # one maximum
    # maxima cut by the window's ends do not count
    t1, per, cnt = F.oscillation(np.cos(np.linspace(0, 2 * np.pi, 81)), 0.0, 0.1)
    assert cnt == 0


def test_oscillation_ignores_wiggles():
    """A fast small ripple adds local maxima but no excursions that peak
    above the mean/maximum midpoint: the shedding period is unchanged."""
    f0, dt = 3.0, 0.002
    t = dt * np.arange(1000)
    clean = -np.cos(2 * np.pi * f0 * t)              # the window starts at a trough
    rippled = clean + 0.05 * np.sin(2 * np.pi * 40 * f0 * t + 0.3)
    a = F.oscillation(clean, 0.0, dt)
    b = F.oscillation(rippled, 0.0, dt)
    assert a[2] == b[2] == 6
    assert abs(a[1] - 1 / f0) < 1e-6 and abs(b[1] - 1 / f0) < 2e-3
