"""Oracle flow functionals (Sec. 3.3, the functionals used to compare the
networks' accuracy), FP64 numpy.  Test infrastructure only.

* J_div(v) = int_Omega |div v|^2 dx: the discrete Q1 velocity, 2x2 Gauss
  quadrature in every cell (the quadrature of the residual).
* Drag and lift on obstacle k:
      J_drag = - int_{Gamma_k} (nu grad v - p I) n . e_x ds,
      J_lift = - int_{Gamma_k} (nu grad v - p I) n . e_y ds,
  with n the unit normal pointing into the obstacle (outward from the
  fluid), nu the kinematic viscosity of the problem (the paper writes 1/Re),
  grad v the full velocity gradient, (grad v n)_i = sum_j dv_i/dx_j n_j.

* Oscillation of a sampled functional (Sec. 3.3 compares the lift of the
  runs over the periodic limit cycle after aligning their first maximum in
  the window): reading F3 below.

Readings (paper silent): F1 the boundary integral is taken over the polygonal
boundary of the mesh, each boundary edge with 2-point Gauss quadrature, grad v
and p from the Q1 fields of the fluid cell the edge belongs to (a line
integral of the discrete fields, not a residual-based evaluation); F2 the
normal of an edge is the outward normal of its cell; F3 a series has one
maximum per excursion above its mean (a maximal run of samples above the
mean, bounded inside the window by samples at or below it) that peaks above
the midpoint of the mean and the series maximum (small wiggles of a noisy
signal do not count); it sits at the vertex of the parabola through the
excursion's largest sample and its two neighbours; the shedding period is the
mean spacing of the maxima, the phase offset of two runs the difference of
their first maxima.
"""
from __future__ import annotations

import numpy as np

from .fem import geometry
from .mesh import Level

_G = 1.0 / np.sqrt(3.0)
_CORNER = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])


def j_div(level: Level, x: np.ndarray) -> float:
    """int |div v|^2 over the mesh (2x2 Gauss per cell)."""
    det, grad = geometry(level.xy, level.cells)          # (C, q), (C, q, a, 2)
    X = x.reshape(-1, 3)
    U, V = X[level.cells, 0], X[level.cells, 1]          # (C, a)
    div = np.einsum('cqa,ca->cq', grad[..., 0], U) + np.einsum('cqa,ca->cq', grad[..., 1], V)
    return float(np.sum(det * div ** 2))


def obstacle_edges(level: Level):
    """(cell, local side a -> a+1, obstacle k) of every obstacle boundary edge."""
    where = {}
    for c, cell in enumerate(level.cells):
        for a in range(4):
            where[frozenset((int(cell[a]), int(cell[(a + 1) % 4])))] = (c, a)
    out = []
    for v0, v1, tag in level.bedges:
        if tag >= 4:
            c, a = where[frozenset((int(v0), int(v1)))]
            out.append((c, a, int(tag) - 4))
    return out


def drag_lift(level: Level, x: np.ndarray, nu, n_obstacles: int):
    """Drag and lift per obstacle; nu a scalar or one viscosity per node."""
    X = x.reshape(-1, 3)
    nu_node = np.broadcast_to(np.asarray(nu, dtype=np.float64), (level.n_nodes,))
    drag = np.zeros(n_obstacles)
    lift = np.zeros(n_obstacles)
    for c, a, k in obstacle_edges(level):
        nodes = level.cells[c]
        P = level.xy[nodes]                              # (4, 2)
        e = P[(a + 1) % 4] - P[a]
        length = np.hypot(e[0], e[1])
        n = np.array([e[1], -e[0]]) / length             # outward from the (CCW) cell
        for t in (-_G, _G):
            xi, eta = 0.5 * (1 - t) * _CORNER[a] + 0.5 * (1 + t) * _CORNER[(a + 1) % 4]
            N = 0.25 * (1 + xi * _CORNER[:, 0]) * (1 + eta * _CORNER[:, 1])
            dxi = 0.25 * _CORNER[:, 0] * (1 + eta * _CORNER[:, 1])
            deta = 0.25 * _CORNER[:, 1] * (1 + xi * _CORNER[:, 0])
            J = np.array([[dxi @ P[:, 0], deta @ P[:, 0]], [dxi @ P[:, 1], deta @ P[:, 1]]])
            # physical gradients: grad N = J^{-T} (dN/dxi, dN/deta)
            G = np.linalg.solve(J.T, np.vstack([dxi, deta]))   # (2, 4)
            gu = G @ X[nodes, 0]
            gv = G @ X[nodes, 1]
            p = N @ X[nodes, 2]
            nu_e = nu_node[nodes[a]]
            tx = nu_e * (gu @ n) - p * n[0]
            ty = nu_e * (gv @ n) - p * n[1]
            w = 0.5 * length                            # Gauss weight 1 on [-1, 1]
            drag[k] -= w * tx
            lift[k] -= w * ty
    return drag, lift


def oscillation(f, t0: float, dt: float):
    """(time of the first maximum, mean period, number of maxima) of
    f[i] = J(t0 + i dt) under reading F3; NaN where undefined."""
    f = np.asarray(f, dtype=np.float64)
    mean = f.mean()
    high = 0.5 * (mean + f.max())
    above = f > mean
    times = []
    # excursions: runs of `above`, kept when bounded on both sides
    starts = [i for i in range(1, len(f)) if above[i] and not above[i - 1]]
    for b in starts:
        e = b
        while e < len(f) and above[e]:
            e += 1
        if e == len(f):
            break
        k = b + int(np.argmax(f[b:e]))
        if f[k] <= high:
            continue
        y0, y1, y2 = f[k - 1], f[k], f[k + 1]
        # vertex of the parabola through (-1, y0), (0, y1), (1, y2)
        curv = y0 - 2 * y1 + y2
        s = (y0 - y2) / (2 * curv) if curv < 0 else 0.0
        times.append(t0 + (k + s) * dt)
    if not times:
        return float("nan"), float("nan"), 0
    period = (times[-1] - times[0]) / (len(times) - 1) if len(times) > 1 else float("nan")
    return times[0], period, len(times)
