"""Seeded macro meshes for the flow-around-an-obstacle test problem.

The paper's experiments use a channel with an elliptic obstacle (a variant of
the Schaefer-Turek benchmark, Sec. 3.1).  Its data is not available, so these
generators stand in for it: a channel [0, 2.2] x [0, 0.41] whose obstacle
centre and size are drawn from a seeded PCG64 stream.

A macro mesh is the coarsest input the solvers receive.  Both the oracle and
the HIP library refine it once to obtain multigrid level 0 (so that level 0
already has 2x2 patches for the local projection stabilisation) and then
uniformly to the finer levels.

Boundary tags of boundary edges:
    1 inflow (x = 0), 2 no-slip wall (y = 0 or y = H), 3 do-nothing outflow
    (x = L), 4 + k the curved boundary of obstacle k.
Curve descriptors are rows (cx, cy, a, b, phi): an ellipse with semi-axes a, b
rotated by phi around its centre (a circle has a = b).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CHANNEL_L = 2.2
CHANNEL_H = 0.41
TAG_INFLOW, TAG_WALL, TAG_OUTFLOW, TAG_OBSTACLE = 1, 2, 3, 4


@dataclass
class MacroMesh:
    xy: np.ndarray            # (V, 2) float64 vertex coordinates
    quads: np.ndarray         # (C, 4) int32, counter-clockwise vertex ids
    bedges: np.ndarray        # (E, 3) int32, (v0, v1, tag)
    curves: np.ndarray        # (K, 5) float64, (cx, cy, a, b, phi)
    nu: float = 1e-3          # kinematic viscosity (the paper's 1/Re)
    info: dict = field(default_factory=dict)

    @property
    def n_vert(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_cell(self) -> int:
        return int(self.quads.shape[0])


def _ray_to_ellipse(cx, cy, a, b, phi, theta):
    """Point where the ray from (cx, cy) in direction theta meets the ellipse."""
    d = np.array([np.cos(theta), np.sin(theta)])
    c, s = np.cos(phi), np.sin(phi)
    dl = np.array([c * d[0] + s * d[1], -s * d[0] + c * d[1]])   # R(-phi) d
    t = 1.0 / np.sqrt((dl[0] / a) ** 2 + (dl[1] / b) ** 2)
    return np.array([cx + t * d[0], cy + t * d[1]])


def _grid_with_hole(xs, ys, hole, curve):
    """Tensor grid xs x ys with the cell `hole` = (i, j) replaced by four quads
    that connect the hole's square boundary to an obstacle inscribed in it."""
    nx, ny = len(xs) - 1, len(ys) - 1
    gid = lambda i, j: j * (nx + 1) + i
    xy = [(x, y) for y in ys for x in xs]
    quads, bedges = [], []
    hi, hj = hole
    for j in range(ny):
        for i in range(nx):
            if (i, j) == (hi, hj):
                continue
            quads.append((gid(i, j), gid(i + 1, j), gid(i + 1, j + 1), gid(i, j + 1)))
    cx, cy, a, b, phi = curve
    # square corners, counter-clockwise starting at the upper right (45 deg)
    corners = [gid(hi + 1, hj + 1), gid(hi, hj + 1), gid(hi, hj), gid(hi + 1, hj)]
    arc = []
    for k in range(4):
        theta = np.pi / 4 + k * np.pi / 2
        arc.append(len(xy))
        xy.append(tuple(_ray_to_ellipse(cx, cy, a, b, phi, theta)))
    for k in range(4):
        k1 = (k + 1) % 4
        quads.append((arc[k], corners[k], corners[k1], arc[k1]))
        bedges.append((arc[k], arc[k1], TAG_OBSTACLE))
    for i in range(nx):
        bedges.append((gid(i, 0), gid(i + 1, 0), TAG_WALL))
        bedges.append((gid(i, ny), gid(i + 1, ny), TAG_WALL))
    for j in range(ny):
        bedges.append((gid(0, j), gid(0, j + 1), TAG_INFLOW))
        bedges.append((gid(nx, j), gid(nx, j + 1), TAG_OUTFLOW))
    return (np.asarray(xy, dtype=np.float64), np.asarray(quads, dtype=np.int32),
            np.asarray(bedges, dtype=np.int32))


def channel_obstacle(seed: int, Re: float = 100.0, box: float = 0.1,
                     n_downstream: int = 4) -> MacroMesh:
    """Channel [0, 2.2] x [0, 0.41] with one circular obstacle.

    Draw order (PCG64, numpy.random.default_rng(seed)): centre x ~ U[0.15, 0.3],
    centre y ~ U[0.15, 0.26], radius ~ U[0.04, 0.06].  The viscosity follows
    nu = U_mean * D_ref / Re with U_mean = 1 and D_ref = 0.1 held fixed.
    The macro mesh has 3 rows and 2 + n_downstream columns of cells around a
    square box of half-width `box` that holds the obstacle (21 quads for the
    default), so level 0 (one refinement) has 84 quads.
    """
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.15, 0.3)
    cy = rng.uniform(0.15, 0.26)
    r = rng.uniform(0.04, 0.06)
    xr = cx + box
    rest = CHANNEL_L - xr
    w = np.arange(1, n_downstream + 1, dtype=np.float64)
    w = np.cumsum(w) / np.sum(w)
    xs = [0.0, cx - box, xr] + list(xr + rest * w[:-1]) + [CHANNEL_L]
    ys = [0.0, cy - box, cy + box, CHANNEL_H]
    curve = (cx, cy, r, r, 0.0)
    xy, quads, bedges = _grid_with_hole(np.array(xs), np.array(ys), (1, 1), curve)
    nu = 1.0 * 0.1 / Re
    return MacroMesh(xy=xy, quads=quads, bedges=bedges,
                     curves=np.array([curve], dtype=np.float64), nu=nu,
                     info=dict(seed=seed, Re=Re, cx=cx, cy=cy, r=r))


def training_channel(seed: int, re_range=(80.0, 120.0)) -> MacroMesh:
    """Geometry of the training workload: channel_obstacle's draws (centre x,
    centre y, radius) followed by Re ~ U[re_range] from the same PCG64
    stream."""
    rng = np.random.default_rng(seed)
    rng.uniform(size=3)                      # the geometry draws of channel_obstacle
    Re = rng.uniform(*re_range)
    return channel_obstacle(seed, Re=Re)


def _strip_mesh(obs, n_downstream):
    """Macro mesh of the channel with one or more obstacles in x-disjoint
    strips.  `obs` rows (cx, cy, a, b, phi, w), sorted by cx; w is the
    half-width of the square box holding the obstacle.  Every vertical grid
    line carries 4 vertices (y = 0, y1, y2, H): inside a strip (y1, y2) is its
    box's y-range; elsewhere the lines move linearly towards the neutral
    (H/3, 2H/3), so no row inherits a thin box margin over a long distance.
    Columns outside the strips are at most 0.3 wide (the downstream ones are
    graded 1:2:..:n_downstream), each a row of 3 quads."""
    xy, quads, bedges, curves = [], [], [], []
    neutral = (CHANNEL_H / 3.0, 2.0 * CHANNEL_H / 3.0)

    def column_line(x, y12):
        base = len(xy)
        for y in (0.0, y12[0], y12[1], CHANNEL_H):
            xy.append((x, y))
        return [base, base + 1, base + 2, base + 3]

    def join(lft, rgt):
        for r in range(3):
            quads.append((lft[r], rgt[r], rgt[r + 1], lft[r + 1]))
        bedges.append((lft[0], rgt[0], TAG_WALL))
        bedges.append((lft[3], rgt[3], TAG_WALL))

    def fill(line, x0, y0, x1, y1, xs=None):
        """Columns from the existing line at x0 (rows y0) to a new line at x1
        (rows y1); returns the last line."""
        if xs is None:
            n = max(1, int(np.ceil((x1 - x0) / 0.3 - 1e-9)))
            xs = [x0 + (x1 - x0) * (k + 1) / n for k in range(n)]
        for x in xs:
            t = (x - x0) / (x1 - x0)
            nxt = column_line(x, ((1 - t) * y0[0] + t * y1[0], (1 - t) * y0[1] + t * y1[1]))
            join(line, nxt)
            line = nxt
        return line

    line = column_line(0.0, neutral)
    for r in range(3):
        bedges.append((line[r], line[r + 1], TAG_INFLOW))
    x_prev, y_prev = 0.0, neutral
    for k, (cx, cy, a, b, phi, w) in enumerate(obs):
        box = (cy - w, cy + w)
        # approach the strip: move to neutral first when there is room, then to the box
        mid = 0.5 * (x_prev + cx - w)
        if cx - w - x_prev > 0.45 and x_prev > 0.0:
            line = fill(line, x_prev, y_prev, mid, neutral)
            x_prev, y_prev = mid, neutral
        left = fill(line, x_prev, y_prev, cx - w, box)
        right = column_line(cx + w, box)
        quads.append((left[0], right[0], right[1], left[1]))
        quads.append((left[2], right[2], right[3], left[3]))
        bedges.append((left[0], right[0], TAG_WALL))
        bedges.append((left[3], right[3], TAG_WALL))
        corners = [right[2], left[2], left[1], right[1]]   # from the upper right, CCW
        arc = []
        for q in range(4):
            arc.append(len(xy))
            xy.append(tuple(_ray_to_ellipse(cx, cy, a, b, phi, np.pi / 4 + q * np.pi / 2)))
        for q in range(4):
            q1 = (q + 1) % 4
            quads.append((arc[q], corners[q], corners[q1], arc[q1]))
            bedges.append((arc[q], arc[q1], TAG_OBSTACLE + k))
        curves.append((cx, cy, a, b, phi))
        line, x_prev, y_prev = right, cx + w, box
    wts = np.cumsum(np.arange(1, n_downstream + 1, dtype=np.float64))
    wts /= wts[-1]
    xs = [x_prev + (CHANNEL_L - x_prev) * t for t in wts]
    # the first downstream column returns to the neutral rows
    line = fill(line, x_prev, y_prev, xs[0], neutral, xs=[xs[0]])
    line = fill(line, xs[0], neutral, CHANNEL_L, neutral, xs=xs[1:])
    for r in range(3):
        bedges.append((line[r], line[r + 1], TAG_OUTFLOW))
    return (np.asarray(xy, dtype=np.float64), np.asarray(quads, dtype=np.int32),
            np.asarray(bedges, dtype=np.int32), np.asarray(curves, dtype=np.float64))


def channel_obstacles(seed: int, n_downstream: int = 4, max_tries: int = 2000) -> MacroMesh:
    """Channel with 1-3 seeded circular or elliptical obstacles, a seeded
    Reynolds number and a seeded mesh depth (the batched-solve workload).

    Draw order (PCG64, numpy.random.default_rng(seed)): n_obs ~ U{1, 2, 3};
    per obstacle: ellipse with probability 1/2, semi-axis a ~ U[0.03, 0.07],
    aspect ~ U[1, 2] (b = a / aspect; a circle has b = a), rotation
    phi ~ U[0, pi), then centres drawn x ~ U[0.15, 1.0], y ~ U[0.1, 0.31]
    until the obstacle keeps 0.05 from both walls and its square box keeps a
    0.05 x-gap to the boxes already placed (so obstacles are >= 0.05 apart);
    then Re ~ U[50, 200] and depth ~ U{4, ..., 7}.  nu = 0.1 / Re as in
    `channel_obstacle`.  Box half-width w = min(1.7 a, a + 0.4 g) with g the
    smaller wall gap cy - a, H - cy - a: the ring around the obstacle gets 40%
    of the gap, the row between box and wall 60%.
    """
    rng = np.random.default_rng(seed)
    n_obs = int(rng.integers(1, 4))
    placed = []
    for _ in range(n_obs):
        ellipse = rng.uniform() < 0.5
        a = rng.uniform(0.03, 0.07)
        aspect = rng.uniform(1.0, 2.0)
        b = a / aspect if ellipse else a
        phi = rng.uniform(0.0, np.pi) if ellipse else 0.0
        for _ in range(max_tries):
            cx = rng.uniform(0.15, 1.0)
            cy = rng.uniform(0.1, 0.31)
            gap = min(cy - a, CHANNEL_H - cy - a)
            if gap < 0.05:
                continue
            w = min(1.7 * a, a + 0.4 * gap)
            if cx - w < 0.05:
                continue
            if all(abs(cx - o[0]) >= w + o[5] + 0.05 for o in placed):
                placed.append((cx, cy, a, b, phi, w))
                break
    placed.sort(key=lambda o: o[0])
    Re = rng.uniform(50.0, 200.0)
    depth = int(rng.integers(4, 8))
    xy, quads, bedges, curves = _strip_mesh(placed, n_downstream)
    return MacroMesh(xy=xy, quads=quads, bedges=bedges, curves=curves, nu=0.1 / Re,
                     info=dict(seed=seed, Re=Re, depth=depth, n_obs=len(placed),
                               obstacles=[tuple(o[:5]) for o in placed]))


def rectangle(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0, nu: float = 0.1,
              x0: float = 0.0, y0: float = 0.0, skew: float = 0.0) -> MacroMesh:
    """Obstacle-free macro mesh of [x0, x0+Lx] x [y0, y0+Ly] with nx x ny cells.

    Tags: left edge inflow, bottom/top walls, right edge outflow.  `skew`
    shifts each interior grid line x_i by skew * (y - y0) to produce an
    all-parallelogram mesh (used for the affine-mesh identities).
    """
    xs = x0 + np.linspace(0.0, Lx, nx + 1)
    ys = y0 + np.linspace(0.0, Ly, ny + 1)
    gid = lambda i, j: j * (nx + 1) + i
    xy = np.array([(x + skew * (y - y0) * (0 < i < nx), y)
                   for j, y in enumerate(ys) for i, x in enumerate(xs)])
    quads = np.array([(gid(i, j), gid(i + 1, j), gid(i + 1, j + 1), gid(i, j + 1))
                      for j in range(ny) for i in range(nx)], dtype=np.int32)
    be = []
    for i in range(nx):
        be.append((gid(i, 0), gid(i + 1, 0), TAG_WALL))
        be.append((gid(i, ny), gid(i + 1, ny), TAG_WALL))
    for j in range(ny):
        be.append((gid(0, j), gid(0, j + 1), TAG_INFLOW))
        be.append((gid(nx, j), gid(nx, j + 1), TAG_OUTFLOW))
    return MacroMesh(xy=xy.astype(np.float64), quads=quads,
                     bedges=np.array(be, dtype=np.int32),
                     curves=np.zeros((0, 5)), nu=nu, info=dict(kind="rectangle"))


def random_state(n_nodes: int, seed: int) -> np.ndarray:
    """Seeded random nodal state, interleaved (u, v, p) per node:
    u, v ~ U[-1.5, 1.5] and p ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    x = np.empty((n_nodes, 3))
    x[:, 0] = rng.uniform(-1.5, 1.5, n_nodes)
    x[:, 1] = rng.uniform(-1.5, 1.5, n_nodes)
    x[:, 2] = rng.uniform(-1.0, 1.0, n_nodes)
    return x.reshape(-1)


def gru_weights(n_in: int, hidden: int, layers: int, n_out: int, seed: int,
                scale: float = 1.0) -> np.ndarray:
    """Seeded bias-free GRU stack + linear head, flat float64 vector.

    Order: for each layer l, W_ih (3H x I_l, gate rows r, z, n) then
    W_hh (3H x H); finally W_out (O x H).  Entries ~ U[-s, s] with
    s = scale / sqrt(H), the usual recurrent-layer initialisation range.
    """
    rng = np.random.default_rng(seed)
    s = scale / np.sqrt(hidden)
    n = 0
    for l in range(layers):
        i_l = n_in if l == 0 else hidden
        n += 3 * hidden * i_l + 3 * hidden * hidden
    n += n_out * hidden
    return rng.uniform(-s, s, n)


# Named workloads (shapes of the configurations the benchmark and tests use).
WORKLOADS = {
    "c1_fp64_parity": dict(seeds=(0, 1, 2, 3), level=3, dt=0.01, steps=10, Re=100.0),
    "c2_mixed_at_scale": dict(seeds=(0,), level=7, dt=0.005, steps=200, Re=100.0,
                              oracle_level=5),
    "c3_batched": dict(seeds=tuple(range(100, 164)), dt=0.005, steps=100,
                       generator="channel_obstacles"),
    "c4_dnnmg_inference": dict(seeds=(0,), coarse_level=5, fine_level=7, dt=0.005,
                               hidden=128, layers=2, n_in=490, n_out=162),
    "c5_training": dict(seeds=tuple(range(200, 216)), batch=8192, seq=32,
                        hidden=(64, 128, 256), layers=2, ckpt=8, generator="training_channel",
                        Re=(80.0, 120.0), held_out=(300, 301, 302, 303)),
}
