"""The seeded multi-obstacle channel generator of the batched workload.

Pins: determinism, a conforming counter-clockwise macro mesh whose boundary
edges are exactly the listed ones, obstacle boundaries on their ellipses,
the clearances the draw promises, the value ranges of the drawn parameters,
and the refined domain area against the exact channel-minus-ellipses area.
"""
import collections

import numpy as np

from oracle import mesh
from synthetic import channel_obstacles
from synthetic.channel import CHANNEL_H, CHANNEL_L

SEEDS = range(100, 164)


def _area(xy, q):
    x, y = xy[q, 0], xy[q, 1]
    return 0.5 * np.sum(x * np.roll(y, -1, axis=1) - np.roll(x, -1, axis=1) * y, axis=1)


def test_deterministic():
    a, b = channel_obstacles(123), channel_obstacles(123)
    assert np.array_equal(a.xy, b.xy) and np.array_equal(a.quads, b.quads)
    assert a.info == b.info


def test_conforming_counter_clockwise_with_tagged_boundary():
    for seed in SEEDS:
        m = channel_obstacles(seed)
        assert (_area(m.xy, m.quads) > 0).all(), seed
        edges = collections.Counter()
        for q in m.quads:
            for k in range(4):
                edges[frozenset((int(q[k]), int(q[(k + 1) % 4])))] += 1
        assert max(edges.values()) <= 2, seed
        boundary = {e for e, c in edges.items() if c == 1}
        listed = {frozenset((int(a), int(b))) for a, b, _ in m.bedges}
        assert boundary == listed, seed
        tags = set(int(t) for t in m.bedges[:, 2])
        assert tags == {1, 2, 3} | {4 + k for k in range(m.info["n_obs"])}, seed


def test_obstacle_vertices_on_ellipses_and_clearances():
    for seed in SEEDS:
        m = channel_obstacles(seed)
        for a_, b_, t in m.bedges:
            if t >= 4:
                cx, cy, A, B, phi = m.curves[t - 4]
                for v in (a_, b_):
                    dx, dy = m.xy[v] - (cx, cy)
                    c, s = np.cos(phi), np.sin(phi)
                    u, w = c * dx + s * dy, -s * dx + c * dy
                    assert abs((u / A) ** 2 + (w / B) ** 2 - 1.0) < 1e-12
        obs = m.info["obstacles"]
        assert 1 <= len(obs) <= 3
        for cx, cy, A, B, phi in obs:
            assert 0.03 <= A <= 0.07 and A / 2 <= B <= A
            assert cy - A >= 0.05 and CHANNEL_H - cy - A >= 0.05
        for i in range(len(obs)):
            for j in range(i + 1, len(obs)):
                d = np.hypot(obs[i][0] - obs[j][0], obs[i][1] - obs[j][1])
                assert d - obs[i][2] - obs[j][2] >= 0.05


def test_parameter_ranges_over_the_batch():
    ms = [channel_obstacles(s) for s in SEEDS]
    assert {m.info["n_obs"] for m in ms} == {1, 2, 3}
    assert {m.info["depth"] for m in ms} == {4, 5, 6, 7}
    assert all(50 <= m.info["Re"] <= 200 and abs(m.nu - 0.1 / m.info["Re"]) < 1e-15 for m in ms)


def test_refined_area_converges_to_channel_minus_ellipses():
    m = channel_obstacles(100)
    exact = CHANNEL_L * CHANNEL_H - sum(np.pi * o[2] * o[3] for o in m.info["obstacles"])
    errs = []
    for lvl in (1, 2, 3):
        L = mesh.hierarchy(m, lvl)[lvl]
        errs.append(abs(_area(L.xy, L.cells).sum() - exact))
    # inscribed polygon of the ellipses: the area defect shrinks ~4x per level
    assert errs[2] < errs[1] < errs[0]
    assert errs[1] / errs[2] > 3.0, errs
