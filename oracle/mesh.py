"""Oracle mesh hierarchy: uniform refinement of the macro mesh (FP64, numpy).

Follows the paper's use of a nested mesh hierarchy for geometric multigrid
(Sec. 2.2) with patches made of the 2x2 children of one coarser cell (the
patch of Sec. 2.2 and of the local projection stabilisation, Sec. 2.1).
Readings (paper silent): G3 (level 0 is the macro mesh refined once so that it
already has patches), G9 (new midpoints of curved obstacle edges are projected
radially onto the ellipse in its scaled frame; a new cell centre is the Coons
point 1/2 sum(edge midpoints) - 1/4 sum(corners)).

Numbering convention of a refinement (a format both implementations follow so
that their nodal vectors can be compared entry by entry):
  * old vertices keep their ids 0..V-1;
  * each undirected edge gets id V + e, edges numbered in order of first
    appearance when visiting cells c = 0..C-1 and local edges k = 0..3, where
    local edge k joins local vertices k and k+1 (mod 4);
  * the centre of cell c gets id V + E + c;
  * cell c has children 4c + k; child k holds the parent's vertex k at its
    local position k (child 0 = (n0, m01, c, m30), child 1 = (m01, n1, m12, c),
    child 2 = (c, m12, n2, m23), child 3 = (m30, c, m23, n3));
  * each boundary edge (v0, v1, tag) becomes (v0, m, tag), (m, v1, tag).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

TAG_INFLOW, TAG_WALL, TAG_OUTFLOW, TAG_OBSTACLE = 1, 2, 3, 4

# patch-local (lexicographic 3x3 in the parent's frame) index of each child's
# local vertices: child k, local vertex a -> q = i + 3 j
CHILD_TO_PATCH = np.array([[0, 1, 4, 3], [1, 2, 5, 4], [4, 5, 8, 7], [3, 4, 7, 6]])


@dataclass
class Level:
    xy: np.ndarray          # (N, 2)
    cells: np.ndarray       # (C, 4)
    bedges: np.ndarray      # (E_b, 3)
    curves: np.ndarray      # (K, 5)
    # refinement record of the *coarser* level that produced this one
    n_coarse: int = 0
    edge_ends: np.ndarray | None = None     # (E_c, 2) coarse node ids of each new edge node
    coarse_cells: np.ndarray | None = None  # (C_c, 4) coarse cells (for new centre nodes)

    @property
    def n_nodes(self):
        return self.xy.shape[0]

    @property
    def n_cells(self):
        return self.cells.shape[0]

    def patches(self) -> np.ndarray:
        """(C/4, 9) node ids of each patch in lexicographic parent-frame order."""
        P = self.n_cells // 4
        pat = np.empty((P, 9), dtype=np.int64)
        c4 = self.cells.reshape(P, 4, 4)
        for k in range(4):
            for a in range(4):
                pat[:, CHILD_TO_PATCH[k, a]] = c4[:, k, a]
        return pat

    def dirichlet_nodes(self) -> np.ndarray:
        """Boolean mask: nodes on an inflow, wall or obstacle edge (eq. boundary:
        Dirichlet part of the boundary; outflow nodes stay free)."""
        m = np.zeros(self.n_nodes, dtype=bool)
        be = self.bedges[self.bedges[:, 2] != TAG_OUTFLOW]
        m[be[:, 0]] = True
        m[be[:, 1]] = True
        return m

    def inflow_nodes(self) -> np.ndarray:
        m = np.zeros(self.n_nodes, dtype=bool)
        be = self.bedges[self.bedges[:, 2] == TAG_INFLOW]
        m[be[:, 0]] = True
        m[be[:, 1]] = True
        return m

    def prolongation(self) -> sp.csr_matrix:
        """Nodal bilinear interpolation from the coarser level in the parent's
        reference coordinates: old vertices copied, edge nodes averaged from
        the two edge ends, centres averaged from the four cell corners."""
        Nc, Nf = self.n_coarse, self.n_nodes
        E = self.edge_ends.shape[0]
        rows = [np.arange(Nc)]
        cols = [np.arange(Nc)]
        vals = [np.ones(Nc)]
        for k in range(2):
            rows.append(Nc + np.arange(E)); cols.append(self.edge_ends[:, k])
            vals.append(np.full(E, 0.5))
        Cc = self.coarse_cells.shape[0]
        for k in range(4):
            rows.append(Nc + E + np.arange(Cc)); cols.append(self.coarse_cells[:, k])
            vals.append(np.full(Cc, 0.25))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                     np.concatenate(cols))),
                             shape=(Nf, Nc))


def project_to_ellipse(p, curve):
    """Radial projection in the ellipse's scaled frame (reading G9)."""
    cx, cy, a, b, phi = curve
    c, s = np.cos(phi), np.sin(phi)
    dx, dy = p[0] - cx, p[1] - cy
    qx, qy = c * dx + s * dy, -s * dx + c * dy
    r = np.sqrt((qx / a) ** 2 + (qy / b) ** 2)
    qx, qy = qx / r, qy / r
    return np.array([cx + c * qx - s * qy, cy + s * qx + c * qy])


def refine(xy, cells, bedges, curves) -> Level:
    """One uniform refinement step (numbering convention in the module doc)."""
    V = xy.shape[0]
    C = cells.shape[0]
    edge_id = {}
    ends = []
    for c in range(C):
        for k in range(4):
            a, b = int(cells[c, k]), int(cells[c, (k + 1) % 4])
            key = (min(a, b), max(a, b))
            if key not in edge_id:
                edge_id[key] = len(ends)
                ends.append((a, b))
    E = len(ends)
    ends = np.array(ends, dtype=np.int64)
    fxy = np.zeros((V + E + C, 2))
    fxy[:V] = xy
    fxy[V:V + E] = 0.5 * (xy[ends[:, 0]] + xy[ends[:, 1]])
    fb = []
    for v0, v1, tag in bedges:
        m = V + edge_id[(min(v0, v1), max(v0, v1))]
        if tag >= TAG_OBSTACLE:
            fxy[m] = project_to_ellipse(fxy[m], curves[tag - TAG_OBSTACLE])
        fb.append((v0, m, tag))
        fb.append((m, v1, tag))
    mid = np.empty((C, 4), dtype=np.int64)
    for c in range(C):
        for k in range(4):
            a, b = int(cells[c, k]), int(cells[c, (k + 1) % 4])
            mid[c, k] = V + edge_id[(min(a, b), max(a, b))]
    ctr = V + E + np.arange(C)
    fxy[ctr] = 0.5 * fxy[mid].sum(axis=1) - 0.25 * xy[cells].sum(axis=1)
    n0, n1, n2, n3 = (cells[:, k].astype(np.int64) for k in range(4))
    m01, m12, m23, m30 = (mid[:, k] for k in range(4))
    ch = np.stack([
        np.stack([n0, m01, ctr, m30], 1),
        np.stack([m01, n1, m12, ctr], 1),
        np.stack([ctr, m12, n2, m23], 1),
        np.stack([m30, ctr, m23, n3], 1)], axis=1).reshape(4 * C, 4)
    return Level(xy=fxy, cells=ch, bedges=np.array(fb, dtype=np.int64), curves=curves,
                 n_coarse=V, edge_ends=ends, coarse_cells=cells.astype(np.int64))


def hierarchy(macro, finest: int) -> list[Level]:
    """Levels 0..finest; level 0 is the macro mesh refined once (reading G3)."""
    lev = [refine(macro.xy, macro.quads.astype(np.int64), macro.bedges.astype(np.int64),
                  macro.curves)]
    for _ in range(finest):
        L = lev[-1]
        lev.append(refine(L.xy, L.cells, L.bedges, L.curves))
    return lev


def cell_areas(xy, cells):
    """Exact area of each (bilinear) quadrilateral by the shoelace formula."""
    x = xy[cells, 0]
    y = xy[cells, 1]
    return 0.5 * np.sum(x * np.roll(y, -1, axis=1) - np.roll(x, -1, axis=1) * y, axis=1)
