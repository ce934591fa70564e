"""Oracle solvers (FP64, numpy/scipy).

* `newton_step`: one time step, A_n(x_n) = f_n solved by Newton's method
  (eq. newton) from x^(0) = (v_{n-1}, p_{n-1}) with the boundary values at
  t_n imposed, each linear system solved by a sparse *direct* solve.  The
  discrete x_n is unique, so this is the plain definition any Newton-Krylov-
  multigrid solver converges to (reading N1: full steps; N2: absolute l2
  tolerance on R).
* The iterative components the paper names for the linear solves (Sec. 2.2:
  GMRES with a geometric multigrid preconditioner, one V-cycle per
  application), in the paper's terms plus the readings N3 (V(2,2), additive
  averaged cell-Vanka, omega = 0.6, coarse operators re-discretised at the
  injected iterate, dense LU on level 0):
  `vanka_sweep`, `vcycle`, `gmres`; and the coloured multiplicative variant
  of the cell-Vanka sweep (`cell_colours`, `vanka_sweep_coloured`): cells in
  index order take the smallest colour no cell sharing a node has taken
  (reading N17); per colour the residual is recomputed and every cell of the
  colour adds omega times its local correction (the cells of a colour share
  no node).  Optionally (reading N18) the levels below the one a V-cycle is
  called on take nu_coarse sweeps before and after instead of (nu1, nu2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from .mesh import Level


def newton_step(level: Level, prob: fem.Problem, x_old: np.ndarray, t_new: float,
                tol: float = 1e-10, maxit: int = 20, return_history: bool = False):
    """x_n from x_{n-1}: Newton with direct linear solves (eq. newton)."""
    x = fem.impose_bc(level, prob, x_old, t_new)
    hist = []
    for it in range(maxit + 1):
        R = fem.residual(level, prob, x, x_old, t_new)
        nr = float(np.linalg.norm(R))
        hist.append(nr)
        if nr <= tol:
            return (x, hist) if return_history else x
        if it == maxit:
            break
        J = fem.jacobian(level, prob, x, x_old)
        x = x + spla.spsolve(J.tocsc(), R)
    raise RuntimeError(f"Newton did not converge: {hist}")


# ---------------------------------------------------------------- multigrid
def cell_dofs(cells):
    return (3 * cells[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)


def cell_blocks(J: sp.csr_matrix, cells) -> np.ndarray:
    """J restricted to the 12 unknowns of every cell: (C, 12, 12)."""
    Jc = J.tocoo()
    n = J.shape[0]
    key = Jc.row.astype(np.int64) * n + Jc.col
    order = np.argsort(key)
    key, val = key[order], Jc.data[order]
    d = cell_dofs(cells).astype(np.int64)
    q = (d[:, :, None] * n + d[:, None, :]).reshape(-1)
    pos = np.searchsorted(key, q)
    pos = np.minimum(pos, key.size - 1)
    found = key[pos] == q
    out = np.where(found, val[pos], 0.0)
    return out.reshape(-1, 12, 12)


def vanka_sweep(J, blocks, cells, x, b, omega=0.6):
    """Additive averaged cell-Vanka: r = b - J x; for every cell solve the local
    12x12 system (LU with partial pivoting); each node receives omega times the
    mean of the corrections of the cells that contain it."""
    r = b - J @ x
    d = cell_dofs(cells)
    delta = np.linalg.solve(blocks, r[d][:, :, None])[:, :, 0]
    acc = np.zeros_like(x)
    np.add.at(acc, d, delta)
    mult = np.zeros(x.size // 3)
    np.add.at(mult, cells.reshape(-1), 1.0)
    return x + omega * acc / np.repeat(mult, 3)


def cell_colours(cells) -> np.ndarray:
    """Greedy colouring in cell order: the smallest colour not taken by an
    earlier cell that shares a node with the cell."""
    cells = np.asarray(cells)
    node_cells = {}
    for c, cell in enumerate(cells):
        for v in cell:
            node_cells.setdefault(int(v), []).append(c)
    colour = np.full(len(cells), -1, dtype=np.int64)
    for c, cell in enumerate(cells):
        taken = {int(colour[o]) for v in cell for o in node_cells[int(v)] if o < c}
        k = 0
        while k in taken:
            k += 1
        colour[c] = k
    return colour


def vanka_sweep_coloured(J, blocks, cells, colours, x, b, omega=0.6):
    """Multiplicative cell-Vanka over the colours: for each colour in turn,
    r = b - J x, then each cell of the colour adds omega times the solution
    of its 12x12 system (LU with partial pivoting) to its unknowns."""
    d = cell_dofs(cells)
    x = x.copy()
    for k in range(int(colours.max()) + 1):
        sel = np.nonzero(colours == k)[0]
        r = b - J @ x
        delta = np.linalg.solve(blocks[sel], r[d[sel]][:, :, None])[:, :, 0]
        x[d[sel]] += omega * delta                 # no two cells of a colour share an unknown
    return x


class MGHierarchy:
    """Operators of all levels at one linearisation point (the fine iterate
    injected to each level: coarse vertices keep their ids, so injection is
    the prefix of the fine vector).  The finest level carries the Jacobian of
    the problem being solved; the levels below it are re-discretised with the
    bounded LPS parameter (fem.coarse_operator_problem, reading G4)."""

    def __init__(self, levels, prob, x_fine, nu1=2, nu2=2, omega=0.6, smoother="additive", nu_coarse=0,
                 coarse=0, x_old=None):
        self.levels = levels
        self.coarse = coarse                # level of the direct solve (Sec. 2: coarse-grid solver)
        self.prob = prob
        self.nu1, self.nu2, self.omega = nu1, nu2, omega
        self.nu_coarse = nu_coarse          # > 0: sweeps before and after on the levels below the top
        self.smoother = smoother
        self.colours = [cell_colours(L.cells) for L in levels] if smoother == "coloured" else None
        self.J = []
        self.blocks = []
        cprob = fem.coarse_operator_problem(prob)
        for l, L in enumerate(levels):
            xl = x_fine[:3 * L.n_nodes]
            xol = None if x_old is None else x_old[:3 * L.n_nodes]
            Jl = fem.jacobian(L, prob if l == len(levels) - 1 else cprob, xl, xol)
            self.J.append(Jl)
            self.blocks.append(cell_blocks(Jl, L.cells))
        self.P = [None] + [levels[l].prolongation() for l in range(1, len(levels))]
        self.dmask = [L.dirichlet_nodes() for L in levels]
        self.lu0 = sla.lu_factor(self.J[coarse].toarray())

    def _prolong(self, l, e):
        return (self.P[l] @ e.reshape(-1, 3)).reshape(-1)

    def _restrict(self, l, r):
        rc = (self.P[l].T @ r.reshape(-1, 3))
        rc[self.dmask[l - 1], :2] = 0.0
        return rc.reshape(-1)

    def sweep(self, l, x, b):
        L = self.levels[l]
        if self.smoother == "coloured":
            return vanka_sweep_coloured(self.J[l], self.blocks[l], L.cells, self.colours[l], x, b, self.omega)
        return vanka_sweep(self.J[l], self.blocks[l], L.cells, x, b, self.omega)

    def vcycle(self, l, b, x=None, top=None):
        """One V(nu1, nu2) cycle on level l for J_l x = b (V(nu_coarse,
        nu_coarse) on the levels below the one it is called on, if set)."""
        top = l if top is None else top
        if l < self.coarse:
            raise ValueError("V-cycle below the coarse level")
        if l == self.coarse:
            return sla.lu_solve(self.lu0, b)
        nu1, nu2 = (self.nu_coarse, self.nu_coarse) if self.nu_coarse > 0 and l != top else (self.nu1, self.nu2)
        x = np.zeros_like(b) if x is None else x.copy()
        for _ in range(nu1):
            x = self.sweep(l, x, b)
        r = b - self.J[l] @ x
        e = self.vcycle(l - 1, self._restrict(l, r), top=top)
        x = x + self._prolong(l, e)
        for _ in range(nu2):
            x = self.sweep(l, x, b)
        return x


def gmres(A, b, precond, rtol=1e-2, restart=30, maxit=100):
    """Right-preconditioned restarted GMRES (Saad) with classical Gram-Schmidt
    applied twice and Givens rotations; stops when the Arnoldi residual
    estimate |g_{j+1}| <= rtol * ||b|| or after maxit iterations.
    Returns (x, iterations, residual estimate history)."""
    n = b.size
    x = np.zeros(n)
    beta0 = np.linalg.norm(b)
    hist = [beta0]
    if beta0 == 0.0:
        return x, 0, hist
    it = 0
    while it < maxit:
        r = b - A @ x
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        Hm = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = A @ Z[j]
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            Hm[:j + 1, j] = h
            Hm[j + 1, j] = hn
            if hn > 0:
                V[j + 1] = w / hn
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            den = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j], sn[j] = Hm[j, j] / den, Hm[j + 1, j] / den
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= rtol * beta0 or it >= maxit:
                break
        y = sla.solve_triangular(Hm[:j_end, :j_end], g[:j_end])
        x = x + Z[:j_end].T @ y
        if hist[-1] <= rtol * beta0:
            break
    return x, it, hist


def newton_step_mg(levels, prob, x_old, t_new, tol=1e-10, maxit=20, gmres_rtol=1e-2,
                   restart=30, gmres_max=100, nu1=2, nu2=2, omega=0.6, smoother="additive", nu_coarse=0,
                   coarse=0):
    """Newton's method (eq. newton) with GMRES + V-cycle linear solves, as in
    the coarse solve of Algorithm 1 (full steps, reading N1)."""
    fine = levels[-1]
    x = fem.impose_bc(fine, prob, x_old, t_new)
    stats = dict(newton=0, gmres=[], res=[])
    for it in range(maxit + 1):
        R = fem.residual(fine, prob, x, x_old, t_new)
        nr = float(np.linalg.norm(R))
        stats["res"].append(nr)
        if nr <= tol:
            stats["newton"] = it
            return x, stats
        if it == maxit:
            break
        mg = MGHierarchy(levels, prob, x, nu1, nu2, omega, smoother, nu_coarse, coarse, x_old)
        w, k, _ = gmres(mg.J[-1], R, lambda v: mg.vcycle(len(levels) - 1, v),
                        gmres_rtol, restart, gmres_max)
        stats["gmres"].append(k)
        x = x + w
    raise RuntimeError(f"Newton-MG did not converge: {stats}")
