"""Oracle DNN-MG correction (Algorithm 1, the steps after the coarse solve; Sec. 2.2), FP64 numpy.

State of a DNN-MG simulation on coarse level L with fine level F = L + m:
x^L (the coarse iterate), the previous corrected fine velocity v^F_prev, the
GRU hidden states (one set per patch), and the pending coarse right-hand side
b^L for the next Newton solve.

One correction, after Newton on level L produced x^L_n (Algorithm 1):
  1. x~ = P^m x^L_n (prolongated velocity and pressure);
  2. r^F = f^F_n(v^F_prev) - A^F_n(x~) (the fine residual of eq.
     nonlinearshort), Dirichlet rows set to zero;
  3. per patch: inputs [v~1, v~2, p~, r1, r2, rp] at the patch's fine nodes
     (residual rows divided by the node's lumped mass) and 4 geometry
     features, standardised per channel (reading N5);
  4. the GRU stack and head give a velocity correction per patch node
     (velocity only);
  5. d = mean of the predictions of all patches containing a node, 0 on
     Dirichlet nodes (reading N6);
  6. b^F = Rhs(v~ + d) (the explicit velocity rows of f^F of eq. varformv),
     pressure rows 0 (the Rhs of Algorithm 1);
  7. b^L = (P^m)^T b^F (restriction, Algorithm 1); v^F_prev <- v~ + d.

Readings (paper silent): N4 patch = the 2x2 level-L cells of one level-(L-1)
cell, i.e. (2^(m+1) + 1)^2 fine nodes in the parent's lexicographic order;
N5 the four features are the patch aspect ratio (longest / shortest side),
|cos| of the angle between the patch mid-lines, h_P / mean_P h_P with
h_P = sqrt(area of the corner quadrilateral), and the patch Peclet number
max_P |v~| h_P / nu; channel standardisation x^ = (x - mu) / sigma with the
net's 10 (mu, sigma) pairs; the prediction is scaled by the net's 2 output
scales.

Cell patches (the patch of the paper's own experiments, Sec. 2.2: one
level-L element): (2^m + 1)^2 fine nodes; reading N16 inputs
[v~1, v~2, r1, r2, rp] at the nodes (the pressure enters through the
residual only) and six features, the four above plus cos 2phi and sin 2phi
of the angle phi of the left -> right mid-line; 11 (mu, sigma) pairs.  At
m = 1 this is I = 5 * 9 + 6 = 51 inputs and O = 18 outputs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fem, gru
from .mesh import Level

PATCH_BLOCK, PATCH_CELL = 0, 1


def patch_grid(levels, L: int, m: int, kind: int = PATCH_BLOCK) -> np.ndarray:
    """(P, S*S) fine-level node ids of every patch, lexicographic (i along
    the root cell's first edge, j along its last edge).  Block patches: the
    root is a level-(L-1) cell, S = 2^(m+1) + 1; cell patches: the root is a
    level-L cell, S = 2^m + 1."""
    # level-(L-1) cell c refined j times covers a (2^j + 1)^2 grid on level L-1+j
    def grid(lvl, j):
        # lvl: level whose cells are the roots; returns (C_lvl, 2^j+1, 2^j+1)
        if j == 1:
            pat = levels[lvl + 1].patches()          # (C_lvl, 9)
            return pat.reshape(-1, 3, 3)
        sub = grid(lvl + 1, j - 1)                   # children grids (4 C_lvl, s, s)
        s = sub.shape[1]
        n = 2 * (s - 1) + 1
        Cn = sub.shape[0] // 4
        out = np.empty((Cn, n, n), dtype=np.int64)
        sub = sub.reshape(Cn, 4, s, s)
        off = {0: (0, 0), 1: (s - 1, 0), 2: (s - 1, s - 1), 3: (0, s - 1)}
        for k, (ox, oy) in off.items():
            out[:, oy:oy + s, ox:ox + s] = sub[:, k]
        return out
    g = grid(L - 1, m + 1) if kind == PATCH_BLOCK else grid(L, m)
    return g.reshape(g.shape[0], -1)


def lumped_mass(level: Level) -> np.ndarray:
    det, _ = fem.geometry(level.xy, level.cells)
    w = np.einsum('cq,qa->ca', det, fem.NQ)
    m = np.zeros(level.n_nodes)
    np.add.at(m, level.cells, w)
    return m


def static_features(xyF, grid, S):
    """(P, 3) aspect ratio, mid-line skew and h_P (before normalisation by
    its mean), from the patch corner nodes."""
    c00, c10 = xyF[grid[:, 0]], xyF[grid[:, S - 1]]
    c01, c11 = xyF[grid[:, S * (S - 1)]], xyF[grid[:, S * S - 1]]
    sides = np.stack([np.linalg.norm(c10 - c00, axis=1), np.linalg.norm(c11 - c10, axis=1),
                      np.linalg.norm(c11 - c01, axis=1), np.linalg.norm(c01 - c00, axis=1)], 1)
    aspect = sides.max(1) / sides.min(1)
    a = 0.5 * (c10 + c11) - 0.5 * (c00 + c01)      # left -> right mid-line
    b = 0.5 * (c01 + c11) - 0.5 * (c00 + c10)      # bottom -> top mid-line
    skew = np.abs(np.sum(a * b, 1)) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
    quad = np.stack([c00, c10, c11, c01], 1)
    area = 0.5 * np.abs(np.sum(quad[:, :, 0] * np.roll(quad[:, :, 1], -1, 1)
                               - np.roll(quad[:, :, 0], -1, 1) * quad[:, :, 1], 1))
    h = np.sqrt(area)
    return aspect, skew, h


def orientation(xyF, grid, S):
    """(cos 2 phi, sin 2 phi) of the left -> right mid-line of each patch."""
    c00, c10 = xyF[grid[:, 0]], xyF[grid[:, S - 1]]
    c01, c11 = xyF[grid[:, S * (S - 1)]], xyF[grid[:, S * S - 1]]
    a = 0.5 * (c10 + c11) - 0.5 * (c00 + c01)
    phi = np.arctan2(a[:, 1], a[:, 0])
    return np.cos(2 * phi), np.sin(2 * phi)


def rhs_rows(level: Level, prob: fem.Problem, v):
    """(N, 2) explicit velocity rows of f_n (eq. varformv) for the velocity
    field v: 1/k (v, phi) - (1 - theta)((v.grad) v, phi)
    - (1 - theta) nu (grad v, grad phi), no external force."""
    det, grad = fem.geometry(level.xy, level.cells)
    X = v.reshape(-1, 3)[level.cells]
    th, nu, idt = prob.theta, prob.nu, prob.inv_dt
    vq = np.einsum('qa,caf->cqf', fem.NQ, X[:, :, :2])
    gv = np.einsum('cqad,caf->cqfd', grad, X[:, :, :2])
    conv = np.einsum('cqd,cqfd->cqf', vq, gv)
    ml = idt * vq - (1 - th) * conv
    f = np.einsum('cq,qa,cqf->caf', det, fem.NQ, ml)
    f -= np.einsum('cq,cqfd,cqad->caf', det, (1 - th) * nu * gv, grad)
    out = np.zeros((level.n_nodes, 2))
    np.add.at(out, level.cells, f)
    return out


@dataclass
class NetSpec:
    weights: np.ndarray      # flat, gru.unpack order
    hidden: int
    layers: int
    mu: np.ndarray           # channel means: nodal channels, then features
    sigma: np.ndarray        # channel scales (same order)
    out_scale: np.ndarray    # (2,) scale of the predicted u, v corrections


class DnnmgOracle:
    """Prolongation, fine residual, patch network and restricted rhs of
    Algorithm 1 for one geometry (levels 0..F)."""

    def __init__(self, levels, prob: fem.Problem, L: int, m: int, kind: int = PATCH_BLOCK):
        self.levels, self.prob, self.L, self.m, self.kind = levels, prob, L, m, kind
        self.F = L + m
        self.S = 2 ** (m + 1) + 1 if kind == PATCH_BLOCK else 2 ** m + 1
        self.n_ch = 6 if kind == PATCH_BLOCK else 5
        self.n_feat = 4 if kind == PATCH_BLOCK else 6
        self.grid = patch_grid(levels, L, m, kind)
        LF = levels[self.F]
        self.mass = lumped_mass(LF)
        self.aspect, self.skew, self.h = static_features(LF.xy, self.grid, self.S)
        self.c2, self.s2 = orientation(LF.xy, self.grid, self.S)
        self.hrel = self.h / self.h.mean()
        self.dir_f = LF.dirichlet_nodes()
        self.P = [None] + [levels[l].prolongation() for l in range(1, len(levels))]
        cnt = np.zeros(LF.n_nodes)
        np.add.at(cnt, self.grid.reshape(-1), 1.0)
        self.count = cnt

    @property
    def n_patches(self):
        return self.grid.shape[0]

    @property
    def n_in(self):
        return self.n_ch * self.S * self.S + self.n_feat

    @property
    def n_stats(self):
        return self.n_ch + self.n_feat

    @property
    def n_out(self):
        return 2 * self.S * self.S

    def prolong(self, x_coarse):
        x = x_coarse.reshape(-1, 3)
        for l in range(self.L + 1, self.F + 1):
            x = self.P[l] @ x
        return x.reshape(-1)

    def restrict(self, b_fine):
        b = b_fine.reshape(-1, 3)
        for l in range(self.F, self.L, -1):
            b = self.P[l].T @ b
        return b.reshape(-1)

    def inputs(self, xt, vprev, t):
        """Network input matrix (P, I) before standardisation, and r^F."""
        LF = self.levels[self.F]
        r = fem.residual(LF, self.prob, xt, vprev, t).reshape(-1, 3)
        r[self.dir_f, :2] = 0.0
        r = r / self.mass[:, None]
        X3 = xt.reshape(-1, 3)
        g = self.grid
        chans = [X3[g, 0], X3[g, 1], X3[g, 2], r[g, 0], r[g, 1], r[g, 2]]
        if self.kind == PATCH_CELL:
            del chans[2]                                # no prolongated pressure
        nodal = np.concatenate(chans, axis=1)
        speed = np.sqrt(X3[:, 0] ** 2 + X3[:, 1] ** 2)
        pe = speed[g].max(axis=1) * self.h / self.prob.nu
        feats = [self.aspect, self.skew, self.hrel, pe]
        if self.kind == PATCH_CELL:
            feats += [self.c2, self.s2]
        return np.concatenate([nodal, np.stack(feats, axis=1)], axis=1), r

    def standardise(self, X, net: NetSpec):
        n, c = self.S * self.S, self.n_ch
        mu = np.concatenate([np.repeat(net.mu[:c], n), net.mu[c:]])
        sg = np.concatenate([np.repeat(net.sigma[:c], n), net.sigma[c:]])
        return (X - mu) / sg

    def scatter(self, Y, net: NetSpec):
        """Mean over patches of the predicted (u, v) corrections, 0 on Dirichlet."""
        n = self.S * self.S
        LF = self.levels[self.F]
        d = np.zeros((LF.n_nodes, 2))
        for f in range(2):
            np.add.at(d[:, f], self.grid.reshape(-1), (Y[:, f * n:(f + 1) * n] * net.out_scale[f]).reshape(-1))
        d /= np.maximum(self.count, 1.0)[:, None]
        d[self.dir_f] = 0.0
        return d

    def rhs(self, v):
        """Explicit velocity rows of f^F (eq. varformv) for velocity v (no
        external force) on every fine node; pressure rows 0."""
        out = np.zeros((self.levels[self.F].n_nodes, 3))
        out[:, :2] = rhs_rows(self.levels[self.F], self.prob, v)
        return out.reshape(-1)

    def correct(self, x_coarse, vprev, h, net: NetSpec, t):
        """One correction.  Returns (b^L, v_corrected, h_new, extras)."""
        xt = self.prolong(x_coarse)
        Xraw, r = self.inputs(xt, vprev, t)
        Xn = self.standardise(Xraw, net)
        dims = (self.n_in, net.hidden, net.layers, self.n_out)
        Y, h_new = gru.forward(net.weights, Xn[None], dims, h0=h)
        d = self.scatter(Y[0], net)
        vc = xt.reshape(-1, 3).copy()
        vc[:, :2] += d
        vc[:, 2] = 0.0
        bF = self.rhs(vc.reshape(-1))
        bL = self.restrict(bF)
        return bL, vc.reshape(-1), h_new, dict(xt=xt, Xraw=Xraw, Xn=Xn, Y=Y[0], d=d, bF=bF)


def dnnmg_residual(levels, prob, L, x, x_old, bL, t_new):
    """Residual of Newton on level L when a DNN-MG right-hand side replaces
    f_n (the coarse solve of Algorithm 1 with b_L^n): R = b^L - A^L_impl(x), Dirichlet
    rows g - x.  A^L_impl is A_n without the old-state terms."""
    Lv = levels[L]
    z = np.zeros_like(x)
    # f(x_old=0) - A(x) = -A_impl(x) because every old-state term is linear
    # in x_old and vanishes for x_old = 0
    R = fem.residual(Lv, prob, x, z, t_new, x_conv=x_old).reshape(-1, 3)
    dn = Lv.dirichlet_nodes()
    Rb = bL.reshape(-1, 3)
    R[~dn, :2] += Rb[~dn, :2]
    R[:, 2] += Rb[:, 2]
    return R.reshape(-1)


def dnnmg_newton(levels, prob, L, x_old, bL, t_new, tol=1e-10, maxit=20):
    """Newton with direct solves for A^L_impl(x) = b^L (or the plain f^L(x_old)
    if bL is None), the coarse solve of Algorithm 1."""
    import scipy.sparse.linalg as spla
    from . import solver
    Lv = levels[L]
    if bL is None:
        return solver.newton_step(Lv, prob, x_old, t_new, tol=tol, maxit=maxit)
    x = fem.impose_bc(Lv, prob, x_old, t_new)
    for it in range(maxit + 1):
        R = dnnmg_residual(levels, prob, L, x, x_old, bL, t_new)
        if np.linalg.norm(R) <= tol:
            return x
        J = fem.jacobian(Lv, prob, x, x_old)
        x = x + spla.spsolve(J.tocsc(), R)
    raise RuntimeError("DNN-MG Newton did not converge")
