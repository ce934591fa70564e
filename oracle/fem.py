"""Oracle Q1/Q1 finite elements with local projection stabilisation (FP64).

The discrete problem of Sec. 2.1: at time step n find x_n = (v^1, v^2, p) with
A_n(x_n) = f_n (eq. nonlinearshort), where for every pressure test function
xi_i (eq. varform)

    [A_n(x)]_i = (div v, xi_i) + sum_T alpha_T (grad(p - pi p), grad(xi_i - pi xi_i))_T,
    [f_n]_i   = 0,

and for every velocity test function phi_i e_c (eq. varformv, Crank-Nicolson
with weight theta = 1/2, written for a general theta)

    [A_n(x)]  = 1/k (v, phi) + theta ((v.grad) v, phi) + theta nu (grad v, grad phi)
                - (p, div phi),
    [f_n]     = 1/k (v_old, phi) + theta (f_n, phi) + (1 - theta)(f_{n-1}, phi)
                - (1 - theta)((v_old.grad) v_old, phi) - (1 - theta) nu (grad v_old, grad phi).

The Jacobian A_n'(x) (eq. newton) is the analytic linearisation.

Readings (paper silent or garbled): G1 Q1/Q1 elements, 3 unknowns per vertex;
G2 p trial / xi test; G3 two-level projection: on each patch of 2x2 sibling
cells pi is bilinear interpolation from the 4 patch corners in the parent's
reference coordinates; G4 alpha_T = alpha0 * Re * h_T^2 as in Sec. 2.1, with
Re read as 1/nu, h_T^2 = area(T) and the free constant alpha0 = 0.5
(`lps_mode="paper"`, the default).  The re-discretised coarse operators of the
multigrid preconditioner (solver.MGHierarchy) use the bounded form
alpha0 / (nu / h_T^2 + 1/k) (`lps_mode="bounded"`); they do not change the
discrete solution, only how fast the linear solves converge; G6 theta = 1/2, pressure fully implicit; G7 inflow U(y,t) = 6 s(t) y (H - y) / H^2
with ramp s(t) = (1 - cos(pi t)) / 2 for t < 1, else 1, no-slip walls and
obstacle, do-nothing outflow (no boundary term); G8 2x2 Gauss quadrature.

Unknowns are interleaved: dof 3 i + f for node i, field f (0 = u, 1 = v, 2 = p).
Dirichlet velocity rows hold R = g - x in the residual and identity rows in the
Jacobian.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

from .mesh import CHILD_TO_PATCH, Level

CHANNEL_H = 0.41

_G = 1.0 / np.sqrt(3.0)
QXI = np.array([-_G, _G, _G, -_G])
QETA = np.array([-_G, -_G, _G, _G])
VXI = np.array([-1.0, 1.0, 1.0, -1.0])
VETA = np.array([-1.0, -1.0, 1.0, 1.0])
# basis values / reference derivatives at the 4 Gauss points: [q, a]
NQ = 0.25 * (1 + np.outer(QXI, VXI)) * (1 + np.outer(QETA, VETA))
DXI = 0.25 * VXI[None, :] * (1 + np.outer(QETA, VETA))
DETA = 0.25 * VETA[None, :] * (1 + np.outer(QXI, VXI))


def fluctuation_matrix() -> np.ndarray:
    """K = I - I_2h on a patch (reading G3): kappa q = K q with patch nodes in
    lexicographic order; corners have zero fluctuation, edge nodes subtract the
    mean of their two corners, the centre the mean of all four."""
    K = np.eye(9)
    for q, (a, b) in {1: (0, 2), 3: (0, 6), 5: (2, 8), 7: (6, 8)}.items():
        K[q, a] -= 0.5
        K[q, b] -= 0.5
    for a in (0, 2, 6, 8):
        K[4, a] -= 0.25
        K[a, a] = 0.0
    return K


@dataclass
class Problem:
    nu: float
    dt: float                       # time step k (np.inf: steady problem)
    theta: float = 0.5
    alpha0: float = 0.5
    H: float = CHANNEL_H
    u_mean: float = 1.0
    lps_mode: str = "paper"                 # "paper": alpha0 h^2/nu; "bounded": alpha0/(nu/h^2 + 1/k)
    delta0: float = 0.0                     # convective stabilisation scale (0: off, the paper's method)
    force: Optional[Callable] = None        # f(x, y, t) -> (fx, fy)
    dirichlet: Optional[Callable] = None    # g(x, y, t) -> (u, v) on Dirichlet nodes

    @property
    def inv_dt(self):
        return 0.0 if np.isinf(self.dt) else 1.0 / self.dt


def ramp(t):
    return 0.5 * (1.0 - np.cos(np.pi * t)) if t < 1.0 else 1.0


def dirichlet_values(level: Level, prob: Problem, t: float) -> np.ndarray:
    """(N, 2) velocity values on Dirichlet nodes (reading G7); zero elsewhere."""
    g = np.zeros((level.n_nodes, 2))
    dn = level.dirichlet_nodes()
    if prob.dirichlet is not None:
        gx, gy = prob.dirichlet(level.xy[:, 0], level.xy[:, 1], t)
        g[:, 0] = np.where(dn, gx, 0.0)
        g[:, 1] = np.where(dn, gy, 0.0)
        return g
    inn = level.inflow_nodes()
    y = level.xy[:, 1]
    H = prob.H
    g[inn, 0] = 6.0 * prob.u_mean * ramp(t) * y[inn] * (H - y[inn]) / H ** 2
    return g


def impose_bc(level: Level, prob: Problem, x: np.ndarray, t: float) -> np.ndarray:
    x = x.copy().reshape(-1, 3)
    dn = level.dirichlet_nodes()
    g = dirichlet_values(level, prob, t)
    x[dn, :2] = g[dn]
    return x.reshape(-1)


def geometry(xy, cells):
    """Per cell and Gauss point: w*det(J) (C, 4) and physical basis gradients
    (C, 4q, 4a, 2)."""
    X = xy[cells]                                        # (C, 4, 2)
    j11 = np.einsum('qa,ca->cq', DXI, X[:, :, 0])        # dx/dxi
    j12 = np.einsum('qa,ca->cq', DETA, X[:, :, 0])       # dx/deta
    j21 = np.einsum('qa,ca->cq', DXI, X[:, :, 1])        # dy/dxi
    j22 = np.einsum('qa,ca->cq', DETA, X[:, :, 1])       # dy/deta
    det = j11 * j22 - j12 * j21
    # grad N = J^{-T} (dN/dxi, dN/deta)
    gx = (j22[:, :, None] * DXI[None] - j21[:, :, None] * DETA[None]) / det[:, :, None]
    gy = (-j12[:, :, None] * DXI[None] + j11[:, :, None] * DETA[None]) / det[:, :, None]
    return det, np.stack([gx, gy], axis=-1)


def lps_alpha(prob: "Problem", area):
    """alpha_T per cell with h_T^2 = area(T) (Sec. 2.1, reading G4).
    "paper": alpha0 * Re * h_T^2 = alpha0 * h_T^2 / nu, the stabilisation of
    the discrete problem.  "bounded": alpha0 / (nu / h_T^2 + 1/k), which equals
    the paper's value where h_T^2 / nu << k and is at most alpha0 * k; used
    only for the coarse operators of the multigrid preconditioner."""
    if prob.lps_mode == "paper":
        return prob.alpha0 * area / prob.nu
    if prob.lps_mode == "bounded":
        return prob.alpha0 / (prob.nu / area + prob.inv_dt)
    raise ValueError(f"unknown lps_mode {prob.lps_mode!r}")


def coarse_operator_problem(prob: "Problem") -> "Problem":
    """The problem whose Jacobian a multigrid preconditioner re-discretises on
    the levels below the one it solves on: the bounded LPS parameter."""
    return replace(prob, lps_mode="bounded")


def _lps_patch_matrices(level: Level, prob: Problem, det, grad):
    """(P, 9, 9) patch matrices s_P = K^T (sum_T alpha_T S_T) K of the LPS term."""
    area = det.sum(axis=1)                               # 2x2 Gauss, weights 1
    alpha = lps_alpha(prob, area)
    S = np.einsum('cq,cqad,cqbd->cab', det, grad, grad)  # cell stiffness (C, 4, 4)
    S *= alpha[:, None, None]
    P = level.n_cells // 4
    SP = np.zeros((P, 9, 9))
    S4 = S.reshape(P, 4, 4, 4)
    for k in range(4):
        idx = CHILD_TO_PATCH[k]
        SP[:, idx[:, None], idx[None, :]] += S4[:, k]
    K = fluctuation_matrix()
    return np.einsum('mi,pmn,nj->pij', K, SP, K)


def convective_matrices(level: Level, prob: Problem, x_old: np.ndarray) -> np.ndarray:
    """(C, 4, 4) cell matrices of the convective stabilisation (an optional
    member of the local-projection family of Sec. 2.1, off unless delta0 > 0):

        s_T(v, phi) = delta_T (kappa_T(b_T . grad v), kappa_T(b_T . grad phi))_T,

    kappa_T g = g - (mean of g over T), b_T the mean of the old velocity over
    the cell's 4 nodes (frozen: the term is linear in v, its Jacobian exact),
    delta_T = delta0 / (nu / h_T^2 + |b_T| / h_T), h_T^2 = area(T), 2x2 Gauss.
    Entry [c, a, b] multiplies the component's value at node b in the row of
    node a; the same matrix acts on u and on v."""
    det, grad = geometry(level.xy, level.cells)
    Vo = x_old.reshape(-1, 3)[level.cells][:, :, :2]            # (C, 4, 2)
    bT = Vo.mean(axis=1)                                          # (C, 2)
    area = det.sum(axis=1)
    h = np.sqrt(area)
    bn = np.linalg.norm(bT, axis=1)
    delta = prob.delta0 / (prob.nu / area + bn / h)
    psi = np.einsum('cd,cqad->cqa', bT, grad)                     # b . grad N_a at each point
    mean = np.einsum('cq,cqa->ca', det, psi) / area[:, None]
    kpsi = psi - mean[:, None, :]
    return delta[:, None, None] * np.einsum('cq,cqa,cqb->cab', det, kpsi, kpsi)


def _forcing(level, prob, t_new):
    C = level.n_cells
    if prob.force is None:
        return np.zeros((C, 4, 2))
    X = level.xy[level.cells]
    qx = np.einsum('qa,ca->cq', NQ, X[:, :, 0])
    qy = np.einsum('qa,ca->cq', NQ, X[:, :, 1])
    fn = np.stack(prob.force(qx, qy, t_new), axis=-1)
    fo = np.stack(prob.force(qx, qy, t_new - (0 if np.isinf(prob.dt) else prob.dt)), axis=-1)
    return prob.theta * fn + (1 - prob.theta) * fo


def residual(level: Level, prob: Problem, x: np.ndarray, x_old: np.ndarray,
             t_new: float, x_conv: Optional[np.ndarray] = None) -> np.ndarray:
    """R = f_n - A_n(x) (eqs. varform, varformv); Dirichlet velocity rows hold
    g(t_new) - x.  With delta0 > 0 the convective stabilisation's frozen field
    comes from x_conv (x_old if not given)."""
    cells = level.cells
    det, grad = geometry(level.xy, cells)
    X = x.reshape(-1, 3)[cells]                          # (C, 4a, 3)
    Xo = x_old.reshape(-1, 3)[cells]
    th, nu, idt = prob.theta, prob.nu, prob.inv_dt
    v = np.einsum('qa,caf->cqf', NQ, X[:, :, :2])        # (C, q, 2)
    vo = np.einsum('qa,caf->cqf', NQ, Xo[:, :, :2])
    p = np.einsum('qa,ca->cq', NQ, X[:, :, 2])
    gv = np.einsum('cqad,caf->cqfd', grad, X[:, :, :2])  # d v_f / d x_d
    gvo = np.einsum('cqad,caf->cqfd', grad, Xo[:, :, :2])
    conv = np.einsum('cqd,cqfd->cqf', v, gv)
    convo = np.einsum('cqd,cqfd->cqf', vo, gvo)
    fbar = _forcing(level, prob, t_new)
    # velocity rows, integrand multiplying N_a and grad N_a
    mass_like = idt * (v - vo) + th * conv + (1 - th) * convo - fbar       # (C, q, f)
    Av = np.einsum('cq,qa,cqf->caf', det, NQ, mass_like)
    Av += np.einsum('cq,cqfd,cqad->caf', det, nu * (th * gv + (1 - th) * gvo), grad)
    Av -= np.einsum('cq,cq,cqaf->caf', det, p, grad)
    div = gv[:, :, 0, 0] + gv[:, :, 1, 1]
    Ap = np.einsum('cq,qa,cq->ca', det, NQ, div)
    Ael = np.concatenate([Av, Ap[:, :, None]], axis=2)  # (C, 4, 3)
    A = np.zeros((level.n_nodes, 3))
    np.add.at(A, cells, Ael)
    sP = _lps_patch_matrices(level, prob, det, grad)
    pat = level.patches()
    pp = x.reshape(-1, 3)[pat, 2]                        # (P, 9)
    np.add.at(A[:, 2], pat, np.einsum('pij,pj->pi', sP, pp))
    if prob.delta0 > 0:
        Sc = convective_matrices(level, prob, x_old if x_conv is None else x_conv)
        sc = np.einsum('cab,cbf->caf', Sc, X[:, :, :2])
        np.add.at(A[:, :2], cells, sc)
    R = -A
    dn = level.dirichlet_nodes()
    g = dirichlet_values(level, prob, t_new)
    xr = x.reshape(-1, 3)
    R[dn, :2] = g[dn] - xr[dn, :2]
    return R.reshape(-1)


def jacobian(level: Level, prob: Problem, x: np.ndarray, x_old: Optional[np.ndarray] = None) -> sp.csr_matrix:
    """Analytic Jacobian A_n'(x) (eq. newton), as a CSR matrix on interleaved dofs.
    Dirichlet velocity rows are identity rows.  With delta0 > 0 the convective
    stabilisation's frozen field comes from x_old (x itself if not given)."""
    cells = level.cells
    C = level.n_cells
    det, grad = geometry(level.xy, cells)
    X = x.reshape(-1, 3)[cells]
    th, nu, idt = prob.theta, prob.nu, prob.inv_dt
    v = np.einsum('qa,caf->cqf', NQ, X[:, :, :2])
    gv = np.einsum('cqad,caf->cqfd', grad, X[:, :, :2])
    Je = np.zeros((C, 4, 3, 4, 3))
    mass = np.einsum('cq,qa,qb->cab', det, NQ, NQ)
    vgradNb = np.einsum('cqd,cqbd->cqb', v, grad)
    adv = np.einsum('cq,qa,cqb->cab', det, NQ, vgradNb)
    lap = np.einsum('cq,cqad,cqbd->cab', det, grad, grad)
    diag = idt * mass + th * adv + th * nu * lap
    for f in range(2):
        Je[:, :, f, :, f] += diag
        for d in range(2):
            # theta (N_b dv_f/dx_d) N_a  for column (b, d)
            Je[:, :, f, :, d] += th * np.einsum('cq,qa,qb,cq->cab', det, NQ, NQ, gv[:, :, f, d])
        Je[:, :, f, :, 2] -= np.einsum('cq,qb,cqa->cab', det, NQ, grad[:, :, :, f])
        Je[:, :, 2, :, f] += np.einsum('cq,qa,cqb->cab', det, NQ, grad[:, :, :, f])
    dof = (3 * cells[:, :, None] + np.arange(3)[None, None, :]).reshape(C, 12)
    if prob.delta0 > 0:
        Sc = convective_matrices(level, prob, x if x_old is None else x_old)
        for f in range(2):
            Je[:, :, f, :, f] += Sc
    Je = Je.reshape(C, 12, 12)
    rows = np.repeat(dof, 12, axis=1).reshape(-1)
    cols = np.tile(dof, (1, 12)).reshape(-1)
    vals = Je.reshape(-1)
    sP = _lps_patch_matrices(level, prob, det, grad)
    pat = level.patches()
    pr = np.repeat(3 * pat + 2, 9, axis=1).reshape(-1)
    pc = np.tile(3 * pat + 2, (1, 9)).reshape(-1)
    n = 3 * level.n_nodes
    Jm = sp.coo_matrix((np.concatenate([vals, sP.reshape(-1)]),
                        (np.concatenate([rows, pr]), np.concatenate([cols, pc]))),
                       shape=(n, n)).tocsr()
    Jm.sum_duplicates()
    dn = np.nonzero(level.dirichlet_nodes())[0]
    drows = np.concatenate([3 * dn, 3 * dn + 1])
    keep = np.ones(n)
    keep[drows] = 0.0
    Jm = sp.diags(keep) @ Jm
    Jm = Jm + sp.csr_matrix((np.ones(drows.size), (drows, drows)), shape=(n, n))
    Jm = Jm.tocsr()
    Jm.sum_duplicates()
    return Jm


def mass_matrix(level: Level) -> sp.csr_matrix:
    """Scalar Q1 mass matrix (2x2 Gauss), used for L2 norms (reading N13)."""
    det, _ = geometry(level.xy, level.cells)
    Me = np.einsum('cq,qa,qb->cab', det, NQ, NQ)
    C = level.n_cells
    rows = np.repeat(level.cells, 4, axis=1).reshape(-1)
    cols = np.tile(level.cells, (1, 4)).reshape(-1)
    return sp.coo_matrix((Me.reshape(-1), (rows, cols)),
                         shape=(level.n_nodes, level.n_nodes)).tocsr()
