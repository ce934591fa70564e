/*
 * dnnmg.h -- C-ABI of the MI355X (gfx950) DNN-MG hot path.
 *
 * The library advances the discrete incompressible Navier-Stokes system of
 * Sec. 2.1 of "Deep neural networks for geometric multigrid methods"
 * (Q1/Q1 finite elements with local projection stabilisation, Crank-Nicolson
 * in time, eqs. nonlinearshort, varform, varformv) by Newton's method
 * (eq. newton) whose linear systems are solved by GMRES preconditioned with a
 * geometric multigrid V-cycle (Sec. 2.2), and applies the DNN-MG correction
 * of Algorithm 1 (prolongation, patch-wise recurrent network, right-hand side
 * on the fine level, restriction).
 *
 * Conventions shared by all calls
 *   - Status: every call returns 0 (DNNMG_OK) or a negative DNNMG_E* code.
 *     Arguments are validated before any device work; on error the message
 *     is available from dnnmg_last_error().  No C++ exception or abort
 *     crosses this boundary.
 *   - Nodal vectors are interleaved: 3 doubles per node, (u, v, p), in the
 *     library's node numbering of that level (dnnmg_level_coords gives the
 *     coordinates).  Node numbering of a refinement: old vertices keep their
 *     ids, then one node per edge in order of first appearance over the
 *     cells, then one node per cell; cell c has children 4c..4c+3.
 *   - Host pointers are borrowed for the duration of the call and copied.
 *     Device pointers (the *_dev calls) are borrowed for the call only.
 *   - The context owns every device allocation it makes (hipMalloc); states
 *     and networks belong to their context and must be destroyed before it.
 *   - Work is enqueued on params.stream (NULL: the default stream).  Calls
 *     that return host data or statistics synchronise that stream.
 */
#ifndef DNNMG_H
#define DNNMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DNNMG_OK 0
#define DNNMG_EINVAL (-1)   /* bad argument (checked before device work)      */
#define DNNMG_ENOMEM (-2)   /* device or host allocation failed               */
#define DNNMG_EDEVICE (-3)  /* a HIP runtime call or kernel launch failed     */
#define DNNMG_ENOCONV (-4)  /* Newton or GMRES did not converge; state rolled back */
#define DNNMG_ESTATE (-5)   /* call out of order (e.g. no mesh set up yet)    */

typedef struct dnnmg_ctx dnnmg_ctx;
typedef struct dnnmg_state dnnmg_state;
typedef struct dnnmg_net dnnmg_net;
typedef struct dnnmg_batch dnnmg_batch;

/* Solver parameters.  Defaults (dnnmg_params_default) follow the readings of
 * the paper's unstated constants: theta = 1/2 (Crank-Nicolson, Sec. 2.1),
 * LPS parameter alpha_T = alpha0 Re h_T^2 (Sec. 2.1; Re = 1/nu, h_T^2 the
 * cell area) with alpha0 = 0.5 on the level whose discrete problem is solved
 * (and in every residual); the re-discretised coarser levels of its multigrid
 * preconditioner use alpha0 / (nu / h_T^2 + 1/k), which changes how fast the
 * linear solves converge, not the solution,
 * Newton with full steps and absolute tolerance 1e-10 on the l2 norm of the
 * nonlinear residual, started from the linear extrapolation of the last two
 * states, GMRES(30) with relative tolerance 1e-2 and at most 100 iterations,
 * V(2,2) cycles with additive cell-Vanka (omega = 0.6); graphs, autotuning. */
typedef struct {
  double nu;              /* kinematic viscosity (the paper's 1/Re)              */
  double alpha0;          /* LPS scale alpha0 of alpha_T = alpha0 h_T^2 / nu      */
  double theta;           /* time-stepping weight, 0.5 = Crank-Nicolson          */
  double u_mean;          /* mean inflow velocity of the parabolic profile       */
  double channel_h;       /* channel height H of the inflow profile              */
  double newton_tol;      /* absolute l2 tolerance on R = f - A(x)               */
  int newton_max;         /* maximum Newton iterations per step                 */
  double gmres_rtol;      /* relative GMRES tolerance                           */
  int gmres_restart;      /* Krylov dimension before restart (<= 64)            */
  int gmres_max;          /* maximum GMRES iterations per Newton step           */
  int nu_pre, nu_post;    /* Vanka sweeps before / after the coarse correction */
  double vanka_omega;     /* damping of the additive Vanka update               */
  int precision;          /* 0: FP64 throughout; 1: mixed (FP32 smoother,
                             transfers, Krylov vectors; FP64 residual, Newton
                             update, coarse solve and Gram-Schmidt dots)        */
  int use_graphs;         /* 1: replay V-cycles and the level-0 Gauss-Jordan
                             sweep from HIP graphs captured on first use (same
                             kernels, same order, bitwise the same results);
                             0: launch every kernel directly                    */
  int autotune;           /* 1: at mesh setup, time the SpMV (one and four
                             threads per row), Vanka and transfer kernels of
                             every level at workgroup sizes 64, 128 and 256,
                             the fused residual + Vanka apply against the
                             separate kernels, a coarse level's last update
                             fused into the prolongation against the two
                             launches, and the bottom of the V-cycle
                             (levels <= 2 and the coarse solve) in a single
                             workgroup against its launches, and keep the
                             fastest (scheduling only: results are bitwise the
                             same); 0: 256 throughout, separate kernels, one
                             thread per row; 2: as 0 with the fused apply
                             (sixteen lanes per cell), four threads per
                             SpMV row, the fused update + prolongation,
                             four cells per thread in the FP32 Vanka apply
                             and the update in cell order on every level;
                             3: as 0 with the single-workgroup bottom cycle  */
  int newton_predictor;   /* 0: Newton starts from x_{n-1}; 1: from the linear
                             extrapolation x_{n-1} + (k_n/k_{n-1})(x_{n-1} -
                             x_{n-2}) once a state has taken a step (the
                             converged x_n is the same to the tolerance)      */
  int jacobian_reuse;     /* 0: every step rebuilds the multigrid hierarchy at
                             its first Newton iterate and re-assembles the
                             finest Jacobian at later ones; 1: Newton keeps the
                             Jacobians, Vanka inverses and level-0 inverse it
                             last built for the same state, level and time step
                             (across iterations and steps) while the residual
                             contracts by reuse_contraction or better per
                             iteration, and rebuilds everything at the current
                             iterate otherwise; a step that fails with a kept
                             hierarchy is redone with fresh ones (the converged
                             x_n is the same to the tolerance)               */
  double reuse_contraction; /* largest ||R_k|| / ||R_{k-1}|| that keeps a
                             Jacobian, in (0, 1); default 0.1                 */
  int switch_off_newton;  /* DNN-MG switch-off (Sec. 3.3): a step with a pending
                             network right-hand side whose Newton iteration has
                             not converged after this many iterations is redone
                             with the plain right-hand side (stats.fallback =
                             1); 0: only when Newton fails (newton_max)      */
  int nu_coarse;          /* 0: every level of a V-cycle takes nu_pre / nu_post
                             sweeps; k in 1..8: the levels below the one the
                             cycle is called on take k sweeps before and k
                             after (the level the Krylov solver works on keeps
                             nu_pre / nu_post)                                */
  int smoother;           /* 0: additive cell-Vanka (every cell's correction,
                             averaged over the cells of a node, omega times);
                             1: coloured multiplicative cell-Vanka (greedy cell
                             colouring in cell order, no two cells of a colour
                             share a node; per colour the residual is
                             recomputed and each cell of the colour adds omega
                             times its correction); same vanka_omega          */
  int coarse_level;       /* level of the direct solve at the bottom of every
                             V-cycle (FP64 dense inverse of its Jacobian, built
                             with each hierarchy); 0: the level-0 mesh, k > 0:
                             levels below k are not used by the solver, and
                             a solve on a level below k is DNNMG_EINVAL.  Fixed
                             at creation, at most 2, and 0 for batches        */
  void *stream;           /* hipStream_t, or NULL for the default stream       */
  double delta0;          /* convective stabilisation (an optional member of the
                             local-projection family of Sec. 2.1; the paper's
                             method has none): 0 (default) off; > 0 adds
                             delta_T (kappa_T(b.grad v), kappa_T(b.grad phi))_T
                             to both velocity rows of A_n, kappa_T g = g minus
                             its mean over cell T, b the mean of the old
                             velocity over the cell's nodes (frozen, so the
                             Jacobian is exact), delta_T = delta0 / (nu / h_T^2
                             + |b| / h_T), h_T^2 = area(T); every level uses it
                             (dnnmg_linearize takes the state's own velocity
                             as b)                                            */
} dnnmg_params;

/* Macro (coarsest) mesh.  Level 0 is this mesh refined once; finer levels are
 * uniform refinements.  quad: 4 counter-clockwise vertex ids per cell.
 * bedge: (v0, v1, tag) per boundary edge, tag 1 inflow, 2 wall, 3 outflow,
 * 4 + k boundary of obstacle k.  curve: (cx, cy, a, b, phi) per obstacle, an
 * ellipse onto which new boundary midpoints of tag 4 + k are projected. */
typedef struct {
  int n_vert;
  const double *xy;       /* 2 * n_vert */
  int n_cell;
  const int *quad;        /* 4 * n_cell */
  int n_bedge;
  const int *bedge;       /* 3 * n_bedge */
  int n_curve;
  const double *curve;    /* 5 * n_curve */
} dnnmg_coarse_mesh;

typedef struct {
  int newton_iters;       /* Newton iterations taken                            */
  int gmres_iters;        /* total GMRES iterations over all Newton iterations  */
  int gmres_iters_max;    /* largest GMRES count of a single Newton iteration  */
  double res_initial;     /* ||R|| at the first Newton iterate                  */
  double res_final;       /* ||R|| at the returned state                        */
  int converged;          /* 1 if ||R|| <= newton_tol                           */
  int fallback;           /* DNN-MG: 1 if the correction was switched off       */
  int jacobian_builds;    /* multigrid hierarchies (all levels' Jacobians,
                             Vanka and level-0 inverses) built in this step  */
} dnnmg_step_stats;

typedef struct {
  int iters;              /* GMRES iterations                                   */
  double res0;            /* ||rhs||                                            */
  double res;             /* final GMRES residual estimate                      */
} dnnmg_solve_stats;

/* Fills *p with the defaults listed above (nu = 1e-3, u_mean = 1, H = 0.41,
 * precision = 1, stream = NULL). */
int dnnmg_params_default(dnnmg_params *p);

/* Creates a context; the device is the current HIP device. */
int dnnmg_create(const dnnmg_params *p, dnnmg_ctx **out);
int dnnmg_destroy(dnnmg_ctx *ctx);
/* Message of the last failed call on this context ("" if none). */
const char *dnnmg_last_error(const dnnmg_ctx *ctx);
/* Replaces nu, alpha0, theta, tolerances, omega and the stream; precision and
 * coarse_level are fixed at creation (a different value is DNNMG_EINVAL).  Returns DNNMG_EINVAL for out-of-range values. */
int dnnmg_set_params(dnnmg_ctx *ctx, const dnnmg_params *p);

/* Mesh hierarchy setup (once): refines the macro mesh to levels
 * 0..finest_level (Sec. 2.2 multigrid hierarchy; patches of 2x2 sibling
 * cells, Sec. 2.1 LPS and Sec. 2.2 network patches), projecting new midpoints
 * of obstacle edges onto the obstacle curve, and uploads all tables.
 * finest_level in [0, 9]. */
int dnnmg_setup_mesh(dnnmg_ctx *ctx, const dnnmg_coarse_mesh *macro, int finest_level);
int dnnmg_level_info(const dnnmg_ctx *ctx, int level, int *n_nodes, int *n_cells,
                     int *n_patches);
/* Host copies of a level's node coordinates (2 * n_nodes doubles) and cells
 * (4 * n_cells ints). */
int dnnmg_level_coords(const dnnmg_ctx *ctx, int level, double *xy);
int dnnmg_level_cells(const dnnmg_ctx *ctx, int level, int *quads);

/* Solver state on one level: x (3 doubles per node, device-resident) and its
 * time t.  Created as zero at t = 0. */
int dnnmg_state_create(dnnmg_ctx *ctx, int level, dnnmg_state **out);
int dnnmg_state_destroy(dnnmg_state *s);
int dnnmg_state_set(dnnmg_state *s, const double *uvp, double t);
int dnnmg_state_get(const dnnmg_state *s, double *uvp, double *t);
/* Device-to-device copy of the state's vector (3 doubles per node) into
 * caller-owned device memory, enqueued on the context's stream (no
 * synchronisation; the copy is ordered before later work on that stream). */
int dnnmg_state_get_dev(const dnnmg_state *s, double *uvp_dev);
/* Device address of the state's vector (owned by the state). */
int dnnmg_state_device_ptr(dnnmg_state *s, double **uvp_dev);

/* One time step t -> t + dt of the plain method on the state's level
 * (the coarse solve of Algorithm 1): Newton (eq. newton) from x^(0) = x_{n-1} with the
 * Dirichlet values of t + dt imposed; each Newton system solved by GMRES with
 * one multigrid V-cycle per preconditioner application.  If the state holds a
 * pending DNN-MG right-hand side (set by dnnmg_correct) it replaces f_n
 * (Algorithm 1 with b_L^n).  On DNNMG_ENOCONV the state is restored
 * to its value before the call. */
int dnnmg_step(dnnmg_ctx *ctx, dnnmg_state *s, double dt, dnnmg_step_stats *stats);

/* Assembles the Jacobian A'(x) (eq. newton) on levels 0..level at the state
 * x (injected to coarser levels: their nodes are a prefix of the fine
 * numbering), factorises the Vanka blocks and the level-0 LU.  dt enters
 * through the mass term 1/k and the bounded alpha_T of the levels below
 * `level`. */
int dnnmg_linearize(dnnmg_ctx *ctx, const dnnmg_state *s, int level, double dt);
/* Solves A'(x) w = rhs on `level` with the operators of the last
 * dnnmg_linearize by GMRES + V-cycle; host in/out, 3 doubles per node. */
int dnnmg_solve(dnnmg_ctx *ctx, int level, const double *rhs, double *w,
                dnnmg_solve_stats *stats);

/* Single-operation entry points used for parity checks (host in/out).
 * Nonlinear residual R = f_n - A_n(x) (eqs. varform, varformv), Dirichlet
 * velocity rows g(t_new) - x. */
int dnnmg_residual(dnnmg_ctx *ctx, int level, const double *x, const double *x_old,
                   double t_new, double dt, double *r);
/* y = A'(x) w with the operator of the last dnnmg_linearize on `level`. */
int dnnmg_jacobian_apply(dnnmg_ctx *ctx, int level, const double *w, double *y);
/* One additive cell-Vanka sweep on `level` (operator of the last linearize). */
int dnnmg_vanka_sweep(dnnmg_ctx *ctx, int level, const double *x, const double *b,
                      double *x_out);
/* One V(nu_pre, nu_post)-cycle on `level` from a zero initial guess. */
int dnnmg_vcycle(dnnmg_ctx *ctx, int level, const double *b, double *x);
/* Prolongation level-1 -> level (bilinear in parent coordinates) and
 * restriction level -> level-1 (its transpose, Dirichlet rows zeroed). */
int dnnmg_prolong(dnnmg_ctx *ctx, int level, const double *coarse, double *fine);
int dnnmg_restrict(dnnmg_ctx *ctx, int level, const double *fine, double *coarse);

/* ---------------------------------------------------------------- DNN-MG
 * Patch network of Sec. 2.2 / Sec. 3.1: a stack of bias-free GRU cells with
 * hidden size `hidden` and `layers` layers followed by a bias-free dense head
 * (the structure whose parameter count 3H(I+H) + 6H^2(n-1) + HO reproduces
 * Table 1).  Patches are the 2x2 level-L cells of one level-(L-1) cell; the
 * network corrects the velocity on level F = L + m_levels, so a patch has
 * S x S fine nodes with S = 2^(m_levels+1) + 1, input size
 * I = 6 S^2 + 4 ([u, v, p, r_u, r_v, r_p] at the patch nodes, channel-major,
 * then aspect ratio, mid-line skew, h_P / mean h_P and the patch Peclet
 * number) and output size O = 2 S^2 (u then v corrections).
 * Requires coarse_level >= 1 and coarse_level + m_levels <= finest level;
 * hidden a multiple of 32.  Weights start at zero. */
int dnnmg_net_create(dnnmg_ctx *ctx, int coarse_level, int m_levels, int hidden, int layers,
                     dnnmg_net **out);

#define DNNMG_PATCH_BLOCK 0   /* the 2x2 level-L cells of one level-(L-1) cell  */
#define DNNMG_PATCH_CELL 1    /* one level-L cell                                */
/* As dnnmg_net_create with a choice of patch.  DNNMG_PATCH_CELL is the patch
 * of the paper's own experiments (Sec. 2.2: a mesh element on level L): S =
 * 2^m_levels + 1 fine nodes per side, input size I = 5 S^2 + 6 ([u, v, r_u,
 * r_v, r_p] at the patch nodes, channel-major: the pressure enters through
 * the residual only; then aspect ratio, mid-line skew, h_P / mean h_P, the
 * Peclet number, cos 2phi and sin 2phi of the angle phi of the left -> right
 * mid-line), O = 2 S^2; with m_levels = 1, I = 51 and O = 18 (Table 1);
 * coarse_level >= 0.  DNNMG_PATCH_BLOCK is dnnmg_net_create. */
int dnnmg_net_create_patch(dnnmg_ctx *ctx, int coarse_level, int m_levels, int hidden, int layers,
                           int patch, dnnmg_net **out);
int dnnmg_net_destroy(dnnmg_net *net);
int dnnmg_net_info(const dnnmg_net *net, int *n_in, int *n_out, int *n_patches,
                   long long *n_params);
/* Patch kind, fine nodes per patch side S and the number of standardisation
 * pairs (10 for block patches, 11 for cell patches); NULL outputs skipped. */
int dnnmg_net_patch_info(const dnnmg_net *net, int *patch, int *nodes_per_side, int *n_stats);
/* Host FP32 weights in the order: per layer W_ih (3H x I_l, gate rows r, z, n)
 * then W_hh (3H x H); then W_out (O x H), all row-major.  mu / sigma: the
 * standardisation pairs, nodal channels then features (10 for block
 * patches: 6 + 4; 11 for cell patches: 5 + 6), x^ = (x - mu) / sigma;
 * out_scale: scales of the predicted u and v.  NULL leaves a part
 * unchanged.  The device keeps FP32 masters and BF16 working copies. */
int dnnmg_net_set_weights(dnnmg_net *net, const float *w, const float *mu, const float *sigma,
                          const float *out_scale);
int dnnmg_net_get_weights(const dnnmg_net *net, float *w);
/* Starts a DNN-MG simulation from the coarse state: GRU hidden states 0 and
 * the stored previous fine velocity v_prev = P^m x (coarse). */
int dnnmg_net_reset(dnnmg_net *net, const dnnmg_state *coarse);
/* One GRU time step of all patches on host inputs X (n_patches x n_in,
 * already standardised); writes Y (n_patches x n_out) and advances the
 * hidden states (BF16 MFMA GEMMs, FP32 accumulation and gates). */
int dnnmg_net_forward(dnnmg_net *net, const float *X, float *Y);

/* Optional host copies of the intermediate results of dnnmg_correct. */
typedef struct {
  float *inputs;          /* n_patches x n_in standardised inputs (FP32)     */
  float *outputs;         /* n_patches x n_out network outputs               */
  double *correction;     /* 2 x N_F scatter-averaged (u, v) corrections     */
  double *rhs_coarse;     /* 3 x N_L restricted right-hand side b^L          */
} dnnmg_correct_out;

/* DNN-MG correction after a coarse step (Algorithm 1, the correction after the coarse step): x~ = P^m x
 * on level F; fine residual r^F = f^F(v_prev) - A^F(x~) (Dirichlet rows 0,
 * divided by the lumped mass); per-patch network; scatter-average of the
 * velocity corrections d (0 on Dirichlet nodes); b^F = Rhs(x~ + d) (explicit
 * velocity rows of eq. varformv with time step dt); b^L = (P^m)^T b^F stored
 * in the state as the right-hand side of its next dnnmg_step; v_prev <-
 * x~ + d.  dbg may be NULL. */
int dnnmg_correct(dnnmg_ctx *ctx, dnnmg_state *coarse, dnnmg_net *net, double dt,
                  dnnmg_correct_out *dbg);

/* Device address (owned by the net) of the fine-level state the next
 * correction starts from: after dnnmg_correct the corrected velocity
 * v~ + d of Algorithm 1 (3 doubles per fine node, pressure entries 0), after
 * dnnmg_rhs_from_fine the given fine velocity, after dnnmg_net_reset P^m x.
 * Valid until the next call that changes it.  DNNMG_ESTATE before the first
 * dnnmg_net_reset. */
int dnnmg_net_fine_velocity(dnnmg_net *net, const double **v_dev);

/* The Rhs and restriction of Algorithm 1 for a given fine velocity (teacher forcing when
 * generating training data from fine solutions): b^F = Rhs(v_fine) on level
 * F, b^L = (P^m)^T b^F stored as the coarse state's pending right-hand side,
 * and v_prev <- v_fine.  v_fine: host, 3 doubles per fine node (pressure
 * ignored). */
int dnnmg_rhs_from_fine(dnnmg_ctx *ctx, dnnmg_state *coarse, dnnmg_net *net, const double *v_fine,
                        double dt);
/* Training targets of the loss (eq. loss) for the coarse state: the velocity
 * correction d* = v_fine - P^m x (coarse) at every patch node, divided by the
 * net's output scales, written as n_patches x n_out floats (host) in the
 * network's output layout.  v_fine: host, 3 doubles per fine node.  The
 * network's inference state is not changed. */
int dnnmg_net_targets(dnnmg_ctx *ctx, const dnnmg_state *coarse, dnnmg_net *net, const double *v_fine,
                      float *D);

/* Training (loss of eq. loss): X holds T x B standardised input rows
 * (T time steps of B patch sequences, n_in floats each, step-major), D the
 * T x B x n_out target rows in network output units.  Loss =
 * sum_t sum_b ||Y_t,b - D_t,b||^2 / B with the hidden state of every sequence
 * starting at 0 (independent of the network's inference state).  Exact
 * backpropagation through time with the forward pass recomputed from
 * checkpoints every `ckpt` steps; BF16 MFMA GEMMs with FP32 accumulation,
 * FP32 gates and gradients.  1 <= T <= 4096, 1 <= B <= 2^22, T B <= 2^26
 * and ckpt >= 1, else DNNMG_EINVAL.
 * dnnmg_net_gradient: host inputs, writes the FP32 gradient (n_params, flat
 * weight order) and the loss; no update.
 * dnnmg_train_step / _dev: one Adam step (beta = 0.9, 0.999, eps = 1e-8,
 * bias-corrected) on the FP32 masters with learning rate lr, then refreshes
 * the BF16 copies; _dev takes device pointers (borrowed for the call). */
int dnnmg_net_gradient(dnnmg_net *net, const float *X, const float *D, int T, int B, int ckpt,
                       float *grad, float *loss);
int dnnmg_train_step(dnnmg_net *net, const float *X, const float *D, int T, int B, int ckpt,
                     float lr, float *loss);
int dnnmg_train_step_dev(dnnmg_net *net, const float *X_dev, const float *D_dev, int T, int B,
                         int ckpt, float lr, float *loss);

/* Flow functionals of a state (Sec. 3.3, the accuracy comparison): J_div =
 * int |div v|^2 dx (2x2 Gauss per cell) and, per obstacle k, drag and lift
 * -int_{Gamma_k} (nu grad v - p I) n . e_{x,y} ds with n the unit normal into
 * the obstacle (2-point Gauss per boundary edge of the mesh, grad v and p of
 * the fluid cell).  FP64.  drag / lift: n_obstacles doubles each (caller-
 * owned; n_obstacles must equal the macro mesh's curve count, else
 * DNNMG_EINVAL).  Synchronises the stream. */
int dnnmg_functionals(dnnmg_ctx *ctx, const dnnmg_state *s, double *jdiv, double *drag, double *lift,
                      int n_obstacles);
/* The same for a host state vector (3 N doubles, node-interleaved) on level. */
int dnnmg_functionals_host(dnnmg_ctx *ctx, int level, const double *uvp, double *jdiv, double *drag,
                           double *lift, int n_obstacles);

/* Velocity error of a nodal field against a reference (Sec. 3.4: relative
 * errors of the velocity against the fine solution).  x_dev: 3 doubles per
 * node on `level`, prolongated bilinearly to ref_level when coarser (the Q1
 * field itself; level <= ref_level); ref_dev: 3 doubles per node on
 * ref_level.  Both device pointers (e.g. dnnmg_state_device_ptr,
 * dnnmg_net_fine_velocity), borrowed for the call.  out[4] (host) receives
 * the squared norms int |v - v_ref|^2 dx and int |v_ref|^2 dx (2x2 Gauss per
 * cell, the mass-weighted L2 norm of the Q1 fields) and the nodal sums
 * sum_i |v_i - v_ref,i|^2 and sum_i |v_ref,i|^2.  Pressure is ignored.  FP64;
 * synchronises the stream. */
int dnnmg_velocity_error(dnnmg_ctx *ctx, int level, const double *x_dev, int ref_level, const double *ref_dev,
                         double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * dnnmg_velocity_error for a field on the reference's own level, allocating
 * nothing.  Its reduction's partial sums live in a fixed static device array
 * of the library (1 MiB per GPU, held until the process ends) instead of
 * memory the context allocates; the four sums (same order and meaning as
 * dnnmg_velocity_error's out) are written to out_dev, a device pointer to 4
 * doubles.  Enqueued on the context's stream without synchronisation.  Limit:
 * max(cells, nodes) of the level at most 8,388,352 (32,767 workgroups of 256
 * threads), else DNNMG_EINVAL.  All calls on one GPU share the array:
 * overlapping calls (other threads or streams) race. */
int dnnmg_velocity_error_noalloc(dnnmg_ctx *ctx, int level, const double *x_dev, const double *ref_dev,
                                 double *out_dev);

/* ------------------------------------------------------------------ batches
 * Many independent simulations of the plain method (Sec. 2: each one the
 * time step of eqs. nonlinearshort/newton on its own mesh and viscosity),
 * advanced together.  Simulations of equal depth are merged into one group
 * whose launches cover all of them (the level-0 direct solve is block
 * diagonal, one block per simulation, each at most 1536 unknowns); the groups
 * run concurrently on streams the batch creates (params->stream is ignored).
 * A group's Newton and GMRES norms span its members: a group step converges
 * when the union's residual meets newton_tol, so each member's does. */
typedef struct {
  const dnnmg_coarse_mesh *mesh;   /* macro mesh (borrowed for the create call) */
  double nu;                       /* viscosity of this simulation              */
  int depth;                       /* finest level (0..9)                      */
} dnnmg_sim_desc;
/* Creates the batch: groups by depth, merged meshes, one context and one
 * zero state per group.  DNNMG_EINVAL on a bad description (message through
 * dnnmg_batch_last_error when *out could not be made: NULL handle). */
int dnnmg_batch_create(const dnnmg_params *p, const dnnmg_sim_desc *sims, int n_sims, dnnmg_batch **out);
int dnnmg_batch_destroy(dnnmg_batch *b);
const char *dnnmg_batch_last_error(const dnnmg_batch *b);
int dnnmg_batch_groups(const dnnmg_batch *b, int *n_groups);
/* Depth, member count and node count (union) of group g. */
int dnnmg_batch_group_info(const dnnmg_batch *b, int g, int *depth, int *n_sims, int *n_nodes);
/* Group of simulation `sim` and its node count at its depth. */
int dnnmg_batch_info(const dnnmg_batch *b, int sim, int *group, int *n_nodes);
/* Host copies of one simulation's state (3 N doubles, node-interleaved, in
 * the node numbering a context of that mesh alone would use); _set also sets
 * the time of the simulation's whole group. */
int dnnmg_batch_set(dnnmg_batch *b, int sim, const double *uvp, double t);
int dnnmg_batch_get(const dnnmg_batch *b, int sim, double *uvp, double *t);
/* One time step of every simulation; stats (optional) receives one entry per
 * group.  On DNNMG_ENOCONV the failing group's states are rolled back; the
 * other groups have advanced. */
int dnnmg_batch_step(dnnmg_batch *b, double dt, dnnmg_step_stats *stats);

/* Instrumentation (not part of the method).  When enabled, the library
 * records a pair of HIP events on its stream around every launch of its main
 * kernels and accumulates their durations per "kernel@Llevel" key; enabling
 * clears earlier totals.  Levels that hold a profiled key are launched
 * directly, not from graphs. */
int dnnmg_profile_enable(dnnmg_ctx *ctx, int on);
/* Restricts the timing to a comma-separated list of "kernel@Llevel" keys;
 * NULL or "" times every key.  Kernels replayed from graphs (levels with no
 * selected key) are not timed. */
int dnnmg_profile_select(dnnmg_ctx *ctx, const char *keys);
/* Writes "key launches total_ms\n" lines into buf (NUL-terminated, at most
 * len bytes; DNNMG_EINVAL if it does not fit).  Synchronises the stream. */
int dnnmg_profile_report(dnnmg_ctx *ctx, char *buf, size_t len);
/* Workgroup sizes in use on `level`: block_sizes[0..12] = SpMV, Vanka apply,
 * Vanka update, restriction from `level`, prolongation to `level`, the fused
 * residual + Vanka apply (0: SpMV and apply run separately), the
 * single-workgroup bottom V-cycle (1024 when `level` is part of it, else 0),
 * the fused residual + restriction (0: separate), the SpMV with four
 * threads per row (0: one thread per row), and the lanes per cell of the
 * fused residual + Vanka apply (4 or 16; 0 when not fused), and the fused
 * last update of the next coarser level + prolongation to `level` (0:
 * separate), the FP32 Vanka apply with four cells per thread (0: one
 * cell per thread), and the Vanka update over the nodes in cell order (0:
 * in node order) (13 ints, caller-owned).
 * DNNMG_ESTATE before dnnmg_setup_mesh. */
int dnnmg_launch_config(const dnnmg_ctx *ctx, int level, int *block_sizes);
/* Storage statistics of a level's operator, for traffic models:
 * q_blocks = number of 3x3 Q1 blocks (sum of the node neighbour counts),
 * x_entries = LPS-extra pressure entries, q_slots / x_slots = the same with
 * the SELL padding included. */
int dnnmg_level_stats(const dnnmg_ctx *ctx, int level, long long *q_blocks, long long *x_entries,
                      long long *q_slots, long long *x_slots);

/* ------------------------------------------------------- diagnostics
 * Oscillation of a sampled functional f[i] = J(t0 + i dt), i < n (Sec. 3.3:
 * the lift over the periodic limit cycle, where runs are compared after
 * aligning their first maximum in the window).  One maximum per excursion
 * above the series mean (a maximal run of samples above the mean, with a
 * sample at or below the mean on both sides inside the window) whose largest
 * sample exceeds the midpoint of the mean and the largest sample of the
 * series; its time comes from the parabola through that sample and its two
 * neighbours.  Outputs (NULL skipped): time of the first maximum (NaN if
 * none), mean period = (last - first) / (count - 1) (NaN if fewer than two),
 * and the number of maxima.  Host arrays only; no device work.  DNNMG_EINVAL
 * for n < 3, dt <= 0 or non-finite samples. */
int dnnmg_oscillation(const double *f, int n, double t0, double dt, double *t_first_max,
                      double *period, int *n_max);

#ifdef __cplusplus
}
#endif
#endif /* DNNMG_H */
