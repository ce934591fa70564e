// gfx950 kernels of the Newton-GMRES-multigrid time step (Sec. 2.1, 2.2).
//
// Operator storage ("node-row SELL-64"): the Jacobian of a level is stored by
// node rows.  Nodes are grouped in slices of 64 consecutive nodes (one
// wavefront).  For slice s the Q1 part has wq[s] slots; slot k of node i holds
// the 3x3 block J[(i,f),(j,g)] for the k-th node j sharing a cell with i, at
//     JQ[((oq[s] + k) * 9 + 3 f + g) * 64 + lane],  lane = i mod 64,
// so that one load instruction of a wavefront reads 256 (FP32) or 512 (FP64)
// contiguous bytes.  The LPS-extra part holds the pressure-pressure entries to
// nodes that share a patch but no cell with i (wx[s] slots, JX / colx).
// Padding slots point at the row's own node and hold zeros.
//
// Vectors are interleaved, 3 values per node (u, v, p).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dnnmg {
constexpr int kS = 64;

// Explicit fused multiply-add (the rounding must not depend on whether the
// compiler contracts a product that other code also uses).
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------- geometry
struct LevelView {
  int N, C, NP;
  const double2 *xy;        // N
  const int4 *cells;        // C
  const uint8_t *flag;      // N
  const int *cadj_ptr, *cadj;
  const uint8_t *cslot;     // 4 per cadj entry
  const int *padj_ptr, *padj;
  const uint8_t *pslot;     // 9 per padj entry
  const int *patch_nodes;   // 9 * NP (row-major per patch)
  const int *wq, *wx, *oq, *ox;
  const int *colq, *colx;
  const uint8_t *vslot;     // 16 per cell
  const double *nnu;        // N: viscosity per node (simulation batches), or null: Phys::nu
};

struct Phys {
  double nu, theta, inv_dt, alpha0, u_mean, H, t;
  double delta0;   // convective stabilisation scale (0: off)
};

struct TransferView {
  int Nc, Ec, Nf;
  const int *edge_ends;   // 2 Ec
  const int4 *ccells;     // coarse cells
  const int *rptr, *ridx; // restriction lists
  const uint8_t *cflag;   // coarse node flags
};

// Internal linkage: every translation unit that launches kernels gets its own
// copy of the (non-template) kernels and constant tables.
namespace {

__device__ __forceinline__ double ramp(double t) {
  return t < 1.0 ? 0.5 * (1.0 - cos(M_PI * t)) : 1.0;
}

// Reference corner signs of the bilinear basis on [-1, 1]^2.
__device__ __constant__ double kVX[4] = {-1.0, 1.0, 1.0, -1.0};
__device__ __constant__ double kVY[4] = {-1.0, -1.0, 1.0, 1.0};

// Values, physical gradients and det J of the Q1 basis at Gauss point q.
__device__ __forceinline__ void q1_point(const double X[4], const double Y[4], int q,
                                         double N[4], double gx[4], double gy[4],
                                         double &det) {
  const double g = 0.57735026918962576451;   // 1 / sqrt(3)
  const double xi = (q == 1 || q == 2) ? g : -g;
  const double eta = (q >= 2) ? g : -g;
  double dxi[4], deta[4];
  double j11 = 0, j12 = 0, j21 = 0, j22 = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    N[a] = 0.25 * (1.0 + kVX[a] * xi) * (1.0 + kVY[a] * eta);
    dxi[a] = 0.25 * kVX[a] * (1.0 + kVY[a] * eta);
    deta[a] = 0.25 * kVY[a] * (1.0 + kVX[a] * xi);
    j11 += dxi[a] * X[a];
    j12 += deta[a] * X[a];
    j21 += dxi[a] * Y[a];
    j22 += deta[a] * Y[a];
  }
  det = j11 * j22 - j12 * j21;
  const double id = 1.0 / det;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gx[a] = (j22 * dxi[a] - j21 * deta[a]) * id;
    gy[a] = (-j12 * dxi[a] + j11 * deta[a]) * id;
  }
}

__device__ __forceinline__ void dirichlet_value(const Phys &ph, uint8_t fl, double y, double &gu,
                                                double &gv) {
  gu = 0.0;
  gv = 0.0;
  if (fl & 2) gu = 6.0 * ph.u_mean * ramp(ph.t) * y * (ph.H - y) / (ph.H * ph.H);
}

// Convective stabilisation of one cell (an optional member of the local-
// projection family, off unless delta0 > 0): delta_T (kappa_T(b.grad v),
// kappa_T(b.grad phi))_T with kappa_T g = g - mean_T(g), b the mean of the
// old velocity over the 4 nodes, delta_T = delta0 / (nu / h^2 + |b| / h),
// h^2 = area.  Given det_q and psi[q][a] = b.grad N_a at the 4 Gauss points,
// returns delta_T and the fluctuations kpsi[q][a] = psi - its cell mean.
__device__ __forceinline__ double conv_fluct(const double det[4], const double psi[4][4], double bn, double nu,
                                             double delta0, double kpsi[4][4]) {
  double area = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) area += det[q];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double m = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) m += det[q] * psi[q][a];
    m /= area;
#pragma unroll
    for (int q = 0; q < 4; ++q) kpsi[q][a] = psi[q][a] - m;
  }
  return delta0 / (nu / area + bn / sqrt(area));
}

// ------------------------------------------------------------------ LPS
// Fluctuation K = I - I_2h on a patch (lexicographic 3x3 nodes): corners 0,
// edge nodes minus the mean of their two corners, centre minus the mean of
// the four corners.  kK[m][q] = K_{m q}.
__device__ __constant__ double kK[9][9] = {
    {0, 0, 0, 0, 0, 0, 0, 0, 0},
    {-0.5, 1, -0.5, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0},
    {-0.5, 0, 0, 1, 0, 0, -0.5, 0, 0},
    {-0.25, 0, -0.25, 0, 1, 0, -0.25, 0, -0.25},
    {0, 0, -0.5, 0, 0, 1, 0, 0, -0.5},
    {0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, -0.5, 1, -0.5},
    {0, 0, 0, 0, 0, 0, 0, 0, 0}};
__device__ __constant__ int kChildToPatch[4][4] = {{0, 1, 4, 3}, {1, 2, 5, 4}, {4, 5, 8, 7}, {3, 4, 7, 6}};

// Patch matrix s_P = K^T (sum_T alpha_T S_T) K of the LPS term, one thread per
// patch, stored SoA: sP[(9 q + m) * NP + P].  alpha_T (Sec. 2.1, h_T^2 =
// area(T), Re = 1/nu): bounded = 0 gives the paper's alpha0 Re h_T^2, the
// stabilisation of the level's own discrete problem; bounded = 1 gives
// alpha0 / (nu / h_T^2 + 1/k), used only for the re-discretised operators a
// finer level's multigrid preconditioner solves with on this level.
__global__ void __launch_bounds__(64) k_lps_patch(LevelView L, Phys ph, int bounded, double *__restrict__ sP) {
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= L.NP) return;
  const double nu = L.nnu ? L.nnu[L.cells[4 * P].x] : ph.nu;
  double S[9][9];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j) S[i][j] = 0.0;
  for (int k = 0; k < 4; ++k) {
    const int4 cn = L.cells[4 * P + k];
    const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
    double X[4], Y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      X[a] = L.xy[nn[a]].x;
      Y[a] = L.xy[nn[a]].y;
    }
    double St[4][4] = {};
    double area = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double N[4], gx[4], gy[4], det;
      q1_point(X, Y, q, N, gx, gy, det);
      area += det;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) St[a][b] += det * (gx[a] * gx[b] + gy[a] * gy[b]);
    }
    const double alpha = bounded ? ph.alpha0 / (nu / area + ph.inv_dt) : ph.alpha0 * area / nu;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) S[kChildToPatch[k][a]][kChildToPatch[k][b]] += alpha * St[a][b];
  }
  // SK = S K ; out = K^T SK
  for (int q = 0; q < 9; ++q) {
    double row[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < 9; ++m) {
        double skmj = 0.0;
#pragma unroll
        for (int n = 0; n < 9; ++n) skmj += S[m][n] * kK[n][j];
        s += kK[m][q] * skmj;
      }
      row[j] = s;
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) sP[(9 * q + j) * L.NP + P] = row[j];
  }
}

// -------------------------------------------------------------- residual
// R = f_n - A_n(x) for every node (eqs. varform, varformv) and the Rhs of
// Algorithm 1; Dirichlet velocity rows hold g(t_new) - x.  FP64 throughout.
//
// Element vectors of the nonlinear residual and of Rhs (eqs. varform,
// varformv; 2x2 Gauss): one thread per cell evaluates each quadrature point
// once and writes the cell's contribution to the rows of its 4 vertices a as
// E[12 c + 3a + f] (f = u, v, p), so that a node reads 24 contiguous bytes per
// cell; a node pass then sums its cells' entries in its adjacency order (no
// atomics).  The
// viscosity of row a is that of vertex a (per-node viscosity of batches).
// kKind 0: the A_n(x) part of the residual rows, with the old-state terms
// (old_terms = 1, x_old = xo) or without them (old_terms = 0: a DNN-MG
// right-hand side replaces them); kKind 1: the explicit velocity rows of f_n
// for v = x (Rhs of Algorithm 1; p entries not written).
// Launched with 256 threads per workgroup.
template <int kKind>
__global__ void __launch_bounds__(256) k_cell_vectors(LevelView L, Phys ph, const double *__restrict__ x,
                                                      const double *__restrict__ xo, int old_terms,
                                                      double *__restrict__ E) {
  __shared__ double stage[256 * 12];
  const int c0 = blockIdx.x * 256, t = threadIdx.x;
  const int c = c0 + t;
  const bool live = c < L.C;
  const int4 cn = L.cells[live ? c : 0];
  const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
  const double th = ph.theta, idt = ph.inv_dt;
  const double tho = kKind == 1 ? 1.0 - th : (old_terms ? 1.0 - th : 0.0);
  double X[4], Y[4], U[4], V[4], P[4], Uo[4], Vo[4], nu[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const double2 pt = L.xy[nn[b]];
    X[b] = pt.x;
    Y[b] = pt.y;
    U[b] = x[3 * nn[b]];
    V[b] = x[3 * nn[b] + 1];
    P[b] = kKind == 0 ? x[3 * nn[b] + 2] : 0.0;
    Uo[b] = kKind == 0 && old_terms ? xo[3 * nn[b]] : 0.0;
    Vo[b] = kKind == 0 && old_terms ? xo[3 * nn[b] + 1] : 0.0;
    nu[b] = L.nnu ? L.nnu[nn[b]] : ph.nu;
  }
  double Au[4] = {0, 0, 0, 0}, Av[4] = {0, 0, 0, 0}, Ap[4] = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double N[4], gx[4], gy[4], det;
    q1_point(X, Y, q, N, gx, gy, det);
    double u = 0, v = 0, p = 0, uo = 0, vo = 0;
    double ux = 0, uy = 0, vx = 0, vy = 0, uox = 0, uoy = 0, vox = 0, voy = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      u += N[b] * U[b];
      v += N[b] * V[b];
      p += N[b] * P[b];
      uo += N[b] * Uo[b];
      vo += N[b] * Vo[b];
      ux += gx[b] * U[b];
      uy += gy[b] * U[b];
      vx += gx[b] * V[b];
      vy += gy[b] * V[b];
      uox += gx[b] * Uo[b];
      uoy += gy[b] * Uo[b];
      vox += gx[b] * Vo[b];
      voy += gy[b] * Vo[b];
    }
    if (kKind == 0) {
      const double mu = idt * (u - uo) + th * (u * ux + v * uy) + tho * (uo * uox + vo * uoy);
      const double mv = idt * (v - vo) + th * (u * vx + v * vy) + tho * (uo * vox + vo * voy);
      const double su = th * ux + tho * uox, tu = th * uy + tho * uoy;
      const double sv = th * vx + tho * vox, tv = th * vy + tho * voy;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        Au[a] += det * (mu * N[a] + nu[a] * (su * gx[a] + tu * gy[a]) - p * gx[a]);
        Av[a] += det * (mv * N[a] + nu[a] * (sv * gx[a] + tv * gy[a]) - p * gy[a]);
        Ap[a] += det * (ux + vy) * N[a];
      }
    } else {
      const double mu = idt * u - tho * (u * ux + v * uy), mv = idt * v - tho * (u * vx + v * vy);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        Au[a] += det * (mu * N[a] - tho * nu[a] * (ux * gx[a] + uy * gy[a]));
        Av[a] += det * (mv * N[a] - tho * nu[a] * (vx * gx[a] + vy * gy[a]));
      }
    }
  }
  // the block's 256 x 12 values are contiguous in E: stage them in LDS and
  // write them with consecutive lanes on consecutive addresses
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    stage[12 * t + 3 * a] = Au[a];
    stage[12 * t + 3 * a + 1] = Av[a];
    stage[12 * t + 3 * a + 2] = kKind == 0 ? Ap[a] : 0.0;
  }
  __syncthreads();
  const size_t base = 12 * static_cast<size_t>(c0), end = 12 * static_cast<size_t>(L.C);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const size_t idx = base + k * 256 + t;
    if (idx < end) E[idx] = stage[k * 256 + t];
  }
}

// Convective stabilisation rows of the residual (delta0 > 0 only), added to
// the element vectors of k_cell_vectors<0>: E[12 c + 3 a + f] += delta_T
// (kappa_T(b.grad v_f), kappa_T(b.grad N_a))_T for f = u, v, with the frozen
// field b from xo (one thread per cell).
__global__ void __launch_bounds__(256) k_conv_vectors(LevelView L, Phys ph, const double *__restrict__ x,
                                                      const double *__restrict__ xo, double *__restrict__ E) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= L.C) return;
  const int4 cn = L.cells[c];
  const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
  double X[4], Y[4], U[4], V[4], Bu = 0.0, Bv = 0.0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const double2 pt = L.xy[nn[b]];
    X[b] = pt.x;
    Y[b] = pt.y;
    U[b] = x[3 * nn[b]];
    V[b] = x[3 * nn[b] + 1];
    Bu += xo[3 * nn[b]];
    Bv += xo[3 * nn[b] + 1];
  }
  Bu *= 0.25;
  Bv *= 0.25;
  double cdet[4], cpsi[4][4], gu[4], gv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double N[4], gx[4], gy[4], det;
    q1_point(X, Y, q, N, gx, gy, det);
    cdet[q] = det;
    gu[q] = 0.0;
    gv[q] = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      cpsi[q][a] = Bu * gx[a] + Bv * gy[a];
      gu[q] += cpsi[q][a] * U[a];
      gv[q] += cpsi[q][a] * V[a];
    }
  }
  double kpsi[4][4];
  const double delta = conv_fluct(cdet, cpsi, sqrt(Bu * Bu + Bv * Bv), L.nnu ? L.nnu[nn[0]] : ph.nu, ph.delta0,
                                  kpsi);
  double mu = 0.0, mv = 0.0, area = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    mu += cdet[q] * gu[q];
    mv += cdet[q] * gv[q];
    area += cdet[q];
  }
  mu /= area;
  mv /= area;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double su = 0.0, sv = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      su += cdet[q] * (gu[q] - mu) * kpsi[q][a];
      sv += cdet[q] * (gv[q] - mv) * kpsi[q][a];
    }
    E[12 * static_cast<size_t>(c) + 3 * a] += delta * su;
    E[12 * static_cast<size_t>(c) + 3 * a + 1] += delta * sv;
  }
}

// LPS rows of the pressure equation per patch: S[q NP + P] = sum_m
// s_P(q, m) p_m over the patch's 9 nodes (one thread per patch; the sums of
// the node rows then add these in the node's patch order).
__global__ void __launch_bounds__(256) k_lps_vectors(LevelView L, const double *__restrict__ sP,
                                                     const double *__restrict__ x, double *__restrict__ S) {
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= L.NP) return;
  double p[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) p[m] = x[3 * L.patch_nodes[9 * P + m] + 2];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 9; ++m) s += sP[(9 * q + m) * L.NP + P] * p[m];
    S[q * static_cast<size_t>(L.NP) + P] = s;
  }
}

// Residual rows R = f_n - A_n(x) (eq. nonlinearshort) from the element
// vectors of k_cell_vectors<0> and the patch vectors of k_lps_vectors: per
// node the sum of its cells' entries, then of its patches' LPS entries, the
// DNN-MG right-hand side if given, and the Dirichlet rows R = g - x.
__global__ void __launch_bounds__(256) k_residual_nodes(LevelView L, Phys ph, const double *__restrict__ x,
                                                        const double *__restrict__ rhs,
                                                        const double *__restrict__ S,
                                                        const double *__restrict__ E, double *__restrict__ R,
                                                        const int *__restrict__ order) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= L.N) return;
  const int i = order ? order[g] : g;   // nodes in cell order on large levels (as k_vanka_update_ordered)
  double Au = 0.0, Av = 0.0, Ap = 0.0;
  for (int e = L.cadj_ptr[i]; e < L.cadj_ptr[i + 1]; ++e) {
    const int c = L.cadj[e] >> 2, a = L.cadj[e] & 3;
    const double *ec = E + 12 * static_cast<size_t>(c) + 3 * a;
    Au += ec[0];
    Av += ec[1];
    Ap += ec[2];
  }
  for (int e = L.padj_ptr[i]; e < L.padj_ptr[i + 1]; ++e) {
    const int Pp = L.padj[e] / 9, q = L.padj[e] % 9;
    Ap += S[q * static_cast<size_t>(L.NP) + Pp];
  }
  double ru = -Au, rv = -Av;
  if (rhs) {
    ru += rhs[3 * i];
    rv += rhs[3 * i + 1];
  }
  const uint8_t fl = L.flag[i];
  if (fl & 1) {
    double gu, gv;
    dirichlet_value(ph, fl, L.xy[i].y, gu, gv);
    ru = gu - x[3 * i];
    rv = gv - x[3 * i + 1];
  }
  R[3 * i] = ru;
  R[3 * i + 1] = rv;
  R[3 * i + 2] = -Ap;
}

// Rhs rows from the element vectors of k_cell_vectors<1>; pressure rows 0.
__global__ void __launch_bounds__(256) k_rhs_nodes(LevelView L, const double *__restrict__ E,
                                                   double *__restrict__ out, const int *__restrict__ order) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= L.N) return;
  const int i = order ? order[g] : g;   // nodes in cell order on large levels
  double fu = 0.0, fv = 0.0;
  for (int e = L.cadj_ptr[i]; e < L.cadj_ptr[i + 1]; ++e) {
    const int c = L.cadj[e] >> 2, a = L.cadj[e] & 3;
    const double *ec = E + 12 * static_cast<size_t>(c) + 3 * a;
    fu += ec[0];
    fv += ec[1];
  }
  out[3 * i] = fu;
  out[3 * i + 1] = fv;
  out[3 * i + 2] = 0.0;
}

// Sets the Dirichlet velocity values of time ph.t.
__global__ void k_impose_bc(LevelView L, Phys ph, double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.N) return;
  const uint8_t fl = L.flag[i];
  if (fl & 1) {
    double gu, gv;
    dirichlet_value(ph, fl, L.xy[i].y, gu, gv);
    x[3 * i] = gu;
    x[3 * i + 1] = gv;
  }
}

// -------------------------------------------------------------- Jacobian
template <typename T>
__global__ void k_fill(T *__restrict__ a, size_t n, T v) {
  size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) a[i] = v;
}

// A_n'(x) (eq. newton) in the node-row SELL layout, written once.  One
// wavefront per slice of 64 node rows (lane = row): each of the row's cells
// contributes row a of its element matrix (2x2 Gauss, FP64), each of its
// patches row q of s_P.  A lane accumulates its own row in a private column of
// LDS, acc[(k * 9 + r) * 64 + lane] for slot k and entry r of the 3x3 block
// (plus the LPS-extra slots), so lanes never touch each other's data and no
// barrier is needed; every contribution is added as
// acc = T(double(acc) + value) in cell then patch order.  The slice's slots,
// padding included, are then stored with one 64-lane contiguous store per
// (slot, entry): no zero fill and no read-modify-write of the operator.
// With cblk, the lane also copies, for each of its cells c (local vertex a),
// its row restricted to the cell's 12 unknowns into the cell's 12x12 block:
// cblk[144 c + 12 (3 a + f) + 3 b + g] (rows of the cell block contiguous,
// for the Vanka factorisation).
// Dynamic LDS: (maxwq * 9 + maxwx) * 64 * sizeof(T) bytes.
template <typename T>
__global__ void __launch_bounds__(64) k_assemble(LevelView L, Phys ph, const double *__restrict__ x,
                                                 const double *__restrict__ sP, const double *__restrict__ xo,
                                                 T *__restrict__ JQ, T *__restrict__ JX, T *__restrict__ cblk) {
  extern __shared__ unsigned char lds_raw[];
  T *accq = reinterpret_cast<T *>(lds_raw);
  const int s = blockIdx.x, lane = threadIdx.x;
  const int i = s * kS + lane;
  const int wq = L.wq[s], wx = L.wx[s];
  T *accx = accq + static_cast<size_t>(wq) * 9 * kS;
  for (int k = 0; k < 9 * wq; ++k) accq[k * kS + lane] = T(0);
  for (int k = 0; k < wx; ++k) accx[k * kS + lane] = T(0);
  auto add = [&](T *a, double v) { *a = static_cast<T>(static_cast<double>(*a) + v); };
  if (i < L.N) {
    const double th = ph.theta, nu = L.nnu ? L.nnu[i] : ph.nu, idt = ph.inv_dt;
    const bool dir = L.flag[i] & 1;
    for (int e = L.cadj_ptr[i]; e < L.cadj_ptr[i + 1]; ++e) {
      const int c = L.cadj[e] >> 2, a = L.cadj[e] & 3;
      const int4 cn = L.cells[c];
      const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
      double X[4], Y[4], U[4], V[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double2 p = L.xy[nn[b]];
        X[b] = p.x;
        Y[b] = p.y;
        U[b] = x[3 * nn[b]];
        V[b] = x[3 * nn[b] + 1];
      }
      double blk[4][8];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int k = 0; k < 8; ++k) blk[b][k] = 0.0;
      // convective stabilisation (delta0 > 0): frozen field b from xo
      const bool conv = ph.delta0 > 0.0 && xo != nullptr;
      double Bu = 0.0, Bv = 0.0;
      if (conv) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          Bu += xo[3 * nn[b]];
          Bv += xo[3 * nn[b] + 1];
        }
        Bu *= 0.25;
        Bv *= 0.25;
      }
      double cdet[4], cpsi[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double N[4], gx[4], gy[4], det;
        q1_point(X, Y, q, N, gx, gy, det);
        cdet[q] = det;
#pragma unroll
        for (int b = 0; b < 4; ++b) cpsi[q][b] = Bu * gx[b] + Bv * gy[b];
        double u = 0, v = 0, ux = 0, uy = 0, vx = 0, vy = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          u += N[b] * U[b];
          v += N[b] * V[b];
          ux += gx[b] * U[b];
          uy += gy[b] * U[b];
          vx += gx[b] * V[b];
          vy += gy[b] * V[b];
        }
        double Na = 0.0, ga = 0.0, ha = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (b == a) {
            Na = N[b];
            ga = gx[b];
            ha = gy[b];
          }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double Nb = N[b];
          const double d = det * (idt * Nb * Na + th * (u * gx[b] + v * gy[b]) * Na +
                                  th * nu * (gx[b] * ga + gy[b] * ha));
          const double r = det * th * Nb * Na;
          blk[b][0] += d + r * ux;       // (u,u)
          blk[b][1] += r * uy;           // (u,v)
          blk[b][2] -= det * Nb * ga;    // (u,p)
          blk[b][3] += r * vx;           // (v,u)
          blk[b][4] += d + r * vy;       // (v,v)
          blk[b][5] -= det * Nb * ha;    // (v,p)
          blk[b][6] += det * gx[b] * Na;  // (p,u)
          blk[b][7] += det * gy[b] * Na;  // (p,v)
        }
      }
      if (conv) {
        double kpsi[4][4];
        const double delta = conv_fluct(cdet, cpsi, sqrt(Bu * Bu + Bv * Bv), nu, ph.delta0, kpsi);
        double ka[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ka[q] = 0.0;
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (b == a) ka[q] = kpsi[q][b];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          double cab = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) cab += cdet[q] * ka[q] * kpsi[q][b];
          blk[b][0] += delta * cab;
          blk[b][4] += delta * cab;
        }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        T *dst = accq + static_cast<size_t>(L.cslot[4 * e + b]) * 9 * kS + lane;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          if (dir && r < 6) continue;
          add(dst + r * kS, blk[b][r]);
        }
      }
    }
    for (int e = L.padj_ptr[i]; e < L.padj_ptr[i + 1]; ++e) {
      const int Pp = L.padj[e] / 9, q = L.padj[e] % 9;
#pragma unroll
      for (int m = 0; m < 9; ++m) {
        const double v = sP[(9 * q + m) * L.NP + Pp];
        const int sl = L.pslot[9 * e + m];
        T *dst = (sl & 0x80) ? accx + (sl & 0x7f) * kS + lane : accq + (static_cast<size_t>(sl) * 9 + 8) * kS + lane;
        add(dst, v);
      }
    }
    if (dir) {
      // identity velocity rows: the self slot holds 1 on (u,u) and (v,v)
      for (int k = 0; k < wq; ++k)
        if (L.colq[(L.oq[s] + k) * kS + lane] == i) {
          accq[(k * 9) * kS + lane] = T(1);
          accq[(k * 9 + 4) * kS + lane] = T(1);
          break;
        }
    }
  }
  if (cblk && i < L.N) {
    for (int e = L.cadj_ptr[i]; e < L.cadj_ptr[i + 1]; ++e) {
      const int c = L.cadj[e] >> 2, a = L.cadj[e] & 3;
      T *dst = cblk + static_cast<size_t>(c) * 144 + 36 * a;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const T *src = accq + static_cast<size_t>(L.cslot[4 * e + b]) * 9 * kS + lane;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
          for (int g = 0; g < 3; ++g) dst[12 * f + 3 * b + g] = src[(3 * f + g) * kS];
      }
    }
  }
  T *oq = JQ + static_cast<size_t>(L.oq[s]) * 9 * kS + lane;
  for (int k = 0; k < 9 * wq; ++k) oq[static_cast<size_t>(k) * kS] = accq[k * kS + lane];
  T *ox = JX + static_cast<size_t>(L.ox[s]) * kS + lane;
  for (int k = 0; k < wx; ++k) ox[static_cast<size_t>(k) * kS] = accx[k * kS + lane];
}

// -------------------------------------------------------------- SpMV
// y = b - J x (if b) or y = J x, T precision.
constexpr int kSpmvChunk = 16;
// Row i of J x (3 values).  The row sum has one canonical order, whatever the
// number of threads per row: entry k (the Q1 blocks, then the LPS extra
// entries, each counted from 0) goes into partial sum k mod 4, in increasing
// k, each block contribution as fma(m2, x2, fma(m1, x1, m0 x0)) and each extra
// entry as one fma; the row is (s0 + s1) + (s2 + s3).  spmv_row evaluates the
// four partial sums in one thread, spmv_row_part the partial sum q in thread
// q of four: both give the same bits.  Chunks of kSpmvChunk entries: all
// column indices of a chunk, then all x values, then the products, so that a
// thread waits on two memory latencies per chunk, not two per entry.
// Operator loads, optionally non-temporal (see kStreamCells).
template <bool kStream, typename T>
__device__ __forceinline__ T op_load(const T *p) {
  if constexpr (kStream) return __builtin_nontemporal_load(p);
  else return *p;
}

template <typename T, bool kStream = false>
__device__ __forceinline__ void spmv_row(const LevelView &L, const T *__restrict__ JQ, const T *__restrict__ JX,
                                         const T *__restrict__ x, int i, T &a0, T &a1, T &a2) {
  const int s = i / kS, lane = i % kS;
  const int wq = L.wq[s], wx = L.wx[s];
  const T *jq = JQ + static_cast<size_t>(L.oq[s]) * 9 * kS + lane;
  const int *cq = L.colq + static_cast<size_t>(L.oq[s]) * kS + lane;
  T p[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) p[q][0] = p[q][1] = p[q][2] = 0;
  for (int k0 = 0; k0 < wq; k0 += kSpmvChunk) {
    int jv[kSpmvChunk];
#pragma unroll
    for (int u = 0; u < kSpmvChunk; ++u) jv[u] = k0 + u < wq ? cq[(k0 + u) * kS] : -1;
    T xv[kSpmvChunk][3];
#pragma unroll
    for (int u = 0; u < kSpmvChunk; ++u)
#pragma unroll
      for (int f = 0; f < 3; ++f) xv[u][f] = jv[u] >= 0 ? x[3 * jv[u] + f] : T(0);
#pragma unroll
    for (int u = 0; u < kSpmvChunk; ++u) {
      if (jv[u] >= 0) {
        const T *m = jq + static_cast<size_t>(k0 + u) * 9 * kS;
#pragma unroll
        for (int f = 0; f < 3; ++f)
          p[u & 3][f] += fma_t(op_load<kStream>(m + (3 * f + 2) * kS), xv[u][2],
                               fma_t(op_load<kStream>(m + (3 * f + 1) * kS), xv[u][1],
                                     op_load<kStream>(m + 3 * f * kS) * xv[u][0]));
      }
    }
  }
  const T *jx = JX + static_cast<size_t>(L.ox[s]) * kS + lane;
  const int *cx = L.colx + static_cast<size_t>(L.ox[s]) * kS + lane;
  for (int k0 = 0; k0 < wx; k0 += kSpmvChunk) {
    int jv[kSpmvChunk];
#pragma unroll
    for (int u = 0; u < kSpmvChunk; ++u) jv[u] = k0 + u < wx ? cx[(k0 + u) * kS] : -1;
    T xv[kSpmvChunk];
#pragma unroll
    for (int u = 0; u < kSpmvChunk; ++u) xv[u] = jv[u] >= 0 ? x[3 * jv[u] + 2] : T(0);
#pragma unroll
    for (int u = 0; u < kSpmvChunk; ++u)
      if (jv[u] >= 0) p[u & 3][2] = fma_t(op_load<kStream>(jx + (k0 + u) * kS), xv[u], p[u & 3][2]);
  }
  a0 = (p[0][0] + p[1][0]) + (p[2][0] + p[3][0]);
  a1 = (p[0][1] + p[1][1]) + (p[2][1] + p[3][1]);
  a2 = (p[0][2] + p[1][2]) + (p[2][2] + p[3][2]);
}

// Partial sum q (entries k = q mod 4) of row i, for four threads per row.
template <typename T>
__device__ __forceinline__ void spmv_row_part(const LevelView &L, const T *__restrict__ JQ,
                                              const T *__restrict__ JX, const T *__restrict__ x, int i, int q,
                                              T &a0, T &a1, T &a2) {
  const int s = i / kS, lane = i % kS;
  const int wq = L.wq[s], wx = L.wx[s];
  const T *jq = JQ + static_cast<size_t>(L.oq[s]) * 9 * kS + lane;
  const int *cq = L.colq + static_cast<size_t>(L.oq[s]) * kS + lane;
  T p[3] = {0, 0, 0};
  constexpr int kPer = kSpmvChunk / 4;
  for (int k0 = 0; k0 < wq; k0 += kSpmvChunk) {
    int jv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = k0 + 4 * u + q;
      jv[u] = k < wq ? cq[k * kS] : -1;
    }
    T xv[kPer][3];
#pragma unroll
    for (int u = 0; u < kPer; ++u)
#pragma unroll
      for (int f = 0; f < 3; ++f) xv[u][f] = jv[u] >= 0 ? x[3 * jv[u] + f] : T(0);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (jv[u] >= 0) {
        const T *m = jq + static_cast<size_t>(k0 + 4 * u + q) * 9 * kS;
#pragma unroll
        for (int f = 0; f < 3; ++f)
          p[f] += fma_t(m[(3 * f + 2) * kS], xv[u][2], fma_t(m[(3 * f + 1) * kS], xv[u][1], m[3 * f * kS] * xv[u][0]));
      }
    }
  }
  const T *jx = JX + static_cast<size_t>(L.ox[s]) * kS + lane;
  const int *cx = L.colx + static_cast<size_t>(L.ox[s]) * kS + lane;
  for (int k0 = 0; k0 < wx; k0 += kSpmvChunk) {
    int jv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = k0 + 4 * u + q;
      jv[u] = k < wx ? cx[k * kS] : -1;
    }
    T xv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) xv[u] = jv[u] >= 0 ? x[3 * jv[u] + 2] : T(0);
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (jv[u] >= 0) p[2] = fma_t(jx[(k0 + 4 * u + q) * kS], xv[u], p[2]);
  }
  a0 = p[0];
  a1 = p[1];
  a2 = p[2];
}

// Each kernel below is a grid over items (nodes, cells) calling the item
// function of the same name; the single-workgroup coarse V-cycle calls the
// same item functions, so both paths compute bitwise the same values.
template <typename T, bool kStream = false>
__device__ __forceinline__ void spmv_item(const LevelView &L, const T *__restrict__ JQ, const T *__restrict__ JX,
                                          const T *__restrict__ x, const T *__restrict__ b, T *__restrict__ y,
                                          int i) {
  T a0, a1, a2;
  spmv_row<T, kStream>(L, JQ, JX, x, i, a0, a1, a2);
  if (b) {
    y[3 * i] = b[3 * i] - a0;
    y[3 * i + 1] = b[3 * i + 1] - a1;
    y[3 * i + 2] = b[3 * i + 2] - a2;
  } else {
    y[3 * i] = a0;
    y[3 * i + 1] = a1;
    y[3 * i + 2] = a2;
  }
}

template <typename T, bool kStream = false>
__global__ void __launch_bounds__(256) k_spmv(LevelView L, const T *__restrict__ JQ, const T *__restrict__ JX,
                       const T *__restrict__ x, const T *__restrict__ b, T *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L.N) spmv_item<T, kStream>(L, JQ, JX, x, b, y, i);
}

// The same rows with four threads per node (more loads in flight on small
// levels): lane q of a group of four sums the entries k = q mod 4; lane 0
// combines (s0 + s1) + (s2 + s3), bitwise the value of k_spmv.  The
// workgroup size is a multiple of 4.
// Four lanes per node: gid = 4 i + q (gid and threadIdx.x agree modulo 64).
// Every lane of the wavefront must take part (shuffles).
template <typename T>
__device__ __forceinline__ void spmv4_item(const LevelView &L, const T *__restrict__ JQ, const T *__restrict__ JX,
                                           const T *__restrict__ x, const T *__restrict__ b, T *__restrict__ y,
                                           int gid) {
  const int i = gid >> 2, q = gid & 3;
  T a0 = 0, a1 = 0, a2 = 0;
  if (i < L.N) spmv_row_part(L, JQ, JX, x, i, q, a0, a1, a2);
  const int lb = (threadIdx.x & 63) & ~3;
  T s[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    s[k][0] = __shfl(a0, lb + k);
    s[k][1] = __shfl(a1, lb + k);
    s[k][2] = __shfl(a2, lb + k);
  }
  if (i >= L.N || q != 0) return;
  const T r0 = (s[0][0] + s[1][0]) + (s[2][0] + s[3][0]);
  const T r1 = (s[0][1] + s[1][1]) + (s[2][1] + s[3][1]);
  const T r2 = (s[0][2] + s[1][2]) + (s[2][2] + s[3][2]);
  if (b) {
    y[3 * i] = b[3 * i] - r0;
    y[3 * i + 1] = b[3 * i + 1] - r1;
    y[3 * i + 2] = b[3 * i + 2] - r2;
  } else {
    y[3 * i] = r0;
    y[3 * i + 1] = r1;
    y[3 * i + 2] = r2;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_spmv4(LevelView L, const T *__restrict__ JQ, const T *__restrict__ JX,
                                               const T *__restrict__ x, const T *__restrict__ b,
                                               T *__restrict__ y) {
  spmv4_item(L, JQ, JX, x, b, y, static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x));
}

// -------------------------------------------------------------- Vanka
// Factorisation of the 12x12 cell blocks J|_{c,c} (4 nodes x 3 fields) by
// Gauss-Jordan elimination with partial pivoting (largest |entry| of the
// column among the rows not yet used as pivots, the lowest row on ties), in
// place.  A group of 4 lanes works on one cell; lane l holds rows
// 3 l .. 3 l + 2 of the block, read from the cell blocks the assembly wrote
// (cblk[144 c + 12 r + j]: a group reads 576 contiguous bytes).  Per column
// k: each lane picks its best row, two butterfly shuffles pick the group's
// row p, the pivot row is broadcast from its lane, scaled by 1 / a_pk and
// subtracted from every other row, and column k turns into the column of
// the identity's unit vector e_p (the classic in-place inversion: it holds
// 1 / a_pk in row p and -a_ik / a_pk elsewhere).  Rows are never swapped: a
// row records the column it pivoted (order) and the group the row that
// pivoted each column (pc), so that at the end entry (i, k) of the array is
// entry (order[i], pc[k]) of the inverse, stored SoA:
// inv[(12 r + j) * C + c] (entry-major: each of the 144 loads of a wavefront
// in the apply reads one contiguous 256-byte segment).
template <typename T>
__global__ void __launch_bounds__(256) k_vanka_factor(LevelView L, const T *__restrict__ cblk, T *__restrict__ inv) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = gid >> 2;
  const int l = threadIdx.x & 3;
  const bool live = c < L.C;
  double A[3][12];
  if (live) {
    const T *row = cblk + static_cast<size_t>(c) * 144 + 36 * l;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 12; ++j) A[i][j] = static_cast<double>(row[12 * i + j]);
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 12; ++j) A[i][j] = (j == 3 * l + i) ? 1.0 : 0.0;
  }
  bool used[3] = {false, false, false};
  int order[3] = {0, 0, 0};
  int pc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double val = -2.0;
    int idx = 12;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double v = used[i] ? -1.0 : fabs(A[i][k]);
      if (v > val) {   // rows in increasing order: ties keep the lower row
        val = v;
        idx = 3 * l + i;
      }
    }
#pragma unroll
    for (int off = 2; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(val, off, 4);
      const int oi = __shfl_xor(idx, off, 4);
      if (ov > val || (ov == val && oi < idx)) {
        val = ov;
        idx = oi;
      }
    }
    pc[k] = idx;
    const int owner = idx / 3, li = idx - 3 * owner;
    double pr[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      const double send = li == 0 ? A[0][j] : (li == 1 ? A[1][j] : A[2][j]);
      pr[j] = __shfl(send, owner, 4);
    }
    const double piv = pr[k];
    const double ip = piv != 0.0 ? 1.0 / piv : 0.0;
#pragma unroll
    for (int j = 0; j < 12; ++j) pr[j] = (j == k) ? ip : pr[j] * ip;   // the new pivot row
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const bool me = 3 * l + i == idx;
      if (me) {
        used[i] = true;
        order[i] = k;
      }
      const double f = A[i][k];
#pragma unroll
      for (int j = 0; j < 12; ++j) {
        const double e = (j == k) ? 0.0 : A[i][j];   // column k of the other rows: 0 - f / a_pk
        A[i][j] = me ? pr[j] : e - f * pr[j];
      }
    }
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 12; ++k)
        inv[static_cast<size_t>(12 * order[i] + pc[k]) * L.C + c] = static_cast<T>(A[i][k]);
  }
}

// delta_c = inv_c r|_c, one thread per cell, stored entry-major
// delta[(3 a + f) * C + c].  With kStream the inverse is read with
// non-temporal loads (for levels whose inverses are far larger than the
// caches: streamed once per sweep, they would only evict the residual).
template <typename T, bool kStream = false>
__device__ __forceinline__ void apply_item(const LevelView &L, const T *__restrict__ inv, const T *__restrict__ r,
                                           T *__restrict__ delta, int c) {
  const int4 cn = L.cells[c];
  const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
  T rc[12];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int f = 0; f < 3; ++f) rc[3 * a + f] = r[3 * nn[a] + f];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      const T *p = inv + static_cast<size_t>(12 * i + j) * L.C + c;
      s += (kStream ? __builtin_nontemporal_load(p) : *p) * rc[j];
    }
    delta[static_cast<size_t>(i) * L.C + c] = s;
  }
}

template <typename T, bool kStream = false>
__global__ void __launch_bounds__(256) k_vanka_apply(LevelView L, const T *__restrict__ inv, const T *__restrict__ r,
                              T *__restrict__ delta) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < L.C) apply_item<T, kStream>(L, inv, r, delta, c);
}

// Levels with at least this many cells read their Vanka inverses with
// non-temporal loads (576 B per cell in FP32: 134 MB and more).
constexpr int kStreamCells = 1 << 18;

// The same (FP32) with four consecutive cells per thread: 16-byte loads of
// the entry-major inverses and 16-byte stores of the corrections (C a
// multiple of 4, so every row of the layout starts 16-byte aligned); each
// cell's rows are summed as in apply_item.
typedef float v4f __attribute__((ext_vector_type(4)));
template <bool kStream = false>
__global__ void __launch_bounds__(256) k_vanka_apply4(LevelView L, const float *__restrict__ inv,
                                                      const float *__restrict__ r, float *__restrict__ delta) {
  const int c0 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
  if (c0 >= L.C) return;
  const size_t C = static_cast<size_t>(L.C);
  float rc[4][12];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int4 cn = L.cells[c0 + q];
    const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int f = 0; f < 3; ++f) rc[q][3 * a + f] = r[3 * nn[a] + f];
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    float s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      const v4f m = op_load<kStream>(reinterpret_cast<const v4f *>(inv + static_cast<size_t>(12 * i + j) * C + c0));
      s0 += m[0] * rc[0][j];
      s1 += m[1] * rc[1][j];
      s2 += m[2] * rc[2][j];
      s3 += m[3] * rc[3][j];
    }
    *reinterpret_cast<float4 *>(delta + static_cast<size_t>(i) * C + c0) = make_float4(s0, s1, s2, s3);
  }
}

// Fused residual + Vanka apply (for small levels, where launches and memory
// latency dominate): 4 threads per cell, thread a evaluates the residual row
// b - J x of the cell's node a with the row arithmetic of k_spmv; the four
// rows are exchanged between the cell's lanes; thread a then forms the
// correction rows 3a..3a+2 with the arithmetic of k_vanka_apply.  Results are
// bitwise those of k_spmv followed by k_vanka_apply (a node shared by several
// cells is evaluated by each of them).  The workgroup size is a multiple of 4.
template <typename T>
__global__ void __launch_bounds__(256) k_vanka_smooth(LevelView L, const T *__restrict__ JQ, const T *__restrict__ JX,
                                                      const T *__restrict__ x, const T *__restrict__ b,
                                                      const T *__restrict__ inv, T *__restrict__ delta) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = gid >> 2, a = gid & 3;
  const bool live = c < L.C;
  T r0 = 0, r1 = 0, r2 = 0;
  if (live) {
    const int4 cn = L.cells[c];
    const int node = a == 0 ? cn.x : a == 1 ? cn.y : a == 2 ? cn.z : cn.w;
    T a0, a1, a2;
    spmv_row(L, JQ, JX, x, node, a0, a1, a2);
    r0 = b[3 * node] - a0;
    r1 = b[3 * node + 1] - a1;
    r2 = b[3 * node + 2] - a2;
  }
  const int lb = (threadIdx.x & 63) & ~3;
  T rc[12];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    rc[3 * q] = __shfl(r0, lb + q);
    rc[3 * q + 1] = __shfl(r1, lb + q);
    rc[3 * q + 2] = __shfl(r2, lb + q);
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int i = 3 * a + q;
    T s = 0;
#pragma unroll
    for (int j = 0; j < 12; ++j) s += inv[static_cast<size_t>(12 * i + j) * L.C + c] * rc[j];
    delta[static_cast<size_t>(i) * L.C + c] = s;
  }
}

// The same with sixteen lanes per cell: lane 4a + q sums partial q of the
// residual row of the cell's node a (the split of k_spmv4), the four
// partials are combined as (s0 + s1) + (s2 + s3) and the twelve residual
// values exchanged between the cell's lanes; lane i < 12 forms correction row
// i with the arithmetic of k_vanka_apply.  Bitwise k_spmv followed by
// k_vanka_apply.  The workgroup size is a multiple of 16.
template <typename T>
__device__ __forceinline__ void smooth16_item(const LevelView &L, const T *__restrict__ JQ,
                                              const T *__restrict__ JX, const T *__restrict__ x,
                                              const T *__restrict__ b, const T *__restrict__ inv,
                                              T *__restrict__ delta, int gid) {
  const int c = gid >> 4, sub = gid & 15, a = sub >> 2, q = sub & 3;
  const bool live = c < L.C;
  T p0 = 0, p1 = 0, p2 = 0;
  int node = 0;
  if (live) {
    const int4 cn = L.cells[c];
    node = a == 0 ? cn.x : a == 1 ? cn.y : a == 2 ? cn.z : cn.w;
    spmv_row_part(L, JQ, JX, x, node, q, p0, p1, p2);
  }
  const int lc = (threadIdx.x & 63) & ~15;   // first lane of the cell's sixteen
  const int la = lc + 4 * a;                 // first lane of node a's four
  T s[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    s[k][0] = __shfl(p0, la + k);
    s[k][1] = __shfl(p1, la + k);
    s[k][2] = __shfl(p2, la + k);
  }
  T r0 = 0, r1 = 0, r2 = 0;
  if (live) {
    r0 = b[3 * node] - ((s[0][0] + s[1][0]) + (s[2][0] + s[3][0]));
    r1 = b[3 * node + 1] - ((s[0][1] + s[1][1]) + (s[2][1] + s[3][1]));
    r2 = b[3 * node + 2] - ((s[0][2] + s[1][2]) + (s[2][2] + s[3][2]));
  }
  T rc[12];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rc[3 * k] = __shfl(r0, lc + 4 * k);
    rc[3 * k + 1] = __shfl(r1, lc + 4 * k);
    rc[3 * k + 2] = __shfl(r2, lc + 4 * k);
  }
  if (!live || sub >= 12) return;
  T acc = 0;
#pragma unroll
  for (int j = 0; j < 12; ++j) acc += inv[static_cast<size_t>(12 * sub + j) * L.C + c] * rc[j];
  delta[static_cast<size_t>(sub) * L.C + c] = acc;
}

template <typename T>
__global__ void __launch_bounds__(256) k_vanka_smooth16(LevelView L, const T *__restrict__ JQ,
                                                        const T *__restrict__ JX, const T *__restrict__ x,
                                                        const T *__restrict__ b, const T *__restrict__ inv,
                                                        T *__restrict__ delta) {
  smooth16_item(L, JQ, JX, x, b, inv, delta, static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x));
}

// x_j += omega / m_j * sum over the cells containing j of their corrections.
// The first kCadj (cell, slot) entries of a node are loaded before any of
// their corrections, so that a thread waits on two memory latencies, not on
// two per cell (small levels have too few waves to hide a dependent chain).
constexpr int kCadj = 8;

// Coloured multiplicative cell-Vanka, one colour: the cells of a colour
// share no node, so each adds omega times its correction inv_c r|_c to its
// own unknowns (no averaging, no write conflicts).  The products are summed
// as in apply_item.
template <typename T>
__global__ void __launch_bounds__(256) k_vanka_colour(LevelView L, const T *__restrict__ inv,
                                                      const T *__restrict__ r, const int *__restrict__ cells_k,
                                                      int n, T omega, T *__restrict__ x) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int c = cells_k[k];
  const int4 cn = L.cells[c];
  const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
  T rc[12];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int f = 0; f < 3; ++f) rc[3 * a + f] = r[3 * nn[a] + f];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < 12; ++j) s += inv[static_cast<size_t>(12 * i + j) * L.C + c] * rc[j];
    T *xi = x + 3 * nn[i / 3] + i % 3;
    *xi = fma_t(omega, s, *xi);
  }
}

// set: x is zero on entry (first sweep from a zero iterate): store instead of add.
// The updated values of node i (update_item without the store).
template <typename T>
__device__ __forceinline__ void update_row(const LevelView &L, const T *__restrict__ delta, T omega,
                                             const T *__restrict__ x, int i, bool set, T &v0, T &v1, T &v2) {
  T a0 = 0, a1 = 0, a2 = 0;
  const int e0 = L.cadj_ptr[i], e1 = L.cadj_ptr[i + 1];
  const size_t C = static_cast<size_t>(L.C);
  int ce[kCadj];
#pragma unroll
  for (int u = 0; u < kCadj; ++u) ce[u] = e0 + u < e1 ? L.cadj[e0 + u] : -1;
  T dv[kCadj][3];
#pragma unroll
  for (int u = 0; u < kCadj; ++u) {
    const int c = ce[u] >> 2, a = ce[u] & 3;
#pragma unroll
    for (int f = 0; f < 3; ++f) dv[u][f] = ce[u] >= 0 ? delta[static_cast<size_t>(3 * a + f) * C + c] : T(0);
  }
#pragma unroll
  for (int u = 0; u < kCadj; ++u) {
    if (ce[u] >= 0) {
      a0 += dv[u][0];
      a1 += dv[u][1];
      a2 += dv[u][2];
    }
  }
  for (int e = e0 + kCadj; e < e1; ++e) {
    const int c = L.cadj[e] >> 2, a = L.cadj[e] & 3;
    a0 += delta[static_cast<size_t>(3 * a) * C + c];
    a1 += delta[static_cast<size_t>(3 * a + 1) * C + c];
    a2 += delta[static_cast<size_t>(3 * a + 2) * C + c];
  }
  const T w = omega / static_cast<T>(e1 - e0);
  if (set) {
    v0 = w * a0;
    v1 = w * a1;
    v2 = w * a2;
  } else {
    v0 = fma_t(w, a0, x[3 * i]);
    v1 = fma_t(w, a1, x[3 * i + 1]);
    v2 = fma_t(w, a2, x[3 * i + 2]);
  }
}

template <typename T>
__device__ __forceinline__ void update_item(const LevelView &L, const T *__restrict__ delta, T omega,
                                            T *__restrict__ x, int i, bool set = false) {
  T v0, v1, v2;
  update_row(L, delta, omega, x, i, set, v0, v1, v2);
  x[3 * i] = v0;
  x[3 * i + 1] = v1;
  x[3 * i + 2] = v2;
}

template <typename T>
__global__ void __launch_bounds__(256) k_vanka_update(LevelView L, const T *__restrict__ delta, T omega, T *__restrict__ x,
                                                      int set) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L.N) update_item(L, delta, omega, x, i, set != 0);
}

// The same over the nodes in the order `order` (a permutation of the nodes,
// sorted by their lowest adjacent cell): the refinement numbers the coarse
// vertices, edge midpoints and centres in separate ranges, so consecutive
// node ids lie far apart, while consecutive cells are neighbours; in cell
// order a wavefront gathers the corrections of nearby cells.  Each node's
// update is update_item's.
template <typename T>
__global__ void __launch_bounds__(256) k_vanka_update_ordered(LevelView L, const int *__restrict__ order,
                                                              const T *__restrict__ delta, T omega,
                                                              T *__restrict__ x, int set) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < L.N) update_item(L, delta, omega, x, order[g], set != 0);
}

// -------------------------------------------------------------- transfers


// x_fine += P e_coarse (bilinear interpolation in parent coordinates).
template <typename T>
__device__ __forceinline__ void prolong_item(const TransferView &tv, const T *__restrict__ ec, T *__restrict__ xf,
                                             int f) {
  T v0, v1, v2;
  if (f < tv.Nc) {
    v0 = ec[3 * f];
    v1 = ec[3 * f + 1];
    v2 = ec[3 * f + 2];
  } else if (f < tv.Nc + tv.Ec) {
    const int a = tv.edge_ends[2 * (f - tv.Nc)], b = tv.edge_ends[2 * (f - tv.Nc) + 1];
    v0 = T(0.5) * (ec[3 * a] + ec[3 * b]);
    v1 = T(0.5) * (ec[3 * a + 1] + ec[3 * b + 1]);
    v2 = T(0.5) * (ec[3 * a + 2] + ec[3 * b + 2]);
  } else {
    const int4 cn = tv.ccells[f - tv.Nc - tv.Ec];
    v0 = T(0.25) * (ec[3 * cn.x] + ec[3 * cn.y] + ec[3 * cn.z] + ec[3 * cn.w]);
    v1 = T(0.25) * (ec[3 * cn.x + 1] + ec[3 * cn.y + 1] + ec[3 * cn.z + 1] + ec[3 * cn.w + 1]);
    v2 = T(0.25) * (ec[3 * cn.x + 2] + ec[3 * cn.y + 2] + ec[3 * cn.z + 2] + ec[3 * cn.w + 2]);
  }
  xf[3 * f] += v0;
  xf[3 * f + 1] += v1;
  xf[3 * f + 2] += v2;
}

template <typename T>
__global__ void k_prolong_add(TransferView tv, const T *__restrict__ ec, T *__restrict__ xf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < tv.Nf) prolong_item(tv, ec, xf, f);
}

// The coarse level's last node update (not a first sweep) fused into the
// prolongation that follows it: fine node f adds P e, where each coarse
// value it interpolates is that node's updated value, formed with the
// arithmetic of update_item (a coarse node is updated by each fine node that
// uses it).  Bitwise k_vanka_update followed by k_prolong_add; the coarse
// iterate itself is not written (nothing reads it afterwards).
template <typename T>
__global__ void k_update_prolong_add(TransferView tv, LevelView Lc, const T *__restrict__ delta, T omega,
                                     const T *__restrict__ xc, T *__restrict__ xf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tv.Nf) return;
  T v0, v1, v2;
  if (f < tv.Nc) {
    update_row(Lc, delta, omega, xc, f, false, v0, v1, v2);
  } else if (f < tv.Nc + tv.Ec) {
    const int a = tv.edge_ends[2 * (f - tv.Nc)], b = tv.edge_ends[2 * (f - tv.Nc) + 1];
    T a0, a1, a2, b0, b1, b2;
    update_row(Lc, delta, omega, xc, a, false, a0, a1, a2);
    update_row(Lc, delta, omega, xc, b, false, b0, b1, b2);
    v0 = T(0.5) * (a0 + b0);
    v1 = T(0.5) * (a1 + b1);
    v2 = T(0.5) * (a2 + b2);
  } else {
    const int4 cn = tv.ccells[f - tv.Nc - tv.Ec];
    T p[4][3];
    update_row(Lc, delta, omega, xc, cn.x, false, p[0][0], p[0][1], p[0][2]);
    update_row(Lc, delta, omega, xc, cn.y, false, p[1][0], p[1][1], p[1][2]);
    update_row(Lc, delta, omega, xc, cn.z, false, p[2][0], p[2][1], p[2][2]);
    update_row(Lc, delta, omega, xc, cn.w, false, p[3][0], p[3][1], p[3][2]);
    v0 = T(0.25) * (p[0][0] + p[1][0] + p[2][0] + p[3][0]);
    v1 = T(0.25) * (p[0][1] + p[1][1] + p[2][1] + p[3][1]);
    v2 = T(0.25) * (p[0][2] + p[1][2] + p[2][2] + p[3][2]);
  }
  xf[3 * f] += v0;
  xf[3 * f + 1] += v1;
  xf[3 * f + 2] += v2;
}

// r_coarse = P^T r_fine with the Dirichlet velocity rows of the coarse level zeroed.
template <typename T>
__device__ __forceinline__ void restrict_item(const TransferView &tv, const T *__restrict__ rf, T *__restrict__ rc,
                                              int j) {
  T a0 = 0, a1 = 0, a2 = 0;
  for (int e = tv.rptr[j]; e < tv.rptr[j + 1]; ++e) {
    const int f = tv.ridx[e];
    const T w = f < tv.Nc ? T(1) : (f < tv.Nc + tv.Ec ? T(0.5) : T(0.25));
    a0 += w * rf[3 * f];
    a1 += w * rf[3 * f + 1];
    a2 += w * rf[3 * f + 2];
  }
  if (tv.cflag[j] & 1) {
    a0 = 0;
    a1 = 0;
  }
  rc[3 * j] = a0;
  rc[3 * j + 1] = a1;
  rc[3 * j + 2] = a2;
}

// order: the coarse nodes in cell order (large levels, as for the Vanka
// update: the fine centres and edge midpoints a coarse node gathers are then
// close to those of its neighbours in the wavefront), or null.
template <typename T>
__global__ void k_restrict(TransferView tv, const T *__restrict__ rf, T *__restrict__ rc,
                           const int *__restrict__ order) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < tv.Nc) restrict_item(tv, rf, rc, order ? order[g] : g);
}

// r_coarse = P^T (b - J x) without storing the fine residual: each coarse
// node evaluates the residual rows of the fine nodes it restricts from (a fine
// node is evaluated by each coarse node that weights it) with the row
// arithmetic of k_spmv and sums them as k_restrict does: bitwise the result
// of k_spmv followed by k_restrict.
template <typename T>
__global__ void __launch_bounds__(256) k_restrict_residual(TransferView tv, LevelView Lf, const T *__restrict__ JQ,
                                                           const T *__restrict__ JX, const T *__restrict__ x,
                                                           const T *__restrict__ b, T *__restrict__ rc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= tv.Nc) return;
  T a0 = 0, a1 = 0, a2 = 0;
  for (int e = tv.rptr[j]; e < tv.rptr[j + 1]; ++e) {
    const int f = tv.ridx[e];
    T s0, s1, s2;
    spmv_row(Lf, JQ, JX, x, f, s0, s1, s2);
    const T r0 = b[3 * f] - s0, r1 = b[3 * f + 1] - s1, r2 = b[3 * f + 2] - s2;
    const T w = f < tv.Nc ? T(1) : (f < tv.Nc + tv.Ec ? T(0.5) : T(0.25));
    a0 += w * r0;
    a1 += w * r1;
    a2 += w * r2;
  }
  if (tv.cflag[j] & 1) {
    a0 = 0;
    a1 = 0;
  }
  rc[3 * j] = a0;
  rc[3 * j + 1] = a1;
  rc[3 * j + 2] = a2;
}

// -------------------------------------------------------------- coarse solve
// Dense copy of the level-0 operator (FP64, row-major n x n, n = 3 N); padding
// slots add zeros.
template <typename T>
__global__ void __launch_bounds__(64) k_dense_from_sell(LevelView L, const T *__restrict__ JQ, const T *__restrict__ JX,
                                  double *__restrict__ A, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.N) return;   // row stride n (= 2 * 3 N for the Gauss-Jordan workspace)
  const int s = i / kS, lane = i % kS;
  for (int k = 0; k < L.wq[s]; ++k) {
    const int j = L.colq[(L.oq[s] + k) * kS + lane];
    for (int f = 0; f < 3; ++f)
      for (int g = 0; g < 3; ++g)
        A[static_cast<size_t>(3 * i + f) * n + 3 * j + g] +=
            static_cast<double>(JQ[(static_cast<size_t>(L.oq[s] + k) * 9 + 3 * f + g) * kS + lane]);
  }
  for (int k = 0; k < L.wx[s]; ++k) {
    const int j = L.colx[(L.ox[s] + k) * kS + lane];
    A[static_cast<size_t>(3 * i + 2) * n + 3 * j + 2] +=
        static_cast<double>(JX[static_cast<size_t>(L.ox[s] + k) * kS + lane]);
  }
}

// Block-diagonal level 0 (simulation batches; one block for a single mesh):
// node i belongs to block blk[i] with local index g2l[i].  Block s of the
// workspace is [A_s | I] padded to nb unknowns (nb x 2 nb, row-major; the
// padding rows and columns hold the identity).
template <typename T>
__global__ void __launch_bounds__(64) k_dense_from_sell_blk(LevelView L, const T *__restrict__ JQ,
                                                           const T *__restrict__ JX, const int *__restrict__ g2l,
                                                           const int *__restrict__ blk, int nb,
                                                           double *__restrict__ W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.N) return;
  const int s = i / kS, lane = i % kS;
  const size_t w2 = 2 * static_cast<size_t>(nb);
  double *Ws = W + static_cast<size_t>(blk[i]) * nb * w2;
  const int li = g2l[i];
  for (int k = 0; k < L.wq[s]; ++k) {
    const int lj = g2l[L.colq[(L.oq[s] + k) * kS + lane]];
    for (int f = 0; f < 3; ++f)
      for (int g = 0; g < 3; ++g)
        Ws[(3 * li + f) * w2 + 3 * lj + g] +=
            static_cast<double>(JQ[(static_cast<size_t>(L.oq[s] + k) * 9 + 3 * f + g) * kS + lane]);
  }
  for (int k = 0; k < L.wx[s]; ++k) {
    const int lj = g2l[L.colx[(L.ox[s] + k) * kS + lane]];
    Ws[(3 * li + 2) * w2 + 3 * lj + 2] += static_cast<double>(JX[static_cast<size_t>(L.ox[s] + k) * kS + lane]);
  }
}

// Identity right halves and identity padding rows of every block
// (bdof[s nb + r] < 0 marks a padding unknown).
__global__ void k_gjb_init(int nblk, int nb, const int *__restrict__ bdof, double *__restrict__ W) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int sb = blockIdx.y;
  if (r >= nb || sb >= nblk) return;
  const size_t w2 = 2 * static_cast<size_t>(nb);
  double *Ws = W + static_cast<size_t>(sb) * nb * w2;
  Ws[r * w2 + nb + r] = 1.0;
  if (bdof[static_cast<size_t>(sb) * nb + r] < 0) Ws[r * w2 + r] = 1.0;
}

// Multi-workgroup Gauss-Jordan, one pivot column k per pair of launches.
// Pivot step (one workgroup): partial pivoting on column k, row swap,
// normalisation of the pivot row, copies of the pivot row (prow) and of
// column k (colk, 0 at the pivot row).
__global__ void __launch_bounds__(256) k_gj_pivot(int n, int k, double *__restrict__ W,
                                                  double *__restrict__ prow, double *__restrict__ colk) {
  __shared__ double sval[256];
  __shared__ int sidx[256];
  const int tid = threadIdx.x, w = 2 * n;
  double best = -1.0;
  int bi = k;
  for (int i = k + tid; i < n; i += 256) {
    const double v = fabs(W[static_cast<size_t>(i) * w + k]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  sval[tid] = best;
  sidx[tid] = bi;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      const double ov = sval[tid + off];
      const int oi = sidx[tid + off];
      if (ov > sval[tid] || (ov == sval[tid] && oi < sidx[tid])) {
        sval[tid] = ov;
        sidx[tid] = oi;
      }
    }
    __syncthreads();
  }
  const int p = sidx[0];
  const double piv = W[static_cast<size_t>(p) * w + k];
  const double ip = 1.0 / piv;
  for (int j = tid; j < w; j += 256) {
    const double a = W[static_cast<size_t>(k) * w + j];
    const double b = W[static_cast<size_t>(p) * w + j];
    const double nb = b * ip;
    W[static_cast<size_t>(p) * w + j] = a;
    W[static_cast<size_t>(k) * w + j] = nb;
    prow[j] = nb;
  }
  __syncthreads();
  for (int i = tid; i < n; i += 256) colk[i] = (i == k) ? 0.0 : W[static_cast<size_t>(i) * w + k];
}

// Elimination step: W[i][j] -= colk[i] * prow[j] for all rows i != k.
__global__ void k_gj_elim(int n, int k, double *__restrict__ W, const double *__restrict__ prow,
                          const double *__restrict__ colk) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  const int w = 2 * n;
  if (j >= w || i == k) return;
  const double f = colk[i];
  if (f != 0.0) W[static_cast<size_t>(i) * w + j] -= f * prow[j];
}

// Blocked Gauss-Jordan on [A | I] (n x 2n, row-major) with implicit
// pivoting: rows stay in place; column k's pivot is a not yet used row of
// largest |value| (see the panel's pivot key), recorded in piv[k].  After
// all columns, row piv[k] of the right half is row k of A^{-1}.
//
// Panel step (one workgroup; thread t holds rows t + r * blockDim, r < RPT,
// of the panel's kGjB columns in registers): the panel's column steps are
// run on the panel alone, in place.  Their composite is
// G = I + sum_r (G e_{p_r} - e_{p_r}) e_{p_r}^T (p_r the panel's pivot rows),
// and G e_{p_r} is the unit column e_{p_r} carried along from step r on (the
// steps before r leave it unchanged): in place, column r of the panel turns
// into G e_{p_r} at step r (the classic in-place inversion update).  Output
// Z = [G e_{p_r}] - [e_{p_r}] and the pivot rows.  The pivot is chosen on a
// 32-bit key: |value| rounded to FP32 with its low kGjRowBits<RPT> mantissa
// bits replaced by (2^bits - 1 - row) (rows within 2^-13 relative for
// RPT = 1, 2^-12 for RPT = 2, count as equal; the lower row wins), reduced by
// one integer maximum.  RPT = 1 takes
// n <= 1024 (1024 threads), RPT = 2 takes n <= 1536 (768 threads: three
// wavefronts per SIMD leave room for the 64 FP64 panel values per thread).
constexpr int kGjB = 32;
template <int RPT>
constexpr int kGjRowBits = RPT == 1 ? 10 : 11;
template <int RPT>
constexpr int kGjMaxRows = RPT == 1 ? 1024 : 1536;
// a[c] for a runtime c without dynamic register indexing
__device__ __forceinline__ double gj_pick(const double (&a)[kGjB], int c) {
  double v = 0.0;
#pragma unroll
  for (int t = 0; t < kGjB; ++t) v = (t == c) ? a[t] : v;
  return v;
}

template <int RPT>
__global__ void __launch_bounds__(RPT == 1 ? 1024 : 768)
    k_gjb_panel(int n, int k0, int b, const double *__restrict__ W, int *__restrict__ used_g, int *__restrict__ piv,
                double *__restrict__ Z) {
  constexpr unsigned kMask = (1u << kGjRowBits<RPT>) - 1u;
  // block blockIdx.x of a block-diagonal batch: its own workspace and records
  W += static_cast<size_t>(blockIdx.x) * n * 2 * n;
  used_g += static_cast<size_t>(blockIdx.x) * n;
  piv += static_cast<size_t>(blockIdx.x) * n;
  Z += static_cast<size_t>(blockIdx.x) * n * kGjB;
  __shared__ double prow[2][kGjB];
  __shared__ unsigned rk[2][16];
  __shared__ int spiv[kGjB];
  const int nt = blockDim.x;
  const int nw = nt >> 6;
  const size_t w2 = 2 * static_cast<size_t>(n);
  double R[RPT][kGjB];
  bool used[RPT], live[RPT];
  int row[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    row[r] = threadIdx.x + r * nt;
    live[r] = row[r] < n;
#pragma unroll
    for (int c = 0; c < kGjB; ++c) R[r][c] = (live[r] && c < b) ? W[row[r] * w2 + k0 + c] : 0.0;
    used[r] = !live[r] || (k0 > 0 && used_g[row[r]] != 0);
  }
  // fully unrolled over the panel's columns: every register index below is a
  // constant (b is the same for the whole workgroup, so the barriers inside
  // the guard are reached by every thread)
#pragma clang loop unroll(full)
  for (int c = 0; c < kGjB; ++c) {
    if (c < b) {
      const int q = c & 1;
      double rc[RPT];
      unsigned key = 0u;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        rc[r] = gj_pick(R[r], c);
        const unsigned kr = used[r] ? 0u
                                    : ((__float_as_uint(fabsf(static_cast<float>(rc[r]))) & ~kMask) |
                                       (kMask - static_cast<unsigned>(row[r])));
        key = max(key, kr);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) key = max(key, static_cast<unsigned>(__shfl_xor(static_cast<int>(key), off)));
      if ((threadIdx.x & 63) == 0) rk[q][threadIdx.x >> 6] = key;
      __syncthreads();
      key = rk[q][0];
      for (int w = 1; w < nw; ++w) key = max(key, rk[q][w]);
      const int p = static_cast<int>(kMask - (key & kMask));
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        if (row[r] == p) {
          const double ip = 1.0 / rc[r];
#pragma unroll
          for (int cc = 0; cc < kGjB; ++cc) {
            R[r][cc] = (cc == c) ? ip : R[r][cc] * ip;
            prow[q][cc] = R[r][cc];
          }
          used[r] = true;
          piv[k0 + c] = p;
          spiv[c] = p;
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        if (row[r] != p && live[r]) {
#pragma unroll
          for (int cc = 0; cc < kGjB; ++cc) R[r][cc] = ((cc == c) ? 0.0 : R[r][cc]) - rc[r] * prow[q][cc];
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r)
    if (live[r]) used_g[row[r]] = used[r] ? 1 : 0;
  __syncthreads();   // spiv[] of the last step is visible
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (!live[r]) continue;
#pragma unroll
    for (int t = 0; t < kGjB; ++t)
      if (t < b) Z[static_cast<size_t>(row[r]) * b + t] = R[r][t] - ((row[r] == spiv[t]) ? 1.0 : 0.0);
  }
}

// Trailing update of a panel, out of place: for the columns j >= k0 + b,
// Wn[i, j] = Wo[i, j] + sum_r Z[i, r] Wo[p_r, j].  A block holds 64 columns x
// 16 rows; the b pivot-row values of its columns are staged in LDS.
__global__ void __launch_bounds__(256) k_gjb_update(int n, int k0, int b, const double *__restrict__ Wo,
                                                    const double *__restrict__ Z, const int *__restrict__ piv,
                                                    double *__restrict__ Wn) {
  const size_t sb = blockIdx.z;   // block of a block-diagonal batch
  Wo += sb * n * 2 * n;
  Wn += sb * n * 2 * n;
  Z += sb * n * kGjB;
  piv += sb * n;
  __shared__ double pr[kGjB][64];
  const size_t w2 = 2 * static_cast<size_t>(n);
  const int jl = threadIdx.x & 63, ig = threadIdx.x >> 6;
  const int j = k0 + b + blockIdx.x * 64 + jl;
  const bool colok = j < 2 * n;
  for (int r = ig; r < b; r += 4) pr[r][jl] = colok ? Wo[piv[k0 + r] * w2 + j] : 0.0;
  __syncthreads();
  if (!colok) return;
  for (int t = 0; t < 4; ++t) {
    const int i = blockIdx.y * 16 + ig * 4 + t;
    if (i >= n) break;
    double acc = Wo[i * w2 + j];
    const double *zi = Z + static_cast<size_t>(i) * b;
    for (int r = 0; r < b; ++r) acc += zi[r] * pr[r][jl];
    Wn[i * w2 + j] = acc;
  }
}

// Compact inverse: Ainv[k, :] = W[piv[k], n:2n].
__global__ void k_gjb_extract(int n, const double *__restrict__ W, const int *__restrict__ piv,
                              double *__restrict__ Ainv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  const size_t sb = blockIdx.z;
  W += sb * n * 2 * n;
  piv += sb * n;
  Ainv += sb * n * n;
  if (j >= n) return;
  Ainv[static_cast<size_t>(k) * n + j] = W[piv[k] * 2 * static_cast<size_t>(n) + n + j];
}

// x = A^{-1} b, the inverse row-major with leading dimension ld: one
// wavefront per row (four rows per workgroup); lane l sums the columns
// k = l (mod 64) in four independent partial sums (more loads in flight),
// combined as (s0 + s1) + (s2 + s3), then a butterfly over the wavefront.
template <typename T>
__global__ void __launch_bounds__(256) k_dense_solve_w(int n, const double *__restrict__ Ainv, size_t ld,
                                                       const T *__restrict__ b, T *__restrict__ x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (row < n) {
    const double *r = Ainv + static_cast<size_t>(row) * ld;
    int k = lane;
    for (; k + 192 < n; k += 256) {
      s0 += r[k] * static_cast<double>(b[k]);
      s1 += r[k + 64] * static_cast<double>(b[k + 64]);
      s2 += r[k + 128] * static_cast<double>(b[k + 128]);
      s3 += r[k + 192] * static_cast<double>(b[k + 192]);
    }
    for (; k < n; k += 64) s0 += r[k] * static_cast<double>(b[k]);
  }
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (row < n && lane == 0) x[row] = static_cast<T>(s);
}

// x = blockdiag(A_s)^{-1} b on the padded blocks (compact inverses, nb x nb
// each): 32 lanes per row split the dot product; padding unknowns skipped.
template <typename T>
__device__ __forceinline__ void dense_row_blk(int nblk, int nb, const double *__restrict__ Ainv,
                                              const int *__restrict__ bdof, const T *__restrict__ b,
                                              T *__restrict__ x, int row, int lane) {
  const bool ok = row < nblk * nb;
  const int sb = ok ? row / nb : 0;
  const int dst = ok ? bdof[row] : -1;
  double s = 0.0;
  if (dst >= 0) {
    const double *r = Ainv + static_cast<size_t>(row) * nb;
    const int *bd = bdof + static_cast<size_t>(sb) * nb;
    for (int k = lane; k < nb; k += 32) {
      const int g = bd[k];
      if (g >= 0) s += r[k] * static_cast<double>(b[g]);
    }
  }
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, 32);
  if (dst >= 0 && lane == 0) x[dst] = static_cast<T>(s);
}

template <typename T>
__global__ void __launch_bounds__(256) k_dense_solve_blk(int nblk, int nb, const double *__restrict__ Ainv,
                                                         const int *__restrict__ bdof, const T *__restrict__ b,
                                                         T *__restrict__ x) {
  dense_row_blk(nblk, nb, Ainv, bdof, b, x, blockIdx.x * 8 + (threadIdx.x >> 5), threadIdx.x & 31);
}

__global__ void k_identity_right(int n, double *__restrict__ W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  W[static_cast<size_t>(i) * 2 * n + n + i] = 1.0;
}

// -------------------------------------------------------------- BLAS-1
// partial[b * m + v] = sum over this block's chunk of V[v] . w  (FP64 accumulation)
template <typename T>
__global__ void k_multidot(int n, int m, const T *__restrict__ Vb, size_t ld, const T *__restrict__ w,
                           double *__restrict__ partial) {
  __shared__ double sh[256];
  const int v = blockIdx.y;
  const T *vv = Vb + static_cast<size_t>(v) * ld;
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    s += static_cast<double>(vv[i]) * static_cast<double>(w[i]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[static_cast<size_t>(blockIdx.x) * m + v] = sh[0];
}

// out[v] = sum_b partial[b * m + v]  (one block per v, deterministic order)
__global__ void k_reduce_partials(int nb, int m, const double *__restrict__ partial,
                                  double *__restrict__ out) {
  __shared__ double sh[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[static_cast<size_t>(b) * m + v];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sh[0];
}

// w -= sum_v h[v] V[v]   (h read from device memory)
template <typename T>
__global__ void k_multi_axpy(int n, int m, const T *__restrict__ Vb, size_t ld,
                             const double *__restrict__ h, T *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int v = 0; v < m; ++v) s += h[v] * static_cast<double>(Vb[static_cast<size_t>(v) * ld + i]);
  w[i] = static_cast<T>(static_cast<double>(w[i]) - s);
}

// x = sum_v y[v] Z[v]  (y on device)
template <typename T>
__global__ void k_combine(int n, int m, const T *__restrict__ Zb, size_t ld,
                          const double *__restrict__ y, T *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int v = 0; v < m; ++v) s += y[v] * static_cast<double>(Zb[static_cast<size_t>(v) * ld + i]);
  x[i] = static_cast<T>(static_cast<double>(x[i]) + s);
}

// y = x / sqrt(h2) (y untouched when h2 <= 0): the next Krylov basis vector,
// normalised with the squared norm the device has just reduced.
template <typename T>
__global__ void k_scale_by_norm(int n, const double *__restrict__ h2, const T *__restrict__ x, T *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double hn = sqrt(fmax(*h2, 0.0));
  if (i < n && hn > 0.0) y[i] = static_cast<T>((1.0 / hn) * static_cast<double>(x[i]));
}

template <typename T>
__global__ void k_scale_copy(int n, double a, const T *__restrict__ x, T *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = static_cast<T>(a * static_cast<double>(x[i]));
}

template <typename A, typename B>
__global__ void k_convert(int n, const A *__restrict__ x, B *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = static_cast<B>(x[i]);
}

// x <- x + a (x - y): linear extrapolation from the two previous states.
__global__ void k_extrapolate(int n, double a, const double *__restrict__ y, double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += a * (x[i] - y[i]);
}

template <typename T>
__global__ void k_add_to_f64(int n, const T *__restrict__ w, double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += static_cast<double>(w[i]);
}

// --------------------------------------------- single-workgroup coarse cycle
// The bottom of a V-cycle (levels top..1 and the level-0 solve, top <= 2) in
// one workgroup: the phases of the multi-launch V-cycle (zero the iterate,
// Vanka sweeps, residual, restriction, coarse solve, prolongation) run in the
// same order, separated by workgroup barriers instead of kernel boundaries,
// each phase looping over its items with the item functions of the kernels
// above (one thread per cell or node: in one workgroup, one pass with long
// independent load chains beats several passes with short ones), whose sums
// are ordered as in every launch variant, so every value is bitwise the one
// of the multi-launch path.
constexpr int kSmallLevels = 3;
template <typename T>
struct SmallLevel {
  LevelView L;
  TransferView tv;            // from the next coarser level (unused on level 0)
  const T *JQ, *JX, *inv;
  T *delta, *r, *b, *x;
};
template <typename T>
struct SmallCycle {
  SmallLevel<T> lv[kSmallLevels];
  int top, nu_pre, nu_post, nblk, nb;
  T omega;
  const double *Ainv;
  const int *bdof;
};

template <typename T>
__device__ void small_sweep(const SmallLevel<T> &V, T omega, bool zero_start) {
  const T *r = V.b;
  if (!zero_start) {
    for (int i = threadIdx.x; i < V.L.N; i += blockDim.x) spmv_item(V.L, V.JQ, V.JX, V.x, V.b, V.r, i);
    __syncthreads();
    r = V.r;
  }
  for (int c = threadIdx.x; c < V.L.C; c += blockDim.x) apply_item(V.L, V.inv, r, V.delta, c);
  __syncthreads();
  for (int i = threadIdx.x; i < V.L.N; i += blockDim.x) update_item(V.L, V.delta, omega, V.x, i, zero_start);
  __syncthreads();
}

// Capacity (doubles) of the workgroup's copy of the coarse right-hand side.
constexpr int kSmallDenseLds = 4096;

template <typename T>
__global__ void __launch_bounds__(1024) k_vcycle_small(SmallCycle<T> P) {
  __shared__ double bl[kSmallDenseLds];
  const int tid = threadIdx.x, nt = blockDim.x;
#pragma unroll
  for (int l = kSmallLevels - 1; l >= 1; --l) {
    if (l > P.top) continue;
    const SmallLevel<T> &V = P.lv[l];
    if (P.nu_pre == 0) {   // otherwise the first sweep stores into x
      for (int i = tid; i < 3 * V.L.N; i += nt) V.x[i] = T(0);
      __syncthreads();
    }
    for (int k = 0; k < P.nu_pre; ++k) small_sweep(V, P.omega, k == 0);
    for (int i = tid; i < V.L.N; i += nt) spmv_item(V.L, V.JQ, V.JX, V.x, V.b, V.r, i);
    __syncthreads();
    for (int j = tid; j < V.tv.Nc; j += nt) restrict_item(V.tv, V.r, P.lv[l - 1].b, j);
    __syncthreads();
  }
  const int rows = P.nblk * P.nb;
  if (rows <= kSmallDenseLds) {
    // coarse solve x = A^-1 b with b gathered once into LDS (zero where a
    // block row is unused) and four rows per 32-lane group in flight; each
    // row is summed as in dense_row_blk (an unused column adds an exact
    // zero to a sum that starts at +0, which leaves it unchanged)
    for (int k = tid; k < rows; k += nt) {
      const int g = P.bdof[k];
      bl[k] = g >= 0 ? static_cast<double>(P.lv[0].b[g]) : 0.0;
    }
    __syncthreads();
    const int grp = tid >> 5, lane = tid & 31, ngrp = nt >> 5;
    for (int r0 = grp; r0 < rows; r0 += 4 * ngrp) {
      double s[4] = {0.0, 0.0, 0.0, 0.0};
      int dst[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = r0 + u * ngrp;
        dst[u] = row < rows ? P.bdof[row] : -1;
        if (dst[u] >= 0) {
          const double *ar = P.Ainv + static_cast<size_t>(row) * P.nb;
          const double *bb = bl + (row / P.nb) * P.nb;
          for (int k = lane; k < P.nb; k += 32) s[u] += ar[k] * bb[k];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) s[u] += __shfl_xor(s[u], off, 32);
        if (dst[u] >= 0 && lane == 0) P.lv[0].x[dst[u]] = static_cast<T>(s[u]);
      }
    }
  } else {
    for (int row = tid >> 5; row < rows; row += nt >> 5)
      dense_row_blk(P.nblk, P.nb, P.Ainv, P.bdof, P.lv[0].b, P.lv[0].x, row, tid & 31);
  }
  __syncthreads();
#pragma unroll
  for (int l = 1; l < kSmallLevels; ++l) {
    if (l > P.top) continue;
    const SmallLevel<T> &V = P.lv[l];
    for (int f = tid; f < V.tv.Nf; f += nt) prolong_item(V.tv, P.lv[l - 1].x, V.x, f);
    __syncthreads();
    for (int k = 0; k < P.nu_post; ++k) small_sweep(V, P.omega, false);
  }
}

// --------------------------------------------------------- flow functionals
// J_div = int |div v|^2 (Sec. 3.3): per cell sum over the 2x2 Gauss points of
// det J (u_x + v_y)^2, reduced per workgroup in a fixed order into partial[].
__global__ void __launch_bounds__(256) k_jdiv_partial(LevelView L, const double *__restrict__ x,
                                                      double *__restrict__ partial) {
  __shared__ double sh[256];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (c < L.C) {
    const int4 cn = L.cells[c];
    const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
    double X[4], Y[4], U[4], V[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double2 p = L.xy[nn[a]];
      X[a] = p.x;
      Y[a] = p.y;
      U[a] = x[3 * nn[a]];
      V[a] = x[3 * nn[a] + 1];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double N[4], gx[4], gy[4], det;
      q1_point(X, Y, q, N, gx, gy, det);
      double d = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) d += gx[a] * U[a] + gy[a] * V[a];
      s += det * d * d;
    }
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Velocity error of a field a against a reference b on one level (Sec. 3.4:
// relative errors of the velocity against the fine solution), partial sums per
// workgroup: partial[4 w + 0] = int |v_a - v_b|^2, [1] = int |v_b|^2 (2x2 Gauss
// per cell, the Q1 fields of the nodal values), [2] = sum_i |v_a,i - v_b,i|^2,
// [3] = sum_i |v_b,i|^2 over the nodes.  Thread i covers cell i and node i.
__global__ void __launch_bounds__(256) k_vel_error_partial(LevelView L, const double *__restrict__ a,
                                                           const double *__restrict__ b,
                                                           double *__restrict__ partial) {
  __shared__ double sh[4][256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < L.C) {
    const int4 cn = L.cells[i];
    const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
    double X[4], Y[4], DU[4], DV[4], BU[4], BV[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 p = L.xy[nn[k]];
      X[k] = p.x;
      Y[k] = p.y;
      BU[k] = b[3 * nn[k]];
      BV[k] = b[3 * nn[k] + 1];
      DU[k] = a[3 * nn[k]] - BU[k];
      DV[k] = a[3 * nn[k] + 1] - BV[k];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double N[4], gx[4], gy[4], det;
      q1_point(X, Y, q, N, gx, gy, det);
      double du = 0.0, dv = 0.0, bu = 0.0, bv = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        du += N[k] * DU[k];
        dv += N[k] * DV[k];
        bu += N[k] * BU[k];
        bv += N[k] * BV[k];
      }
      s[0] += det * (du * du + dv * dv);
      s[1] += det * (bu * bu + bv * bv);
    }
  }
  if (i < L.N) {
    const double bu = b[3 * i], bv = b[3 * i + 1];
    const double du = a[3 * i] - bu, dv = a[3 * i + 1] - bv;
    s[2] = du * du + dv * dv;
    s[3] = bu * bu + bv * bv;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
#pragma unroll
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// Drag and lift contributions of each obstacle edge (Sec. 3.3):
// -int_e (nu grad v - p I) n . e_{x,y} ds with 2-point Gauss quadrature on the
// edge, grad v and p of the fluid cell, n its outward normal (into the
// obstacle).  edges[2 e] = cell, edges[2 e + 1] = local side a (corners a,
// a + 1 counter-clockwise).  out[2 e] = drag part, out[2 e + 1] = lift part.
__global__ void k_edge_forces(LevelView L, int ne, const int *__restrict__ edges, const double *__restrict__ x,
                              double nu_const, double *__restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int c = edges[2 * e], a = edges[2 * e + 1], a1 = (a + 1) & 3;
  const int4 cn = L.cells[c];
  const int nn[4] = {cn.x, cn.y, cn.z, cn.w};
  double X[4], Y[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const double2 p = L.xy[nn[b]];
    X[b] = p.x;
    Y[b] = p.y;
  }
  const double ex = X[a1] - X[a], ey = Y[a1] - Y[a];
  const double len = sqrt(ex * ex + ey * ey);
  const double nx = ey / len, ny = -ex / len;
  const double nu = L.nnu ? L.nnu[nn[a]] : nu_const;
  const double g = 0.57735026918962576451;
  double fx = 0.0, fy = 0.0;
  for (int k = 0; k < 2; ++k) {
    const double t = k == 0 ? -g : g;
    const double xi = 0.5 * (1.0 - t) * kVX[a] + 0.5 * (1.0 + t) * kVX[a1];
    const double eta = 0.5 * (1.0 - t) * kVY[a] + 0.5 * (1.0 + t) * kVY[a1];
    double N[4], dxi[4], deta[4], j11 = 0, j12 = 0, j21 = 0, j22 = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      N[b] = 0.25 * (1.0 + kVX[b] * xi) * (1.0 + kVY[b] * eta);
      dxi[b] = 0.25 * kVX[b] * (1.0 + kVY[b] * eta);
      deta[b] = 0.25 * kVY[b] * (1.0 + kVX[b] * xi);
      j11 += dxi[b] * X[b];
      j12 += deta[b] * X[b];
      j21 += dxi[b] * Y[b];
      j22 += deta[b] * Y[b];
    }
    const double id = 1.0 / (j11 * j22 - j12 * j21);
    double ux = 0, uy = 0, vx = 0, vy = 0, p = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double gxb = (j22 * dxi[b] - j21 * deta[b]) * id;
      const double gyb = (-j12 * dxi[b] + j11 * deta[b]) * id;
      const double u = x[3 * nn[b]], v = x[3 * nn[b] + 1];
      ux += gxb * u;
      uy += gyb * u;
      vx += gxb * v;
      vy += gyb * v;
      p += N[b] * x[3 * nn[b] + 2];
    }
    const double w = 0.5 * len;
    fx -= w * (nu * (ux * nx + uy * ny) - p * nx);
    fy -= w * (nu * (vx * nx + vy * ny) - p * ny);
  }
  out[2 * e] = fx;
  out[2 * e + 1] = fy;
}

// out[2 k + f] = sum over the edges of obstacle k (ptr CSR) of vals[2 e + f],
// in edge order (one thread per obstacle and component).
__global__ void k_sum_ranges(int nk, const int *__restrict__ ptr, const double *__restrict__ vals,
                             double *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * nk) return;
  const int k = t >> 1, f = t & 1;
  double s = 0.0;
  for (int e = ptr[k]; e < ptr[k + 1]; ++e) s += vals[2 * e + f];
  out[t] = s;
}

// ---------------------------------------------------- per-simulation BLAS-1
// Batches: the unknowns of one simulation ("segment") form runs of the node
// order; runs are cut into chunks (start and length in unknowns) listed
// segment by segment in increasing position.  Segmented reductions sum each
// chunk in a fixed order, then each segment's chunks in list order, so the
// result does not depend on scheduling.  segn holds the segment of each node.

// partial[c * m + v] = V[v] . w over chunk c  (FP64 accumulation)
template <typename T>
__global__ void k_multidot_chunks(const int *__restrict__ cstart, const int *__restrict__ clen, int m,
                                  const T *__restrict__ Vb, size_t ld, const T *__restrict__ w,
                                  double *__restrict__ partial) {
  __shared__ double sh[256];
  const int c = blockIdx.x, v = blockIdx.y;
  const T *vv = Vb + static_cast<size_t>(v) * ld;
  const int i0 = cstart[c], i1 = i0 + clen[c];
  double s = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x)
    s += static_cast<double>(vv[i]) * static_cast<double>(w[i]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[static_cast<size_t>(c) * m + v] = sh[0];
}

// out[g * m + v] = sum over the chunks of segment g (seg_ptr CSR) of partial
__global__ void k_reduce_seg(const int *__restrict__ seg_ptr, int m, const double *__restrict__ partial,
                             double *__restrict__ out) {
  __shared__ double sh[256];
  const int g = blockIdx.x, v = blockIdx.y;
  double s = 0.0;
  for (int c = seg_ptr[g] + threadIdx.x; c < seg_ptr[g + 1]; c += blockDim.x)
    s += partial[static_cast<size_t>(c) * m + v];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[static_cast<size_t>(g) * m + v] = sh[0];
}

// w -= sum_v h[seg, v] V[v]  (coefficients per segment, stride hs)
template <typename T>
__global__ void k_multi_axpy_seg(int n, int m, const T *__restrict__ Vb, size_t ld, const double *__restrict__ h,
                                 int hs, const int *__restrict__ segn, T *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *hg = h + static_cast<size_t>(segn[i / 3]) * hs;
  double s = 0.0;
  for (int v = 0; v < m; ++v) s += hg[v] * static_cast<double>(Vb[static_cast<size_t>(v) * ld + i]);
  w[i] = static_cast<T>(static_cast<double>(w[i]) - s);
}

// x += sum_v y[seg, v] Z[v]
template <typename T>
__global__ void k_combine_seg(int n, int m, const T *__restrict__ Zb, size_t ld, const double *__restrict__ y,
                              int ys, const int *__restrict__ segn, T *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *yg = y + static_cast<size_t>(segn[i / 3]) * ys;
  double s = 0.0;
  for (int v = 0; v < m; ++v) s += yg[v] * static_cast<double>(Zb[static_cast<size_t>(v) * ld + i]);
  x[i] = static_cast<T>(static_cast<double>(x[i]) + s);
}

// y = a[seg] x
template <typename T>
__global__ void k_scale_copy_seg(int n, const double *__restrict__ a, const int *__restrict__ segn,
                                 const T *__restrict__ x, T *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = static_cast<T>(a[segn[i / 3]] * static_cast<double>(x[i]));
}

}  // namespace
}  // namespace dnnmg
