// DNN-MG correction (Algorithm 1, the correction after the coarse step): patch tables, the GRU patch
// network in BF16 MFMA GEMMs, and the C-ABI calls dnnmg_net_* / dnnmg_correct.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "net.h"

using namespace dnnmg;

namespace dnnmg {

namespace {

// Fine-level grid of level-(L-1) cell `c` refined `depth` times, written into
// g (stride S) at offset (ox, oy) with `size` fine cells per side.
void fill_grid(const std::vector<std::unique_ptr<DevLevel>> &lv, int lvl, int c, int depth, int ox,
               int oy, int size, int S, int *g) {
  if (depth == 0) {
    const int *q = &lv[lvl]->h.cells[4 * c];
    g[oy * S + ox] = q[0];
    g[oy * S + ox + size] = q[1];
    g[(oy + size) * S + ox + size] = q[2];
    g[(oy + size) * S + ox] = q[3];
    return;
  }
  const int half = size / 2;
  const int offs[4][2] = {{0, 0}, {half, 0}, {half, half}, {0, half}};
  for (int k = 0; k < 4; ++k)
    fill_grid(lv, lvl + 1, 4 * c + k, depth - 1, ox + offs[k][0], oy + offs[k][1], half, S, g);
}

void build_patch_tables(Net &n) {
  Ctx &c = *n.ctx;
  // patch roots: level-(L-1) cells (block patches) or level-L cells
  const int root = n.patch == DNNMG_PATCH_CELL ? n.L : n.L - 1;
  const HostLevel &hp = c.levels[root]->h;
  const HostLevel &hf = c.levels[n.F]->h;
  n.B = hp.C;
  std::vector<int> grid(static_cast<size_t>(n.B) * n.S2, -1);
  for (int p = 0; p < n.B; ++p)
    fill_grid(c.levels, root, p, n.F - root, 0, 0, n.S - 1, n.S, &grid[static_cast<size_t>(p) * n.S2]);
  for (int v : grid)
    if (v < 0 || v >= hf.N) throw DnnmgError{DNNMG_EDEVICE, "patch grid construction failed"};
  std::vector<int> ptr(hf.N + 1, 0);
  for (int v : grid) ptr[v + 1]++;
  for (int i = 0; i < hf.N; ++i) ptr[i + 1] += ptr[i];
  std::vector<int> adj(ptr[hf.N]);
  {
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (size_t e = 0; e < grid.size(); ++e) adj[fill[grid[e]]++] = static_cast<int>(e);
  }
  // lumped mass: integral of each basis function (2x2 Gauss)
  std::vector<double> mass(hf.N, 0.0);
  const double g = 1.0 / std::sqrt(3.0);
  const double vx[4] = {-1, 1, 1, -1}, vy[4] = {-1, -1, 1, 1};
  for (int cc = 0; cc < hf.C; ++cc) {
    const int *q = &hf.cells[4 * cc];
    for (int qp = 0; qp < 4; ++qp) {
      const double xi = (qp == 1 || qp == 2) ? g : -g, eta = qp >= 2 ? g : -g;
      double j11 = 0, j12 = 0, j21 = 0, j22 = 0, N[4];
      for (int a = 0; a < 4; ++a) {
        N[a] = 0.25 * (1 + vx[a] * xi) * (1 + vy[a] * eta);
        const double dxi = 0.25 * vx[a] * (1 + vy[a] * eta), deta = 0.25 * vy[a] * (1 + vx[a] * xi);
        j11 += dxi * hf.xy[2 * q[a]];
        j12 += deta * hf.xy[2 * q[a]];
        j21 += dxi * hf.xy[2 * q[a] + 1];
        j22 += deta * hf.xy[2 * q[a] + 1];
      }
      const double det = j11 * j22 - j12 * j21;
      for (int a = 0; a < 4; ++a) mass[q[a]] += det * N[a];
    }
  }
  std::vector<double> inv(hf.N);
  for (int i = 0; i < hf.N; ++i) inv[i] = 1.0 / mass[i];
  // static features from the patch corners
  const int nf = n.nfeat;
  std::vector<double> feat(static_cast<size_t>(nf) * n.B, 0.0);
  double hsum = 0.0;
  for (int p = 0; p < n.B; ++p) {
    const int *gp = &grid[static_cast<size_t>(p) * n.S2];
    const int ids[4] = {gp[0], gp[n.S - 1], gp[n.S2 - 1], gp[n.S * (n.S - 1)]};   // c00 c10 c11 c01
    double X[4], Y[4];
    for (int k = 0; k < 4; ++k) {
      X[k] = hf.xy[2 * ids[k]];
      Y[k] = hf.xy[2 * ids[k] + 1];
    }
    double side[4];
    for (int k = 0; k < 4; ++k) side[k] = std::hypot(X[(k + 1) % 4] - X[k], Y[(k + 1) % 4] - Y[k]);
    const double aspect = *std::max_element(side, side + 4) / *std::min_element(side, side + 4);
    // mid-lines: left->right and bottom->top
    const double ax = 0.5 * (X[1] + X[2]) - 0.5 * (X[0] + X[3]), ay = 0.5 * (Y[1] + Y[2]) - 0.5 * (Y[0] + Y[3]);
    const double bx = 0.5 * (X[3] + X[2]) - 0.5 * (X[0] + X[1]), by = 0.5 * (Y[3] + Y[2]) - 0.5 * (Y[0] + Y[1]);
    const double skew = std::fabs(ax * bx + ay * by) / (std::hypot(ax, ay) * std::hypot(bx, by));
    double area = 0.0;
    for (int k = 0; k < 4; ++k) area += X[k] * Y[(k + 1) % 4] - X[(k + 1) % 4] * Y[k];
    const double h = std::sqrt(0.5 * std::fabs(area));
    double *f = &feat[static_cast<size_t>(nf) * p];
    f[0] = aspect;
    f[1] = skew;
    f[3] = h;
    if (nf == 6) {   // direction of the left -> right mid-line, as (cos 2phi, sin 2phi)
      const double a2 = ax * ax + ay * ay;
      f[4] = (ax * ax - ay * ay) / a2;
      f[5] = 2.0 * ax * ay / a2;
    }
    hsum += h;
  }
  const double hmean = hsum / n.B;
  for (int p = 0; p < n.B; ++p) feat[static_cast<size_t>(nf) * p + 2] = feat[static_cast<size_t>(nf) * p + 3] / hmean;
  n.grid.upload(grid, c.stream);
  n.nadj_ptr.upload(ptr, c.stream);
  n.nadj.upload(adj, c.stream);
  n.inv_mass.upload(inv, c.stream);
  n.feat.upload(feat, c.stream);
}

void gemm(hipStream_t s, int M, int N, int K, const uint16_t *A, int lda, const uint16_t *Bm, int ldb,
          float *C, int ldc, bool acc) {
  launch_gemm_nt(s, M, N, K, A, lda, Bm, ldb, C, ldc, acc);
  check(hipGetLastError(), "k_gemm_nt_bf16");
}

}  // namespace

void net_repack(Net &n) {
  hipStream_t s = n.ctx->stream;
  for (int l = 0; l < n.layers; ++l) {
    const int il = l == 0 ? n.I : n.H, kl = l == 0 ? n.K0 : n.H;
    const size_t rows = 3 * static_cast<size_t>(n.H);
    hipLaunchKernelGGL(k_pack_bf16, dim3(blocks(rows * kl, 256)), dim3(256), 0, s, static_cast<int>(rows), il,
                       n.w32.p + n.off_ih[l], kl, n.wih_b[l].p);
    hipLaunchKernelGGL(k_pack_bf16, dim3(blocks(rows * n.H, 256)), dim3(256), 0, s, static_cast<int>(rows),
                       n.H, n.w32.p + n.off_hh[l], n.H, n.whh_b[l].p);
    hipLaunchKernelGGL(k_pack_bf16_t, dim3(blocks(rows * n.H, 256)), dim3(256), 0, s, static_cast<int>(rows), n.H,
                       n.w32.p + n.off_hh[l], n.whh_t[l].p);
    if (l > 0)
      hipLaunchKernelGGL(k_pack_bf16_t, dim3(blocks(rows * n.H, 256)), dim3(256), 0, s, static_cast<int>(rows),
                         n.H, n.w32.p + n.off_ih[l], n.wih_t[l].p);
  }
  hipLaunchKernelGGL(k_pack_bf16, dim3(blocks(static_cast<size_t>(n.O) * n.H, 256)), dim3(256), 0, s, n.O,
                     n.H, n.w32.p + n.off_out, n.H, n.wout_b.p);
  check(hipGetLastError(), "repack");
}

namespace {

// One GRU time step of all patches on the BF16 input rows in n.X.
void net_forward(Net &n) {
  hipStream_t s = n.ctx->stream;
  const int H3 = 3 * n.H;
  for (int l = 0; l < n.layers; ++l) {
    const uint16_t *in = l == 0 ? n.X.p : n.hb[l - 1].p;
    const int K = l == 0 ? n.K0 : n.H;
    // keys "name<layer>@L<fine level>": the patches live on the fine level
    const std::string lay = std::to_string(l);
    {
      ProfScope ps(n.ctx->prof, s, ("gru_gemm_in" + lay).c_str(), n.F);
      gemm(s, n.B, H3, K, in, K, n.wih_b[l].p, K, n.Gi.p, H3, false);
    }
    // recurrent product and gate update in one kernel (H is a multiple of 32)
    ProfScope ps(n.ctx->prof, s, ("gru_step" + lay).c_str(), n.F);
    hipLaunchKernelGGL(k_gru_step_fused, dim3(n.H / 32, blocks(n.B, 64)), dim3(256), 0, s, n.B, n.H, n.Gi.p,
                       n.hb[l].p, n.h[l].p, n.whh_b[l].p, n.h[l].p, n.hb_next[l].p, nullptr);
    check(hipGetLastError(), "k_gru_step_fused");
    std::swap(n.hb[l], n.hb_next[l]);
  }
  ProfScope ps(n.ctx->prof, s, "gru_head", n.F);
  gemm(s, n.B, n.O, n.H, n.hb[n.layers - 1].p, n.H, n.wout_b.p, n.H, n.Y.p, n.O, false);
}

void zero_state(Net &n) {
  hipStream_t s = n.ctx->stream;
  for (int l = 0; l < n.layers; ++l) {
    hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, s, n.h[l].p, n.h[l].n, 0.0f);
    hipLaunchKernelGGL(k_fill<uint16_t>, dim3(1024), dim3(256), 0, s, n.hb[l].p, n.hb[l].n, uint16_t(0));
  }
  check(hipGetLastError(), "zero_state");
}

// x_fine = P^m x_coarse (FP64), chain buffers xt[0] = level L copy.
void prolong_chain(Net &n, const double *xL) {
  Ctx &c = *n.ctx;
  hipStream_t s = c.stream;
  const size_t nL = 3 * static_cast<size_t>(c.levels[n.L]->h.N);
  check(hipMemcpyAsync(n.xt[0].p, xL, nL * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
  for (int l = n.L + 1; l <= n.F; ++l) {
    DevLevel &Fl = *c.levels[l];
    DevLevel &Cl = *c.levels[l - 1];
    TransferView tv{Fl.h.Nc, Fl.h.Ec, Fl.h.N, Fl.edge_ends.p, Cl.cells.p, Fl.rptr.p, Fl.ridx.p, Cl.flag.p};
    double *dst = n.xt[l - n.L].p;
    hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, s, dst, n.xt[l - n.L].n, 0.0);
    hipLaunchKernelGGL(k_prolong_add<double>, dim3(blocks(Fl.h.N, 256)), dim3(256), 0, s, tv,
                       n.xt[l - 1 - n.L].p, dst);
  }
  check(hipGetLastError(), "prolong_chain");
}

// b^F = Rhs(n.vc) on level F (Algorithm 1), b^L = (P^m)^T b^F into the
// coarse state's pending right-hand side, then v_prev <- n.vc.
void rhs_and_restrict(Net &n, State &st, double dt) {
  Ctx &c = *n.ctx;
  hipStream_t s = c.stream;
  const DevLevel &LF = *c.levels[n.F];
  {
    ProfScope ps(c.prof, s, "dnnmg_rhs", n.F);
    double *E = c.cell_vectors(n.F);
    hipLaunchKernelGGL(k_cell_vectors<1>, dim3(blocks(LF.h.C, 256)), dim3(256), 0, s, LF.view(),
                       c.phys(dt, st.t + dt), n.vc.p, nullptr, 0, E);
    hipLaunchKernelGGL(k_rhs_nodes, dim3(blocks(LF.h.N, 256)), dim3(256), 0, s, LF.view(), E, n.bF.p,
                       LF.large_order());
    check(hipGetLastError(), "rhs");
  }
  const double *src = n.bF.p;
  for (int l = n.F; l > n.L; --l) {
    DevLevel &Fl = *c.levels[l];
    DevLevel &Cl = *c.levels[l - 1];
    TransferView tv{Fl.h.Nc, Fl.h.Ec, Fl.h.N, Fl.edge_ends.p, Cl.cells.p, Fl.rptr.p, Fl.ridx.p, Cl.flag.p};
    double *dst = (l - 1 == n.L) ? st.pending_rhs.p : n.rchain[l - 1 - n.L].p;
    hipLaunchKernelGGL(k_restrict<double>, dim3(blocks(Fl.h.Nc, 256)), dim3(256), 0, s, tv, src, dst,
                       Cl.large_order());
    src = dst;
  }
  check(hipGetLastError(), "restrict chain");
  std::swap(n.vprev, n.vc);
  st.has_pending = true;
}

}  // namespace
}  // namespace dnnmg

extern "C" {

int dnnmg_net_targets(dnnmg_ctx *ctx, const dnnmg_state *coarse, dnnmg_net *net, const double *v_fine,
                      float *D) {
  if (!ctx || !coarse || !net || !v_fine || !D) return DNNMG_EINVAL;
  Net &n = net->impl;
  Ctx &c = ctx->impl;
  if (n.ctx != &c || coarse->impl.ctx != &c || coarse->impl.level != n.L) {
    c.last_error = "state / network do not belong to this context and coarse level";
    return DNNMG_EINVAL;
  }
  try {
    hipStream_t s = c.stream;
    const size_t nf = 3 * static_cast<size_t>(c.levels[n.F]->h.N);
    check(hipMemcpyAsync(n.vc.p, v_fine, nf * sizeof(double), hipMemcpyHostToDevice, s), "v H2D");
    prolong_chain(n, coarse->impl.x.p);
    const size_t cnt = static_cast<size_t>(n.B) * n.S2;
    hipLaunchKernelGGL(k_patch_targets, dim3(blocks(cnt, 256)), dim3(256), 0, s, n.view(), n.vc.p,
                       n.xt[n.m].p, n.oscale.p, n.Y.p);
    check(hipGetLastError(), "k_patch_targets");
    check(hipMemcpyAsync(D, n.Y.p, sizeof(float) * n.B * n.O, hipMemcpyDeviceToHost, s), "D D2H");
    check(hipStreamSynchronize(s), "targets");
  } catch (const DnnmgError &e) {
    c.last_error = e.msg;
    return e.code;
  }
  return DNNMG_OK;
}

int dnnmg_net_fine_velocity(dnnmg_net *net, const double **v_dev) {
  if (!net || !v_dev) return DNNMG_EINVAL;
  Net &n = net->impl;
  if (!n.has_vprev) {
    n.ctx->last_error = "no corrected fine velocity yet (dnnmg_net_reset first)";
    return DNNMG_ESTATE;
  }
  *v_dev = n.vprev.p;
  return DNNMG_OK;
}

int dnnmg_rhs_from_fine(dnnmg_ctx *ctx, dnnmg_state *coarse, dnnmg_net *net, const double *v_fine,
                        double dt) {
  if (!ctx || !coarse || !net || !v_fine || !(dt > 0)) return DNNMG_EINVAL;
  Net &n = net->impl;
  Ctx &c = ctx->impl;
  if (n.ctx != &c || coarse->impl.ctx != &c || coarse->impl.level != n.L) {
    c.last_error = "state / network do not belong to this context and coarse level";
    return DNNMG_EINVAL;
  }
  try {
    const size_t nf = 3 * static_cast<size_t>(c.levels[n.F]->h.N);
    check(hipMemcpyAsync(n.vc.p, v_fine, nf * sizeof(double), hipMemcpyHostToDevice, c.stream), "v H2D");
    rhs_and_restrict(n, coarse->impl, dt);
    n.has_vprev = true;
    check(hipStreamSynchronize(c.stream), "rhs_from_fine");
  } catch (const DnnmgError &e) {
    c.last_error = e.msg;
    return e.code;
  }
  return DNNMG_OK;
}

int dnnmg_net_create(dnnmg_ctx *ctx, int coarse_level, int m_levels, int hidden, int layers,
                     dnnmg_net **out) {
  return dnnmg_net_create_patch(ctx, coarse_level, m_levels, hidden, layers, DNNMG_PATCH_BLOCK, out);
}

int dnnmg_net_create_patch(dnnmg_ctx *ctx, int coarse_level, int m_levels, int hidden, int layers, int patch,
                           dnnmg_net **out) {
  if (!ctx || !out) return DNNMG_EINVAL;
  if (ctx->impl.finest < 0) return DNNMG_ESTATE;
  if ((patch != DNNMG_PATCH_BLOCK && patch != DNNMG_PATCH_CELL) ||
      coarse_level < (patch == DNNMG_PATCH_BLOCK ? 1 : 0) || m_levels < 1 ||
      coarse_level + m_levels > ctx->impl.finest || hidden < 32 || hidden % 32 != 0 || hidden > 1024 ||
      layers < 1 || layers > 8) {
    ctx->impl.last_error = "invalid network / level configuration";
    return DNNMG_EINVAL;
  }
  dnnmg_net *h = new (std::nothrow) dnnmg_net();
  if (!h) return DNNMG_ENOMEM;
  Ctx &c = ctx->impl;
  try {
    Net &n = h->impl;
    n.ctx = &c;
    n.L = coarse_level;
    n.m = m_levels;
    n.F = coarse_level + m_levels;
    n.patch = patch;
    n.S = (1 << (patch == DNNMG_PATCH_CELL ? m_levels : m_levels + 1)) + 1;
    n.S2 = n.S * n.S;
    n.nch = patch == DNNMG_PATCH_CELL ? 5 : 6;
    n.nfeat = patch == DNNMG_PATCH_CELL ? 6 : 4;
    n.nstat = n.nch + n.nfeat;
    n.I = n.nch * n.S2 + n.nfeat;
    n.O = 2 * n.S2;
    n.H = hidden;
    n.layers = layers;
    n.K0 = (n.I + 31) / 32 * 32;
    build_patch_tables(n);
    long long o = 0;
    for (int l = 0; l < layers; ++l) {
      const int il = l == 0 ? n.I : n.H;
      n.off_ih.push_back(o);
      o += 3LL * n.H * il;
      n.off_hh.push_back(o);
      o += 3LL * n.H * n.H;
    }
    n.off_out = o;
    o += static_cast<long long>(n.O) * n.H;
    n.nparam = o;
    n.w32.alloc(static_cast<size_t>(o));
    hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, c.stream, n.w32.p, n.w32.n, 0.0f);
    n.wih_b.resize(layers);
    n.whh_b.resize(layers);
    n.whh_t.resize(layers);
    n.wih_t.resize(layers);
    n.h.resize(layers);
    n.hb.resize(layers);
    n.hb_next.resize(layers);
    for (int l = 0; l < layers; ++l) {
      n.wih_b[l].alloc(3 * static_cast<size_t>(n.H) * (l == 0 ? n.K0 : n.H));
      n.whh_b[l].alloc(3 * static_cast<size_t>(n.H) * n.H);
      n.whh_t[l].alloc(3 * static_cast<size_t>(n.H) * n.H);
      if (l > 0) n.wih_t[l].alloc(3 * static_cast<size_t>(n.H) * n.H);
      n.h[l].alloc(static_cast<size_t>(n.B) * n.H);
      n.hb[l].alloc(static_cast<size_t>(n.B) * n.H);
      n.hb_next[l].alloc(static_cast<size_t>(n.B) * n.H);
    }
    n.wout_b.alloc(static_cast<size_t>(n.O) * n.H);
    n.mu.alloc(n.nstat);
    n.sg.alloc(n.nstat);
    n.oscale.alloc(2);
    std::vector<float> zeros(n.nstat, 0.0f), ones(n.nstat, 1.0f);
    n.mu.upload(zeros, c.stream);
    n.sg.upload(ones, c.stream);
    n.oscale.upload(std::vector<float>{1.0f, 1.0f}, c.stream);
    n.X.alloc(static_cast<size_t>(n.B) * n.K0);
    n.Xf.alloc(static_cast<size_t>(n.B) * n.K0);
    n.Gi.alloc(static_cast<size_t>(n.B) * 3 * n.H);
    n.Y.alloc(static_cast<size_t>(n.B) * n.O);
    n.xt.resize(m_levels + 1);
    n.rchain.resize(m_levels + 1);
    for (int l = n.L; l <= n.F; ++l) {
      n.xt[l - n.L].alloc(3 * static_cast<size_t>(c.levels[l]->h.N));
      n.rchain[l - n.L].alloc(3 * static_cast<size_t>(c.levels[l]->h.N));
    }
    const size_t nf = 3 * static_cast<size_t>(c.levels[n.F]->h.N);
    n.vprev.alloc(nf);
    n.vc.alloc(nf);
    n.bF.alloc(nf);
    n.dcorr.alloc(2 * static_cast<size_t>(c.levels[n.F]->h.N));
    net_repack(n);
    zero_state(n);
    check(hipStreamSynchronize(c.stream), "net create");
  } catch (const DnnmgError &e) {
    c.last_error = e.msg;
    delete h;
    return e.code;
  } catch (...) {
    delete h;
    return DNNMG_ENOMEM;
  }
  *out = h;
  return DNNMG_OK;
}

int dnnmg_net_destroy(dnnmg_net *net) {
  if (!net) return DNNMG_EINVAL;
  delete net;
  return DNNMG_OK;
}

int dnnmg_net_info(const dnnmg_net *net, int *n_in, int *n_out, int *n_patches, long long *n_params) {
  if (!net) return DNNMG_EINVAL;
  const Net &n = net->impl;
  if (n_in) *n_in = n.I;
  if (n_out) *n_out = n.O;
  if (n_patches) *n_patches = n.B;
  if (n_params) *n_params = n.nparam;
  return DNNMG_OK;
}

int dnnmg_net_patch_info(const dnnmg_net *net, int *patch, int *nodes_per_side, int *n_stats) {
  if (!net) return DNNMG_EINVAL;
  const Net &n = net->impl;
  if (patch) *patch = n.patch;
  if (nodes_per_side) *nodes_per_side = n.S;
  if (n_stats) *n_stats = n.nstat;
  return DNNMG_OK;
}

int dnnmg_net_set_weights(dnnmg_net *net, const float *w, const float *mu, const float *sigma,
                          const float *out_scale) {
  if (!net) return DNNMG_EINVAL;
  Net &n = net->impl;
  Ctx &c = *n.ctx;
  if (sigma)
    for (int k = 0; k < n.nstat; ++k)
      if (!(sigma[k] > 0.0f)) {
        c.last_error = "sigma must be positive";
        return DNNMG_EINVAL;
      }
  try {
    if (w)
      check(hipMemcpyAsync(n.w32.p, w, sizeof(float) * n.nparam, hipMemcpyHostToDevice, c.stream), "w H2D");
    if (mu) check(hipMemcpyAsync(n.mu.p, mu, sizeof(float) * n.nstat, hipMemcpyHostToDevice, c.stream), "mu");
    if (sigma)
      check(hipMemcpyAsync(n.sg.p, sigma, sizeof(float) * n.nstat, hipMemcpyHostToDevice, c.stream), "sg");
    if (out_scale)
      check(hipMemcpyAsync(n.oscale.p, out_scale, sizeof(float) * 2, hipMemcpyHostToDevice, c.stream), "os");
    net_repack(n);
    check(hipStreamSynchronize(c.stream), "set weights");
  } catch (const DnnmgError &e) {
    c.last_error = e.msg;
    return e.code;
  }
  return DNNMG_OK;
}

int dnnmg_net_get_weights(const dnnmg_net *net, float *w) {
  if (!net || !w) return DNNMG_EINVAL;
  const Net &n = net->impl;
  if (hipMemcpyAsync(w, n.w32.p, sizeof(float) * n.nparam, hipMemcpyDeviceToHost, n.ctx->stream) != hipSuccess ||
      hipStreamSynchronize(n.ctx->stream) != hipSuccess)
    return DNNMG_EDEVICE;
  return DNNMG_OK;
}

int dnnmg_net_reset(dnnmg_net *net, const dnnmg_state *coarse) {
  if (!net || !coarse) return DNNMG_EINVAL;
  Net &n = net->impl;
  Ctx &c = *n.ctx;
  if (coarse->impl.ctx != &c || coarse->impl.level != n.L) {
    c.last_error = "state is not on the network's coarse level";
    return DNNMG_EINVAL;
  }
  try {
    zero_state(n);
    prolong_chain(n, coarse->impl.x.p);
    const size_t nf = 3 * static_cast<size_t>(c.levels[n.F]->h.N);
    check(hipMemcpyAsync(n.vprev.p, n.xt[n.m].p, nf * sizeof(double), hipMemcpyDeviceToDevice, c.stream),
          "vprev");
    check(hipStreamSynchronize(c.stream), "reset");
    n.has_vprev = true;
  } catch (const DnnmgError &e) {
    c.last_error = e.msg;
    return e.code;
  }
  return DNNMG_OK;
}

int dnnmg_net_forward(dnnmg_net *net, const float *X, float *Y) {
  if (!net || !X || !Y) return DNNMG_EINVAL;
  Net &n = net->impl;
  Ctx &c = *n.ctx;
  try {
    const size_t rows = static_cast<size_t>(n.B);
    std::vector<float> pad(rows * n.K0, 0.0f);
    for (size_t p = 0; p < rows; ++p) std::memcpy(&pad[p * n.K0], X + p * n.I, sizeof(float) * n.I);
    check(hipMemcpyAsync(n.Xf.p, pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice, c.stream),
          "X H2D");
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks(pad.size(), 256)), dim3(256), 0, c.stream, pad.size(), n.Xf.p,
                       n.X.p);
    net_forward(n);
    check(hipMemcpyAsync(Y, n.Y.p, sizeof(float) * rows * n.O, hipMemcpyDeviceToHost, c.stream), "Y D2H");
    check(hipStreamSynchronize(c.stream), "forward");
  } catch (const DnnmgError &e) {
    c.last_error = e.msg;
    return e.code;
  }
  return DNNMG_OK;
}

int dnnmg_correct(dnnmg_ctx *ctx, dnnmg_state *coarse, dnnmg_net *net, double dt,
                  dnnmg_correct_out *dbg) {
  if (!ctx || !coarse || !net || !(dt > 0)) return DNNMG_EINVAL;
  Net &n = net->impl;
  Ctx &c = ctx->impl;
  if (n.ctx != &c || coarse->impl.ctx != &c || coarse->impl.level != n.L) {
    c.last_error = "state / network do not belong to this context and coarse level";
    return DNNMG_EINVAL;
  }
  if (!n.has_vprev) {
    c.last_error = "dnnmg_net_reset must be called before the first correction";
    return DNNMG_ESTATE;
  }
  try {
    hipStream_t s = c.stream;
    State &st = coarse->impl;
    const DevLevel &LF = *c.levels[n.F];
    const int NF = LF.h.N;
    {
      ProfScope ps(c.prof, s, "dnnmg_prolong", n.F);
      prolong_chain(n, st.x.p);
    }
    const double *xt = n.xt[n.m].p;
    // fine residual r^F = f^F(v_prev) - A^F(x~) at the coarse state's time
    c.residual(n.F, xt, n.vprev.p, nullptr, st.t, dt, c.R.p);
    const PatchView pv = n.view();
    {
      ProfScope ps(c.prof, s, "patch_gather", n.F);
      hipLaunchKernelGGL(k_patch_gather, dim3(n.B), dim3(128), 0, s, pv, xt, c.R.p, n.mu.p, n.sg.p, c.prm.nu,
                         n.X.p, n.K0, dbg && dbg->inputs ? n.Xf.p : nullptr);
      check(hipGetLastError(), "k_patch_gather");
    }
    net_forward(n);
    {
      ProfScope ps(c.prof, s, "patch_scatter", n.F);
      hipLaunchKernelGGL(k_patch_scatter, dim3(blocks(NF, 256)), dim3(256), 0, s, pv, n.Y.p, n.O, n.oscale.p, xt,
                         n.vc.p, n.dcorr.p);
      check(hipGetLastError(), "k_patch_scatter");
    }
    rhs_and_restrict(n, st, dt);
    if (dbg) {
      if (dbg->inputs) {
        std::vector<float> tmp(static_cast<size_t>(n.B) * n.K0);
        check(hipMemcpyAsync(tmp.data(), n.Xf.p, tmp.size() * sizeof(float), hipMemcpyDeviceToHost, s), "dbg");
        check(hipStreamSynchronize(s), "dbg");
        for (int p = 0; p < n.B; ++p)
          std::memcpy(dbg->inputs + static_cast<size_t>(p) * n.I, &tmp[static_cast<size_t>(p) * n.K0],
                      sizeof(float) * n.I);
      }
      if (dbg->outputs)
        check(hipMemcpyAsync(dbg->outputs, n.Y.p, sizeof(float) * n.B * n.O, hipMemcpyDeviceToHost, s), "dbg");
      if (dbg->correction)
        check(hipMemcpyAsync(dbg->correction, n.dcorr.p, sizeof(double) * 2 * NF, hipMemcpyDeviceToHost, s),
              "dbg");
      if (dbg->rhs_coarse)
        check(hipMemcpyAsync(dbg->rhs_coarse, st.pending_rhs.p, sizeof(double) * st.pending_rhs.n,
                             hipMemcpyDeviceToHost, s),
              "dbg");
    }
    check(hipStreamSynchronize(s), "correct");
  } catch (const DnnmgError &e) {
    c.last_error = e.msg;
    return e.code;
  }
  return DNNMG_OK;
}

}  // extern "C"
