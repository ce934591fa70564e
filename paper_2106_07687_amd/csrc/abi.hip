// extern "C" entry points of include/dnnmg.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include <mutex>

#include "context.h"

using namespace dnnmg;

// Scratch of dnnmg_velocity_error_noalloc: the per-workgroup partial sums of
// its reduction (4 doubles per workgroup of 256 threads).  One copy per GPU,
// held until the process ends.  Host code never passes this name to a
// kernel: the device address of each GPU's copy is taken with
// hipGetSymbolAddress (scratch_address) and used instead.
static constexpr int kScratchDoubles = 131072;   // 1 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

template <typename F>
int guarded(dnnmg_ctx *ctx, F &&f) {
  try {
    if (ctx) ctx->impl.last_error.clear();
    return f();
  } catch (const DnnmgError &e) {
    if (ctx) ctx->impl.last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    if (ctx) ctx->impl.last_error = "host allocation failed";
    return DNNMG_ENOMEM;
  } catch (...) {
    if (ctx) ctx->impl.last_error = "unexpected exception";
    return DNNMG_EDEVICE;
  }
}

int fail(dnnmg_ctx *ctx, int code, const char *msg) {
  if (ctx) ctx->impl.last_error = msg;
  return code;
}

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) on the first allocation-free call
// there.
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
double *scratch_ptr[kMaxDevices] = {};

double *scratch_address() {
  int dev = 0;
  check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) throw DnnmgError{DNNMG_EDEVICE, "device index out of range"};
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    scratch_ptr[dev] = static_cast<double *>(p);
  }
  return scratch_ptr[dev];
}

bool params_ok(const dnnmg_params *p) {
  return p && p->nu > 0 && p->alpha0 >= 0 && p->delta0 >= 0 && std::isfinite(p->delta0) && p->theta > 0 && p->theta <= 1 && p->u_mean >= 0 &&
         p->channel_h > 0 && p->newton_tol > 0 && p->newton_max >= 0 && p->newton_max <= 1000 &&
         p->gmres_rtol > 0 && p->gmres_rtol < 1 && p->gmres_restart >= 1 &&
         p->gmres_restart <= 64 && p->gmres_max >= 1 && p->nu_pre >= 0 && p->nu_post >= 0 &&
         p->nu_pre + p->nu_post >= 1 && p->vanka_omega > 0 && p->vanka_omega <= 2 &&
         (p->precision == 0 || p->precision == 1) && (p->use_graphs == 0 || p->use_graphs == 1) &&
         (p->autotune >= 0 && p->autotune <= 3) && (p->newton_predictor == 0 || p->newton_predictor == 1) &&
         (p->jacobian_reuse == 0 || p->jacobian_reuse == 1) && (p->smoother == 0 || p->smoother == 1) &&
         p->switch_off_newton >= 0 && p->nu_coarse >= 0 && p->nu_coarse <= 8 && p->coarse_level >= 0 &&
         p->coarse_level <= 2 &&
         p->reuse_contraction > 0 &&
         p->reuse_contraction < 1;
}

void upload_level(DevLevel &D, hipStream_t s) {
  const HostLevel &h = D.h;
  std::vector<double2> xy(h.N);
  for (int i = 0; i < h.N; ++i) xy[i] = make_double2(h.xy[2 * i], h.xy[2 * i + 1]);
  D.xy.upload(xy, s);
  std::vector<int4> cells(h.C);
  for (int c = 0; c < h.C; ++c)
    cells[c] = make_int4(h.cells[4 * c], h.cells[4 * c + 1], h.cells[4 * c + 2], h.cells[4 * c + 3]);
  D.cells.upload(cells, s);
  D.flag.upload(h.flag, s);
  D.cadj_ptr.upload(h.cadj_ptr, s);
  D.cadj.upload(h.cadj, s);
  D.colour_cells.upload(h.colour_cells, s);
  {   // nodes in the order of their lowest adjacent cell (ties by id): the
      // Vanka update's lanes then gather corrections of nearby cells
    std::vector<int> first(h.N), order(h.N);
    for (int i = 0; i < h.N; ++i) {
      int m = h.C;
      for (int e = h.cadj_ptr[i]; e < h.cadj_ptr[i + 1]; ++e) m = std::min(m, h.cadj[e] >> 2);
      first[i] = m;
      order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return first[a] < first[b]; });
    D.node_order.upload(order, s);
  }
  D.cslot.upload(h.cslot, s);
  D.padj_ptr.upload(h.padj_ptr, s);
  D.padj.upload(h.padj, s);
  D.pslot.upload(h.pslot, s);
  D.patch_nodes.upload(h.patch_nodes, s);
  D.wq.upload(h.wq, s);
  D.wx.upload(h.wx, s);
  D.oq.upload(h.oq, s);
  D.ox.upload(h.ox, s);
  D.colq.upload(h.colq, s);
  D.colx.upload(h.colx, s);
  D.vslot.upload(h.vslot, s);
  D.edge_ends.upload(h.edge_ends, s);
  D.rptr.upload(h.rptr, s);
  D.ridx.upload(h.ridx, s);
}

bool mesh_ready(const dnnmg_ctx *ctx) { return ctx && ctx->impl.finest >= 0; }

template <typename T>
Solver<T> &solver(Ctx &c);
template <>
Solver<float> &solver<float>(Ctx &c) {
  return *c.s32;
}
template <>
Solver<double> &solver<double>(Ctx &c) {
  return *c.s64;
}

template <typename T>
int step_impl(Ctx &c, State &st, double dt, dnnmg_step_stats *stats) {
  Solver<T> &S = solver<T>(c);
  const int l = st.level;
  const int N = c.levels[l]->h.N;
  const int n = 3 * N;
  hipStream_t s = c.stream;
  const double t_new = st.t + dt;
  check(hipMemcpyAsync(c.xo_save.p, st.x.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "save");
  dnnmg_step_stats loc{};
  bool ok = false;
  OpLevel<T> &o = S.op(l);
  bool use_pending = st.has_pending;
  const bool reuse = c.prm.jacobian_reuse != 0;
  bool fresh_only = !reuse;   // set when an attempt with kept Jacobians failed
  if (c.prm.newton_predictor && st.has_prev && st.dt_prev > 0.0) {
    // Newton starts from x_{n-1} + (k_n / k_{n-1}) (x_{n-1} - x_{n-2})
    hipLaunchKernelGGL(k_extrapolate, dim3(blocks(n, 256)), dim3(256), 0, s, n, dt / st.dt_prev, st.xprev.p,
                       st.x.p);
    check(hipGetLastError(), "predictor");
  }
  bool kept_used;   // this attempt iterated with a hierarchy built before its first iterate
  double nr_prev;
retry:
  kept_used = false;
  nr_prev = 0.0;
  hipLaunchKernelGGL(k_impose_bc, dim3(blocks(N, 256)), dim3(256), 0, s, c.levels[l]->view(),
                     c.phys(dt, t_new), st.x.p);
  // with a network right-hand side, Newton may stop early (switch-off)
  const int it_max = use_pending && c.prm.switch_off_newton > 0
                         ? std::min(c.prm.switch_off_newton, c.prm.newton_max)
                         : c.prm.newton_max;
  for (int it = 0; it <= it_max; ++it) {
    c.residual(l, st.x.p, c.xo_save.p, use_pending ? st.pending_rhs.p : nullptr, t_new, dt,
               c.R.p);
    const double nr = c.norm2_max_seg(l, c.R.p);   // batches: every simulation's own norm
    if (it == 0) loc.res_initial = nr;
    loc.res_final = nr;
    loc.newton_iters = it;
    if (!std::isfinite(nr)) break;
    if (nr <= c.prm.newton_tol) {
      ok = true;
      break;
    }
    if (it > 0) st.reuse_ok = nr <= c.prm.reuse_contraction * nr_prev;
    nr_prev = nr;
    if (it == it_max) break;
    if (fresh_only) {
      // the multigrid preconditioner is refreshed at the first Newton
      // iteration of a step; later iterations re-assemble only the finest
      // Jacobian
      S.linearize(st.x.p, c.xo_save.p, l, dt, it == 0);
      if (it == 0) ++loc.jacobian_builds;
    } else if (S.jacobian_kept(st.key, l, dt) && st.reuse_ok) {
      kept_used = true;   // chord iteration with the kept hierarchy
    } else {
      S.linearize(st.x.p, c.xo_save.p, l, dt, true);
      S.keep_jacobian(st.key, l, dt);
      st.reuse_ok = true;
      ++loc.jacobian_builds;
    }
    hipLaunchKernelGGL((k_convert<double, T>), dim3(blocks(n, 256)), dim3(256), 0, s, n, c.R.p, o.b.p);
    double r0, r1;
    const int k = S.gmres(l, o.b.p, o.x.p, c.prm.gmres_rtol, c.prm.gmres_restart, c.prm.gmres_max,
                          &r0, &r1);
    loc.gmres_iters += k;
    loc.gmres_iters_max = std::max(loc.gmres_iters_max, k);
    hipLaunchKernelGGL(k_add_to_f64<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, o.x.p, st.x.p);
    check(hipGetLastError(), "newton update");
  }
  if (!ok && kept_used) {
    // the kept Jacobians did not carry Newton to the tolerance: redo the step
    // from x_{n-1} with a fresh hierarchy at every step's first iterate
    check(hipMemcpyAsync(st.x.p, c.xo_save.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s),
          "reuse restore");
    S.forget_jacobian();
    st.reuse_ok = false;
    fresh_only = true;
    loc.gmres_iters_max = 0;
    goto retry;
  }
  if (!ok && use_pending) {
    // switch-off of the network for this step (Sec. 3.3): redo the step with
    // the plain right-hand side f_n(x_{n-1}), from x_{n-1}
    check(hipMemcpyAsync(st.x.p, c.xo_save.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s),
          "fallback restore");
    use_pending = false;
    loc.fallback = 1;
    loc.gmres_iters_max = 0;
    goto retry;
  }
  loc.converged = ok ? 1 : 0;
  if (stats) *stats = loc;
  if (!ok) {
    check(hipMemcpyAsync(st.x.p, c.xo_save.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s),
          "rollback");
    check(hipStreamSynchronize(s), "rollback sync");
    throw DnnmgError{DNNMG_ENOCONV, "Newton did not converge"};
  }
  st.t = t_new;
  st.has_pending = false;
  if (c.prm.newton_predictor) {
    if (st.xprev.n != static_cast<size_t>(n)) st.xprev.alloc(n);
    check(hipMemcpyAsync(st.xprev.p, c.xo_save.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "xprev");
    st.has_prev = true;
    st.dt_prev = dt;
  }
  return DNNMG_OK;
}

// Host-vector helpers for the single-operation entry points.
struct HostIO {
  Ctx &c;
  explicit HostIO(Ctx &cc) : c(cc) {}
  void up(double *dev, const double *host, size_t n) {
    check(hipMemcpyAsync(dev, host, n * sizeof(double), hipMemcpyHostToDevice, c.stream), "H2D");
  }
  void down(double *host, const double *dev, size_t n) {
    check(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, c.stream), "D2H");
    check(hipStreamSynchronize(c.stream), "sync");
  }
};

template <typename T>
void to_T(Ctx &c, const double *src, T *dst, int n) {
  hipLaunchKernelGGL((k_convert<double, T>), dim3(blocks(n, 256)), dim3(256), 0, c.stream, n, src, dst);
  check(hipGetLastError(), "convert");
}
template <typename T>
void from_T(Ctx &c, const T *src, double *dst, int n) {
  hipLaunchKernelGGL((k_convert<T, double>), dim3(blocks(n, 256)), dim3(256), 0, c.stream, n, src, dst);
  check(hipGetLastError(), "convert");
}

int check_level(const dnnmg_ctx *ctx, int level) {
  if (!mesh_ready(ctx)) return DNNMG_ESTATE;
  if (level < 0 || level > ctx->impl.finest) return DNNMG_EINVAL;
  return DNNMG_OK;
}

}  // namespace

extern "C" {

int dnnmg_params_default(dnnmg_params *p) {
  if (!p) return DNNMG_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->nu = 1e-3;
  p->alpha0 = 0.5;
  p->theta = 0.5;
  p->u_mean = 1.0;
  p->channel_h = 0.41;
  p->newton_tol = 1e-10;
  p->newton_max = 20;
  p->gmres_rtol = 1e-2;
  p->gmres_restart = 30;
  p->gmres_max = 100;
  p->nu_pre = 2;
  p->nu_post = 2;
  p->vanka_omega = 0.6;
  p->precision = 1;
  p->use_graphs = 1;
  p->autotune = 1;
  p->newton_predictor = 1;
  p->jacobian_reuse = 0;
  p->reuse_contraction = 0.1;
  p->smoother = 0;
  p->switch_off_newton = 0;
  p->nu_coarse = 0;
  p->coarse_level = 0;
  p->stream = nullptr;
  p->delta0 = 0.0;
  return DNNMG_OK;
}

int dnnmg_create(const dnnmg_params *p, dnnmg_ctx **out) {
  if (!out || !params_ok(p)) return DNNMG_EINVAL;
  dnnmg_ctx *c = new (std::nothrow) dnnmg_ctx();
  if (!c) return DNNMG_ENOMEM;
  c->impl.owner = c;
  c->impl.prm = *p;
  c->impl.stream = static_cast<hipStream_t>(p->stream);
  *out = c;
  return DNNMG_OK;
}

int dnnmg_destroy(dnnmg_ctx *ctx) {
  if (!ctx) return DNNMG_EINVAL;
  if (ctx->impl.finest >= 0) (void)hipStreamSynchronize(ctx->impl.stream);
  delete ctx;
  return DNNMG_OK;
}

const char *dnnmg_last_error(const dnnmg_ctx *ctx) {
  return ctx ? ctx->impl.last_error.c_str() : "null context";
}

int dnnmg_set_params(dnnmg_ctx *ctx, const dnnmg_params *p) {
  if (!ctx) return DNNMG_EINVAL;
  if (!params_ok(p)) return fail(ctx, DNNMG_EINVAL, "invalid parameters");
  if (p->coarse_level != ctx->impl.prm.coarse_level)
    return fail(ctx, DNNMG_EINVAL, "coarse_level is fixed at creation");
  const int prec = ctx->impl.prm.precision;
  ctx->impl.prm = *p;
  ctx->impl.prm.precision = prec;
  ctx->impl.stream = static_cast<hipStream_t>(p->stream);
  ++ctx->impl.graph_gen;   // captured graphs hold the old Vanka damping and sweep counts
  ctx->impl.forget_jacobians();   // viscosity or stabilisation may have changed
  return DNNMG_OK;
}

int dnnmg_setup_mesh(dnnmg_ctx *ctx, const dnnmg_coarse_mesh *m, int finest_level) {
  if (!ctx || !m) return DNNMG_EINVAL;
  if (finest_level < 0 || finest_level > 9 || m->n_vert < 4 || m->n_cell < 1 || !m->xy ||
      !m->quad || m->n_bedge < 0 || (m->n_bedge > 0 && !m->bedge) || m->n_curve < 0 ||
      (m->n_curve > 0 && !m->curve))
    return fail(ctx, DNNMG_EINVAL, "invalid macro mesh or level");
  for (int i = 0; i < 4 * m->n_cell; ++i)
    if (m->quad[i] < 0 || m->quad[i] >= m->n_vert) return fail(ctx, DNNMG_EINVAL, "quad vertex out of range");
  for (int e = 0; e < m->n_bedge; ++e) {
    const int *b = m->bedge + 3 * e;
    if (b[0] < 0 || b[0] >= m->n_vert || b[1] < 0 || b[1] >= m->n_vert || b[2] < 1 ||
        (b[2] >= 4 && b[2] - 4 >= m->n_curve))
      return fail(ctx, DNNMG_EINVAL, "boundary edge out of range");
  }
  if (ctx->impl.finest >= 0) return fail(ctx, DNNMG_ESTATE, "mesh already set up");
  if (!ctx->impl.macro_blk.empty() && static_cast<int>(ctx->impl.macro_blk.size()) != m->n_cell)
    return fail(ctx, DNNMG_EINVAL, "batch cell map does not match the macro mesh");
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    std::string err;
    std::vector<double> xy(m->xy, m->xy + 2 * m->n_vert);
    std::vector<int> q(m->quad, m->quad + 4 * m->n_cell);
    std::vector<int> be(m->bedge, m->bedge + 3 * m->n_bedge);
    std::vector<double> cv(m->curve, m->curve + 5 * m->n_curve);
    c.n_curve = m->n_curve;
    c.levels.clear();
    for (int l = 0; l <= finest_level; ++l) {
      auto D = std::make_unique<DevLevel>();
      if (l == 0)
        D->h = refine(xy, q, be, cv, &err);
      else {
        const HostLevel &P = c.levels[l - 1]->h;
        D->h = refine(P.xy, P.cells, P.bedges, cv, &err);
      }
      if (D->h.N == 0 || !build_tables(D->h, &err)) throw DnnmgError{DNNMG_EINVAL, err};
      if (l == 0) {   // level 0 has no coarser multigrid level
        D->h.rptr.clear();
        D->h.ridx.clear();
      }
      if (!c.macro_blk.empty()) {   // simulation batch: viscosity per node, level-0 blocks
        const HostLevel &h = D->h;
        std::vector<double> nu(h.N);
        std::vector<int> b0(l == 0 ? h.N : 0);
        for (int i = 0; i < h.N; ++i) {
          const int cell = h.cadj[h.cadj_ptr[i]] >> 2;   // cells descend as 4 c + k
          const int blk = c.macro_blk[cell >> (2 * l + 2)];
          nu[i] = c.blk_nu[blk];
          if (l == 0) b0[i] = blk;
        }
        D->nnu.upload(nu, c.stream);
        // per-simulation reduction chunks: runs of equal simulation in node
        // order, cut at 1024 nodes, listed simulation by simulation
        std::vector<int> seg(h.N);
        for (int i = 0; i < h.N; ++i) seg[i] = c.macro_blk[(h.cadj[h.cadj_ptr[i]] >> 2) >> (2 * l + 2)];
        const int nseg = static_cast<int>(c.blk_nu.size());
        std::vector<std::vector<std::pair<int, int>>> runs(nseg);
        for (int i = 0; i < h.N;) {
          int j = i;
          while (j < h.N && seg[j] == seg[i] && j - i < 1024) ++j;
          runs[seg[i]].push_back({3 * i, 3 * (j - i)});
          i = j;
        }
        std::vector<int> cs, cl, sp(1, 0);
        for (int g = 0; g < nseg; ++g) {
          for (auto &r : runs[g]) {
            cs.push_back(r.first);
            cl.push_back(r.second);
          }
          sp.push_back(static_cast<int>(cs.size()));
        }
        D->nseg = nseg;
        D->nchunk = static_cast<int>(cs.size());
        D->segn.upload(seg, c.stream);
        D->cstart.upload(cs, c.stream);
        D->clen.upload(cl, c.stream);
        D->seg_ptr.upload(sp, c.stream);
        if (l == 0) c.blk0 = std::move(b0);
      }
      upload_level(*D, c.stream);
      c.levels.push_back(std::move(D));
    }
    check(hipStreamSynchronize(c.stream), "upload");
    c.finest = finest_level;
    const size_t n = 3 * static_cast<size_t>(c.levels[finest_level]->h.N);
    c.R.alloc(n);
    c.xo_save.alloc(n);
    c.tmp64a.alloc(n);
    c.tmp64b.alloc(n);
    if (c.prm.precision == 1) {
      c.s32 = std::make_unique<Solver<float>>(&c);
      c.s32->setup(finest_level);
      if (c.prm.autotune == 1) c.s32->autotune();
      if (c.prm.autotune == 2) c.s32->fuse_all();
      if (c.prm.autotune == 3) c.s32->set_small_top(kSmallLevels - 1);
    } else {
      c.s64 = std::make_unique<Solver<double>>(&c);
      c.s64->setup(finest_level);
      if (c.prm.autotune == 1) c.s64->autotune();
      if (c.prm.autotune == 2) c.s64->fuse_all();
      if (c.prm.autotune == 3) c.s64->set_small_top(kSmallLevels - 1);
    }
    return DNNMG_OK;
  });
}

int dnnmg_level_info(const dnnmg_ctx *ctx, int level, int *n_nodes, int *n_cells, int *n_patches) {
  const int e = check_level(ctx, level);
  if (e) return e;
  const HostLevel &h = ctx->impl.levels[level]->h;
  if (n_nodes) *n_nodes = h.N;
  if (n_cells) *n_cells = h.C;
  if (n_patches) *n_patches = h.NP;
  return DNNMG_OK;
}

int dnnmg_level_coords(const dnnmg_ctx *ctx, int level, double *xy) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!xy) return DNNMG_EINVAL;
  const HostLevel &h = ctx->impl.levels[level]->h;
  std::memcpy(xy, h.xy.data(), sizeof(double) * 2 * h.N);
  return DNNMG_OK;
}

int dnnmg_level_cells(const dnnmg_ctx *ctx, int level, int *quads) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!quads) return DNNMG_EINVAL;
  const HostLevel &h = ctx->impl.levels[level]->h;
  std::memcpy(quads, h.cells.data(), sizeof(int) * 4 * h.C);
  return DNNMG_OK;
}

int dnnmg_state_create(dnnmg_ctx *ctx, int level, dnnmg_state **out) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!out) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    auto *s = new dnnmg_state();
    s->impl.ctx = &ctx->impl;
    s->impl.level = level;
    s->impl.key = ++ctx->impl.state_keys;
    const size_t n = 3 * static_cast<size_t>(ctx->impl.levels[level]->h.N);
    try {
      s->impl.x.alloc(n);
      s->impl.pending_rhs.alloc(n);
      hipLaunchKernelGGL(k_fill<double>, dim3(blocks(n, 256)), dim3(256), 0, ctx->impl.stream,
                         s->impl.x.p, n, 0.0);
      check(hipStreamSynchronize(ctx->impl.stream), "state zero");
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
    return DNNMG_OK;
  });
}

int dnnmg_state_destroy(dnnmg_state *s) {
  if (!s) return DNNMG_EINVAL;
  delete s;
  return DNNMG_OK;
}

int dnnmg_state_set(dnnmg_state *s, const double *uvp, double t) {
  if (!s || !uvp) return DNNMG_EINVAL;
  dnnmg_ctx *ctx = s->impl.ctx->owner;
  return guarded(ctx, [&]() {
    Ctx &c = *s->impl.ctx;
    check(hipMemcpyAsync(s->impl.x.p, uvp, sizeof(double) * s->impl.x.n, hipMemcpyHostToDevice,
                         c.stream),
          "state H2D");
    check(hipStreamSynchronize(c.stream), "state sync");
    s->impl.t = t;
    s->impl.has_pending = false;
    s->impl.has_prev = false;
    s->impl.key = ++c.state_keys;   // a Jacobian built from the old values is not reused
    s->impl.reuse_ok = false;
    return DNNMG_OK;
  });
}

int dnnmg_state_get(const dnnmg_state *s, double *uvp, double *t) {
  if (!s) return DNNMG_EINVAL;
  dnnmg_ctx *ctx = s->impl.ctx->owner;
  return guarded(ctx, [&]() {
    Ctx &c = *s->impl.ctx;
    if (uvp) {
      check(hipMemcpyAsync(uvp, s->impl.x.p, sizeof(double) * s->impl.x.n, hipMemcpyDeviceToHost,
                           c.stream),
            "state D2H");
      check(hipStreamSynchronize(c.stream), "state sync");
    }
    if (t) *t = s->impl.t;
    return DNNMG_OK;
  });
}

int dnnmg_state_get_dev(const dnnmg_state *s, double *uvp_dev) {
  if (!s || !uvp_dev) return DNNMG_EINVAL;
  dnnmg_ctx *ctx = s->impl.ctx->owner;
  return guarded(ctx, [&]() {
    Ctx &c = *s->impl.ctx;
    check(hipMemcpyAsync(uvp_dev, s->impl.x.p, sizeof(double) * s->impl.x.n, hipMemcpyDeviceToDevice, c.stream),
          "state D2D");
    return DNNMG_OK;
  });
}

int dnnmg_state_device_ptr(dnnmg_state *s, double **p) {
  if (!s || !p) return DNNMG_EINVAL;
  *p = s->impl.x.p;
  return DNNMG_OK;
}

int dnnmg_step(dnnmg_ctx *ctx, dnnmg_state *s, double dt, dnnmg_step_stats *stats) {
  if (!ctx || !s || !(dt > 0)) return DNNMG_EINVAL;
  if (!mesh_ready(ctx)) return DNNMG_ESTATE;
  if (s->impl.ctx != &ctx->impl) return fail(ctx, DNNMG_EINVAL, "state belongs to another context");
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    return c.prm.precision == 1 ? step_impl<float>(c, s->impl, dt, stats)
                                : step_impl<double>(c, s->impl, dt, stats);
  });
}

int dnnmg_linearize(dnnmg_ctx *ctx, const dnnmg_state *s, int level, double dt) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!s || !(dt > 0) || level > s->impl.level) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    if (c.prm.precision == 1)
      c.s32->linearize(s->impl.x.p, s->impl.x.p, level, dt);
    else
      c.s64->linearize(s->impl.x.p, s->impl.x.p, level, dt);
    check(hipStreamSynchronize(c.stream), "linearize");
    return DNNMG_OK;
  });
}

int dnnmg_solve(dnnmg_ctx *ctx, int level, const double *rhs, double *w, dnnmg_solve_stats *st) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!rhs || !w) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    const int n = 3 * c.levels[level]->h.N;
    HostIO io(c);
    io.up(c.tmp64a.p, rhs, n);
    auto run = [&](auto &S) {
      auto &o = S.op(level);
      to_T(c, c.tmp64a.p, o.b.p, n);
      double r0, r1;
      const int it = S.gmres(level, o.b.p, o.x.p, c.prm.gmres_rtol, c.prm.gmres_restart,
                             c.prm.gmres_max, &r0, &r1);
      from_T(c, o.x.p, c.tmp64b.p, n);
      io.down(w, c.tmp64b.p, n);
      if (st) {
        st->iters = it;
        st->res0 = r0;
        st->res = r1;
      }
      return DNNMG_OK;
    };
    return c.prm.precision == 1 ? run(*c.s32) : run(*c.s64);
  });
}

int dnnmg_residual(dnnmg_ctx *ctx, int level, const double *x, const double *xo, double t_new,
                   double dt, double *r) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!x || !xo || !r || !(dt > 0)) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    const int n = 3 * c.levels[level]->h.N;
    HostIO io(c);
    io.up(c.tmp64a.p, x, n);
    io.up(c.tmp64b.p, xo, n);
    c.residual(level, c.tmp64a.p, c.tmp64b.p, nullptr, t_new, dt, c.R.p);
    io.down(r, c.R.p, n);
    return DNNMG_OK;
  });
}

int dnnmg_jacobian_apply(dnnmg_ctx *ctx, int level, const double *w, double *y) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!w || !y) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    const int n = 3 * c.levels[level]->h.N;
    HostIO io(c);
    io.up(c.tmp64a.p, w, n);
    auto run = [&](auto &S) {
      auto &o = S.op(level);
      to_T(c, c.tmp64a.p, o.t.p, n);
      S.spmv(level, o.t.p, nullptr, o.r.p);
      from_T(c, o.r.p, c.tmp64b.p, n);
      io.down(y, c.tmp64b.p, n);
      return DNNMG_OK;
    };
    return c.prm.precision == 1 ? run(*c.s32) : run(*c.s64);
  });
}

int dnnmg_vanka_sweep(dnnmg_ctx *ctx, int level, const double *x, const double *b, double *xout) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (level < 1 || !x || !b || !xout) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    const int n = 3 * c.levels[level]->h.N;
    HostIO io(c);
    io.up(c.tmp64a.p, x, n);
    io.up(c.tmp64b.p, b, n);
    auto run = [&](auto &S) {
      auto &o = S.op(level);
      to_T(c, c.tmp64a.p, o.x.p, n);
      to_T(c, c.tmp64b.p, o.b.p, n);
      S.vanka_sweep(level, o.x.p, o.b.p, false);
      from_T(c, o.x.p, c.tmp64a.p, n);
      io.down(xout, c.tmp64a.p, n);
      return DNNMG_OK;
    };
    return c.prm.precision == 1 ? run(*c.s32) : run(*c.s64);
  });
}

int dnnmg_vcycle(dnnmg_ctx *ctx, int level, const double *b, double *x) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!b || !x) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    const int n = 3 * c.levels[level]->h.N;
    HostIO io(c);
    io.up(c.tmp64a.p, b, n);
    auto run = [&](auto &S) {
      auto &o = S.op(level);
      to_T(c, c.tmp64a.p, o.b.p, n);
      S.vcycle(level, o.b.p, o.x.p);
      from_T(c, o.x.p, c.tmp64a.p, n);
      io.down(x, c.tmp64a.p, n);
      return DNNMG_OK;
    };
    return c.prm.precision == 1 ? run(*c.s32) : run(*c.s64);
  });
}

int dnnmg_prolong(dnnmg_ctx *ctx, int level, const double *coarse, double *fine) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (level < 1 || !coarse || !fine) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    const int nf = 3 * c.levels[level]->h.N, nc = 3 * c.levels[level - 1]->h.N;
    HostIO io(c);
    io.up(c.tmp64a.p, coarse, nc);
    auto run = [&](auto &S) {
      auto &of = S.op(level);
      auto &oc = S.op(level - 1);
      to_T(c, c.tmp64a.p, oc.t.p, nc);
      using T = std::remove_reference_t<decltype(*of.t.p)>;
      hipLaunchKernelGGL(k_fill<T>, dim3(blocks(nf, 256)), dim3(256), 0, c.stream, of.t.p,
                         static_cast<size_t>(nf), T(0));
      S.prolong_add(level, oc.t.p, of.t.p);
      from_T(c, of.t.p, c.tmp64b.p, nf);
      io.down(fine, c.tmp64b.p, nf);
      return DNNMG_OK;
    };
    return c.prm.precision == 1 ? run(*c.s32) : run(*c.s64);
  });
}

int dnnmg_restrict(dnnmg_ctx *ctx, int level, const double *fine, double *coarse) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (level < 1 || !coarse || !fine) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    const int nf = 3 * c.levels[level]->h.N, nc = 3 * c.levels[level - 1]->h.N;
    HostIO io(c);
    io.up(c.tmp64a.p, fine, nf);
    auto run = [&](auto &S) {
      auto &of = S.op(level);
      auto &oc = S.op(level - 1);
      to_T(c, c.tmp64a.p, of.t.p, nf);
      S.restrict_to(level, of.t.p, oc.t.p);
      from_T(c, oc.t.p, c.tmp64b.p, nc);
      io.down(coarse, c.tmp64b.p, nc);
      return DNNMG_OK;
    };
    return c.prm.precision == 1 ? run(*c.s32) : run(*c.s64);
  });
}

}  // extern "C"

extern "C" {

int dnnmg_profile_enable(dnnmg_ctx *ctx, int on) {
  if (!ctx) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    if (on) c.prof.clear();
    c.prof.on = on != 0;
    return DNNMG_OK;
  });
}

int dnnmg_profile_select(dnnmg_ctx *ctx, const char *keys) {
  if (!ctx) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    std::vector<std::string> only;
    if (keys) {
      std::string all(keys), cur;
      for (char ch : all + ",") {
        if (ch == ',') {
          if (!cur.empty()) only.push_back(cur);
          cur.clear();
        } else if (ch != ' ') {
          cur += ch;
        }
      }
    }
    ctx->impl.prof.only = std::move(only);
    return DNNMG_OK;
  });
}

int dnnmg_profile_report(dnnmg_ctx *ctx, char *buf, size_t len) {
  if (!ctx || !buf || len == 0) return DNNMG_EINVAL;
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    if (c.finest >= 0) check(hipStreamSynchronize(c.stream), "profile sync");
    c.prof.resolve();
    std::string out;
    char line[256];
    for (const auto &kv : c.prof.acc) {
      std::snprintf(line, sizeof(line), "%s %ld %.6f\n", kv.first.c_str(), kv.second.second,
                    kv.second.first);
      out += line;
    }
    if (out.size() + 1 > len) return fail(ctx, DNNMG_EINVAL, "profile buffer too small");
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return DNNMG_OK;
  });
}

int dnnmg_functionals(dnnmg_ctx *ctx, const dnnmg_state *s, double *jdiv, double *drag, double *lift,
                      int n_obstacles) {
  if (!ctx || !s || s->impl.ctx != &ctx->impl) return DNNMG_EINVAL;
  if (n_obstacles != ctx->impl.n_curve || (n_obstacles > 0 && (!drag || !lift)))
    return fail(ctx, DNNMG_EINVAL, "n_obstacles must equal the mesh's obstacle count");
  return guarded(ctx, [&]() {
    ctx->impl.functionals(s->impl.level, s->impl.x.p, jdiv, drag, lift);
    return DNNMG_OK;
  });
}

int dnnmg_functionals_host(dnnmg_ctx *ctx, int level, const double *uvp, double *jdiv, double *drag,
                           double *lift, int n_obstacles) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!uvp) return DNNMG_EINVAL;
  if (n_obstacles != ctx->impl.n_curve || (n_obstacles > 0 && (!drag || !lift)))
    return fail(ctx, DNNMG_EINVAL, "n_obstacles must equal the mesh's obstacle count");
  return guarded(ctx, [&]() {
    Ctx &c = ctx->impl;
    const size_t n = 3 * static_cast<size_t>(c.levels[level]->h.N);
    DevBuf<double> xd;
    xd.alloc(n);
    check(hipMemcpyAsync(xd.p, uvp, n * sizeof(double), hipMemcpyHostToDevice, c.stream), "H2D");
    c.functionals(level, xd.p, jdiv, drag, lift);
    return DNNMG_OK;
  });
}

int dnnmg_velocity_error(dnnmg_ctx *ctx, int level, const double *x_dev, int ref_level, const double *ref_dev,
                         double *out) {
  const int e = check_level(ctx, ref_level);
  if (e) return e;
  if (level < 0 || level > ref_level || !x_dev || !ref_dev || !out)
    return fail(ctx, DNNMG_EINVAL, "velocity_error: need 0 <= level <= ref_level and non-null pointers");
  return guarded(ctx, [&]() {
    ctx->impl.velocity_error(level, x_dev, ref_level, ref_dev, out);
    return DNNMG_OK;
  });
}

int dnnmg_velocity_error_noalloc(dnnmg_ctx *ctx, int level, const double *x_dev, const double *ref_dev,
                                 double *out_dev) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!x_dev || !ref_dev || !out_dev) return fail(ctx, DNNMG_EINVAL, "velocity_error_noalloc: null pointer");
  const DevLevel &R = *ctx->impl.levels[level];
  const int nb = blocks(std::max(R.h.C, R.h.N), 256);
  if (4 * static_cast<size_t>(nb) > static_cast<size_t>(kScratchDoubles))
    return fail(ctx, DNNMG_EINVAL, "velocity_error_noalloc: level larger than the static scratch allows");
  return guarded(ctx, [&]() {
    double *partial = scratch_address();
    hipStream_t s = ctx->impl.stream;
    hipLaunchKernelGGL(k_vel_error_partial, dim3(nb), dim3(256), 0, s, R.view(), x_dev, ref_dev, partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3(4), dim3(256), 0, s, nb, 4, partial, out_dev);
    check(hipGetLastError(), "velocity_error_noalloc");
    return DNNMG_OK;
  });
}

int dnnmg_launch_config(const dnnmg_ctx *ctx, int level, int *block_sizes) {
  const int e = check_level(ctx, level);
  if (e) return e;
  if (!block_sizes) return DNNMG_EINVAL;
  const Ctx &c = ctx->impl;
  auto fill = [&](const auto &S) {
    const auto &o = S.op(level);
    block_sizes[0] = o.bs_spmv;
    block_sizes[1] = o.bs_apply;
    block_sizes[2] = o.bs_update;
    block_sizes[3] = o.bs_restrict;
    block_sizes[4] = o.bs_prolong;
    block_sizes[5] = o.bs_smooth;
    block_sizes[6] = (level >= 1 && level <= S.small_top()) ? 1024 : 0;
    block_sizes[7] = o.bs_rres;
    block_sizes[8] = o.bs_spmv4;
    block_sizes[9] = o.bs_smooth > 0 ? o.smooth_lanes : 0;
    block_sizes[10] = o.bs_upro;
    block_sizes[11] = o.bs_apply4;
    block_sizes[12] = o.bs_update_ord;
  };
  if (c.s32)
    fill(*c.s32);
  else if (c.s64)
    fill(*c.s64);
  else
    return DNNMG_ESTATE;
  return DNNMG_OK;
}

int dnnmg_level_stats(const dnnmg_ctx *ctx, int level, long long *q_blocks, long long *x_entries,
                      long long *q_slots, long long *x_slots) {
  const int e = check_level(ctx, level);
  if (e) return e;
  const HostLevel &h = ctx->impl.levels[level]->h;
  if (q_blocks) *q_blocks = h.nnzq;
  if (x_entries) *x_entries = h.nnzx;
  if (q_slots) *q_slots = static_cast<long long>(h.totq) * kSlice;
  if (x_slots) *x_slots = static_cast<long long>(h.totx) * kSlice;
  return DNNMG_OK;
}

}  // extern "C"
