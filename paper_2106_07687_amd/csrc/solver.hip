// Host drivers: mesh upload, Jacobian linearisation, additive cell-Vanka,
// V-cycle, right-preconditioned GMRES (Sec. 2.2) and the FP64 residual.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "context.h"

namespace dnnmg {

void check(hipError_t e, const char *what) {
  if (e != hipSuccess)
    throw DnnmgError{DNNMG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

#define LAUNCH_CHECK(name) check(hipGetLastError(), name)

hipEvent_t Profiler::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

void Profiler::resolve() {
  for (auto &r : pending) {
    check(hipEventSynchronize(r.b), "profiler sync");
    float ms = 0.0f;
    check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
    auto &v = acc[r.key];
    v.first += ms;
    v.second += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}

void Profiler::clear() {
  resolve();
  acc.clear();
}

Profiler::~Profiler() {
  for (auto &r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

bool Profiler::wants(const std::string &key) const {
  if (!on) return false;
  if (only.empty()) return true;
  return std::find(only.begin(), only.end(), key) != only.end();
}

bool Profiler::wants_level(int level) const {
  if (!on) return false;
  if (only.empty()) return true;
  const std::string suffix = "@L" + std::to_string(level);
  for (const auto &k : only)
    if (k.size() > suffix.size() && k.compare(k.size() - suffix.size(), suffix.size(), suffix) == 0)
      return true;
  return false;
}

ProfScope::ProfScope(Profiler &pr, hipStream_t st, const char *name, int level)
    : p(pr.on ? &pr : nullptr), s(st) {
  if (!p) return;
  key = std::string(name) + "@L" + std::to_string(level);
  if (!p->wants(key)) {
    p = nullptr;
    return;
  }
  a = p->take();
  check(hipEventRecord(a, s), "hipEventRecord");
}

ProfScope::~ProfScope() {
  if (!p) return;
  hipEvent_t b = p->take();
  if (hipEventRecord(b, s) != hipSuccess) return;
  p->pending.push_back({key, a, b});
  if (p->pending.size() > 8192) p->resolve();
}

LevelView DevLevel::view() const {
  LevelView v;
  v.N = h.N;
  v.C = h.C;
  v.NP = h.NP;
  v.xy = xy.p;
  v.cells = cells.p;
  v.flag = flag.p;
  v.cadj_ptr = cadj_ptr.p;
  v.cadj = cadj.p;
  v.cslot = cslot.p;
  v.padj_ptr = padj_ptr.p;
  v.padj = padj.p;
  v.pslot = pslot.p;
  v.patch_nodes = patch_nodes.p;
  v.wq = wq.p;
  v.wx = wx.p;
  v.oq = oq.p;
  v.ox = ox.p;
  v.colq = colq.p;
  v.colx = colx.p;
  v.vslot = vslot.p;
  v.nnu = nnu.p;
  return v;
}

hipStream_t Ctx::capture_stream() {
  if (!cap_stream) check(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking), "hipStreamCreate");
  return cap_stream;
}

Ctx::~Ctx() {
  s32.reset();
  s64.reset();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

const double *Ctx::ensure_lps(int l, double dt, int role) {
  DevLevel &L = *levels[l];
  DevLevel::LpsCache &c = L.lps[role ? 1 : 0];
  const double key_dt = role ? dt : 0.0;   // the paper's alpha_T does not depend on k
  if (c.m.p && c.dt == key_dt && c.nu == prm.nu && c.alpha0 == prm.alpha0) return c.m.p;
  if (!c.m.p) c.m.alloc(static_cast<size_t>(81) * L.h.NP);
  hipLaunchKernelGGL(k_lps_patch, dim3(blocks(L.h.NP, 64)), dim3(64), 0, stream, L.view(), phys(dt, 0.0),
                     role ? 1 : 0, c.m.p);
  LAUNCH_CHECK("k_lps_patch");
  c.dt = key_dt;
  c.nu = prm.nu;
  c.alpha0 = prm.alpha0;
  return c.m.p;
}

double Ctx::norm2_f64(const double *x, int n) {
  const int nb = std::min(blocks(n, 256), 1024);
  if (red_partial.n < static_cast<size_t>(nb)) red_partial.alloc(1024);
  if (!red_out.p) red_out.alloc(64);
  hipLaunchKernelGGL(k_multidot<double>, dim3(nb, 1), dim3(256), 0, stream, n, 1, x, size_t(0), x,
                     red_partial.p);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, stream, nb, 1, red_partial.p,
                     red_out.p);
  LAUNCH_CHECK("norm");
  double h = 0.0;
  check(hipMemcpyAsync(&h, red_out.p, sizeof(double), hipMemcpyDeviceToHost, stream), "norm D2H");
  check(hipStreamSynchronize(stream), "norm sync");
  return std::sqrt(h);
}

double Ctx::norm2_max_seg(int l, const double *x) {
  DevLevel &L = *levels[l];
  if (L.nseg <= 1) return norm2_f64(x, 3 * L.h.N);
  if (seg_partial.n < static_cast<size_t>(L.nchunk)) seg_partial.alloc(L.nchunk);
  if (seg_out.n < static_cast<size_t>(L.nseg)) seg_out.alloc(L.nseg);
  hipLaunchKernelGGL(k_multidot_chunks<double>, dim3(L.nchunk, 1), dim3(256), 0, stream, L.cstart.p, L.clen.p, 1, x,
                     size_t(0), x, seg_partial.p);
  hipLaunchKernelGGL(k_reduce_seg, dim3(L.nseg, 1), dim3(256), 0, stream, L.seg_ptr.p, 1, seg_partial.p,
                     seg_out.p);
  LAUNCH_CHECK("segmented norm");
  seg_host.resize(L.nseg);
  check(hipMemcpyAsync(seg_host.data(), seg_out.p, sizeof(double) * L.nseg, hipMemcpyDeviceToHost, stream),
        "norm D2H");
  check(hipStreamSynchronize(stream), "norm sync");
  double mx = 0.0;
  for (double v : seg_host) mx = std::max(mx, std::sqrt(v));
  for (double v : seg_host)
    if (!std::isfinite(v)) return v;
  return mx;
}

void Ctx::functionals(int l, const double *x, double *jdiv, double *drag, double *lift) {
  DevLevel &L = *levels[l];
  if (L.n_obst < 0) {   // obstacle edges of this level, grouped by obstacle
    const HostLevel &h = L.h;
    std::map<std::pair<int, int>, std::pair<int, int>> side;   // (v0, v1) -> (cell, a)
    for (int c = 0; c < h.C; ++c)
      for (int a = 0; a < 4; ++a) {
        const int v0 = h.cells[4 * c + a], v1 = h.cells[4 * c + (a + 1) % 4];
        side[{std::min(v0, v1), std::max(v0, v1)}] = {c, a};
      }
    std::vector<std::vector<int>> per(n_curve);
    for (int e = 0; e < h.Eb; ++e) {
      const int v0 = h.bedges[3 * e], v1 = h.bedges[3 * e + 1], tag = h.bedges[3 * e + 2];
      if (tag < 4 || tag - 4 >= n_curve) continue;
      const auto it = side.find({std::min(v0, v1), std::max(v0, v1)});
      if (it == side.end()) throw DnnmgError{DNNMG_EINVAL, "obstacle edge without a cell"};
      per[tag - 4].push_back(it->second.first);
      per[tag - 4].push_back(it->second.second);
    }
    std::vector<int> ed, ptr(1, 0);
    for (auto &v : per) {
      ed.insert(ed.end(), v.begin(), v.end());
      ptr.push_back(static_cast<int>(ed.size() / 2));
    }
    L.obst_edges.upload(ed, stream);
    L.obst_ptr.upload(ptr, stream);
    L.obst_vals.alloc(std::max<size_t>(ed.size(), 2) + 2 * static_cast<size_t>(n_curve) + 2);
    L.n_obst = n_curve;
  }
  const int nb = blocks(L.h.C, 256);
  if (red_partial.n < static_cast<size_t>(nb)) red_partial.alloc(nb);
  if (!red_out.p) red_out.alloc(64);
  ProfScope ps(prof, stream, "functionals", l);
  hipLaunchKernelGGL(k_jdiv_partial, dim3(nb), dim3(256), 0, stream, L.view(), x, red_partial.p);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, stream, nb, 1, red_partial.p, red_out.p);
  const int ne = static_cast<int>(L.obst_edges.n / 2);
  double *vals = L.obst_vals.p, *sums = L.obst_vals.p + 2 * static_cast<size_t>(std::max(ne, 1));
  if (ne > 0) {
    hipLaunchKernelGGL(k_edge_forces, dim3(blocks(ne, 256)), dim3(256), 0, stream, L.view(), ne,
                       L.obst_edges.p, x, prm.nu, vals);
  }
  if (n_curve > 0)
    hipLaunchKernelGGL(k_sum_ranges, dim3(blocks(2 * n_curve, 64)), dim3(64), 0, stream, n_curve, L.obst_ptr.p,
                       vals, sums);
  LAUNCH_CHECK("functionals");
  std::vector<double> h(1 + 2 * static_cast<size_t>(n_curve));
  check(hipMemcpyAsync(h.data(), red_out.p, sizeof(double), hipMemcpyDeviceToHost, stream), "D2H");
  if (n_curve > 0)
    check(hipMemcpyAsync(h.data() + 1, sums, sizeof(double) * 2 * n_curve, hipMemcpyDeviceToHost, stream),
          "D2H");
  check(hipStreamSynchronize(stream), "functionals sync");
  if (jdiv) *jdiv = h[0];
  for (int k = 0; k < n_curve; ++k) {
    if (drag) drag[k] = h[1 + 2 * k];
    if (lift) lift[k] = h[2 + 2 * k];
  }
}

void Ctx::velocity_error(int l, const double *x, int ref_level, const double *ref, double out[4]) {
  DevLevel &R = *levels[ref_level];
  const size_t nr = 3 * static_cast<size_t>(R.h.N);
  const double *a = x;
  if (l < ref_level) {   // bilinear prolongation level by level (FP64)
    if (verr_a.n < nr) verr_a.alloc(nr);
    if (verr_b.n < nr) verr_b.alloc(nr);
    double *bufs[2] = {verr_a.p, verr_b.p};
    for (int k = l + 1; k <= ref_level; ++k) {
      DevLevel &Fl = *levels[k];
      DevLevel &Cl = *levels[k - 1];
      TransferView tv{Fl.h.Nc, Fl.h.Ec, Fl.h.N, Fl.edge_ends.p, Cl.cells.p, Fl.rptr.p, Fl.ridx.p, Cl.flag.p};
      double *dst = bufs[k & 1];
      const size_t nf = 3 * static_cast<size_t>(Fl.h.N);
      hipLaunchKernelGGL(k_fill<double>, dim3(std::min(blocks(nf, 256), 1024)), dim3(256), 0, stream, dst, nf,
                         0.0);
      hipLaunchKernelGGL(k_prolong_add<double>, dim3(blocks(Fl.h.N, 256)), dim3(256), 0, stream, tv, a, dst);
      a = dst;
    }
  }
  const int nb = blocks(std::max(R.h.C, R.h.N), 256);
  if (red_partial.n < 4 * static_cast<size_t>(nb)) red_partial.alloc(4 * static_cast<size_t>(nb));
  if (!red_out.p) red_out.alloc(64);
  hipLaunchKernelGGL(k_vel_error_partial, dim3(nb), dim3(256), 0, stream, R.view(), a, ref, red_partial.p);
  hipLaunchKernelGGL(k_reduce_partials, dim3(4), dim3(256), 0, stream, nb, 4, red_partial.p, red_out.p);
  LAUNCH_CHECK("velocity error");
  check(hipMemcpyAsync(out, red_out.p, 4 * sizeof(double), hipMemcpyDeviceToHost, stream), "D2H");
  check(hipStreamSynchronize(stream), "velocity error sync");
}

void Ctx::residual(int l, const double *x, const double *xo, const double *rhs, double t_new,
                   double dt, double *Rout) {
  const double *sP = ensure_lps(l, dt, 0);
  DevLevel &L = *levels[l];
  double *E = cell_vectors(l);
  double *S = E + 12 * static_cast<size_t>(L.h.C);
  ProfScope ps(prof, stream, "residual", l);
  hipLaunchKernelGGL(k_cell_vectors<0>, dim3(blocks(L.h.C, 256)), dim3(256), 0, stream, L.view(),
                     phys(dt, t_new), x, xo, rhs ? 0 : 1, E);
  if (prm.delta0 > 0.0 && xo)
    hipLaunchKernelGGL(k_conv_vectors, dim3(blocks(L.h.C, 256)), dim3(256), 0, stream, L.view(), phys(dt, t_new), x,
                       xo, E);
  hipLaunchKernelGGL(k_lps_vectors, dim3(blocks(L.h.NP, 256)), dim3(256), 0, stream, L.view(), sP, x, S);
  hipLaunchKernelGGL(k_residual_nodes, dim3(blocks(L.h.N, 256)), dim3(256), 0, stream, L.view(),
                     phys(dt, t_new), x, rhs, S, E, Rout, L.large_order());
  LAUNCH_CHECK("residual");
}

// ------------------------------------------------------------------ Solver
template <typename T>
Solver<T>::~Solver() {
  clear_graphs();
  free_pipeline();
}

template <typename T>
int Solver<T>::ctx_coarse_sweeps() const {
  return ctx_->prm.nu_coarse;
}

namespace {
// HIP graph calls (capture, instantiate, launch, destroy) are made under one
// process-wide lock: simulation batches step their groups from several host
// threads at once, and the library does not rely on the graph API being safe
// to call concurrently.
std::mutex &graph_api_mutex() {
  static std::mutex m;
  return m;
}
}  // namespace

// Executables launched earlier may still run on the context's stream: it is
// synchronised before any of them is destroyed.
template <typename T>
void Solver<T>::clear_graphs() {
  bool any = ginv_.exec != nullptr;
  for (auto &kv : vgraphs_) any = any || kv.second.exec != nullptr;
  if (any) {
    (void)hipStreamSynchronize(ctx_->stream);
    std::lock_guard<std::mutex> lock(graph_api_mutex());
    for (auto &kv : vgraphs_)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (ginv_.exec) (void)hipGraphExecDestroy(ginv_.exec);
  }
  vgraphs_.clear();
  ginv_ = GraphSlot{};
}

// Graphs are used unless disabled, while not already capturing, and when no
// profiled kernel key lives on the level (profiled launches stay eager so
// that their events bracket them).
template <typename T>
bool Solver<T>::use_graph(int level) const {
  return ctx_->prm.use_graphs != 0 && !capturing_ && !ctx_->prof.wants_level(level);
}

// Captures body() on the context's private capture stream (the kernels it
// enqueues on ctx_->stream are redirected there and only recorded), then
// launches the instantiated graph on the context's stream.
template <typename T>
template <class F>
void Solver<T>::graph_run(GraphSlot &g, F &&body) {
  if (g.exec && g.gen != ctx_->graph_gen) {   // stale: wait for its last launch, then destroy it
    check(hipStreamSynchronize(ctx_->stream), "graph sync");
    std::lock_guard<std::mutex> lock(graph_api_mutex());
    (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
  }
  std::lock_guard<std::mutex> lock(graph_api_mutex());
  if (!g.exec) {
    hipStream_t cap = ctx_->capture_stream();
    hipStream_t saved = ctx_->stream;
    const bool prof_on = ctx_->prof.on;
    hipGraph_t graph = nullptr;
    check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    ctx_->stream = cap;
    ctx_->prof.on = false;
    capturing_ = true;
    auto restore = [&]() {
      ctx_->stream = saved;
      ctx_->prof.on = prof_on;
      capturing_ = false;
    };
    try {
      body();
    } catch (...) {
      (void)hipStreamEndCapture(cap, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      restore();
      throw;
    }
    const hipError_t e = hipStreamEndCapture(cap, &graph);
    restore();
    check(e, "hipStreamEndCapture");
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    check(ei, "hipGraphInstantiate");
    g.gen = ctx_->graph_gen;
  }
  check(hipGraphLaunch(g.exec, ctx_->stream), "hipGraphLaunch");
}

template <typename T>
void Solver<T>::setup(int finest) {
  clear_graphs();
  ops_.clear();
  ops_.resize(finest + 1);
  for (int l = 0; l <= finest; ++l) {
    const HostLevel &h = ctx_->levels[l]->h;
    OpLevel<T> &o = ops_[l];
    o.JQ.alloc(static_cast<size_t>(h.totq) * 9 * kS);
    o.JX.alloc(static_cast<size_t>(std::max(h.totx, 1)) * kS);
    o.inv.alloc(static_cast<size_t>(144) * ((h.C + kS - 1) / kS) * kS);
    o.delta.alloc(static_cast<size_t>(12) * h.C);
    o.r.alloc(3 * static_cast<size_t>(h.N));
    o.b.alloc(3 * static_cast<size_t>(h.N));
    o.x.alloc(3 * static_cast<size_t>(h.N));
    o.t.alloc(3 * static_cast<size_t>(h.N));
  }
  // cell blocks of the Vanka factorisation, shared by the levels (each level
  // is assembled and factorised before the next)
  cblk_.alloc(static_cast<size_t>(144) * ctx_->levels[finest]->h.C);
  // the direct solve at the bottom of the V-cycle: level c_ (0 unless set)
  c_ = ctx_->prm.coarse_level;
  if (c_ > finest) throw DnnmgError{DNNMG_EINVAL, "coarse_level above the finest level"};
  if (c_ > 0 && !ctx_->blk0.empty()) throw DnnmgError{DNNMG_EINVAL, "a batch solves on level 0"};
  n0_ = 3 * ctx_->levels[c_]->h.N;
  // Coarse blocks: one per simulation of a batch (its nodes are those of its
  // own mesh), a single block otherwise.  A block is solved by blocked
  // Gauss-Jordan (panels of kGjB columns; one thread per row up to 1024
  // unknowns, two up to 1536); a single larger block falls back to one pivot
  // and one elimination launch per column.
  const int N0 = ctx_->levels[c_]->h.N;
  std::vector<int> blk(N0, 0);
  if (!ctx_->blk0.empty()) {
    if (static_cast<int>(ctx_->blk0.size()) != N0)
      throw DnnmgError{DNNMG_EINVAL, "level-0 block map does not match the mesh"};
    blk = ctx_->blk0;
  }
  nblk_ = 1 + *std::max_element(blk.begin(), blk.end());
  std::vector<int> cnt(nblk_, 0), g2l(N0);
  for (int i = 0; i < N0; ++i) g2l[i] = cnt[blk[i]]++;
  nb_ = 3 * *std::max_element(cnt.begin(), cnt.end());
  gj_rpt_ = nb_ <= kGjMaxRows<1> ? 1 : 2;
  gj_b_ = nb_ <= kGjMaxRows<2> ? kGjB : 0;
  if (gj_b_ == 0 && nblk_ > 1)
    throw DnnmgError{DNNMG_EINVAL, "a level-0 block of the batch exceeds 1536 unknowns"};
  if (gj_b_ > 0) {
    std::vector<int> bdof(static_cast<size_t>(nblk_) * nb_, -1);
    for (int i = 0; i < N0; ++i)
      for (int f = 0; f < 3; ++f) bdof[static_cast<size_t>(blk[i]) * nb_ + 3 * g2l[i] + f] = 3 * i + f;
    const size_t wsz = static_cast<size_t>(nblk_) * nb_ * 2 * nb_;
    W_.alloc(wsz);
    W2_.alloc(wsz);
    Zp_.alloc(static_cast<size_t>(nblk_) * nb_ * gj_b_);
    Ainv_.alloc(static_cast<size_t>(nblk_) * nb_ * nb_);
    piv_.alloc(static_cast<size_t>(nblk_) * nb_);
    used_.alloc(static_cast<size_t>(nblk_) * nb_);
    g2l_.upload(g2l, ctx_->stream);
    blk_.upload(blk, ctx_->stream);
    bdof_.upload(bdof, ctx_->stream);
  } else {
    W_.alloc(static_cast<size_t>(n0_) * 2 * n0_);
    prow_.alloc(2 * static_cast<size_t>(n0_));
    colk_.alloc(static_cast<size_t>(n0_));
  }
  lin_level_ = -1;
}

// Every fused or vectorised launch variant at workgroup size 256 (no timing).
// The FP32 four-cells-per-thread Vanka apply (C a multiple of 4), streaming
// the inverses on levels with at least kStreamCells cells.
inline void launch_apply4(hipStream_t s, int C, int bs, const LevelView &v, const float *inv, const float *r,
                          float *delta) {
  if (C >= kStreamCells)
    hipLaunchKernelGGL(k_vanka_apply4<true>, dim3(blocks(C / 4, bs)), dim3(bs), 0, s, v, inv, r, delta);
  else
    hipLaunchKernelGGL(k_vanka_apply4<false>, dim3(blocks(C / 4, bs)), dim3(bs), 0, s, v, inv, r, delta);
}

// The one-thread-per-row SpMV, streaming the operator on levels with at
// least kStreamCells nodes.
template <typename T>
void launch_spmv(hipStream_t s, int N, int bs, const LevelView &v, const T *JQ, const T *JX, const T *x,
                 const T *b, T *y) {
  if (N >= kStreamCells)
    hipLaunchKernelGGL((k_spmv<T, true>), dim3(blocks(N, bs)), dim3(bs), 0, s, v, JQ, JX, x, b, y);
  else
    hipLaunchKernelGGL((k_spmv<T, false>), dim3(blocks(N, bs)), dim3(bs), 0, s, v, JQ, JX, x, b, y);
}

// The one-cell-per-thread Vanka apply, streaming the inverses on levels with
// at least kStreamCells cells.
template <typename T>
void launch_apply(hipStream_t s, int C, int bs, const LevelView &v, const T *inv, const T *r, T *delta) {
  if (C >= kStreamCells)
    hipLaunchKernelGGL((k_vanka_apply<T, true>), dim3(blocks(C, bs)), dim3(bs), 0, s, v, inv, r, delta);
  else
    hipLaunchKernelGGL((k_vanka_apply<T, false>), dim3(blocks(C, bs)), dim3(bs), 0, s, v, inv, r, delta);
}

template <typename T>
void Solver<T>::fuse_all() {
  for (size_t l = 0; l < ops_.size(); ++l) {
    OpLevel<T> &o = ops_[l];
    o.bs_smooth = 256;
    o.smooth_lanes = 16;
    o.bs_rres = 256;
    o.bs_spmv4 = 256;
    o.bs_upro = static_cast<int>(l) - 1 > c_ ? 256 : 0;
    o.bs_apply4 = ctx_->levels[l]->h.C % 4 == 0 ? 256 : 0;
    o.bs_update_ord = ctx_->levels[l]->node_order.n == static_cast<size_t>(ctx_->levels[l]->h.N) ? 256 : 0;
  }
}

template <typename T>
void Solver<T>::autotune() {
  hipStream_t s = ctx_->stream;
  for (auto &o : ops_) {   // defined contents for the timing runs
    for (DevBuf<T> *v : {&o.JQ, &o.JX, &o.inv, &o.delta, &o.r, &o.b, &o.x, &o.t})
      hipLaunchKernelGGL(k_fill<T>, dim3(std::min(blocks(v->n, 256), 1024)), dim3(256), 0, s, v->p, v->n,
                         T(0));
  }
  LAUNCH_CHECK("autotune fill");
  hipEvent_t e0, e1;
  check(hipEventCreate(&e0), "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    throw DnnmgError{DNNMG_EDEVICE, "hipEventCreate failed"};
  }
  const int cand[3] = {64, 128, 256};
  // In a V-cycle a level's operator, inverses and vectors have left the L2
  // caches (32 MB in all) by the time they are used again, and on the small
  // levels the dependent load chains then decide which variant is faster.
  // Each timed launch therefore follows a 64 MB fill that evicts the L2s.
  DevBuf<float> evict;
  evict.alloc(size_t(16) << 20);
  float last_t = 0.0f;   // time of the last pick's winner (one launch after eviction, ms)
  auto pick = [&](auto launch) {
    float best_t = 1e30f;
    int best = 256;
    for (int rep = 0; rep < 3; ++rep)
      for (int ci = 0; ci < 3; ++ci) {
        const int bs = cand[rep == 1 ? 2 - ci : ci];
        if (rep == 0) launch(bs);
        hipLaunchKernelGGL(k_fill<float>, dim3(2048), dim3(256), 0, s, evict.p, evict.n, 0.0f);
        check(hipEventRecord(e0, s), "hipEventRecord");
        launch(bs);
        check(hipEventRecord(e1, s), "hipEventRecord");
        check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.0f;
        check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (ms < best_t) {
          best_t = ms;
          best = bs;
        }
      }
    last_t = best_t;
    return best;
  };
  try {
    const T omega = static_cast<T>(ctx_->prm.vanka_omega);
    for (int l = 0; l < static_cast<int>(ops_.size()); ++l) {
      DevLevel &L = *ctx_->levels[l];
      OpLevel<T> &o = ops_[l];
      const LevelView v = L.view();
      o.bs_spmv = pick([&](int bs) {
        launch_spmv<T>(s, L.h.N, bs, v, o.JQ.p, o.JX.p, o.x.p, o.b.p, o.t.p);
      });
      // four threads per row (bitwise the same rows): kept if faster
      o.bs_spmv4 = 0;
      const float t_one = last_t;
      const int bs4 = pick([&](int bs) {
        hipLaunchKernelGGL(k_spmv4<T>, dim3(blocks(4 * static_cast<size_t>(L.h.N), bs)), dim3(bs), 0, s, v, o.JQ.p,
                           o.JX.p, o.x.p, o.b.p, o.t.p);
      });
      if (last_t < t_one) o.bs_spmv4 = bs4;
      if (l == 0) continue;
      o.bs_apply = pick([&](int bs) {
        launch_apply<T>(s, L.h.C, bs, v, o.inv.p, o.r.p, o.delta.p);
      });
      // four cells per thread with 16-byte loads (FP32, C a multiple of 4): kept if faster
      o.bs_apply4 = 0;
      if constexpr (std::is_same_v<T, float>) {
        if (L.h.C % 4 == 0) {
          const float t_one_apply = last_t;
          const int bs4a = pick([&](int bs) {
            launch_apply4(s, L.h.C, bs, v, o.inv.p, o.r.p, o.delta.p);
          });
          if (last_t < t_one_apply) o.bs_apply4 = bs4a;
        }
      }
      // residual + apply: separate kernels at their best sizes, or fused
      o.bs_smooth = 0;
      const int bsp = o.bs_spmv, bap = o.bs_apply, bap4 = o.bs_apply4;
      pick([&](int) {
        launch_spmv<T>(s, L.h.N, bsp, v, o.JQ.p, o.JX.p, o.x.p, o.b.p, o.r.p);
        if constexpr (std::is_same_v<T, float>) {
          if (bap4 > 0) {
            launch_apply4(s, L.h.C, bap4, v, o.inv.p, o.r.p, o.delta.p);
            return;
          }
        }
        launch_apply<T>(s, L.h.C, bap, v, o.inv.p, o.r.p, o.delta.p);
      });
      const float t_sep = last_t;
      const int bsm = pick([&](int bs) {
        hipLaunchKernelGGL(k_vanka_smooth<T>, dim3(blocks(4 * static_cast<size_t>(L.h.C), bs)), dim3(bs), 0, s,
                           v, o.JQ.p, o.JX.p, o.x.p, o.b.p, o.inv.p, o.delta.p);
      });
      const float t_four = last_t;
      const int bsm16 = pick([&](int bs) {
        hipLaunchKernelGGL(k_vanka_smooth16<T>, dim3(blocks(16 * static_cast<size_t>(L.h.C), bs)), dim3(bs), 0,
                           s, v, o.JQ.p, o.JX.p, o.x.p, o.b.p, o.inv.p, o.delta.p);
      });
      const float t_sixteen = last_t;
      o.smooth_lanes = 4;
      if (t_sixteen < t_four && t_sixteen < t_sep) {
        o.bs_smooth = bsm16;
        o.smooth_lanes = 16;
      } else if (t_four < t_sep) {
        o.bs_smooth = bsm;
      }
      o.bs_update = pick([&](int bs) {
        hipLaunchKernelGGL(k_vanka_update<T>, dim3(blocks(L.h.N, bs)), dim3(bs), 0, s, v, o.delta.p, omega,
                           o.t.p, 0);
      });
      // the nodes in cell order: kept if faster
      o.bs_update_ord = 0;
      if (L.node_order.n == static_cast<size_t>(L.h.N)) {
        const float t_nat = last_t;
        const int bso = pick([&](int bs) {
          hipLaunchKernelGGL(k_vanka_update_ordered<T>, dim3(blocks(L.h.N, bs)), dim3(bs), 0, s, v,
                             L.node_order.p, o.delta.p, omega, o.t.p, 0);
        });
        if (last_t < t_nat) o.bs_update_ord = bso;
      }
      DevLevel &Cl = *ctx_->levels[l - 1];
      OpLevel<T> &oc = ops_[l - 1];
      TransferView tv{L.h.Nc, L.h.Ec, L.h.N, L.edge_ends.p, Cl.cells.p, L.rptr.p, L.ridx.p, Cl.flag.p};
      o.bs_restrict = pick([&](int bs) {
        hipLaunchKernelGGL(k_restrict<T>, dim3(blocks(L.h.Nc, bs)), dim3(bs), 0, s, tv, o.r.p, oc.t.p,
                           Cl.large_order());
      });
      o.bs_prolong = pick([&](int bs) {
        hipLaunchKernelGGL(k_prolong_add<T>, dim3(blocks(L.h.N, bs)), dim3(bs), 0, s, tv, oc.x.p, o.t.p);
      });
      // the coarser level's last update + this prolongation: separate, or fused
      o.bs_upro = 0;
      if (l - 1 > c_) {
        const int bsu = oc.bs_update, bsq = o.bs_prolong;
        pick([&](int) {
          hipLaunchKernelGGL(k_vanka_update<T>, dim3(blocks(Cl.h.N, bsu)), dim3(bsu), 0, s, Cl.view(), oc.delta.p,
                             omega, oc.x.p, 0);
          hipLaunchKernelGGL(k_prolong_add<T>, dim3(blocks(L.h.N, bsq)), dim3(bsq), 0, s, tv, oc.x.p, o.t.p);
        });
        const float t_sep_up = last_t;
        const int bsf = pick([&](int bs) {
          hipLaunchKernelGGL(k_update_prolong_add<T>, dim3(blocks(L.h.N, bs)), dim3(bs), 0, s, tv, Cl.view(),
                             oc.delta.p, omega, oc.x.p, o.t.p);
        });
        if (last_t < t_sep_up) o.bs_upro = bsf;
      }
      // residual + restriction: separate at their best sizes, or fused
      o.bs_rres = 0;
      const int bsr = o.bs_restrict;
      pick([&](int) {
        launch_spmv<T>(s, L.h.N, bsp, v, o.JQ.p, o.JX.p, o.x.p, o.b.p, o.r.p);
        hipLaunchKernelGGL(k_restrict<T>, dim3(blocks(L.h.Nc, bsr)), dim3(bsr), 0, s, tv, o.r.p, oc.t.p,
                           Cl.large_order());
      });
      const float t_sep2 = last_t;
      const int bsrr = pick([&](int bs) {
        hipLaunchKernelGGL(k_restrict_residual<T>, dim3(blocks(L.h.Nc, bs)), dim3(bs), 0, s, tv, v, o.JQ.p,
                           o.JX.p, o.x.p, o.b.p, oc.t.p);
      });
      if (last_t < t_sep2) o.bs_rres = bsrr;
      LAUNCH_CHECK("autotune");
    }
    // bottom of the V-cycle in one workgroup (levels 1..top), if faster than
    // the launches it replaces (those replayed from a graph, as in use)
    small_top_ = 0;
    const int tmax = std::min(kSmallLevels - 1, static_cast<int>(ops_.size()) - 1);
    for (int top = 1; top <= tmax && gj_b_ > 0 && c_ == 0; ++top) {
      OpLevel<T> &o = ops_[top];
      const int keep = small_top_;
      pick([&](int) { vcycle(top, o.b.p, o.x.p); });
      const float t_multi = last_t;
      small_top_ = top;
      pick([&](int) { vcycle(top, o.b.p, o.x.p); });
      if (!(last_t < t_multi)) {
        small_top_ = keep;
        break;
      }
    }
    clear_graphs();
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <typename T>
void Solver<T>::linearize(const double *x_dev, const double *xo_dev, int level, double dt, bool full) {
  hipStream_t s = ctx_->stream;
  kept_key_ = 0;
  if (level < c_) throw DnnmgError{DNNMG_EINVAL, "solve level below coarse_level"};
  if (lin_level_ < level) full = true;   // never factorised at this depth
  for (int l = full ? c_ : level; l <= level; ++l) {
    // the level solved on carries its own problem's stabilisation; the
    // coarser levels of its preconditioner the bounded form
    const double *sP = ctx_->ensure_lps(l, dt, l < level ? 1 : 0);
    DevLevel &L = *ctx_->levels[l];
    OpLevel<T> &o = ops_[l];
    {
      // one wavefront per slice, the slice's rows accumulated in LDS
      const size_t lds = static_cast<size_t>(L.h.maxwq * 9 + L.h.maxwx) * kS * sizeof(T);
      if (lds > 65536) throw DnnmgError{DNNMG_EINVAL, "node rows too wide for the LDS assembly"};
      ProfScope ps(ctx_->prof, s, "assemble", l);
      hipLaunchKernelGGL(k_assemble<T>, dim3(L.h.nslice), dim3(kS), lds, s, L.view(), ctx_->phys(dt, 0.0), x_dev,
                         sP, xo_dev, o.JQ.p, o.JX.p, full && l > c_ ? cblk_.p : nullptr);
    }
    LAUNCH_CHECK("k_assemble");
    if (full && l > c_) {
      ProfScope ps(ctx_->prof, s, "vanka_factor", l);
      hipLaunchKernelGGL(k_vanka_factor<T>, dim3(blocks(static_cast<size_t>(L.h.C) * 4, 256)),
                         dim3(256), 0, s, L.view(), cblk_.p, o.inv.p);
      LAUNCH_CHECK("k_vanka_factor");
    }
  }
  if (!full) return;
  if (use_graph(c_))
    graph_run(ginv_, [&]() { coarse_inverse(); });
  else
    coarse_inverse();
  lin_level_ = level;
}

// Dense inverse (FP64) of the coarse level's Jacobian: blocked Gauss-Jordan
// with partial pivoting on [J_c | I] per block, or one pivot kernel and one
// elimination kernel per column for a single large block.
template <typename T>
void Solver<T>::coarse_inverse() {
  hipStream_t s = ctx_->stream;
  DevLevel &L0 = *ctx_->levels[c_];
  ProfScope ps(ctx_->prof, s, "coarse_inverse", c_);
  hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, s, W_.p, W_.n, 0.0);
  if (gj_b_ > 0) {
    const int nb = nb_;
    hipLaunchKernelGGL(k_dense_from_sell_blk<T>, dim3(blocks(L0.h.N, 64)), dim3(64), 0, s, L0.view(),
                       ops_[c_].JQ.p, ops_[c_].JX.p, g2l_.p, blk_.p, nb, W_.p);
    hipLaunchKernelGGL(k_gjb_init, dim3(blocks(nb, 256), nblk_), dim3(256), 0, s, nblk_, nb, bdof_.p, W_.p);
    double *wo = W_.p, *wn = W2_.p;
    for (int k0 = 0; k0 < nb; k0 += gj_b_) {
      const int b = std::min(gj_b_, nb - k0);
      if (gj_rpt_ == 1)
        hipLaunchKernelGGL(k_gjb_panel<1>, dim3(nblk_), dim3(64 * blocks(nb, 64)), 0, s, nb, k0, b, wo, used_.p,
                           piv_.p, Zp_.p);
      else
        hipLaunchKernelGGL(k_gjb_panel<2>, dim3(nblk_), dim3(64 * blocks(blocks(nb, 2), 64)), 0, s, nb, k0, b, wo,
                           used_.p, piv_.p, Zp_.p);
      const dim3 ug(blocks(2 * nb - k0 - b, 64), blocks(nb, 16), nblk_);
      hipLaunchKernelGGL(k_gjb_update, ug, dim3(256), 0, s, nb, k0, b, wo, Zp_.p, piv_.p, wn);
      std::swap(wo, wn);
    }
    hipLaunchKernelGGL(k_gjb_extract, dim3(blocks(nb, 256), nb, nblk_), dim3(256), 0, s, nb, wo, piv_.p,
                       Ainv_.p);
    LAUNCH_CHECK("blocked coarse inverse");
    return;
  }
  hipLaunchKernelGGL(k_dense_from_sell<T>, dim3(blocks(L0.h.N, 64)), dim3(64), 0, s, L0.view(),
                     ops_[c_].JQ.p, ops_[c_].JX.p, W_.p, 2 * n0_);
  hipLaunchKernelGGL(k_identity_right, dim3(blocks(n0_, 256)), dim3(256), 0, s, n0_, W_.p);
  const dim3 eg(blocks(2 * n0_, 256), n0_);
  for (int k = 0; k < n0_; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, n0_, k, W_.p, prow_.p, colk_.p);
    hipLaunchKernelGGL(k_gj_elim, eg, dim3(256), 0, s, n0_, k, W_.p, prow_.p, colk_.p);
  }
  LAUNCH_CHECK("coarse inverse");
}

template <typename T>
void Solver<T>::spmv(int l, const T *x, const T *b, T *y) {
  DevLevel &L = *ctx_->levels[l];
  OpLevel<T> &o = ops_[l];
  ProfScope ps(ctx_->prof, ctx_->stream, b ? "residual_spmv" : "spmv", l);
  if (o.bs_spmv4 > 0)
    hipLaunchKernelGGL(k_spmv4<T>, dim3(blocks(4 * static_cast<size_t>(L.h.N), o.bs_spmv4)), dim3(o.bs_spmv4), 0,
                       ctx_->stream, L.view(), o.JQ.p, o.JX.p, x, b, y);
  else
    launch_spmv<T>(ctx_->stream, L.h.N, o.bs_spmv, L.view(), o.JQ.p, o.JX.p, x, b, y);
  LAUNCH_CHECK("k_spmv");
}

template <typename T>
void Solver<T>::vanka_sweep(int l, T *x, const T *b, bool zero_start, bool defer_update) {
  DevLevel &L = *ctx_->levels[l];
  OpLevel<T> &o = ops_[l];
  hipStream_t s = ctx_->stream;
  if (ctx_->prm.smoother == 1) {   // coloured multiplicative: colour by colour
    if (zero_start) hipLaunchKernelGGL(k_fill<T>, dim3(blocks(3 * static_cast<size_t>(L.h.N), 256)), dim3(256), 0, s,
                                       x, 3 * static_cast<size_t>(L.h.N), T(0));
    const T omega = static_cast<T>(ctx_->prm.vanka_omega);
    for (int k = 0; k < L.h.ncolour; ++k) {
      spmv(l, x, b, o.r.p);
      const int c0 = L.h.colour_ptr[k], n = L.h.colour_ptr[k + 1] - c0;
      ProfScope ps(ctx_->prof, s, "vanka_colour", l);
      hipLaunchKernelGGL(k_vanka_colour<T>, dim3(blocks(n, 256)), dim3(256), 0, s, L.view(), o.inv.p, o.r.p,
                         L.colour_cells.p + c0, n, omega, x);
    }
    LAUNCH_CHECK("coloured vanka");
    return;
  }
  const T *r = b;
  if (!zero_start && o.bs_smooth > 0) {
    ProfScope ps(ctx_->prof, s, "vanka_smooth", l);
    if (o.smooth_lanes == 16)
      hipLaunchKernelGGL(k_vanka_smooth16<T>, dim3(blocks(16 * static_cast<size_t>(L.h.C), o.bs_smooth)),
                         dim3(o.bs_smooth), 0, s, L.view(), o.JQ.p, o.JX.p, x, b, o.inv.p, o.delta.p);
    else
      hipLaunchKernelGGL(k_vanka_smooth<T>, dim3(blocks(4 * static_cast<size_t>(L.h.C), o.bs_smooth)),
                         dim3(o.bs_smooth), 0, s, L.view(), o.JQ.p, o.JX.p, x, b, o.inv.p, o.delta.p);
  } else {
    if (!zero_start) {
      spmv(l, x, b, o.r.p);
      r = o.r.p;
    }
    ProfScope ps(ctx_->prof, s, "vanka_apply", l);
    if constexpr (std::is_same_v<T, float>) {
      if (o.bs_apply4 > 0) {
        launch_apply4(s, L.h.C, o.bs_apply4, L.view(), o.inv.p, r, o.delta.p);
        LAUNCH_CHECK("k_vanka_apply4");
      }
    }
    if (!(std::is_same_v<T, float> && o.bs_apply4 > 0))
      launch_apply<T>(s, L.h.C, o.bs_apply, L.view(), o.inv.p, r, o.delta.p);
  }
  if (!defer_update) {
    ProfScope ps(ctx_->prof, s, "vanka_update", l);
    if (o.bs_update_ord > 0 && L.node_order.n == static_cast<size_t>(L.h.N))
      hipLaunchKernelGGL(k_vanka_update_ordered<T>, dim3(blocks(L.h.N, o.bs_update_ord)), dim3(o.bs_update_ord),
                         0, s, L.view(), L.node_order.p, o.delta.p, static_cast<T>(ctx_->prm.vanka_omega), x,
                         zero_start ? 1 : 0);
    else
      hipLaunchKernelGGL(k_vanka_update<T>, dim3(blocks(L.h.N, o.bs_update)), dim3(o.bs_update), 0, s, L.view(),
                         o.delta.p, static_cast<T>(ctx_->prm.vanka_omega), x, zero_start ? 1 : 0);
  }
  LAUNCH_CHECK("vanka");
}

template <typename T>
void Solver<T>::prolong_add(int l, const T *ec, T *xf) {
  DevLevel &F = *ctx_->levels[l];
  DevLevel &Cl = *ctx_->levels[l - 1];
  TransferView tv{F.h.Nc, F.h.Ec, F.h.N, F.edge_ends.p, Cl.cells.p, F.rptr.p, F.ridx.p, Cl.flag.p};
  ProfScope ps(ctx_->prof, ctx_->stream, "prolong", l);
  const int bs = ops_[l].bs_prolong;
  hipLaunchKernelGGL(k_prolong_add<T>, dim3(blocks(F.h.N, bs)), dim3(bs), 0, ctx_->stream, tv, ec,
                     xf);
  LAUNCH_CHECK("k_prolong_add");
}

template <typename T>
void Solver<T>::restrict_to(int l, const T *rf, T *rc) {
  DevLevel &F = *ctx_->levels[l];
  DevLevel &Cl = *ctx_->levels[l - 1];
  TransferView tv{F.h.Nc, F.h.Ec, F.h.N, F.edge_ends.p, Cl.cells.p, F.rptr.p, F.ridx.p, Cl.flag.p};
  ProfScope ps(ctx_->prof, ctx_->stream, "restrict", l);
  const int bs = ops_[l].bs_restrict;
  hipLaunchKernelGGL(k_restrict<T>, dim3(blocks(F.h.Nc, bs)), dim3(bs), 0, ctx_->stream, tv, rf,
                     rc, Cl.large_order());
  LAUNCH_CHECK("k_restrict");
}

template <typename T>
SmallCycle<T> Solver<T>::small_params(int top, const T *b, T *x) {
  SmallCycle<T> P{};
  for (int l = 0; l <= top; ++l) {
    DevLevel &L = *ctx_->levels[l];
    OpLevel<T> &o = ops_[l];
    SmallLevel<T> &V = P.lv[l];
    V.L = L.view();
    if (l > 0) {
      DevLevel &Cl = *ctx_->levels[l - 1];
      V.tv = TransferView{L.h.Nc, L.h.Ec, L.h.N, L.edge_ends.p, Cl.cells.p, L.rptr.p, L.ridx.p, Cl.flag.p};
    }
    V.JQ = o.JQ.p;
    V.JX = o.JX.p;
    V.inv = o.inv.p;
    V.delta = o.delta.p;
    V.r = o.r.p;
    V.b = l == top ? const_cast<T *>(b) : o.b.p;
    V.x = l == top ? x : o.x.p;
  }
  P.top = top;
  // every level of the one-workgroup cycle lies below the top when nu_coarse is set
  P.nu_pre = ctx_->prm.nu_coarse > 0 ? ctx_->prm.nu_coarse : ctx_->prm.nu_pre;
  P.nu_post = ctx_->prm.nu_coarse > 0 ? ctx_->prm.nu_coarse : ctx_->prm.nu_post;
  P.omega = static_cast<T>(ctx_->prm.vanka_omega);
  P.nblk = nblk_;
  P.nb = nb_;
  P.Ainv = Ainv_.p;
  P.bdof = bdof_.p;
  return P;
}

template <typename T>
void Solver<T>::launch_small(int top, const T *b, T *x) {
  ProfScope ps(ctx_->prof, ctx_->stream, "vcycle_small", top);
  hipLaunchKernelGGL(k_vcycle_small<T>, dim3(1), dim3(1024), 0, ctx_->stream, small_params(top, b, x));
  LAUNCH_CHECK("k_vcycle_small");
}

template <typename T>
bool Solver<T>::vcycle(int l, const T *b, T *x, bool defer) {
  // the outermost call's level is the top of the cycle (nu_pre / nu_post
  // sweeps); the levels below take nu_coarse sweeps when that is set
  struct Depth {
    int &d;
    explicit Depth(int &v) : d(v) { ++d; }
    ~Depth() { --d; }
  };
  if (cycle_depth_ == 0) cycle_top_ = l;
  Depth guard(cycle_depth_);
  // the one-workgroup cycle is additive and uses one sweep count for all its levels
  if (l < c_) throw DnnmgError{DNNMG_EINVAL, "V-cycle below coarse_level"};
  if (c_ == 0 && l >= 1 && l <= small_top_ && ctx_->prm.smoother == 0 &&
      (ctx_->prm.nu_coarse == 0 || l != cycle_top_)) {
    launch_small(l, b, x);
    return false;
  }
  if (l > c_ && use_graph(l)) {
    const auto key = std::make_tuple(l, (l == cycle_top_ ? 1 : 0) + (defer ? 2 : 0), static_cast<const void *>(b),
                                     static_cast<const void *>(x));
    // bound the cache: keys of freed work vectors are never looked up again
    if (vgraphs_.size() >= 512 && vgraphs_.find(key) == vgraphs_.end()) clear_graphs();
    // the body decides from the level and parameters alone (will_defer), so
    // a replay defers exactly when the captured body did
    graph_run(vgraphs_[key], [&]() { vcycle_body(l, b, x, defer); });
    return defer && will_defer(l);
  }
  return vcycle_body(l, b, x, defer);
}

// Whether vcycle_body(l, ..., defer = true) leaves its last update to the
// caller: an additive smoother with at least one post-sweep on a level above
// the direct solve.
template <typename T>
bool Solver<T>::will_defer(int l) const {
  if (l <= c_ || ctx_->prm.smoother != 0) return false;
  const int nu2 = inner_level(l) ? ctx_->prm.nu_coarse : ctx_->prm.nu_post;
  return nu2 > 0;
}

template <typename T>
bool Solver<T>::vcycle_body(int l, const T *b, T *x, bool defer) {
  hipStream_t s = ctx_->stream;
  if (l == c_) {
    ProfScope ps(ctx_->prof, s, "coarse_solve", c_);
    // a single block above level 0 (no padding, unknowns in order): one
    // wavefront per row; level 0 keeps the per-block rows the single-workgroup
    // bottom cycle also uses
    if (gj_b_ > 0 && nblk_ == 1 && c_ > 0)
      hipLaunchKernelGGL(k_dense_solve_w<T>, dim3(blocks(nb_, 4)), dim3(256), 0, s, nb_, Ainv_.p,
                         static_cast<size_t>(nb_), b, x);
    else if (gj_b_ > 0)
      hipLaunchKernelGGL(k_dense_solve_blk<T>, dim3(blocks(static_cast<size_t>(nblk_) * nb_, 8)), dim3(256), 0,
                         s, nblk_, nb_, Ainv_.p, bdof_.p, b, x);
    else
      hipLaunchKernelGGL(k_dense_solve_w<T>, dim3(blocks(n0_, 4)), dim3(256), 0, s, n0_, W_.p + n0_,
                         2 * static_cast<size_t>(n0_), b, x);
    LAUNCH_CHECK("k_dense_solve");
    return false;
  }
  DevLevel &L = *ctx_->levels[l];
  OpLevel<T> &o = ops_[l];
  OpLevel<T> &oc = ops_[l - 1];
  const size_t n = 3 * static_cast<size_t>(L.h.N);
  const bool inner = inner_level(l);
  const int nu1 = inner ? ctx_->prm.nu_coarse : ctx_->prm.nu_pre;
  const int nu2 = inner ? ctx_->prm.nu_coarse : ctx_->prm.nu_post;
  // zero iterate: the first sweep stores its update (no separate fill)
  if (nu1 == 0)
    hipLaunchKernelGGL(k_fill<T>, dim3(std::min(blocks(n, 256), 1024)), dim3(256), 0, s, x, n, T(0));
  for (int k = 0; k < nu1; ++k) vanka_sweep(l, x, b, k == 0);
  if (o.bs_rres > 0) {
    DevLevel &Cl = *ctx_->levels[l - 1];
    TransferView tv{L.h.Nc, L.h.Ec, L.h.N, L.edge_ends.p, Cl.cells.p, L.rptr.p, L.ridx.p, Cl.flag.p};
    ProfScope ps(ctx_->prof, s, "restrict_residual", l);
    hipLaunchKernelGGL(k_restrict_residual<T>, dim3(blocks(L.h.Nc, o.bs_rres)), dim3(o.bs_rres), 0, s, tv,
                       L.view(), o.JQ.p, o.JX.p, x, b, oc.b.p);
    LAUNCH_CHECK("k_restrict_residual");
  } else {
    spmv(l, x, b, o.r.p);
    restrict_to(l, o.r.p, oc.b.p);
  }
  // the coarser level's last update fused into the prolongation, where the
  // autotuner found that faster
  if (vcycle(l - 1, oc.b.p, oc.x.p, o.bs_upro > 0)) {
    DevLevel &Cl = *ctx_->levels[l - 1];
    TransferView tv{L.h.Nc, L.h.Ec, L.h.N, L.edge_ends.p, Cl.cells.p, L.rptr.p, L.ridx.p, Cl.flag.p};
    ProfScope ps(ctx_->prof, s, "update_prolong", l);
    hipLaunchKernelGGL(k_update_prolong_add<T>, dim3(blocks(L.h.N, o.bs_upro)), dim3(o.bs_upro), 0, s, tv,
                       Cl.view(), oc.delta.p, static_cast<T>(ctx_->prm.vanka_omega), oc.x.p, x);
    LAUNCH_CHECK("k_update_prolong_add");
  } else {
    prolong_add(l, oc.x.p, x);
  }
  const bool dfr = defer && will_defer(l);
  for (int k = 0; k < nu2; ++k) vanka_sweep(l, x, b, false, dfr && k == nu2 - 1);
  return dfr;
}

template <typename T>
void Solver<T>::free_pipeline() {
  for (auto e : hev_) (void)hipEventDestroy(e);
  hev_.clear();
  if (hpin_) (void)hipHostFree(hpin_);
  hpin_ = nullptr;
  hslots_ = 0;
}

template <typename T>
void Solver<T>::ensure_gmres(int level, int m) {
  const size_t n = 3 * static_cast<size_t>(ctx_->levels[level]->h.N);
  if (gm_level_ == level && gm_m_ >= m) return;
  V_.alloc((m + 1) * n);
  Z_.alloc(m * n);
  w_.alloc(n);
  partial_.alloc(static_cast<size_t>(1024) * (m + 2));
  hdev_.alloc(static_cast<size_t>(2 * (m + 2)));
  hhost_.assign(2 * (m + 2), 0.0);
  if (hslots_ < m) {
    free_pipeline();
    const size_t stride = 2 * static_cast<size_t>(m + 1) + 1;
    hcol_.alloc(stride * m);
    if (hipHostMalloc(reinterpret_cast<void **>(&hpin_), sizeof(double) * stride * m) != hipSuccess)
      throw DnnmgError{DNNMG_ENOMEM, "hipHostMalloc failed"};
    hev_.resize(m, nullptr);
    for (auto &e : hev_) check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    hslots_ = m;
  }
  gm_level_ = level;
  gm_m_ = m;
}

// Right-preconditioned restarted GMRES (Saad) with classical Gram-Schmidt
// applied twice (FP64 dot products) and Givens rotations.  x = 0 on entry is
// assumed (Newton corrections); returns the iteration count.
//
// Pipelining: each Arnoldi step normalises its new basis vector on the device
// and copies its Hessenberg column (the two Gram-Schmidt passes and the norm)
// to pinned host memory with an event; the host enqueues step j + 1 before it
// reads column j, so the GPU does not wait for the host's Givens rotations.
// It waits for column j at once only when the residual history predicts that
// step j may meet the tolerance (or at a restart or the iteration limit); a
// step enqueued past convergence is discarded (its basis vectors unused).
template <typename T>
int Solver<T>::gmres(int level, const T *b, T *x, double rtol, int restart, int maxit,
                     double *res0, double *res_out) {
  if (ctx_->levels[level]->nseg > 1) return gmres_batched(level, b, x, rtol, restart, maxit, res0, res_out);
  hipStream_t s = ctx_->stream;
  const int n = 3 * ctx_->levels[level]->h.N;
  const size_t ld = static_cast<size_t>(n);
  restart = std::max(1, std::min(restart, 64));
  ensure_gmres(level, restart);
  const int nb = std::min(blocks(n, 256), 1024);
  auto dots = [&](int m, const T *w, double *out_dev) {
    ProfScope ps(ctx_->prof, s, "gs_dots", level);
    hipLaunchKernelGGL(k_multidot<T>, dim3(nb, m), dim3(256), 0, s, n, m, V_.p, ld, w, partial_.p);
    hipLaunchKernelGGL(k_reduce_partials, dim3(m), dim3(256), 0, s, nb, m, partial_.p, out_dev);
  };
  hipLaunchKernelGGL(k_fill<T>, dim3(std::min(blocks(n, 256), 1024)), dim3(256), 0, s, x,
                     static_cast<size_t>(n), T(0));
  // beta0 = ||b||
  hipLaunchKernelGGL(k_multidot<T>, dim3(nb, 1), dim3(256), 0, s, n, 1, b, ld, b, partial_.p);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, nb, 1, partial_.p, hdev_.p);
  double beta0 = 0.0;
  check(hipMemcpyAsync(&beta0, hdev_.p, sizeof(double), hipMemcpyDeviceToHost, s), "gmres D2H");
  check(hipStreamSynchronize(s), "gmres sync");
  beta0 = std::sqrt(beta0);
  if (res0) *res0 = beta0;
  if (res_out) *res_out = beta0;
  if (beta0 == 0.0) return 0;
  const int m = restart;
  const size_t stride = 2 * static_cast<size_t>(m + 1) + 1;
  const double target = rtol * beta0;
  std::vector<double> H(static_cast<size_t>(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), rh;
  int it = 0;            // Arnoldi steps whose columns were used
  double resid = beta0;
  OpLevel<T> &o = ops_[level];
  bool first = true;
  while (it < maxit) {
    double beta;
    if (first) {
      beta = beta0;
      hipLaunchKernelGGL(k_scale_copy<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, 1.0 / beta, b,
                         V_.p);
    } else {
      spmv(level, x, b, o.t.p);   // r = b - J x
      hipLaunchKernelGGL(k_multidot<T>, dim3(nb, 1), dim3(256), 0, s, n, 1, o.t.p, ld, o.t.p,
                         partial_.p);
      hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, nb, 1, partial_.p, hdev_.p);
      check(hipMemcpyAsync(&beta, hdev_.p, sizeof(double), hipMemcpyDeviceToHost, s), "D2H");
      check(hipStreamSynchronize(s), "sync");
      beta = std::sqrt(beta);
      hipLaunchKernelGGL(k_scale_copy<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, 1.0 / beta,
                         o.t.p, V_.p);
    }
    first = false;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    rh.assign(1, beta);
    int jend = 0, done_cols = 0;
    bool conv = false;
    // host side of column c: Hessenberg entries, rotations, residual estimate
    auto process = [&](int c) {
      check(hipEventSynchronize(hev_[c]), "gmres column");
      const double *hc = hpin_ + stride * c;
      const double hn = std::sqrt(std::max(hc[2 * (c + 1)], 0.0));
      for (int i = 0; i <= c; ++i) H[i * m + c] = hc[i] + hc[c + 1 + i];
      H[(c + 1) * m + c] = hn;
      for (int i = 0; i < c; ++i) {
        const double t = cs[i] * H[i * m + c] + sn[i] * H[(i + 1) * m + c];
        H[(i + 1) * m + c] = -sn[i] * H[i * m + c] + cs[i] * H[(i + 1) * m + c];
        H[i * m + c] = t;
      }
      const double den = std::hypot(H[c * m + c], H[(c + 1) * m + c]);
      cs[c] = H[c * m + c] / den;
      sn[c] = H[(c + 1) * m + c] / den;
      H[c * m + c] = den;
      H[(c + 1) * m + c] = 0.0;
      g[c + 1] = -sn[c] * g[c];
      g[c] = cs[c] * g[c];
      ++it;
      jend = c + 1;
      done_cols = c + 1;
      resid = std::fabs(g[c + 1]);
      rh.push_back(resid);
      conv = resid <= target;
    };
    int enq = 0;   // steps enqueued in this cycle
    while (!conv && done_cols < m && it < maxit) {
      if (enq < m && it + (enq - done_cols) < maxit) {
        const int j = enq++;
        T *vj = V_.p + static_cast<size_t>(j) * ld;
        T *zj = Z_.p + static_cast<size_t>(j) * ld;
        double *hc = hcol_.p + stride * j;
        vcycle(level, vj, zj);
        spmv(level, zj, nullptr, w_.p);
        // CGS2, the new vector's norm, its normalisation
        dots(j + 1, w_.p, hc);
        hipLaunchKernelGGL(k_multi_axpy<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, j + 1, V_.p, ld, hc,
                           w_.p);
        dots(j + 1, w_.p, hc + (j + 1));
        hipLaunchKernelGGL(k_multi_axpy<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, j + 1, V_.p, ld,
                           hc + (j + 1), w_.p);
        hipLaunchKernelGGL(k_multidot<T>, dim3(nb, 1), dim3(256), 0, s, n, 1, w_.p, ld, w_.p, partial_.p);
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, nb, 1, partial_.p, hc + 2 * (j + 1));
        hipLaunchKernelGGL(k_scale_by_norm<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, hc + 2 * (j + 1),
                           w_.p, V_.p + static_cast<size_t>(j + 1) * ld);
        LAUNCH_CHECK("gmres iteration");
        check(hipMemcpyAsync(hpin_ + stride * j, hc, sizeof(double) * (2 * (j + 1) + 1),
                             hipMemcpyDeviceToHost, s),
              "gmres D2H");
        check(hipEventRecord(hev_[j], s), "gmres event");
      }
      // columns older than the newest: the GPU already has the next step queued
      while (!conv && done_cols < enq - 1) process(done_cols);
      if (conv || done_cols >= enq) continue;
      // the newest column: wait for it now only if it may finish the solve
      const int c = done_cols;
      bool wait_now = enq >= m || it + (enq - done_cols) >= maxit;
      if (!wait_now && rh.size() >= 3) {
        const double r1 = rh[rh.size() - 1], r2 = rh[rh.size() - 2];
        const double rate = r2 > 0.0 ? r1 / r2 : 1.0;
        wait_now = r1 * std::min(rate, 1.0) <= 3.0 * target;
      }
      if (wait_now) process(c);
    }
    for (int i = jend - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int k = i + 1; k < jend; ++k) sacc -= H[i * m + k] * y[k];
      y[i] = sacc / H[i * m + i];
    }
    check(hipMemcpyAsync(hdev_.p, y.data(), sizeof(double) * jend, hipMemcpyHostToDevice, s), "H2D");
    hipLaunchKernelGGL(k_combine<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, jend, Z_.p, ld,
                       hdev_.p, x);
    LAUNCH_CHECK("gmres combine");
    if (resid <= target) break;
  }
  check(hipStreamSynchronize(s), "gmres end");
  if (res_out) *res_out = resid;
  return it;
}

template <typename T>
void Solver<T>::seg_dots(int level, int m, const T *V, size_t ld, const T *w, double *dev) {
  DevLevel &L = *ctx_->levels[level];
  hipStream_t s = ctx_->stream;
  ProfScope ps(ctx_->prof, s, "gs_dots", level);
  hipLaunchKernelGGL(k_multidot_chunks<T>, dim3(L.nchunk, m), dim3(256), 0, s, L.cstart.p, L.clen.p, m, V, ld, w,
                     spart_.p);
  hipLaunchKernelGGL(k_reduce_seg, dim3(L.nseg, m), dim3(256), 0, s, L.seg_ptr.p, m, spart_.p, dev);
}

// Restarted right-preconditioned GMRES on a batch level: the operator and the
// V-cycle are block diagonal over the simulations, and every inner product,
// Hessenberg column, Givens rotation and least-squares solve is kept per
// simulation, so each simulation iterates in its own Krylov space (as it
// would alone).  A simulation that has converged (or broken down) is frozen:
// its basis vectors are zeroed from then on and its coefficients ignored.
// The launches are shared; the loop ends when every simulation has converged.
template <typename T>
int Solver<T>::gmres_batched(int level, const T *b, T *x, double rtol, int restart, int maxit,
                             double *res0, double *res_out) {
  hipStream_t s = ctx_->stream;
  DevLevel &L = *ctx_->levels[level];
  const int n = 3 * L.h.N, G = L.nseg;
  const size_t ld = static_cast<size_t>(n);
  restart = std::max(1, std::min(restart, 64));
  ensure_gmres(level, restart);
  const int m = restart;
  const size_t sp_need = static_cast<size_t>(L.nchunk) * (m + 1);
  if (spart_.n < sp_need) spart_.alloc(sp_need);
  const size_t sd_need = static_cast<size_t>(G) * (2 * (m + 1) + 1);
  if (sdev_.n < sd_need) sdev_.alloc(sd_need);
  if (scoef_.n < static_cast<size_t>(G) * m) scoef_.alloc(static_cast<size_t>(G) * m);
  shost_.resize(sd_need);
  auto d2h = [&](size_t cnt) {
    check(hipMemcpyAsync(shost_.data(), sdev_.p, sizeof(double) * cnt, hipMemcpyDeviceToHost, s), "gmres D2H");
    check(hipStreamSynchronize(s), "gmres sync");
  };
  auto scale_to = [&](const std::vector<double> &a, const T *src, T *dst) {
    check(hipMemcpyAsync(scoef_.p, a.data(), sizeof(double) * G, hipMemcpyHostToDevice, s), "H2D");
    hipLaunchKernelGGL(k_scale_copy_seg<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, scoef_.p, L.segn.p, src,
                       dst);
  };
  hipLaunchKernelGGL(k_fill<T>, dim3(std::min(blocks(n, 256), 1024)), dim3(256), 0, s, x, static_cast<size_t>(n),
                     T(0));
  seg_dots(level, 1, b, ld, b, sdev_.p);
  d2h(G);
  std::vector<double> beta0(G), target(G), resid(G);
  std::vector<char> done(G);
  double b0max = 0.0;
  for (int g = 0; g < G; ++g) {
    beta0[g] = std::sqrt(std::max(shost_[g], 0.0));
    target[g] = rtol * beta0[g];
    resid[g] = beta0[g];
    done[g] = !(beta0[g] > 0.0);
    b0max = std::max(b0max, beta0[g]);
  }
  if (res0) *res0 = b0max;
  if (res_out) *res_out = b0max;
  if (std::all_of(done.begin(), done.end(), [](char d) { return d != 0; })) return 0;
  std::vector<std::vector<double>> H(G, std::vector<double>(static_cast<size_t>(m + 1) * m)), cs(G),
      sn(G), gv(G);
  std::vector<int> jend(G, 0);
  std::vector<double> sc(G), y(static_cast<size_t>(G) * m);
  int it = 0;
  bool first = true;
  OpLevel<T> &o = ops_[level];
  while (it < maxit) {
    // v_0 = r / ||r|| per simulation (r = b on the first cycle)
    const T *r = b;
    std::vector<double> beta(G);
    if (first) {
      beta = beta0;
    } else {
      spmv(level, x, b, o.t.p);
      seg_dots(level, 1, o.t.p, ld, o.t.p, sdev_.p);
      d2h(G);
      for (int g = 0; g < G; ++g) beta[g] = std::sqrt(std::max(shost_[g], 0.0));
      r = o.t.p;
    }
    first = false;
    for (int g = 0; g < G; ++g) {
      sc[g] = (!done[g] && beta[g] > 0.0) ? 1.0 / beta[g] : 0.0;
      if (!(beta[g] > 0.0)) done[g] = 1;
      cs[g].assign(m, 0.0);
      sn[g].assign(m, 0.0);
      gv[g].assign(m + 1, 0.0);
      gv[g][0] = beta[g];
      std::fill(H[g].begin(), H[g].end(), 0.0);
      jend[g] = 0;
    }
    scale_to(sc, r, V_.p);
    std::vector<char> active(done);   // frozen at the start of this cycle
    int jmax = 0;
    for (int j = 0; j < m; ++j) {
      T *vj = V_.p + static_cast<size_t>(j) * ld;
      T *zj = Z_.p + static_cast<size_t>(j) * ld;
      vcycle(level, vj, zj);
      spmv(level, zj, nullptr, w_.p);
      const int k = j + 1;
      double *h1 = sdev_.p, *h2 = sdev_.p + static_cast<size_t>(G) * k, *hn = sdev_.p + 2 * static_cast<size_t>(G) * k;
      seg_dots(level, k, V_.p, ld, w_.p, h1);
      hipLaunchKernelGGL(k_multi_axpy_seg<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, k, V_.p, ld, h1, k,
                         L.segn.p, w_.p);
      seg_dots(level, k, V_.p, ld, w_.p, h2);
      hipLaunchKernelGGL(k_multi_axpy_seg<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, k, V_.p, ld, h2, k,
                         L.segn.p, w_.p);
      seg_dots(level, 1, w_.p, ld, w_.p, hn);
      LAUNCH_CHECK("batched gmres iteration");
      d2h(2 * static_cast<size_t>(G) * k + G);
      ++it;
      jmax = k;
      for (int g = 0; g < G; ++g) {
        sc[g] = 0.0;
        if (done[g]) continue;
        std::vector<double> &Hg = H[g];
        const double hnorm = std::sqrt(std::max(shost_[2 * static_cast<size_t>(G) * k + g], 0.0));
        for (int i = 0; i <= j; ++i)
          Hg[i * m + j] = shost_[static_cast<size_t>(g) * k + i] + shost_[static_cast<size_t>(G) * k + g * k + i];
        Hg[(j + 1) * m + j] = hnorm;
        for (int i = 0; i < j; ++i) {
          const double t = cs[g][i] * Hg[i * m + j] + sn[g][i] * Hg[(i + 1) * m + j];
          Hg[(i + 1) * m + j] = -sn[g][i] * Hg[i * m + j] + cs[g][i] * Hg[(i + 1) * m + j];
          Hg[i * m + j] = t;
        }
        const double den = std::hypot(Hg[j * m + j], Hg[(j + 1) * m + j]);
        jend[g] = k;
        if (!(den > 0.0)) {   // breakdown: the current iterate is this simulation's best
          jend[g] = j;
          done[g] = 1;
          continue;
        }
        cs[g][j] = Hg[j * m + j] / den;
        sn[g][j] = Hg[(j + 1) * m + j] / den;
        Hg[j * m + j] = den;
        Hg[(j + 1) * m + j] = 0.0;
        gv[g][j + 1] = -sn[g][j] * gv[g][j];
        gv[g][j] = cs[g][j] * gv[g][j];
        resid[g] = std::fabs(gv[g][j + 1]);
        if (resid[g] <= target[g] || !(hnorm > 0.0))
          done[g] = 1;
        else
          sc[g] = 1.0 / hnorm;
      }
      if (std::all_of(done.begin(), done.end(), [](char d) { return d != 0; }) || it >= maxit) break;
      if (j + 1 < m) scale_to(sc, w_.p, V_.p + static_cast<size_t>(j + 1) * ld);
    }
    // per-simulation least squares and x += Z y
    std::fill(y.begin(), y.end(), 0.0);
    for (int g = 0; g < G; ++g) {
      if (active[g]) continue;   // frozen before this cycle: nothing to add
      const std::vector<double> &Hg = H[g];
      double *yg = y.data() + static_cast<size_t>(g) * m;
      for (int i = jend[g] - 1; i >= 0; --i) {
        double acc = gv[g][i];
        for (int k2 = i + 1; k2 < jend[g]; ++k2) acc -= Hg[i * m + k2] * yg[k2];
        yg[i] = acc / Hg[i * m + i];
      }
    }
    check(hipMemcpyAsync(scoef_.p, y.data(), sizeof(double) * G * m, hipMemcpyHostToDevice, s), "H2D");
    hipLaunchKernelGGL(k_combine_seg<T>, dim3(blocks(n, 256)), dim3(256), 0, s, n, jmax, Z_.p, ld, scoef_.p, m,
                       L.segn.p, x);
    LAUNCH_CHECK("batched gmres combine");
    if (std::all_of(done.begin(), done.end(), [](char d) { return d != 0; })) break;
  }
  check(hipStreamSynchronize(s), "gmres end");
  if (res_out) *res_out = *std::max_element(resid.begin(), resid.end());
  return it;
}

template class Solver<float>;
template class Solver<double>;

}  // namespace dnnmg
