// Library context: device copies of the mesh hierarchy, operators, and the
// Newton / GMRES / multigrid drivers (host code that enqueues the kernels of
// kernels.h on the context's stream).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dnnmg.h"
#include "kernels.h"
#include "mesh.h"

namespace dnnmg {

struct DnnmgError {
  int code;
  std::string msg;
};

// Thin owner of one hipMalloc'ed array.
template <typename T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    if (hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T)) != hipSuccess)
      throw DnnmgError{DNNMG_ENOMEM, "hipMalloc failed"};
    n = count;
  }
  // Setup-time copy from a host vector, complete on return: callers pass
  // locals and temporaries, which must not be read by a copy still queued
  // after they are freed.
  void upload(const std::vector<T> &h, hipStream_t s) {
    alloc(h.size());
    if (h.empty()) return;
    if (hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess)
      throw DnnmgError{DNNMG_EDEVICE, "hipMemcpyAsync H2D failed"};
    if (hipStreamSynchronize(s) != hipSuccess) throw DnnmgError{DNNMG_EDEVICE, "upload: stream synchronisation failed"};
  }
};

void check(hipError_t e, const char *what);

// Optional per-kernel timing: HIP events recorded on the launch stream around
// each profiled launch, resolved (synchronising) when queried.  `only` limits
// the timing to the listed "name@Llevel" keys (empty: every key).
struct Profiler {
  bool on = false;
  std::vector<std::string> only;
  bool wants(const std::string &key) const;
  bool wants_level(int level) const;   // some profiled key lives on `level`
  struct Rec {
    std::string key;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<double, long>> acc;   // key -> (total ms, launches)
  hipEvent_t take();
  void resolve();
  void clear();
  ~Profiler();
};

class Ctx;
// RAII: records a start event at construction and a stop event at destruction.
struct ProfScope {
  Profiler *p;
  std::string key;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(Profiler &pr, hipStream_t st, const char *name, int level);
  ~ProfScope();
};

struct DevLevel {
  HostLevel h;
  DevBuf<double2> xy;
  DevBuf<int4> cells;
  DevBuf<uint8_t> flag, cslot, pslot, vslot;
  DevBuf<int> cadj_ptr, cadj, padj_ptr, padj, patch_nodes, wq, wx, oq, ox, colq, colx;
  DevBuf<int> colour_cells;            // cells grouped by colour (h.colour_ptr)
  DevBuf<int> node_order;              // nodes sorted by their lowest adjacent cell (N, or empty)
  // the node order for node-gather kernels on levels of at least 2^18 nodes
  // (where it pays), else null: natural order
  const int *large_order() const {
    return h.N >= (1 << 18) && node_order.n == static_cast<size_t>(h.N) ? node_order.p : nullptr;
  }
  DevBuf<int> edge_ends, rptr, ridx;   // transfer from the coarser level
  // LPS patch matrices (81 per patch) in two roles: [0] the level's own
  // discrete problem (alpha0 h_T^2 / nu), [1] the level as a coarse level of a
  // finer level's multigrid preconditioner (alpha0 / (nu / h_T^2 + 1/k))
  struct LpsCache {
    DevBuf<double> m;
    double dt = -1.0, nu = -1.0, alpha0 = -1.0;
  } lps[2];
  DevBuf<double> nnu;                  // per-node viscosity (batches only; else empty)
  // obstacle boundary edges (cell, side) grouped by obstacle (ptr CSR), built
  // on the first functional evaluation of the level
  int n_obst = -1;
  DevBuf<int> obst_edges, obst_ptr;
  DevBuf<double> obst_vals;
  // batches: simulation of each node and the chunks of per-simulation
  // reductions (starts/lengths in unknowns, grouped by simulation: seg_ptr)
  int nseg = 1, nchunk = 0;
  DevBuf<int> segn, cstart, clen, seg_ptr;
  LevelView view() const;
};

// Operator storage and work vectors of one level in precision T.
template <typename T>
struct OpLevel {
  DevBuf<T> JQ, JX, inv, delta, r, b, x, t;
  // workgroup sizes of the level's streaming kernels (autotuned at setup);
  // restrict / prolong are the transfers between this level and the next
  // coarser one
  int bs_spmv = 256, bs_apply = 256, bs_update = 256, bs_restrict = 256, bs_prolong = 256;
  int bs_spmv4 = 0;    // > 0: four threads per row (k_spmv4) at this size
  int bs_smooth = 0;   // > 0: residual + Vanka apply fused at this size
  int smooth_lanes = 4;   // lanes per cell of the fused kernel: 4 (k_vanka_smooth) or 16 (k_vanka_smooth16)
  int bs_rres = 0;     // > 0: residual + restriction fused (k_restrict_residual)
  int bs_apply4 = 0;   // > 0: FP32 Vanka apply with four cells per thread (k_vanka_apply4)
  int bs_update_ord = 0;   // > 0: Vanka update over the nodes in cell order (k_vanka_update_ordered)
  int bs_upro = 0;     // > 0: the next coarser level's last update fused into
                       // the prolongation to this level (k_update_prolong_add)
};

class Ctx;

// Newton-GMRES-multigrid solver in working precision T (float: mixed mode).
template <typename T>
class Solver {
 public:
  explicit Solver(Ctx *c) : ctx_(c) {}
  void setup(int finest);
  // J on `level` (and, if full, on all coarser levels with the Vanka inverses
  // and the level-0 inverse: the multigrid preconditioner); xo_dev: the
  // frozen field of the convective stabilisation (delta0 > 0)
  void linearize(const double *x_dev, const double *xo_dev, int level, double dt, bool full = true);
  // Jacobian reuse: after linearize(.., full = true) from state `key` the
  // hierarchy is marked as kept for (key, level, dt); any other linearize
  // or forget_jacobian() drops the mark
  void keep_jacobian(unsigned long long key, int level, double dt) {
    kept_key_ = key;
    kept_level_ = level;
    kept_dt_ = dt;
  }
  bool jacobian_kept(unsigned long long key, int level, double dt) const {
    return key != 0 && kept_key_ == key && kept_level_ == level && kept_dt_ == dt;
  }
  void forget_jacobian() { kept_key_ = 0; }
  // defer_update: leave the node update of the sweep to the caller (the
  // corrections are in op(l).delta)
  void vanka_sweep(int l, T *x, const T *b, bool zero_start, bool defer_update = false);
  // x = V(b), zero start.  With defer, the last post-sweep's node update may
  // be left to the caller (returns true if it was).
  bool vcycle(int l, const T *b, T *x, bool defer = false);
  int gmres(int level, const T *b, T *x, double rtol, int restart, int maxit, double *res0,
            double *res);
  void spmv(int l, const T *x, const T *b, T *y);               // y = b - J x or J x
  void prolong_add(int l, const T *ec, T *xf);
  void restrict_to(int l, const T *rf, T *rc);
  OpLevel<T> &op(int l) { return ops_[l]; }
  const OpLevel<T> &op(int l) const { return ops_[l]; }
  ~Solver();
  // Times each streaming kernel of every level at workgroup sizes 64, 128
  // and 256 and keeps the fastest (the choice changes scheduling only: every
  // thread does the same arithmetic, results are bitwise the same).
  void autotune();
  // Fused residual + Vanka apply (sixteen lanes per cell) and four threads
  // per SpMV row on every level, workgroup size 256 (a fixed configuration,
  // e.g. for reproducible comparisons).
  void fuse_all();

  // Levels 1..top of every V-cycle (and the level-0 solve) in one workgroup
  // launch; 0 = off.  Needs the blocked level-0 inverse.
  void set_small_top(int top) { small_top_ = gj_b_ > 0 && c_ == 0 ? std::min(top, kSmallLevels - 1) : 0; }
  int small_top() const { return small_top_; }

 private:
  Ctx *ctx_;
  int lin_level_ = -1;
  unsigned long long kept_key_ = 0;
  int kept_level_ = -1;
  double kept_dt_ = 0.0;
  int small_top_ = 0;
  SmallCycle<T> small_params(int top, const T *b, T *x);
  void launch_small(int top, const T *b, T *x);
  // Launch-bound sequences (a V-cycle from a given level, the level-0
  // Gauss-Jordan sweep) are captured once into HIP graphs and replayed; a
  // slot is rebuilt when the context's graph generation changes.
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    long gen = -1;
  };
  // key: level, whether the level is the top of its cycle, b, x
  std::map<std::tuple<int, int, const void *, const void *>, GraphSlot> vgraphs_;
  int cycle_top_ = -1;   // level of the outermost vcycle call in progress
  int cycle_depth_ = 0;
  bool inner_level(int l) const { return ctx_coarse_sweeps() > 0 && l != cycle_top_; }
  int ctx_coarse_sweeps() const;
  GraphSlot ginv_;
  bool capturing_ = false;
  template <class F>
  void graph_run(GraphSlot &g, F &&body);
  bool use_graph(int level) const;
  void clear_graphs();
  bool vcycle_body(int l, const T *b, T *x, bool defer);
  bool will_defer(int l) const;
  void coarse_inverse();
  std::vector<OpLevel<T>> ops_;
  DevBuf<T> cblk_;   // 12x12 cell blocks written by the assembly for the Vanka factorisation
  DevBuf<double> W_, prow_, colk_;
  int c_ = 0;    // level of the coarse direct solve
  int n0_ = 0;
  // blocked Gauss-Jordan: panel width (0: one pivot + one elimination launch
  // per column), second workspace, panel transforms, pivot rows, used-row
  // flags, and the compact inverse read by the coarse solve
  int gj_b_ = 0, gj_rpt_ = 1;      // rows per panel thread: 1 (<= 1024 unknowns) or 2
  int nblk_ = 1, nb_ = 0;          // level-0 blocks and their padded size (unknowns)
  DevBuf<double> W2_, Zp_, Ainv_;
  DevBuf<int> piv_, used_, g2l_, blk_, bdof_;
  // GMRES workspace
  int gm_level_ = -1, gm_m_ = 0;
  DevBuf<T> V_, Z_, w_;
  DevBuf<double> partial_, hdev_;
  std::vector<double> hhost_;
  // pipelined Hessenberg read-back: one device slot, pinned host slot and
  // event per Arnoldi step
  DevBuf<double> hcol_;
  double *hpin_ = nullptr;
  std::vector<hipEvent_t> hev_;
  int hslots_ = 0;
  void free_pipeline();
  void ensure_gmres(int level, int m);
  // GMRES with per-simulation inner products, Hessenberg matrices and Givens
  // rotations on a batch level (each simulation's own Krylov space).
  int gmres_batched(int level, const T *b, T *x, double rtol, int restart, int maxit, double *res0,
                    double *res);
  DevBuf<double> spart_, sdev_, scoef_;
  std::vector<double> shost_;
  // segmented dots of V[0..m) with w on `level` into dev (segment-major, m per segment)
  void seg_dots(int level, int m, const T *V, size_t ld, const T *w, double *dev);
};

class Ctx {
 public:
  dnnmg_ctx *owner = nullptr;   // the C handle wrapping this context
  dnnmg_params prm{};
  hipStream_t stream = nullptr;
  std::string last_error;
  Profiler prof;
  long graph_gen = 0;              // bumped when captured graphs go stale
  unsigned long long state_keys = 0;   // last key handed to a state (Jacobian reuse)
  // simulation batches (empty otherwise): macro cell -> simulation, its
  // viscosity, and level-0 node -> simulation (the coarse solve's blocks)
  std::vector<int> macro_blk;
  std::vector<double> blk_nu;
  std::vector<int> blk0;
  hipStream_t cap_stream = nullptr;
  hipStream_t capture_stream();    // private stream used only for graph capture
  ~Ctx();
  std::vector<std::unique_ptr<DevLevel>> levels;
  int finest = -1;
  std::unique_ptr<Solver<float>> s32;
  std::unique_ptr<Solver<double>> s64;
  void forget_jacobians() {
    if (s32) s32->forget_jacobian();
    if (s64) s64->forget_jacobian();
  }
  // FP64 scratch for residual evaluation / Newton on the finest used level
  DevBuf<double> R, xo_save, tmp64a, tmp64b;
  DevBuf<double> cellvec;   // element vectors of the residual / Rhs (12 per cell), then
                            // the LPS vectors of the patches (9 per patch)
  // cellvec sized for level l (allocated on first use)
  double *cell_vectors(int l) {
    const size_t need = 12 * static_cast<size_t>(levels[l]->h.C) + 9 * static_cast<size_t>(levels[l]->h.NP);
    if (cellvec.n < need) cellvec.alloc(need);
    return cellvec.p;
  }
  DevBuf<double> red_partial, red_out;

  Phys phys(double dt, double t) const {
    Phys p;
    p.nu = prm.nu;
    p.theta = prm.theta;
    p.inv_dt = dt > 0 ? 1.0 / dt : 0.0;
    p.alpha0 = prm.alpha0;
    p.u_mean = prm.u_mean;
    p.H = prm.channel_h;
    p.t = t;
    p.delta0 = prm.delta0;
    return p;
  }
  // LPS patch matrices of level l in the given role (0: the level's own
  // problem, 1: coarse operator of a finer level's preconditioner), built on
  // first use and when nu, alpha0 or (role 1) the time step change
  const double *ensure_lps(int l, double dt, int role);
  double norm2_f64(const double *x, int n);   // ||x||_2, synchronising
  // largest per-simulation ||x||_2 on a batch level (= ||x||_2 otherwise)
  double norm2_max_seg(int l, const double *x);
  DevBuf<double> seg_partial, seg_out;
  std::vector<double> seg_host;
  int n_curve = 0;                 // obstacles of the mesh
  // J_div, drag[k], lift[k] of x on level l (synchronising)
  void functionals(int l, const double *x, double *jdiv, double *drag, double *lift);
  void residual(int l, const double *x, const double *xo, const double *rhs, double t_new,
                double dt, double *R);
  // Velocity error of x on level l (prolongated to ref_level if coarser)
  // against ref on ref_level: out = {int |v - v_ref|^2, int |v_ref|^2,
  // sum_i |v_i - v_ref,i|^2, sum_i |v_ref,i|^2} (synchronising)
  void velocity_error(int l, const double *x, int ref_level, const double *ref, double out[4]);
  DevBuf<double> verr_a, verr_b;   // prolongation chain of velocity_error
};

struct State {
  Ctx *ctx;
  int level;
  double t = 0.0;
  DevBuf<double> x;
  DevBuf<double> pending_rhs;   // DNN-MG right-hand side for the next step
  bool has_pending = false;
  DevBuf<double> xprev;         // state before the last step (Newton predictor)
  bool has_prev = false;
  double dt_prev = 0.0;
  unsigned long long key = 0;   // identifies the values a kept Jacobian was built from
  bool reuse_ok = false;        // the last Newton iteration contracted well enough to keep J
};

inline int blocks(size_t n, int bs) { return static_cast<int>((n + bs - 1) / bs); }

}  // namespace dnnmg

struct dnnmg_ctx {
  dnnmg::Ctx impl;
};
struct dnnmg_state {
  dnnmg::State impl;
};
