// Batches of independent simulations of uneven mesh depth.
//
// Simulations of equal depth form a group whose meshes are merged into one
// disjoint union: every kernel launch of the group (residual, assembly, Vanka
// sweeps, transfers, GMRES vectors) covers all of its simulations at once,
// the viscosity is read per node, and the level-0 direct solve is block
// diagonal (one dense inverse per simulation, all factorised by the same
// launches).  Groups are independent contexts with their own streams, stepped
// concurrently from one host thread each, so that the latency-bound coarse
// work of shallow groups overlaps the bandwidth-bound fine levels of deep ones.
//
// Newton and GMRES run on each group's union: their norms and inner products
// span the group's simulations, so a group converges when the residual of the
// union meets the tolerance (each member's residual then does too).
#include <algorithm>
#include <cstring>
#include <exception>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "context.h"

namespace dnnmg {
namespace {

struct Group {
  int depth = 0;
  std::vector<int> sims;                  // members, in union order
  std::vector<std::vector<int>> nodes;    // per member: union node of each own node
  dnnmg_ctx *ctx = nullptr;
  dnnmg_state *state = nullptr;
  hipStream_t stream = nullptr;
  int n_nodes = 0;
};

}  // namespace
}  // namespace dnnmg

struct dnnmg_batch {
  std::vector<dnnmg::Group> groups;
  std::vector<std::pair<int, int>> where;   // sim -> (group, member index)
  std::string last_error;
};

namespace {

using dnnmg::Group;

void release(dnnmg_batch *b) {
  for (Group &g : b->groups) {
    if (g.state) dnnmg_state_destroy(g.state);
    if (g.ctx) dnnmg_destroy(g.ctx);
    if (g.stream) (void)hipStreamDestroy(g.stream);
    g.state = nullptr;
    g.ctx = nullptr;
    g.stream = nullptr;
  }
}

int bfail(dnnmg_batch *b, int code, const std::string &msg) {
  if (b) b->last_error = msg;
  return code;
}

bool mesh_ok(const dnnmg_coarse_mesh *m) {
  return m && m->n_vert >= 4 && m->n_cell >= 1 && m->xy && m->quad && m->n_bedge >= 0 &&
         (m->n_bedge == 0 || m->bedge) && m->n_curve >= 0 && (m->n_curve == 0 || m->curve);
}

// Builds group g: the union of its members' macro meshes (vertices and cells
// concatenated in member order, obstacle tags renumbered onto the
// concatenated curve list), its context, state and node maps.
int build_group(dnnmg_batch *b, Group &g, const dnnmg_params *p, const dnnmg_sim_desc *sims) {
  std::vector<double> xy, cv;
  std::vector<int> q, be, cell_blk;
  std::vector<double> nu;
  for (size_t k = 0; k < g.sims.size(); ++k) {
    const dnnmg_sim_desc &d = sims[g.sims[k]];
    const dnnmg_coarse_mesh *m = d.mesh;
    const int voff = static_cast<int>(xy.size() / 2), coff = static_cast<int>(cv.size() / 5);
    xy.insert(xy.end(), m->xy, m->xy + 2 * m->n_vert);
    for (int i = 0; i < 4 * m->n_cell; ++i) {
      if (m->quad[i] < 0 || m->quad[i] >= m->n_vert)
        return bfail(b, DNNMG_EINVAL, "quad vertex out of range in simulation " + std::to_string(g.sims[k]));
      q.push_back(m->quad[i] + voff);
    }
    for (int e = 0; e < m->n_bedge; ++e) {
      const int *t = m->bedge + 3 * e;
      if (t[0] < 0 || t[0] >= m->n_vert || t[1] < 0 || t[1] >= m->n_vert || t[2] < 1 ||
          (t[2] >= 4 && t[2] - 4 >= m->n_curve))
        return bfail(b, DNNMG_EINVAL, "boundary edge out of range in simulation " + std::to_string(g.sims[k]));
      be.push_back(t[0] + voff);
      be.push_back(t[1] + voff);
      be.push_back(t[2] >= 4 ? t[2] + coff : t[2]);
    }
    cv.insert(cv.end(), m->curve, m->curve + 5 * m->n_curve);
    cell_blk.insert(cell_blk.end(), m->n_cell, static_cast<int>(k));
    nu.push_back(d.nu);
  }
  if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess)
    return bfail(b, DNNMG_EDEVICE, "hipStreamCreate failed");
  dnnmg_params gp = *p;
  gp.stream = g.stream;
  int rc = dnnmg_create(&gp, &g.ctx);
  if (rc) return bfail(b, rc, "dnnmg_create failed for a group");
  g.ctx->impl.macro_blk = cell_blk;
  g.ctx->impl.blk_nu = nu;
  dnnmg_coarse_mesh um;
  um.n_vert = static_cast<int>(xy.size() / 2);
  um.xy = xy.data();
  um.n_cell = static_cast<int>(q.size() / 4);
  um.quad = q.data();
  um.n_bedge = static_cast<int>(be.size() / 3);
  um.bedge = be.empty() ? nullptr : be.data();
  um.n_curve = static_cast<int>(cv.size() / 5);
  um.curve = cv.empty() ? nullptr : cv.data();
  rc = dnnmg_setup_mesh(g.ctx, &um, g.depth);
  if (rc) return bfail(b, rc, std::string("group setup: ") + dnnmg_last_error(g.ctx));
  rc = dnnmg_state_create(g.ctx, g.depth, &g.state);
  if (rc) return bfail(b, rc, std::string("group state: ") + dnnmg_last_error(g.ctx));
  // members' nodes: a member's own numbering is its union nodes in increasing
  // order (refinement numbers old vertices, then edge midpoints, then cell
  // centres, each in cell order, and the members' cells are contiguous)
  const dnnmg::HostLevel &h = g.ctx->impl.levels[g.depth]->h;
  g.n_nodes = h.N;
  g.nodes.assign(g.sims.size(), {});
  for (int i = 0; i < h.N; ++i) {
    const int cell = h.cadj[h.cadj_ptr[i]] >> 2;
    g.nodes[cell_blk[cell >> (2 * g.depth + 2)]].push_back(i);
  }
  return DNNMG_OK;
}

}  // namespace

extern "C" {

int dnnmg_batch_create(const dnnmg_params *p, const dnnmg_sim_desc *sims, int n_sims, dnnmg_batch **out) {
  if (!p || !sims || n_sims < 1 || !out || p->coarse_level != 0) return DNNMG_EINVAL;
  for (int s = 0; s < n_sims; ++s)
    if (!mesh_ok(sims[s].mesh) || !(sims[s].nu > 0) || sims[s].depth < 0 || sims[s].depth > 9)
      return DNNMG_EINVAL;
  dnnmg_batch *b = new (std::nothrow) dnnmg_batch();
  if (!b) return DNNMG_ENOMEM;
  std::map<int, std::vector<int>> by_depth;
  for (int s = 0; s < n_sims; ++s) by_depth[sims[s].depth].push_back(s);
  b->where.assign(n_sims, {-1, -1});
  for (auto &kv : by_depth) {
    Group g;
    g.depth = kv.first;
    g.sims = kv.second;
    for (size_t k = 0; k < g.sims.size(); ++k)
      b->where[g.sims[k]] = {static_cast<int>(b->groups.size()), static_cast<int>(k)};
    b->groups.push_back(std::move(g));
  }
  for (Group &g : b->groups) {
    const int rc = build_group(b, g, p, sims);
    if (rc) {
      release(b);
      delete b;
      return rc;
    }
  }
  *out = b;
  return DNNMG_OK;
}

int dnnmg_batch_destroy(dnnmg_batch *b) {
  if (!b) return DNNMG_EINVAL;
  release(b);
  delete b;
  return DNNMG_OK;
}

const char *dnnmg_batch_last_error(const dnnmg_batch *b) { return b ? b->last_error.c_str() : ""; }

int dnnmg_batch_groups(const dnnmg_batch *b, int *n_groups) {
  if (!b || !n_groups) return DNNMG_EINVAL;
  *n_groups = static_cast<int>(b->groups.size());
  return DNNMG_OK;
}

int dnnmg_batch_group_info(const dnnmg_batch *b, int g, int *depth, int *n_sims, int *n_nodes) {
  if (!b || g < 0 || g >= static_cast<int>(b->groups.size())) return DNNMG_EINVAL;
  const Group &G = b->groups[g];
  if (depth) *depth = G.depth;
  if (n_sims) *n_sims = static_cast<int>(G.sims.size());
  if (n_nodes) *n_nodes = G.n_nodes;
  return DNNMG_OK;
}

int dnnmg_batch_info(const dnnmg_batch *b, int sim, int *group, int *n_nodes) {
  if (!b || sim < 0 || sim >= static_cast<int>(b->where.size())) return DNNMG_EINVAL;
  const auto w = b->where[sim];
  if (group) *group = w.first;
  if (n_nodes) *n_nodes = static_cast<int>(b->groups[w.first].nodes[w.second].size());
  return DNNMG_OK;
}

int dnnmg_batch_set(dnnmg_batch *b, int sim, const double *uvp, double t) {
  if (!b || !uvp || sim < 0 || sim >= static_cast<int>(b->where.size())) return DNNMG_EINVAL;
  const auto w = b->where[sim];
  Group &G = b->groups[w.first];
  std::vector<double> all(3 * static_cast<size_t>(G.n_nodes));
  double t_old = 0.0;
  int rc = dnnmg_state_get(G.state, all.data(), &t_old);
  if (rc) return bfail(b, rc, dnnmg_last_error(G.ctx));
  const std::vector<int> &nd = G.nodes[w.second];
  for (size_t k = 0; k < nd.size(); ++k)
    for (int f = 0; f < 3; ++f) all[3 * static_cast<size_t>(nd[k]) + f] = uvp[3 * k + f];
  rc = dnnmg_state_set(G.state, all.data(), t);
  if (rc) return bfail(b, rc, dnnmg_last_error(G.ctx));
  return DNNMG_OK;
}

int dnnmg_batch_get(const dnnmg_batch *b, int sim, double *uvp, double *t) {
  if (!b || !uvp || sim < 0 || sim >= static_cast<int>(b->where.size())) return DNNMG_EINVAL;
  const auto w = b->where[sim];
  const Group &G = b->groups[w.first];
  std::vector<double> all(3 * static_cast<size_t>(G.n_nodes));
  const int rc = dnnmg_state_get(G.state, all.data(), t);
  if (rc) return rc;
  const std::vector<int> &nd = G.nodes[w.second];
  for (size_t k = 0; k < nd.size(); ++k)
    for (int f = 0; f < 3; ++f) uvp[3 * k + f] = all[3 * static_cast<size_t>(nd[k]) + f];
  return DNNMG_OK;
}

int dnnmg_batch_step(dnnmg_batch *b, double dt, dnnmg_step_stats *stats) {
  if (!b || !(dt > 0)) return DNNMG_EINVAL;
  const size_t ng = b->groups.size();
  std::vector<int> rcs(ng, DNNMG_OK);
  std::vector<dnnmg_step_stats> st(ng);
  std::vector<std::thread> th;
  try {
    for (size_t g = 1; g < ng; ++g)
      th.emplace_back([&, g]() { rcs[g] = dnnmg_step(b->groups[g].ctx, b->groups[g].state, dt, &st[g]); });
  } catch (const std::exception &) {
    for (auto &t : th) t.join();
    return bfail(b, DNNMG_ENOMEM, "could not start group threads");
  }
  rcs[0] = dnnmg_step(b->groups[0].ctx, b->groups[0].state, dt, &st[0]);
  for (auto &t : th) t.join();
  if (stats) std::memcpy(stats, st.data(), ng * sizeof(dnnmg_step_stats));
  for (size_t g = 0; g < ng; ++g)
    if (rcs[g]) return bfail(b, rcs[g], "group " + std::to_string(g) + ": " + dnnmg_last_error(b->groups[g].ctx));
  return DNNMG_OK;
}

}  // extern "C"
