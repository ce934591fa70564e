// Host-side refinement and table construction (see mesh.h).
#include "mesh.h"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace dnnmg {

namespace {

inline uint64_t edge_key(int a, int b) {
  const uint32_t lo = static_cast<uint32_t>(std::min(a, b));
  const uint32_t hi = static_cast<uint32_t>(std::max(a, b));
  return (static_cast<uint64_t>(lo) << 32) | hi;
}

// Radial projection onto the ellipse (cx, cy, a, b, phi) in its scaled frame.
void project(const double *cv, double *p) {
  const double c = std::cos(cv[4]), s = std::sin(cv[4]);
  const double dx = p[0] - cv[0], dy = p[1] - cv[1];
  double qx = c * dx + s * dy, qy = -s * dx + c * dy;
  const double r = std::sqrt((qx / cv[2]) * (qx / cv[2]) + (qy / cv[3]) * (qy / cv[3]));
  qx /= r;
  qy /= r;
  p[0] = cv[0] + c * qx - s * qy;
  p[1] = cv[1] + s * qx + c * qy;
}

// Position of each child's local vertex in the 3x3 patch (lexicographic).
constexpr int kChildToPatch[4][4] = {{0, 1, 4, 3}, {1, 2, 5, 4}, {4, 5, 8, 7}, {3, 4, 7, 6}};

}  // namespace

HostLevel refine(const std::vector<double> &xy, const std::vector<int> &cells,
                 const std::vector<int> &bedges, const std::vector<double> &curves,
                 std::string *err) {
  HostLevel F;
  const int V = static_cast<int>(xy.size() / 2);
  const int C = static_cast<int>(cells.size() / 4);
  const int E_b = static_cast<int>(bedges.size() / 3);
  const int K = static_cast<int>(curves.size() / 5);
  std::unordered_map<uint64_t, int> eid;
  eid.reserve(static_cast<size_t>(2 * C + 16));
  std::vector<int> ends;
  ends.reserve(static_cast<size_t>(4 * C + 8));
  std::vector<int> mid(static_cast<size_t>(4) * C);
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < 4; ++k) {
      const int a = cells[4 * c + k], b = cells[4 * c + (k + 1) % 4];
      const uint64_t key = edge_key(a, b);
      auto it = eid.find(key);
      int id;
      if (it == eid.end()) {
        id = static_cast<int>(ends.size() / 2);
        eid.emplace(key, id);
        ends.push_back(a);
        ends.push_back(b);
      } else {
        id = it->second;
      }
      mid[4 * c + k] = V + id;
    }
  const int E = static_cast<int>(ends.size() / 2);
  F.N = V + E + C;
  F.C = 4 * C;
  F.NP = C;
  F.Nc = V;
  F.Ec = E;
  F.edge_ends = ends;
  F.coarse_cells = cells;
  F.xy.assign(static_cast<size_t>(2) * F.N, 0.0);
  std::copy(xy.begin(), xy.end(), F.xy.begin());
  for (int e = 0; e < E; ++e)
    for (int d = 0; d < 2; ++d)
      F.xy[2 * (V + e) + d] = 0.5 * (xy[2 * ends[2 * e] + d] + xy[2 * ends[2 * e + 1] + d]);
  F.Eb = 2 * E_b;
  F.bedges.reserve(static_cast<size_t>(6) * E_b);
  for (int e = 0; e < E_b; ++e) {
    const int v0 = bedges[3 * e], v1 = bedges[3 * e + 1], tag = bedges[3 * e + 2];
    auto it = eid.find(edge_key(v0, v1));
    if (it == eid.end()) {
      if (err) *err = "boundary edge is not an edge of any cell";
      return HostLevel();
    }
    const int m = V + it->second;
    if (tag >= 4) {
      if (tag - 4 >= K) {
        if (err) *err = "boundary tag refers to a missing curve";
        return HostLevel();
      }
      project(&curves[5 * (tag - 4)], &F.xy[2 * m]);
    }
    const int fb[6] = {v0, m, tag, m, v1, tag};
    F.bedges.insert(F.bedges.end(), fb, fb + 6);
  }
  F.cells.resize(static_cast<size_t>(4) * F.C);
  for (int c = 0; c < C; ++c) {
    const int ctr = V + E + c;
    for (int d = 0; d < 2; ++d) {
      double s = 0.0, t = 0.0;
      for (int k = 0; k < 4; ++k) {
        s += F.xy[2 * mid[4 * c + k] + d];
        t += xy[2 * cells[4 * c + k] + d];
      }
      F.xy[2 * ctr + d] = 0.5 * s - 0.25 * t;   // Coons point
    }
    const int n0 = cells[4 * c], n1 = cells[4 * c + 1], n2 = cells[4 * c + 2], n3 = cells[4 * c + 3];
    const int m01 = mid[4 * c], m12 = mid[4 * c + 1], m23 = mid[4 * c + 2], m30 = mid[4 * c + 3];
    const int ch[4][4] = {{n0, m01, ctr, m30}, {m01, n1, m12, ctr}, {ctr, m12, n2, m23},
                          {m30, ctr, m23, n3}};
    for (int k = 0; k < 4; ++k)
      for (int a = 0; a < 4; ++a) F.cells[16 * c + 4 * k + a] = ch[k][a];
  }
  F.flag.assign(static_cast<size_t>(F.N), 0);
  for (int e = 0; e < F.Eb; ++e) {
    const int tag = F.bedges[3 * e + 2];
    for (int k = 0; k < 2; ++k) {
      const int v = F.bedges[3 * e + k];
      if (tag != 3) F.flag[v] |= kFlagDirichlet;
      if (tag == 1) F.flag[v] |= kFlagInflow;
    }
  }
  return F;
}

bool build_tables(HostLevel &L, std::string *err) {
  const int N = L.N, C = L.C;
  // node -> (cell, local) adjacency, in increasing cell order
  L.cadj_ptr.assign(static_cast<size_t>(N) + 1, 0);
  for (int c = 0; c < C; ++c)
    for (int a = 0; a < 4; ++a) L.cadj_ptr[L.cells[4 * c + a] + 1]++;
  for (int i = 0; i < N; ++i) L.cadj_ptr[i + 1] += L.cadj_ptr[i];
  L.cadj.assign(static_cast<size_t>(L.cadj_ptr[N]), 0);
  {
    std::vector<int> fill(L.cadj_ptr.begin(), L.cadj_ptr.end() - 1);
    for (int c = 0; c < C; ++c)
      for (int a = 0; a < 4; ++a) L.cadj[fill[L.cells[4 * c + a]]++] = 4 * c + a;
  }
  // patches: children 4P..4P+3 of coarse cell P
  L.NP = C / 4;
  L.patch_nodes.assign(static_cast<size_t>(9) * L.NP, -1);
  for (int P = 0; P < L.NP; ++P)
    for (int k = 0; k < 4; ++k)
      for (int a = 0; a < 4; ++a)
        L.patch_nodes[9 * P + kChildToPatch[k][a]] = L.cells[4 * (4 * P + k) + a];
  L.padj_ptr.assign(static_cast<size_t>(N) + 1, 0);
  for (int P = 0; P < L.NP; ++P)
    for (int q = 0; q < 9; ++q) L.padj_ptr[L.patch_nodes[9 * P + q] + 1]++;
  for (int i = 0; i < N; ++i) L.padj_ptr[i + 1] += L.padj_ptr[i];
  L.padj.assign(static_cast<size_t>(L.padj_ptr[N]), 0);
  {
    std::vector<int> fill(L.padj_ptr.begin(), L.padj_ptr.end() - 1);
    for (int P = 0; P < L.NP; ++P)
      for (int q = 0; q < 9; ++q) L.padj[fill[L.patch_nodes[9 * P + q]]++] = 9 * P + q;
  }
  // neighbour lists: Q1 (nodes sharing a cell), extra (sharing a patch only)
  std::vector<std::vector<int>> nq(static_cast<size_t>(N)), nx(static_cast<size_t>(N));
  for (int i = 0; i < N; ++i) {
    auto &q = nq[i];
    for (int e = L.cadj_ptr[i]; e < L.cadj_ptr[i + 1]; ++e) {
      const int c = L.cadj[e] >> 2;
      for (int b = 0; b < 4; ++b) q.push_back(L.cells[4 * c + b]);
    }
    std::sort(q.begin(), q.end());
    q.erase(std::unique(q.begin(), q.end()), q.end());
    auto &x = nx[i];
    for (int e = L.padj_ptr[i]; e < L.padj_ptr[i + 1]; ++e) {
      const int P = L.padj[e] / 9;
      for (int m = 0; m < 9; ++m) {
        const int j = L.patch_nodes[9 * P + m];
        if (!std::binary_search(q.begin(), q.end(), j)) x.push_back(j);
      }
    }
    std::sort(x.begin(), x.end());
    x.erase(std::unique(x.begin(), x.end()), x.end());
    if (q.size() > 120 || x.size() > 120) {
      if (err) *err = "node valence too large for the row layout";
      return false;
    }
    L.nnzq += static_cast<long long>(q.size());
    L.nnzx += static_cast<long long>(x.size());
  }
  L.nslice = (N + kSlice - 1) / kSlice;
  L.wq.assign(L.nslice, 0);
  L.wx.assign(L.nslice, 0);
  L.oq.assign(L.nslice, 0);
  L.ox.assign(L.nslice, 0);
  L.totq = L.totx = 0;
  L.maxwq = L.maxwx = 0;
  for (int s = 0; s < L.nslice; ++s) {
    int a = 0, b = 0;
    for (int i = s * kSlice; i < std::min(N, (s + 1) * kSlice); ++i) {
      a = std::max(a, static_cast<int>(nq[i].size()));
      b = std::max(b, static_cast<int>(nx[i].size()));
    }
    L.wq[s] = a;
    L.wx[s] = b;
    L.oq[s] = L.totq;
    L.ox[s] = L.totx;
    L.totq += a;
    L.totx += b;
    L.maxwq = std::max(L.maxwq, a);
    L.maxwx = std::max(L.maxwx, b);
  }
  // padding entries point at the row's own node (value stays zero)
  L.colq.assign(static_cast<size_t>(L.totq) * kSlice, 0);
  L.colx.assign(static_cast<size_t>(std::max(L.totx, 1)) * kSlice, 0);
  for (int s = 0; s < L.nslice; ++s)
    for (int lane = 0; lane < kSlice; ++lane) {
      const int i = s * kSlice + lane;
      const int self = i < N ? i : 0;
      for (int k = 0; k < L.wq[s]; ++k)
        L.colq[static_cast<size_t>(L.oq[s] + k) * kSlice + lane] =
            (i < N && k < static_cast<int>(nq[i].size())) ? nq[i][k] : self;
      for (int k = 0; k < L.wx[s]; ++k)
        L.colx[static_cast<size_t>(L.ox[s] + k) * kSlice + lane] =
            (i < N && k < static_cast<int>(nx[i].size())) ? nx[i][k] : self;
    }
  auto qslot = [&](int i, int j) -> int {
    auto it = std::lower_bound(nq[i].begin(), nq[i].end(), j);
    return (it != nq[i].end() && *it == j) ? static_cast<int>(it - nq[i].begin()) : -1;
  };
  auto xslot = [&](int i, int j) -> int {
    auto it = std::lower_bound(nx[i].begin(), nx[i].end(), j);
    return (it != nx[i].end() && *it == j) ? static_cast<int>(it - nx[i].begin()) : -1;
  };
  L.cslot.assign(static_cast<size_t>(4) * L.cadj.size(), 0);
  for (int i = 0; i < N; ++i)
    for (int e = L.cadj_ptr[i]; e < L.cadj_ptr[i + 1]; ++e) {
      const int c = L.cadj[e] >> 2;
      for (int b = 0; b < 4; ++b) L.cslot[4 * e + b] = static_cast<uint8_t>(qslot(i, L.cells[4 * c + b]));
    }
  L.pslot.assign(static_cast<size_t>(9) * L.padj.size(), 0);
  for (int i = 0; i < N; ++i)
    for (int e = L.padj_ptr[i]; e < L.padj_ptr[i + 1]; ++e) {
      const int P = L.padj[e] / 9;
      for (int m = 0; m < 9; ++m) {
        const int j = L.patch_nodes[9 * P + m];
        const int s = qslot(i, j);
        L.pslot[9 * e + m] = s >= 0 ? static_cast<uint8_t>(s)
                                    : static_cast<uint8_t>(kExtraBit | xslot(i, j));
      }
    }
  L.vslot.assign(static_cast<size_t>(16) * C, 0);
  for (int c = 0; c < C; ++c)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        L.vslot[16 * c + 4 * a + b] =
            static_cast<uint8_t>(qslot(L.cells[4 * c + a], L.cells[4 * c + b]));
  // restriction lists to the coarser level (transpose of the prolongation)
  if (L.Nc > 0) {
    const int Nc = L.Nc, Ec = L.Ec, Cc = static_cast<int>(L.coarse_cells.size() / 4);
    L.rptr.assign(static_cast<size_t>(Nc) + 1, 0);
    for (int j = 0; j < Nc; ++j) L.rptr[j + 1]++;
    for (int e = 0; e < Ec; ++e)
      for (int k = 0; k < 2; ++k) L.rptr[L.edge_ends[2 * e + k] + 1]++;
    for (int c = 0; c < Cc; ++c)
      for (int k = 0; k < 4; ++k) L.rptr[L.coarse_cells[4 * c + k] + 1]++;
    for (int j = 0; j < Nc; ++j) L.rptr[j + 1] += L.rptr[j];
    L.ridx.assign(static_cast<size_t>(L.rptr[Nc]), 0);
    std::vector<int> fill(L.rptr.begin(), L.rptr.end() - 1);
    for (int j = 0; j < Nc; ++j) L.ridx[fill[j]++] = j;
    for (int e = 0; e < Ec; ++e)
      for (int k = 0; k < 2; ++k) L.ridx[fill[L.edge_ends[2 * e + k]]++] = Nc + e;
    for (int c = 0; c < Cc; ++c)
      for (int k = 0; k < 4; ++k) L.ridx[fill[L.coarse_cells[4 * c + k]]++] = Nc + Ec + c;
  }
  // greedy colouring in cell order: a cell takes the smallest colour not taken
  // by an earlier cell that shares one of its nodes
  {
    std::vector<int> colour(static_cast<size_t>(C), -1);
    int ncol = 0;
    for (int c = 0; c < C; ++c) {
      uint64_t taken = 0;
      for (int a = 0; a < 4; ++a) {
        const int v = L.cells[4 * c + a];
        for (int e = L.cadj_ptr[v]; e < L.cadj_ptr[v + 1]; ++e) {
          const int o = L.cadj[e] >> 2;
          if (o < c) taken |= uint64_t(1) << colour[o];
        }
      }
      int k = 0;
      while (k < 64 && ((taken >> k) & 1)) ++k;
      if (k == 64) {
        if (err) *err = "cell colouring needs more than 64 colours";
        return false;
      }
      colour[c] = k;
      ncol = std::max(ncol, k + 1);
    }
    L.ncolour = ncol;
    L.colour_ptr.assign(static_cast<size_t>(ncol) + 1, 0);
    for (int c = 0; c < C; ++c) L.colour_ptr[colour[c] + 1]++;
    for (int k = 0; k < ncol; ++k) L.colour_ptr[k + 1] += L.colour_ptr[k];
    L.colour_cells.assign(static_cast<size_t>(C), 0);
    std::vector<int> fill(L.colour_ptr.begin(), L.colour_ptr.end() - 1);
    for (int c = 0; c < C; ++c) L.colour_cells[fill[colour[c]]++] = c;
  }
  return true;
}

}  // namespace dnnmg
