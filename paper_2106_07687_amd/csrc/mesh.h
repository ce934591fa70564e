// Host-side mesh hierarchy and the index tables the gfx950 kernels use.
//
// Uniform refinement of the macro mesh (level 0 = macro refined once, so that
// level 0 already has patches of 2x2 sibling cells for the local projection
// stabilisation of Sec. 2.1), projection of new obstacle-edge midpoints onto
// the obstacle ellipse, Coons points for new cell centres, and the tables of
// the node-row operator storage described in sell.h.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dnnmg {

constexpr int kSlice = 64;          // nodes per SELL slice (one wavefront)
constexpr uint8_t kFlagDirichlet = 1;
constexpr uint8_t kFlagInflow = 2;
constexpr uint8_t kExtraBit = 0x80; // pslot entry lives in the LPS-extra part

struct MacroInput {
  std::vector<double> xy;           // 2 V
  std::vector<int> quads;           // 4 C
  std::vector<int> bedges;          // 3 E
  std::vector<double> curves;       // 5 K
};

struct HostLevel {
  int N = 0, C = 0, NP = 0, Eb = 0;
  std::vector<double> xy;           // 2 N
  std::vector<int> cells;           // 4 C, counter-clockwise
  std::vector<int> bedges;          // 3 Eb
  std::vector<uint8_t> flag;        // per node
  // refinement record: how this level was made from the coarser one
  int Nc = 0, Ec = 0;
  std::vector<int> edge_ends;       // 2 Ec coarse node ids per new edge node
  std::vector<int> coarse_cells;    // 4 Cc coarse cells (one new centre each)
  // adjacency
  std::vector<int> cadj_ptr, cadj;  // node -> 4 c + a
  std::vector<int> padj_ptr, padj;  // node -> 9 P + q
  std::vector<int> patch_nodes;     // 9 NP, lexicographic in the parent frame
  // SELL-64 row structure: per slice the Q1 width wq and LPS-extra width wx
  int nslice = 0, totq = 0, totx = 0, maxwq = 0, maxwx = 0;
  long long nnzq = 0, nnzx = 0;     // real (unpadded) Q1 blocks and extra entries
  std::vector<int> wq, wx, oq, ox;  // per slice
  std::vector<int> colq, colx;      // [slot][lane] global column node ids
  std::vector<uint8_t> cslot;       // 4 per cadj entry: slot of each cell node in the row
  std::vector<uint8_t> pslot;       // 9 per padj entry: slot of each patch node (kExtraBit)
  std::vector<uint8_t> vslot;       // 16 per cell: slot of node b in node a's Q1 row
  // restriction to the coarser level: fine nodes contributing to coarse node j
  std::vector<int> rptr, ridx;
  // greedy cell colouring in cell order (no two cells of a colour share a
  // node): cells of colour k are colour_cells[colour_ptr[k] .. colour_ptr[k+1])
  int ncolour = 0;
  std::vector<int> colour_ptr, colour_cells;
};

// Refines (xy, cells, bedges) once; numbering: old vertices keep ids, then one
// node per edge in order of first appearance over cells/local edges, then one
// node per cell; cell c has children 4c..4c+3 (child k keeps vertex k).
HostLevel refine(const std::vector<double> &xy, const std::vector<int> &cells,
                 const std::vector<int> &bedges, const std::vector<double> &curves,
                 std::string *err);

// Builds adjacency, patches, SELL layout, slot tables and restriction lists.
bool build_tables(HostLevel &L, std::string *err);

}  // namespace dnnmg
