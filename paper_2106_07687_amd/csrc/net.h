// Device-resident DNN-MG patch network shared by the inference (dnnmg.hip)
// and training (train.hip) translation units.
#pragma once
#include <vector>

#include "context.h"
#include "nn_kernels.h"

namespace dnnmg {

// Opaque owner of the training workspace (defined in train.hip).
struct TrainStateHolder {
  void *p = nullptr;
  TrainStateHolder() = default;
  TrainStateHolder(const TrainStateHolder &) = delete;
  TrainStateHolder &operator=(const TrainStateHolder &) = delete;
  ~TrainStateHolder();
};

// Device-resident patch network of one simulation (weights, GRU state,
// work buffers) for patches of level L and fine level F = L + m.
struct Net {
  Ctx *ctx = nullptr;
  int L = 0, m = 0, F = 0, S = 0, S2 = 0, B = 0;
  int patch = 0;                               // DNNMG_PATCH_BLOCK or DNNMG_PATCH_CELL
  int nch = 6, nfeat = 4, nstat = 10;          // nodal channels, features, (mu, sigma) pairs
  int I = 0, H = 0, layers = 0, O = 0, K0 = 0;   // K0: padded input width
  long long nparam = 0;
  std::vector<long long> off_ih, off_hh;       // offsets in the flat weight vector
  long long off_out = 0;
  DevBuf<float> w32;                           // FP32 master weights (flat)
  std::vector<DevBuf<uint16_t>> wih_b, whh_b;  // BF16 working copies
  std::vector<DevBuf<uint16_t>> whh_t, wih_t;  // transposed BF16 copies (H x 3H), for the backward GEMMs
  DevBuf<uint16_t> wout_b;
  DevBuf<float> mu, sg, oscale;
  std::vector<DevBuf<float>> h;                // [B x H] per layer
  std::vector<DevBuf<uint16_t>> hb, hb_next;   // BF16 state; the fused step writes hb_next, then they swap
  DevBuf<uint16_t> X;
  DevBuf<float> Xf, Gi, Y;
  // fine-level vectors (FP64)
  std::vector<DevBuf<double>> xt;              // prolongation chain, index l - L
  DevBuf<double> vprev, vc, bF, dcorr;
  std::vector<DevBuf<double>> rchain;          // restriction chain
  // patch tables
  DevBuf<int> grid, nadj_ptr, nadj;
  DevBuf<double> inv_mass, feat;
  bool has_vprev = false;
  TrainStateHolder train;
  PatchView view() const {
    const DevLevel &LF = *ctx->levels[F];
    return PatchView{B, S2, LF.h.N, grid.p, nadj_ptr.p, nadj.p, inv_mass.p, feat.p, LF.flag.p, nch, nfeat};
  }
};


// BF16 working copies from the FP32 masters (dnnmg.hip).
void net_repack(Net &n);

}  // namespace dnnmg

struct dnnmg_net {
  dnnmg::Net impl;
};

namespace dnnmg {
inline Net &net_of(dnnmg_net *h) { return h->impl; }
}  // namespace dnnmg
