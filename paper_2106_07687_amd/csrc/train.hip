// BPTT training of the patch GRU network (loss of eq. loss, Sec. 2.2) with
// gradient checkpointing, BF16 MFMA GEMMs (FP32 accumulation) and Adam on
// FP32 master weights.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "net.h"

using namespace dnnmg;

namespace {

// C (+)= A(M,K) B(N,K)^T; M is split into launches of at most 32768 row
// tiles (each row's result does not depend on the split).
void gemm_nt(hipStream_t s, long M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
             float *C, int ldc, bool acc = false) {
  const long chunk = 32768L * GBM;
  for (long m0 = 0; m0 < M; m0 += chunk) {
    const int mc = static_cast<int>(std::min(chunk, M - m0));
    launch_gemm_nt(s, mc, N, K, A + m0 * lda, lda, B, ldb, C + m0 * ldc, ldc, acc);
  }
  check(hipGetLastError(), "k_gemm_nt_bf16");
}

// C (+)= A(m,k) B(n,k) with general strides; split-K through `part`.
void gemm_strided(hipStream_t s, int M, int N, int K, const uint16_t *A, long sAm, long sAk,
                  const uint16_t *B, long sBn, long sBk, float *C, int ldc, bool acc, DevBuf<float> &part) {
  // K-major operands with unit stride along m and n: the kernel with 16-byte
  // row loads (bitwise the same products)
  // (measured: for the input width of the first layer, N not a multiple of 8
  // and read up to the padded row length, the element-gather kernel is as
  // fast, so the 16-byte path is taken for N a multiple of 8 only)
  const int Nl = N;
  const bool tn = sAm == 1 && sBn == 1 && sAk % 8 == 0 && sBk % 8 == 0 && M % 8 == 0 && N % 8 == 0 &&
                  reinterpret_cast<uintptr_t>(A) % 16 == 0 && reinterpret_cast<uintptr_t>(B) % 16 == 0;
  auto launch = [&](dim3 g, int m, int kz, const uint16_t *a, float *c, int ld, long zs, int accf) {
    if (tn)
      hipLaunchKernelGGL(k_gemm_bf16_tn, g, dim3(256), 0, s, m, N, Nl, K, kz, a, sAk, B, sBk, c, ld, zs, accf);
    else
      hipLaunchKernelGGL(k_gemm_bf16_strided, g, dim3(256), 0, s, m, N, K, kz, a, sAm, sAk, B, sBn, sBk, c, ld, zs,
                         accf);
  };
  const long tiles = static_cast<long>((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
  int Z = 1;
  while (tiles * Z < 512 && K / (Z * 2) >= 1024) Z *= 2;
  dim3 grid((N + GBN - 1) / GBN, (M + GBM - 1) / GBM, Z);
  if (Z == 1) {
    // M in launches of at most 32768 row tiles
    const int chunk = 32768 * GBM;
    for (int m0 = 0; m0 < M; m0 += chunk) {
      const int mc = std::min(chunk, M - m0);
      dim3 g1((N + GBN - 1) / GBN, (mc + GBM - 1) / GBM);
      launch(g1, mc, K, A + m0 * sAm, C + static_cast<long>(m0) * ldc, ldc, 0L, acc ? 1 : 0);
    }
    check(hipGetLastError(), "k_gemm_bf16_strided");
    return;
  }
  const int kz = ((K + Z - 1) / Z + GBK - 1) / GBK * GBK;
  const size_t need = static_cast<size_t>(Z) * M * N;
  if (part.n < need) part.alloc(need);
  launch(grid, M, kz, A, part.p, N, static_cast<long>(M) * N, 0);
  hipLaunchKernelGGL(k_reduce_split, dim3(blocks(static_cast<size_t>(M) * N, 256)), dim3(256), 0, s, M, N, N, Z,
                     static_cast<long>(M) * N, part.p, C, ldc, acc ? 1 : 0);
  check(hipGetLastError(), "split-K GEMM");
}

struct Trainer {
  int T = 0, Bt = 0, seg = 0, nseg = 0;
  DevBuf<uint16_t> Xb;                       // T x Bt x K0
  std::vector<DevBuf<float>> hck;            // per layer: (nseg) x Bt x H checkpoints
  std::vector<DevBuf<float>> hs32;           // per layer: (seg + 1) x Bt x H
  std::vector<DevBuf<uint16_t>> hs16;        // per layer: (seg + 1) x Bt x H
  std::vector<DevBuf<float>> sv;             // per layer: seg x Bt x 4H saved gates
  std::vector<DevBuf<uint16_t>> dgi, dgh;    // per layer: seg x Bt x 3H
  std::vector<DevBuf<float>> dh;             // per layer: Bt x H
  DevBuf<float> Gi;                          // seg x Bt x 3H input projections
  DevBuf<float> E;                           // seg x Bt x H gradient from above
  DevBuf<float> Yseg;                        // seg x Bt x O
  DevBuf<uint16_t> dYb;                      // seg x Bt x O
  DevBuf<float> grad, part;
  DevBuf<double> lpart;
};

void ensure(Net &n, Trainer &tr, int T, int Bt, int seg) {
  if (tr.T == T && tr.Bt == Bt && tr.seg == seg) return;
  tr.T = T;
  tr.Bt = Bt;
  tr.seg = seg;
  tr.nseg = (T + seg - 1) / seg;
  const size_t bh = static_cast<size_t>(Bt) * n.H;
  tr.Xb.alloc(static_cast<size_t>(T) * Bt * n.K0);
  tr.hck.resize(n.layers);
  tr.hs32.resize(n.layers);
  tr.hs16.resize(n.layers);
  tr.sv.resize(n.layers);
  tr.dgi.resize(n.layers);
  tr.dgh.resize(n.layers);
  tr.dh.resize(n.layers);
  for (int l = 0; l < n.layers; ++l) {
    tr.hck[l].alloc(static_cast<size_t>(tr.nseg) * bh);
    tr.hs32[l].alloc(static_cast<size_t>(seg + 1) * bh);
    tr.hs16[l].alloc(static_cast<size_t>(seg + 1) * bh);
    tr.sv[l].alloc(static_cast<size_t>(seg) * 4 * bh);
    tr.dgi[l].alloc(static_cast<size_t>(seg) * 3 * bh);
    tr.dgh[l].alloc(static_cast<size_t>(seg) * 3 * bh);
    tr.dh[l].alloc(bh);
  }
  tr.Gi.alloc(static_cast<size_t>(seg) * 3 * bh);
  tr.E.alloc(static_cast<size_t>(seg) * bh);
  tr.Yseg.alloc(static_cast<size_t>(seg) * Bt * n.O);
  tr.dYb.alloc(static_cast<size_t>(seg) * Bt * n.O);
  tr.grad.alloc(static_cast<size_t>(n.nparam));
  tr.lpart.alloc(static_cast<size_t>(T) * 1024);
}

// The ns steps t0 .. t0 + ns - 1 of the whole stack, layer by layer: one
// input-projection GEMM over all ns steps of a layer, then its recurrent
// steps (k_gru_step_fused, BF16 state slot k in, slot k + 1 out).  On entry
// slot 0 of hs32[l] / hs16[l] holds every layer's state before t0.  With
// `keep`, every FP32 state (slots 1 .. ns), the gates and the head outputs
// Yseg are kept for the backward sweep; without, the FP32 state is updated
// in place in slot 0.
void segment_forward(Net &n, Trainer &tr, hipStream_t s, int t0, int ns, bool keep) {
  const int Bt = tr.Bt, H = n.H, H3 = 3 * H;
  const size_t bh = static_cast<size_t>(Bt) * H;
  for (int l = 0; l < n.layers; ++l) {
    const uint16_t *in = l == 0 ? tr.Xb.p + static_cast<size_t>(t0) * Bt * n.K0 : tr.hs16[l - 1].p + bh;
    const int K = l == 0 ? n.K0 : H;
    gemm_nt(s, static_cast<long>(ns) * Bt, H3, K, in, K, n.wih_b[l].p, K, tr.Gi.p, H3);
    for (int k = 0; k < ns; ++k) {
      float *h32_in = tr.hs32[l].p + (keep ? k * bh : 0);
      float *h32_out = tr.hs32[l].p + (keep ? (k + 1) * bh : 0);
      float *save = keep ? tr.sv[l].p + static_cast<size_t>(k) * 4 * bh : nullptr;
      // recurrent product + gates in one kernel (H a multiple of 32; the BF16
      // input and output states are distinct slots)
      hipLaunchKernelGGL(k_gru_step_fused, dim3(H / 32, blocks(Bt, 64)), dim3(256), 0, s, Bt, H,
                         tr.Gi.p + static_cast<size_t>(k) * 3 * bh, tr.hs16[l].p + k * bh, h32_in,
                         n.whh_b[l].p, h32_out, tr.hs16[l].p + (k + 1) * bh, save);
    }
  }
  if (keep)
    gemm_nt(s, static_cast<long>(ns) * Bt, n.O, H, tr.hs16[n.layers - 1].p + bh, H, n.wout_b.p, H, tr.Yseg.p,
            n.O);
  check(hipGetLastError(), "segment_forward");
}

// Loss and gradient (into tr.grad) by BPTT with checkpoints every `seg` steps.
double loss_and_grad(Net &n, Trainer &tr, const float *X, const float *D) {
  Ctx &c = *n.ctx;
  hipStream_t s = c.stream;
  const int T = tr.T, Bt = tr.Bt, seg = tr.seg, L = n.layers, H = n.H;
  const size_t bh = static_cast<size_t>(Bt) * H;
  hipLaunchKernelGGL(k_pack_bf16, dim3(blocks(static_cast<size_t>(T) * Bt * n.K0, 256)), dim3(256), 0, s,
                     T * Bt, n.I, X, n.K0, tr.Xb.p);
  hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, s, tr.grad.p, tr.grad.n, 0.0f);
  // forward sweep storing checkpoints (running state in slot 0 of hs32 /
  // hs16); the last segment keeps what its backward sweep needs
  for (int l = 0; l < L; ++l) {
    hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, s, tr.hs32[l].p, bh, 0.0f);
    hipLaunchKernelGGL(k_fill<uint16_t>, dim3(1024), dim3(256), 0, s, tr.hs16[l].p, bh, uint16_t(0));
  }
  for (int sg = 0; sg < tr.nseg; ++sg) {
    const int t0 = sg * seg, ns = std::min(seg, T - t0);
    for (int l = 0; l < L; ++l)
      check(hipMemcpyAsync(tr.hck[l].p + static_cast<size_t>(sg) * bh, tr.hs32[l].p, bh * sizeof(float),
                           hipMemcpyDeviceToDevice, s),
            "checkpoint");
    const bool last = sg == tr.nseg - 1;
    segment_forward(n, tr, s, t0, ns, last);
    if (!last)
      for (int l = 0; l < L; ++l)
        check(hipMemcpyAsync(tr.hs16[l].p, tr.hs16[l].p + static_cast<size_t>(ns) * bh, bh * sizeof(uint16_t),
                             hipMemcpyDeviceToDevice, s),
              "BF16 state");
  }
  for (int l = 0; l < L; ++l)
    hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, s, tr.dh[l].p, bh, 0.0f);
  double loss = 0.0;
  std::vector<double> lp(1024);
  const int lblocks = std::min(1024, blocks(static_cast<size_t>(Bt) * n.O, 256));
  for (int sg = tr.nseg - 1; sg >= 0; --sg) {
    const int t0 = sg * seg, ns = std::min(seg, T - t0);
    if (sg != tr.nseg - 1) {
      // recompute the segment from its checkpoint, keeping every state
      for (int l = 0; l < L; ++l) {
        check(hipMemcpyAsync(tr.hs32[l].p, tr.hck[l].p + static_cast<size_t>(sg) * bh, bh * sizeof(float),
                             hipMemcpyDeviceToDevice, s),
              "restore");
        hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks(bh, 256)), dim3(256), 0, s, bh, tr.hs32[l].p,
                           tr.hs16[l].p);
      }
      segment_forward(n, tr, s, t0, ns, true);
    }
    // backward through the segment, layer by layer from the top.  Loss
    // gradients of all ns steps (per-block loss partials of step t stay on
    // the device until the end), then the head's gradient dY W_out for all
    // steps as one product into E.
    hipLaunchKernelGGL(k_loss_grad, dim3(lblocks, ns), dim3(256), 0, s, Bt, n.O, tr.Yseg.p,
                       D + static_cast<size_t>(t0) * Bt * n.O, tr.dYb.p,
                       tr.lpart.p + static_cast<size_t>(t0) * lblocks);
    gemm_strided(s, ns * Bt, H, n.O, tr.dYb.p, n.O, 1, n.wout_b.p, 1, H, tr.E.p, H, false, tr.part);
    for (int l = L - 1; l >= 0; --l) {
      for (int k = ns - 1; k >= 0; --k) {
        uint16_t *dgi = tr.dgi[l].p + static_cast<size_t>(k) * 3 * bh;
        uint16_t *dgh = tr.dgh[l].p + static_cast<size_t>(k) * 3 * bh;
        // dL/dh_t = (carried) + E_t; then dh_{t-1} = g z + dgh W_hh (an NT
        // product with the transposed BF16 weights, K = 3H)
        hipLaunchKernelGGL(k_gru_gates_bwd, dim3(blocks(bh, 256)), dim3(256), 0, s, Bt, H, tr.dh[l].p,
                           tr.E.p + static_cast<size_t>(k) * bh, tr.sv[l].p + static_cast<size_t>(k) * 4 * bh,
                           tr.hs32[l].p + k * bh, dgi, dgh, tr.dh[l].p);
        gemm_nt(s, Bt, H, 3 * H, dgh, 3 * H, n.whh_t[l].p, 3 * H, tr.dh[l].p, H, true);
      }
      // gradient into the layer below at every step of the segment: dgi W_ih
      if (l > 0)
        gemm_nt(s, static_cast<long>(ns) * Bt, H, 3 * H, tr.dgi[l].p, 3 * H, n.wih_t[l].p, 3 * H, tr.E.p, H);
    }
    // weight gradients of the segment: K = ns * Bt rows at once
    const int Ks = ns * Bt;
    float *g = tr.grad.p;
    gemm_strided(s, n.O, H, Ks, tr.dYb.p, 1, n.O, tr.hs16[L - 1].p + bh, 1, H, g + n.off_out, H, true, tr.part);
    for (int l = 0; l < L; ++l) {
      const int Il = l == 0 ? n.I : H;
      const uint16_t *in = l == 0 ? tr.Xb.p + static_cast<size_t>(t0) * Bt * n.K0 : tr.hs16[l - 1].p + bh;
      const long ldin = l == 0 ? n.K0 : H;
      gemm_strided(s, 3 * H, Il, Ks, tr.dgi[l].p, 1, 3 * H, in, 1, ldin, g + n.off_ih[l], Il, true, tr.part);
      gemm_strided(s, 3 * H, H, Ks, tr.dgh[l].p, 1, 3 * H, tr.hs16[l].p, 1, H, g + n.off_hh[l], H, true, tr.part);
    }
  }
  // loss: the per-step partials, summed in the order of the backward sweep
  lp.resize(static_cast<size_t>(T) * lblocks);
  check(hipMemcpyAsync(lp.data(), tr.lpart.p, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, s), "loss");
  check(hipStreamSynchronize(s), "loss sync");
  for (int t = T - 1; t >= 0; --t)
    for (int b = 0; b < lblocks; ++b) loss += lp[static_cast<size_t>(t) * lblocks + b];
  return loss / Bt;
}

struct TrainState {
  Trainer tr;
  DevBuf<float> m, v, Xd, Dd;
  long step = 0;
};

}  // namespace

namespace dnnmg {
TrainStateHolder::~TrainStateHolder() { delete static_cast<TrainState *>(p); }
}  // namespace dnnmg

namespace {
TrainState &tstate(Net &n) {
  if (!n.train.p) n.train.p = new TrainState();
  return *static_cast<TrainState *>(n.train.p);
}

int check_batch(Net &n, int T, int Bt, int ckpt) {
  if (T < 1 || Bt < 1 || ckpt < 1 || T > 4096 || Bt > (1 << 22) || static_cast<long>(T) * Bt > (1L << 26)) {
    n.ctx->last_error = "invalid batch shape";
    return DNNMG_EINVAL;
  }
  return DNNMG_OK;
}

int run_grad(Net &n, const float *X, const float *D, int T, int Bt, int ckpt, bool host, float *grad_out,
             float *loss_out, float lr, bool update) {
  Ctx &c = *n.ctx;
  try {
    TrainState &ts = tstate(n);
    ensure(n, ts.tr, T, Bt, std::min(ckpt, T));
    const float *Xd = X, *Dd = D;
    if (host) {
      const size_t nx = static_cast<size_t>(T) * Bt * n.I, nd = static_cast<size_t>(T) * Bt * n.O;
      if (ts.Xd.n < nx) ts.Xd.alloc(nx);
      if (ts.Dd.n < nd) ts.Dd.alloc(nd);
      check(hipMemcpyAsync(ts.Xd.p, X, nx * sizeof(float), hipMemcpyHostToDevice, c.stream), "X H2D");
      check(hipMemcpyAsync(ts.Dd.p, D, nd * sizeof(float), hipMemcpyHostToDevice, c.stream), "D H2D");
      Xd = ts.Xd.p;
      Dd = ts.Dd.p;
    }
    const double loss = loss_and_grad(n, ts.tr, Xd, Dd);
    if (update) {
      if (!ts.m.p) {
        ts.m.alloc(n.nparam);
        ts.v.alloc(n.nparam);
        hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, c.stream, ts.m.p, ts.m.n, 0.0f);
        hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, c.stream, ts.v.p, ts.v.n, 0.0f);
      }
      ts.step += 1;
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.0f - std::pow(b1, static_cast<float>(ts.step));
      const float c2 = 1.0f - std::pow(b2, static_cast<float>(ts.step));
      hipLaunchKernelGGL(k_adam, dim3(blocks(n.nparam, 256)), dim3(256), 0, c.stream, static_cast<size_t>(n.nparam),
                         n.w32.p, ts.tr.grad.p, ts.m.p, ts.v.p, lr, b1, b2, 1e-8f, c1, c2);
      check(hipGetLastError(), "k_adam");
      net_repack(n);
    }
    if (grad_out)
      check(hipMemcpyAsync(grad_out, ts.tr.grad.p, sizeof(float) * n.nparam, hipMemcpyDeviceToHost, c.stream),
            "grad D2H");
    check(hipStreamSynchronize(c.stream), "train sync");
    if (loss_out) *loss_out = static_cast<float>(loss);
  } catch (const DnnmgError &e) {
    c.last_error = e.msg;
    return e.code;
  }
  return DNNMG_OK;
}

}  // namespace

extern "C" {

int dnnmg_net_gradient(dnnmg_net *net, const float *X, const float *D, int T, int B, int ckpt,
                       float *grad, float *loss) {
  if (!net || !X || !D) return DNNMG_EINVAL;
  Net &n = net_of(net);
  const int e = check_batch(n, T, B, ckpt);
  if (e) return e;
  return run_grad(n, X, D, T, B, ckpt, true, grad, loss, 0.0f, false);
}

int dnnmg_train_step(dnnmg_net *net, const float *X, const float *D, int T, int B, int ckpt, float lr,
                     float *loss) {
  if (!net || !X || !D || !(lr > 0)) return DNNMG_EINVAL;
  Net &n = net_of(net);
  const int e = check_batch(n, T, B, ckpt);
  if (e) return e;
  return run_grad(n, X, D, T, B, ckpt, true, nullptr, loss, lr, true);
}

int dnnmg_train_step_dev(dnnmg_net *net, const float *X_dev, const float *D_dev, int T, int B, int ckpt,
                         float lr, float *loss) {
  if (!net || !X_dev || !D_dev || !(lr > 0)) return DNNMG_EINVAL;
  Net &n = net_of(net);
  const int e = check_batch(n, T, B, ckpt);
  if (e) return e;
  return run_grad(n, X_dev, D_dev, T, B, ckpt, false, nullptr, loss, lr, true);
}

}  // extern "C"
