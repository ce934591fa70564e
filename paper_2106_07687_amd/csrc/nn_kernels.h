// gfx950 kernels of the DNN-MG patch network (Algorithm 1, the correction after the coarse step):
// patch gather with input standardisation, BF16 MFMA GEMMs with FP32
// accumulation, GRU gate update, output scatter-average, and the backward
// counterparts used by BPTT training.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace dnnmg {

struct PatchView {
  int B;              // patches
  int S2;             // fine nodes per patch (S * S)
  int NF;             // fine nodes
  const int *grid;    // B * S2 fine node ids (lexicographic in the parent frame)
  const int *nadj_ptr, *nadj;   // fine node -> (patch * S2 + q)
  const double *inv_mass;       // NF, 1 / lumped mass
  const double *feat;           // nfeat * B: aspect, skew, h_rel, h[, cos 2phi, sin 2phi]
  const uint8_t *flag;          // NF fine node flags
  int nch;                      // nodal input channels: 6 (block patches) or 5 (cell patches, no p)
  int nfeat;                    // patch features: 4 or 6
};

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// gfx950 MFMA 16x16x32 BF16 -> FP32.  Operand layout: lane l supplies row
// (or column) l % 16 and the 8 consecutive k = 8 (l / 16) .. 8 (l / 16) + 7 of
// the 32-wide k step; the accumulator holds rows 4 (l / 16) .. + 3 of column
// l % 16.  frag8 reads a lane's 8 BF16 with one 16-byte LDS load (rows of the
// LDS tiles are 16-byte aligned and k offsets multiples of 8).
__device__ __forceinline__ bf16x8 frag8(const uint16_t *p) { return *reinterpret_cast<const bf16x8 *>(p); }
__device__ __forceinline__ f32x4 mfma32(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ float sigmoidf_(float a) { return 1.0f / (1.0f + __expf(-a)); }

// C[M x N] (fp32, ldc) = A[M x K] * B[N x K]^T (+ C if accumulate), A and B
// BF16 row-major with leading dimensions lda, ldb (elements, multiples of 8),
// K a multiple of 32.  64 x 64 tile per workgroup of 256 threads (4 waves,
// each 32 x 32 as 2 x 2 MFMA 16x16x32 blocks), BK = 32 staged through LDS.
constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

__global__ void __launch_bounds__(256) k_gemm_nt_bf16(int M, int N, int K, const uint16_t *__restrict__ A,
                                                      int lda, const uint16_t *__restrict__ Bm, int ldb,
                                                      float *__restrict__ Cm, int ldc, int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GBM][GBK + GPAD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GBN][GBK + GPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int bm = blockIdx.y * GBM, bn = blockIdx.x * GBN;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int lr = tid >> 2, lc = (tid & 3) * 8;   // loader: row, 8-element chunk
  for (int k0 = 0; k0 < K; k0 += GBK) {
    uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
    if (bm + lr < M) va = *reinterpret_cast<const uint4 *>(A + static_cast<size_t>(bm + lr) * lda + k0 + lc);
    if (bn + lr < N) vb = *reinterpret_cast<const uint4 *>(Bm + static_cast<size_t>(bn + lr) * ldb + k0 + lc);
    __syncthreads();
    *reinterpret_cast<uint4 *>(&As[lr][lc]) = va;
    *reinterpret_cast<uint4 *>(&Bs[lr][lc]) = vb;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 32) {
      bf16x8 a[2], b[2];
      const int kq = kk + 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = frag8(&As[wm * 32 + i * 16 + (lane & 15)][kq]);
        b[i] = frag8(&Bs[wn * 32 + i * 16 + (lane & 15)][kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = bn + wn * 32 + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bm + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (row < M) {
          float *c = Cm + static_cast<size_t>(row) * ldc + col;
          *c = accumulate ? *c + acc[i][j][r] : acc[i][j][r];
        }
      }
    }
}

// The same product with a 128 x 128 tile per workgroup (4 waves, each 64 x 64
// as 4 x 4 MFMA 16x16x32 blocks) and 64-wide K chunks, the next chunk loaded
// into registers while the current one is multiplied out of LDS: four times
// the MFMA work per LDS byte and a quarter of the barriers, for products
// with enough tiles to fill the chip.  Every element's MFMA sequence over K
// (32-wide steps in order; a chunk past K is cut at K, a multiple of 32) is
// that of k_gemm_nt_bf16, so the two give bitwise the same C.
constexpr int GBM2 = 128, GBN2 = 128, GBK2 = 64;
__global__ void __launch_bounds__(256) k_gemm_nt_bf16_128(int M, int N, int K, const uint16_t *__restrict__ A,
                                                          int lda, const uint16_t *__restrict__ Bm, int ldb,
                                                          float *__restrict__ Cm, int ldc, int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GBM2][GBK2 + GPAD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GBN2][GBK2 + GPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int bm = blockIdx.y * GBM2, bn = blockIdx.x * GBN2;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int lr = tid >> 3, lc = (tid & 7) * 8;   // loader: rows lr + 32 h, 8-element chunk lc
  uint4 va[4], vb[4];
  auto load = [&](int k0) {
    const bool kin = k0 + lc < K;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int r = lr + 32 * h;
      va[h] = kin && bm + r < M
                  ? *reinterpret_cast<const uint4 *>(A + static_cast<size_t>(bm + r) * lda + k0 + lc)
                  : make_uint4(0, 0, 0, 0);
      vb[h] = kin && bn + r < N
                  ? *reinterpret_cast<const uint4 *>(Bm + static_cast<size_t>(bn + r) * ldb + k0 + lc)
                  : make_uint4(0, 0, 0, 0);
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += GBK2) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      *reinterpret_cast<uint4 *>(&As[lr + 32 * h][lc]) = va[h];
      *reinterpret_cast<uint4 *>(&Bs[lr + 32 * h][lc]) = vb[h];
    }
    __syncthreads();
    if (k0 + GBK2 < K) load(k0 + GBK2);
    const int kend = min(GBK2, K - k0);
#pragma unroll
    for (int kk = 0; kk < GBK2; kk += 32) {
      if (kk >= kend) break;
      bf16x8 a[4], b[4];
      const int kq = kk + 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = frag8(&As[wm * 64 + i * 16 + (lane & 15)][kq]);
        b[i] = frag8(&Bs[wn * 64 + i * 16 + (lane & 15)][kq]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = bn + wn * 64 + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bm + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (row < M) {
          float *c = Cm + static_cast<size_t>(row) * ldc + col;
          *c = accumulate ? *c + acc[i][j][r] : acc[i][j][r];
        }
      }
    }
}

// C (+)= A B^T on stream s: the 128 x 128 tile kernel when the product has at
// least 256 such tiles (enough to fill the chip), else the 64 x 64 one; the
// result is bitwise the same either way.
inline void launch_gemm_nt(hipStream_t s, int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B,
                           int ldb, float *C, int ldc, bool acc) {
  const long tiles128 = static_cast<long>((M + GBM2 - 1) / GBM2) * ((N + GBN2 - 1) / GBN2);
  if (tiles128 >= 256)
    hipLaunchKernelGGL(k_gemm_nt_bf16_128, dim3((N + GBN2 - 1) / GBN2, (M + GBM2 - 1) / GBM2), dim3(256), 0, s, M,
                       N, K, A, lda, B, ldb, C, ldc, acc ? 1 : 0);
  else
    hipLaunchKernelGGL(k_gemm_nt_bf16, dim3((N + GBN - 1) / GBN, (M + GBM - 1) / GBM), dim3(256), 0, s, M, N, K,
                       A, lda, B, ldb, C, ldc, acc ? 1 : 0);
}

// One GRU time step of a layer (gate rows r, z, n): the recurrent product
// Gh = h_in W_hh^T for a tile of 64 rows x 32 hidden units and all three
// gates (MFMA 16x16x32 BF16, the K loop in 32-wide chunks as in
// k_gemm_nt_bf16), then, on the accumulators, with Gi = x W_ih^T from that
// kernel: r = s(gi_r + gh_r), z = s(gi_z + gh_z), n = tanh(gi_n + r gh_n),
// h = (1 - z) n + z h_in (FP32; h may be hin), its BF16 copy into hb_out (not
// hb_in), and optionally r, z, n, gh_n for the backward pass.  Gh never goes
// to memory.  Wave w owns rows 16w..16w+15 of the tile, both 16-unit halves
// and the three gates, so each lane holds r, z, n inputs of the same (row,
// unit).  H must be a multiple of 32.
__global__ void __launch_bounds__(256) k_gru_step_fused(int B, int H, const float *__restrict__ Gi,
                                                        const uint16_t *__restrict__ hb_in,
                                                        const float *hin, const uint16_t *__restrict__ Whh,
                                                        float *h, uint16_t *__restrict__ hb_out,
                                                        float *__restrict__ save) {
  __shared__ __attribute__((aligned(16))) uint16_t As[64][GBK + GPAD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[96][GBK + GPAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = blockIdx.y * 64, u0 = blockIdx.x * 32;
  f32x4 acc[3][2];
#pragma unroll
  for (int g = 0; g < 3; ++g)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[g][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < H; k0 += GBK) {
    // loaders: 64 A rows x 4 chunks of 8; 96 B rows x 4 chunks (threads 0..383 -> two passes)
    uint4 va = make_uint4(0, 0, 0, 0), vb0 = make_uint4(0, 0, 0, 0), vb1 = make_uint4(0, 0, 0, 0);
    const int lr = tid >> 2, lc = (tid & 3) * 8;
    if (r0 + lr < B) va = *reinterpret_cast<const uint4 *>(hb_in + static_cast<size_t>(r0 + lr) * H + k0 + lc);
    {   // B rows 0..63 of the tile: gate lr / 32, unit lr % 32
      const int g = lr >> 5, u = lr & 31;
      if (u0 + u < H) vb0 = *reinterpret_cast<const uint4 *>(Whh + static_cast<size_t>(g * H + u0 + u) * H + k0 + lc);
    }
    if (lr < 32) {   // B rows 64..95: gate 2
      const int u = lr;
      if (u0 + u < H) vb1 = *reinterpret_cast<const uint4 *>(Whh + static_cast<size_t>(2 * H + u0 + u) * H + k0 + lc);
    }
    __syncthreads();
    *reinterpret_cast<uint4 *>(&As[lr][lc]) = va;
    *reinterpret_cast<uint4 *>(&Bs[lr][lc]) = vb0;
    if (lr < 32) *reinterpret_cast<uint4 *>(&Bs[64 + lr][lc]) = vb1;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 32) {
      const int kq = kk + 8 * (lane >> 4);
      const bf16x8 a = frag8(&As[wave * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int g = 0; g < 3; ++g)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[g][j] = mfma32(a, frag8(&Bs[g * 32 + j * 16 + (lane & 15)][kq]), acc[g][j]);
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int unit = u0 + j * 16 + (lane & 15);
    if (unit >= H) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = r0 + wave * 16 + 4 * (lane >> 4) + i;
      if (row >= B) continue;
      const float *gi = Gi + static_cast<size_t>(row) * 3 * H;
      const float ghr = acc[0][j][i], ghz = acc[1][j][i], ghn = acc[2][j][i];
      const float r = sigmoidf_(gi[unit] + ghr);
      const float z = sigmoidf_(gi[H + unit] + ghz);
      const float n = tanhf(gi[2 * H + unit] + r * ghn);
      const size_t t = static_cast<size_t>(row) * H + unit;
      const float hp = hin[t];
      const float hn = (1.0f - z) * n + z * hp;
      h[t] = hn;
      hb_out[t] = f2bf(hn);
      if (save) {
        float *s = save + static_cast<size_t>(row) * 4 * H;
        s[unit] = r;
        s[H + unit] = z;
        s[2 * H + unit] = n;
        s[3 * H + unit] = ghn;
      }
    }
  }
}

// Patch gather (Algorithm 1, the network inputs): one workgroup per patch writes the
// standardised input row as BF16 into X (ld = ldx, padding zeroed): block
// patches [u, v, p, r_u, r_v, r_p at the S2 patch nodes; aspect, skew,
// h_rel, Peclet], cell patches [u, v, r_u, r_v, r_p; aspect, skew, h_rel,
// Peclet, cos 2phi, sin 2phi].  Residual rows are divided by the lumped
// mass; Dirichlet velocity residual rows are zero.
__global__ void __launch_bounds__(128) k_patch_gather(PatchView pv, const double *__restrict__ xt,
                                                      const double *__restrict__ R, const float *__restrict__ mu,
                                                      const float *__restrict__ sg, double nu,
                                                      uint16_t *__restrict__ X, int ldx, float *__restrict__ Xf) {
  __shared__ double smax[128];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int S2 = pv.S2;
  uint16_t *row = X + static_cast<size_t>(p) * ldx;
  float *rowf = Xf ? Xf + static_cast<size_t>(p) * ldx : nullptr;
  double sp = 0.0;
  for (int q = tid; q < S2; q += blockDim.x) {
    const int i = pv.grid[static_cast<size_t>(p) * S2 + q];
    const double u = xt[3 * i], v = xt[3 * i + 1], pr = xt[3 * i + 2];
    const double im = pv.inv_mass[i];
    const bool dir = pv.flag[i] & 1;
    const double ru = dir ? 0.0 : R[3 * i] * im, rv = dir ? 0.0 : R[3 * i + 1] * im;
    const double rp = R[3 * i + 2] * im;
    const bool no_p = pv.nch == 5;
    const double vals[6] = {u, v, no_p ? ru : pr, no_p ? rv : ru, no_p ? rp : rv, rp};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (c < pv.nch) {
        const float s = static_cast<float>((vals[c] - mu[c]) / sg[c]);
        row[c * S2 + q] = f2bf(s);
        if (rowf) rowf[c * S2 + q] = s;
      }
    }
    sp = fmax(sp, sqrt(u * u + v * v));
  }
  smax[tid] = sp;
  __syncthreads();
  for (int off = 64; off > 0; off >>= 1) {
    if (tid < off) smax[tid] = fmax(smax[tid], smax[tid + off]);
    __syncthreads();
  }
  const int nch = pv.nch, I = nch * S2 + pv.nfeat;
  if (tid < pv.nfeat) {
    const double *f = pv.feat + static_cast<size_t>(p) * pv.nfeat;
    const double val = tid == 3 ? smax[0] * f[3] / nu : f[tid];
    const float s = static_cast<float>((val - mu[nch + tid]) / sg[nch + tid]);
    row[nch * S2 + tid] = f2bf(s);
    if (rowf) rowf[nch * S2 + tid] = s;
  }
  for (int c = I + tid; c < ldx; c += blockDim.x) {
    row[c] = 0;
    if (rowf) rowf[c] = 0.0f;
  }
}

// Scatter-average of the predicted corrections to fine nodes, zero on
// Dirichlet nodes, then v_c = x~ + d (velocity), pressure 0:
// vc[3 i + f] = x~[3 i + f] + s_f * mean_{(p, q) ∋ i} Y[p][f * S2 + q].
__global__ void k_patch_scatter(PatchView pv, const float *__restrict__ Y, int ldy,
                                const float *__restrict__ oscale, const double *__restrict__ xt,
                                double *__restrict__ vc, double *__restrict__ d_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pv.NF) return;
  double du = 0.0, dv = 0.0;
  const int e0 = pv.nadj_ptr[i], e1 = pv.nadj_ptr[i + 1];
  for (int e = e0; e < e1; ++e) {
    const int p = pv.nadj[e] / pv.S2, q = pv.nadj[e] % pv.S2;
    du += Y[static_cast<size_t>(p) * ldy + q];
    dv += Y[static_cast<size_t>(p) * ldy + pv.S2 + q];
  }
  const double inv = e1 > e0 ? 1.0 / (e1 - e0) : 0.0;
  du *= inv * oscale[0];
  dv *= inv * oscale[1];
  if (pv.flag[i] & 1) {
    du = 0.0;
    dv = 0.0;
  }
  vc[3 * i] = xt[3 * i] + du;
  vc[3 * i + 1] = xt[3 * i + 1] + dv;
  vc[3 * i + 2] = 0.0;
  if (d_out) {
    d_out[2 * i] = du;
    d_out[2 * i + 1] = dv;
  }
}

// General-stride BF16 GEMM for the backward pass:
// C_z[m][n] = sum_{k in slice z} A(m, k) B(n, k), A(m, k) = A[m sAm + k sAk],
// B(n, k) = B[n sBn + k sBk]; any M, N, K (guarded).  Split-K over
// gridDim.z: slice z covers k in [z kz, min(K, (z + 1) kz)) and writes (or,
// with accumulate and gridDim.z == 1, adds to) C + z * zstride.
__global__ void __launch_bounds__(256) k_gemm_bf16_strided(int M, int N, int K, int kz,
                                                           const uint16_t *__restrict__ A, long sAm, long sAk,
                                                           const uint16_t *__restrict__ Bm, long sBn, long sBk,
                                                           float *__restrict__ Cm, int ldc, long zstride,
                                                           int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GBM][GBK + GPAD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GBN][GBK + GPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int bm = blockIdx.y * GBM, bn = blockIdx.x * GBN;
  const int kb = blockIdx.z * kz, ke = min(K, kb + kz);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += GBK) {
    uint16_t va[8], vb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid * 8 + e;   // 0..2047 over a 64 x 32 tile
      const int r = idx >> 5, cc = idx & 31;
      const int k = k0 + cc;
      va[e] = (bm + r < M && k < ke) ? A[(bm + r) * sAm + k * sAk] : uint16_t(0);
      vb[e] = (bn + r < N && k < ke) ? Bm[(bn + r) * sBn + k * sBk] : uint16_t(0);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid * 8 + e;
      As[idx >> 5][idx & 31] = va[e];
      Bs[idx >> 5][idx & 31] = vb[e];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 32) {
      bf16x8 a[2], b[2];
      const int kq = kk + 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = frag8(&As[wm * 32 + i * 16 + (lane & 15)][kq]);
        b[i] = frag8(&Bs[wn * 32 + i * 16 + (lane & 15)][kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
    }
  }
  float *Cz = Cm + blockIdx.z * zstride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = bn + wn * 32 + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bm + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (row < M) {
          float *c = Cz + static_cast<size_t>(row) * ldc + col;
          *c = accumulate ? *c + acc[i][j][r] : acc[i][j][r];
        }
      }
    }
}

// The same product for K-major operands with unit stride along m and n (A(m,
// k) = A[k lda + m], B(n, k) = B[k ldb + n]; lda, ldb and M multiples of 8;
// B columns are read up to Nl, N rounded up to 8, which each row of B must
// hold): each thread loads 8 consecutive m (or n) of one k row with one
// 16-byte load, so a workgroup reads whole 128-byte rows, and scatters them
// into the [m][k] LDS layout.  The LDS contents of the stored columns, and so
// every MFMA and its order, are those of k_gemm_bf16_strided: bitwise the
// same C.
__global__ void __launch_bounds__(256) k_gemm_bf16_tn(int M, int N, int Nl, int K, int kz,
                                                      const uint16_t *__restrict__ A, long lda,
                                                      const uint16_t *__restrict__ Bm, long ldb,
                                                      float *__restrict__ Cm, int ldc, long zstride,
                                                      int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GBM][GBK + GPAD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GBN][GBK + GPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int bm = blockIdx.y * GBM, bn = blockIdx.x * GBN;
  const int kb = blockIdx.z * kz, ke = min(K, kb + kz);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int lk = tid >> 3, lm = (tid & 7) * 8;   // loader: k row lk, 8 consecutive m (n) from lm
  uint4 va, vb;
  // the next K chunk is loaded into registers while the current one is
  // multiplied out of LDS
  auto load = [&](int k0) {
    const int k = k0 + lk;
    va = make_uint4(0, 0, 0, 0);
    vb = make_uint4(0, 0, 0, 0);
    if (k < ke && bm + lm < M) va = *reinterpret_cast<const uint4 *>(A + static_cast<size_t>(k) * lda + bm + lm);
    if (k < ke && bn + lm < Nl) vb = *reinterpret_cast<const uint4 *>(Bm + static_cast<size_t>(k) * ldb + bn + lm);
  };
  load(kb);
  for (int k0 = kb; k0 < ke; k0 += GBK) {
    __syncthreads();
    const uint16_t *ea = reinterpret_cast<const uint16_t *>(&va);
    const uint16_t *eb = reinterpret_cast<const uint16_t *>(&vb);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[lm + e][lk] = ea[e];
      Bs[lm + e][lk] = eb[e];
    }
    __syncthreads();
    if (k0 + GBK < ke) load(k0 + GBK);
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 32) {
      bf16x8 a[2], b[2];
      const int kq = kk + 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = frag8(&As[wm * 32 + i * 16 + (lane & 15)][kq]);
        b[i] = frag8(&Bs[wn * 32 + i * 16 + (lane & 15)][kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
    }
  }
  float *Cz = Cm + blockIdx.z * zstride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = bn + wn * 32 + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bm + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (row < M) {
          float *c = Cz + static_cast<size_t>(row) * ldc + col;
          *c = accumulate ? *c + acc[i][j][r] : acc[i][j][r];
        }
      }
    }
}

// dst[i] (+)= sum_z part[z * zstride + i] for an M x N block with leading
// dimension ld (fixed z order: deterministic).
__global__ void k_reduce_split(int M, int N, int ld, int Z, long zstride, const float *__restrict__ part,
                               float *__restrict__ dst, int ldd, int accumulate) {
  const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<size_t>(M) * N) return;
  const int m = static_cast<int>(t / N), n = static_cast<int>(t % N);
  float s = 0.0f;
  for (int z = 0; z < Z; ++z) s += part[z * zstride + static_cast<size_t>(m) * ld + n];
  float *d = dst + static_cast<size_t>(m) * ldd + n;
  *d = accumulate ? *d + s : s;
}

// Backward of one GRU gate update.  In: g = dL/dh_t (total), saved gates
// (r, z, n, gh_n) and h_{t-1}.  Out: dgi = dL/d(W_ih x) (3H), dgh =
// dL/d(W_hh h_{t-1}) (3H) as FP32 and BF16, dhp = g * z (the direct part of
// dL/dh_{t-1}; the GEMM dgh W_hh is added to it afterwards).
// g: dL/dh_t in, as the sum g + e (the carried gradient of the same layer plus
// the one arriving from the layer above or the head, added here in FP32);
// dhp: the z-path of dL/dh_{t-1} out (elementwise, may be g).
__global__ void k_gru_gates_bwd(int B, int H, const float *g, const float *__restrict__ e,
                                const float *__restrict__ save, const float *__restrict__ hprev,
                                uint16_t *__restrict__ dgi_b, uint16_t *__restrict__ dgh_b, float *dhp) {
  const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<size_t>(B) * H) return;
  const int b = static_cast<int>(t / H), j = static_cast<int>(t % H);
  const float *s = save + static_cast<size_t>(b) * 4 * H;
  const float r = s[j], z = s[H + j], n = s[2 * H + j], ghn = s[3 * H + j];
  const float gg = g[t] + e[t], hp = hprev[t];
  const float dz = gg * (hp - n);
  const float dn = gg * (1.0f - z);
  const float dan = dn * (1.0f - n * n);
  const float dr = dan * ghn;
  const float dar = dr * r * (1.0f - r);
  const float daz = dz * z * (1.0f - z);
  const size_t o = static_cast<size_t>(b) * 3 * H;
  dgi_b[o + j] = f2bf(dar);
  dgi_b[o + H + j] = f2bf(daz);
  dgi_b[o + 2 * H + j] = f2bf(dan);
  dgh_b[o + j] = f2bf(dar);
  dgh_b[o + H + j] = f2bf(daz);
  dgh_b[o + 2 * H + j] = f2bf(dan * r);
  dhp[t] = gg * z;
}

// dY = 2 (Y - D) / B (BF16 copy) and per-block partial sums of (Y - D)^2,
// for one time step per blockIdx.y (each step's B x O block and gridDim.x
// partials follow the previous step's).
__global__ void k_loss_grad(int B, int O, const float *__restrict__ Y, const float *__restrict__ D,
                            uint16_t *__restrict__ dYb, double *__restrict__ partial) {
  __shared__ double sh[256];
  const size_t n = static_cast<size_t>(B) * O;
  Y += blockIdx.y * n;
  D += blockIdx.y * n;
  dYb += blockIdx.y * n;
  partial += static_cast<size_t>(blockIdx.y) * gridDim.x;
  double s = 0.0;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float d = Y[i] - D[i];
    s += static_cast<double>(d) * d;
    dYb[i] = f2bf(2.0f * d / static_cast<float>(B));
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Adam on the FP32 masters (bias-corrected, step t >= 1).
__global__ void k_adam(size_t n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Training targets (reading N9): D[p][f S2 + q] = (v_fine - x~)_f at the
// patch node q of patch p, divided by the output scale of component f.
__global__ void k_patch_targets(PatchView pv, const double *__restrict__ vf, const double *__restrict__ xt,
                                const float *__restrict__ oscale, float *__restrict__ D) {
  const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<size_t>(pv.B) * pv.S2) return;
  const int p = static_cast<int>(t / pv.S2), q = static_cast<int>(t % pv.S2);
  const int i = pv.grid[t];
  float *row = D + static_cast<size_t>(p) * 2 * pv.S2;
  row[q] = static_cast<float>((vf[3 * i] - xt[3 * i]) / oscale[0]);
  row[pv.S2 + q] = static_cast<float>((vf[3 * i + 1] - xt[3 * i + 1]) / oscale[1]);
}

__global__ void k_f32_to_bf16(size_t n, const float *__restrict__ a, uint16_t *__restrict__ b) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = f2bf(a[i]);
}

// Copy of a row-major [rows x cols] FP32 matrix into a BF16 matrix with
// leading dimension ld >= cols (padding columns zero).
// b (cols x rows) = BF16 of the transpose of a (rows x cols, row-major).
__global__ void k_pack_bf16_t(int rows, int cols, const float *__restrict__ a, uint16_t *__restrict__ b) {
  const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<size_t>(rows) * cols) return;
  const int c = static_cast<int>(t / rows), r = static_cast<int>(t % rows);
  b[t] = f2bf(a[static_cast<size_t>(r) * cols + c]);
}

__global__ void k_pack_bf16(int rows, int cols, const float *__restrict__ a, int ld,
                            uint16_t *__restrict__ b) {
  const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<size_t>(rows) * ld) return;
  const int r = static_cast<int>(t / ld), c = static_cast<int>(t % ld);
  b[t] = c < cols ? f2bf(a[static_cast<size_t>(r) * cols + c]) : 0;
}

}  // namespace
}  // namespace dnnmg
