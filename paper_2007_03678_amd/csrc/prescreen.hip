// Learned pre-screen on the GPU: message passing over the ligand graph,
// sum pooling and an MLP predict each ligand's docking score, so that full
// docking can be spent on the ligands ranked best (the screening setting of
// Sec. 1 / Sec. 2.2: many ligands against one receptor).
//
// Network (BF16 operands, FP32 accumulation; r() = round to BF16):
//   H0 = r(relu(X W0 + b0)); for l = 1..3: M = r(A H), H = r(relu([H|M] W_l + b_l))
//   g = r(sum_atoms H3); z1 = r(relu(g U1 + c1)); z2 = r(relu(z1 U2 + c2)); p = z2 U3 + c3
// Loss: mean (p - y)^2 + lam * mean over (y_i < y_j) of softplus((p_i - p_j)/tau),
// labels standardised; Adam on FP32 master weights, BF16 mirror for the GEMMs.
//
// GEMMs run on the gfx950 MFMA unit (v_mfma_f32_32x32x16_bf16): 64x64 output
// tiles per 256-thread work-group (2x2 wavefronts of 32x32), K in steps of
// 32 through LDS.  Weight gradients reduce over graph nodes in split-K
// chunks written to a partial buffer and summed in a fixed order, so every
// result is deterministic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "api_internal.h"

namespace ad {
namespace {

constexpr int kW = 128;     // message-passing width
constexpr int kH = 256;     // MLP width
constexpr int kLayers = 3;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// GEMM  C[M x N] = A[M x K] . B[K x N]
// A modes: 0 row-major A1[m*lda1 + k] (rows optionally through a_rows),
//          1 two row-major sources side by side (k < split from A1),
//          2 column access A1[k*lda1 + m] (a transposed operand),
//          3 column access of two sources (m < split from A1),
//          4 a message-passing layer's [H | r(A H)]: columns k < split are
//            H = A1 (row-major, lda1), columns k >= split the BF16 rounding
//            of the sum of H over the row's bond neighbours, gathered in
//            the tile loader in neighbour order (the same FP32 sum, hence
//            the same rounding, as a separate gather pass); the work-groups
//            of the first N tile also store that half to Mout when given
//            (the backward pass reads it).
// B modes: 0 B[k*ldb + n], 1 B[n*ldb + k] (a transposed operand).
// ---------------------------------------------------------------------------
struct GemmArgs {
  int M, N, K;
  int a_mode, split;
  const uint16_t *A1, *A2;
  int lda1, lda2;
  const int *a_rows;
  int b_mode;
  const uint16_t *B;
  int ldb;
  int m_ones;             // A row m_ones (column access) is all ones: C row m_ones = column sums of B (-1: none)
  const float *bias;
  int relu;
  const uint16_t *mask;   // zero where mask[m*ldm + n] <= 0
  int ldm;
  float *C32;
  int ldc32;
  uint16_t *C16;
  int ldc16;
  float *part;            // split-K partials [gridDim.z][M][N]
  int k_chunk;
  // a_mode 4: graph layout of the rows and where the gathered half goes
  const int *node_atom, *node_g0;
  const uint8_t *nbr;
  uint16_t *Mout;
};

constexpr int BM = 64, BN = 64, BK = 32, BKP = BK + 8;

__device__ __forceinline__ uint16_t gemm_a(const GemmArgs &g, int m, int k) {
  if (m == g.m_ones) return (uint16_t)0x3F80;   // 1.0 in BF16
  switch (g.a_mode) {
    case 0: {
      const int r = g.a_rows ? g.a_rows[m] : m;
      return g.A1[(size_t)r * g.lda1 + k];
    }
    case 1:
      return k < g.split ? g.A1[(size_t)m * g.lda1 + k] : g.A2[(size_t)m * g.lda2 + (k - g.split)];
    case 2:
      return g.A1[(size_t)k * g.lda1 + m];
    case 4: {
      if (k < g.split) return g.A1[(size_t)m * g.lda1 + k];
      const uint8_t *nb = g.nbr + (size_t)g.node_atom[m] * kMaxDeg;
      float acc = 0.0f;
      for (int d = 0; d < kMaxDeg && nb[d] != 0xff; ++d)
        acc += bf2f(g.A1[(size_t)(g.node_g0[m] + nb[d]) * g.lda1 + (k - g.split)]);
      return f2bf(acc);
    }
    default:
      return m < g.split ? g.A1[(size_t)k * g.lda1 + m] : g.A2[(size_t)k * g.lda2 + (m - g.split)];
  }
}

// Eight consecutive A elements along the operand's contiguous axis as one
// 16-byte load, or null when they have to be gathered one by one (ragged
// edge, the split of a concatenated operand, the ones row, misalignment).
__device__ __forceinline__ const uint16_t *aligned8(const uint16_t *p) {
  return ((uintptr_t)p & 15) == 0 ? p : nullptr;
}
// row-wise modes: A(m, k..k+7)
__device__ __forceinline__ const uint16_t *a_row8(const GemmArgs &g, int m, int k, int kz1) {
  if (m >= g.M || m == g.m_ones || k + 8 > kz1) return nullptr;
  if (g.a_mode == 0 || g.a_mode == 4) {
    if (g.a_rows || (g.lda1 & 7) || (g.a_mode == 4 && k + 8 > g.split)) return nullptr;
    return aligned8(g.A1 + (size_t)m * g.lda1 + k);
  }
  if (k + 8 <= g.split) return (g.lda1 & 7) ? nullptr : aligned8(g.A1 + (size_t)m * g.lda1 + k);
  if (k >= g.split) return (g.lda2 & 7) ? nullptr : aligned8(g.A2 + (size_t)m * g.lda2 + (k - g.split));
  return nullptr;
}
// column modes: A(m..m+7, k)
__device__ __forceinline__ const uint16_t *a_col8(const GemmArgs &g, int m, int k, int kz1) {
  if (k >= kz1 || m + 8 > g.M || (g.m_ones >= m && g.m_ones < m + 8)) return nullptr;
  if (g.a_mode == 2) return (g.lda1 & 7) ? nullptr : aligned8(g.A1 + (size_t)k * g.lda1 + m);
  if (m + 8 <= g.split) return (g.lda1 & 7) ? nullptr : aligned8(g.A1 + (size_t)k * g.lda1 + m);
  if (m >= g.split) return (g.lda2 & 7) ? nullptr : aligned8(g.A2 + (size_t)k * g.lda2 + (m - g.split));
  return nullptr;
}

__device__ __forceinline__ void unpack8(const uint4 v, uint16_t h[8]) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    h[2 * j] = (uint16_t)(w[j] & 0xffffu);
    h[2 * j + 1] = (uint16_t)(w[j] >> 16);
  }
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][BKP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][BKP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kz0 = blockIdx.z * g.k_chunk, kz1 = min(g.K, kz0 + g.k_chunk);
  const bool a_rowwise = g.a_mode <= 1 || g.a_mode == 4;
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
  for (int k0 = kz0; k0 < kz1; k0 += BK) {
    // A tile (64 x 32): each thread moves 8 elements along the contiguous axis
    if (g.a_mode == 4 && k0 >= g.split) {
      // gathered half of a message-passing layer: 8 channels of one row,
      // summed over its neighbours in FP32, in neighbour order
      const int r = tid >> 2, k8 = (tid & 3) * 8;
      const int m = m0 + r, kc = k0 + k8 - g.split;
      const uint16_t *h0 = g.A1 + kc;
      if (m < g.M && k0 + k8 + 8 <= kz1 && !(g.lda1 & 7) && aligned8(h0)) {
        const uint8_t *nb = g.nbr + (size_t)g.node_atom[m] * kMaxDeg;
        const int g0 = g.node_g0[m];
        float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (int d = 0; d < kMaxDeg && nb[d] != 0xff; ++d) {
          uint16_t h[8];
          unpack8(*reinterpret_cast<const uint4 *>(h0 + (size_t)(g0 + nb[d]) * g.lda1), h);
#pragma unroll
          for (int j = 0; j < 8; ++j) acc[j] += bf2f(h[j]);
        }
        uint16_t o[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = f2bf(acc[j]);
        const uint4 packed = {(uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16),
                              (uint32_t)o[4] | ((uint32_t)o[5] << 16), (uint32_t)o[6] | ((uint32_t)o[7] << 16)};
        *reinterpret_cast<uint4 *>(&As[r][k8]) = packed;
        if (g.Mout && blockIdx.x == 0) *reinterpret_cast<uint4 *>(g.Mout + (size_t)m * kW + kc) = packed;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint16_t v = (m < g.M && k0 + k8 + j < kz1) ? gemm_a(g, m, k0 + k8 + j) : (uint16_t)0;
          As[r][k8 + j] = v;
          if (g.Mout && blockIdx.x == 0 && m < g.M && k0 + k8 + j < kz1) g.Mout[(size_t)m * kW + kc + j] = v;
        }
      }
    } else if (a_rowwise) {
      const int r = tid >> 2, k8 = (tid & 3) * 8;
      const int m = m0 + r, k = k0 + k8;
      const uint16_t *src = a_row8(g, m, k, kz1);
      if (src) {
        *reinterpret_cast<uint4 *>(&As[r][k8]) = *reinterpret_cast<const uint4 *>(src);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) As[r][k8 + j] = (m < g.M && k + j < kz1) ? gemm_a(g, m, k + j) : (uint16_t)0;
      }
    } else {
      const int kk = tid >> 3, m8 = (tid & 7) * 8;
      const int m = m0 + m8, k = k0 + kk;
      const uint16_t *src = a_col8(g, m, k, kz1);
      if (src) {
        uint16_t h[8];
        unpack8(*reinterpret_cast<const uint4 *>(src), h);
#pragma unroll
        for (int j = 0; j < 8; ++j) As[m8 + j][kk] = h[j];
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) As[m8 + j][kk] = (m + j < g.M && k < kz1) ? gemm_a(g, m + j, k) : (uint16_t)0;
      }
    }
    // B tile (32 x 64), stored n-major
    if (g.b_mode == 0) {   // B[k * ldb + n]: contiguous along n
      const int kk = tid >> 3, n8 = (tid & 7) * 8;
      const int n = n0 + n8, k = k0 + kk;
      const uint16_t *src =
          (k < kz1 && n + 8 <= g.N && !(g.ldb & 7)) ? aligned8(g.B + (size_t)k * g.ldb + n) : nullptr;
      if (src) {
        uint16_t h[8];
        unpack8(*reinterpret_cast<const uint4 *>(src), h);
#pragma unroll
        for (int j = 0; j < 8; ++j) Bs[n8 + j][kk] = h[j];
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          Bs[n8 + j][kk] = (k < kz1 && n + j < g.N) ? g.B[(size_t)k * g.ldb + n + j] : (uint16_t)0;
      }
    } else {               // B[n * ldb + k]: contiguous along k
      const int nn = tid >> 2, k8 = (tid & 3) * 8;
      const int n = n0 + nn, k = k0 + k8;
      const uint16_t *src =
          (n < g.N && k + 8 <= kz1 && !(g.ldb & 7)) ? aligned8(g.B + (size_t)n * g.ldb + k) : nullptr;
      if (src) {
        *reinterpret_cast<uint4 *>(&Bs[nn][k8]) = *reinterpret_cast<const uint4 *>(src);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          Bs[nn][k8 + j] = (n < g.N && k + j < kz1) ? g.B[(size_t)n * g.ldb + k + j] : (uint16_t)0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < BK; s += 16) {
      const int kk = s + (lane >> 5) * 8;
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&As[wm * 32 + (lane & 31)][kk]);
      const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 32 + (lane & 31)][kk]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = m0 + wm * 32 + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
    const int col = n0 + wn * 32 + (lane & 31);
    if (row >= g.M || col >= g.N) continue;
    float v = acc[i];
    if (g.part) {
      g.part[((size_t)blockIdx.z * g.M + row) * g.N + col] = v;
      continue;
    }
    if (g.bias) v += g.bias[col];
    if (g.relu) v = fmaxf(v, 0.0f);
    if (g.mask && !(bf2f(g.mask[(size_t)row * g.ldm + col]) > 0.0f)) v = 0.0f;
    if (g.C32) g.C32[(size_t)row * g.ldc32 + col] = v;
    if (g.C16) g.C16[(size_t)row * g.ldc16 + col] = f2bf(v);
  }
}

// sum of split-K partials in chunk order
__global__ void k_reduce_parts(const float *part, int Z, size_t MN, float *out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MN) return;
  float s = 0.0f;
  for (int z = 0; z < Z; ++z) s += part[(size_t)z * MN + i];
  out[i] = s;
}

// ---------------------------------------------------------------------------
// graph kernels (minibatch node layout: the nodes of graph b are
// [gstart[b], gstart[b+1]); node m is atom node_atom[m] of the batch)
// ---------------------------------------------------------------------------
struct GraphArgs {
  const int *node_atom;   // [Nn] batch atom index
  const int *node_g0;     // [Nn] first node of the node's graph
  const int *node_graph;  // [Nn] graph of the node
  const int *gstart;      // [B+1]
  const uint8_t *nbr;     // batch [atoms][8] local neighbour indices
  int Nn, B;
};

// rows of the batch features for the minibatch nodes
__global__ void k_gather_x(GraphArgs G, const uint16_t *X, uint16_t *Xmb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)G.Nn * kFeat) return;
  const int m = (int)(i / kFeat), c = (int)(i % kFeat);
  Xmb[i] = X[(size_t)G.node_atom[m] * kFeat + c];
}

// M[m] = r(sum over bonded neighbours of H); at most 8 BF16 terms, summed in FP32
// dP_prev[m] = [H_prev > 0] * r(dHM[m, :128] + sum over neighbours of dHM[., 128:])
__global__ void k_neighbour_bwd(GraphArgs G, const uint16_t *dHM, const uint16_t *Hprev, uint16_t *dP) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)G.Nn * kW) return;
  const int m = (int)(i / kW), c = (int)(i % kW);
  const uint8_t *nb = G.nbr + (size_t)G.node_atom[m] * kMaxDeg;
  float s = bf2f(dHM[(size_t)m * 2 * kW + c]);
  for (int d = 0; d < kMaxDeg && nb[d] != 0xff; ++d)
    s += bf2f(dHM[(size_t)(G.node_g0[m] + nb[d]) * 2 * kW + kW + c]);
  dP[i] = bf2f(Hprev[i]) > 0.0f ? f2bf(s) : (uint16_t)0;
}

// g[b] = r(sum of H over the graph's nodes).  The sum of up to 128 BF16
// values is exact in FP64, so its rounding (FP64 -> FP32 -> BF16) does not
// depend on the summation order.
__global__ void k_pool(GraphArgs G, const uint16_t *H, uint16_t *gp) {
  const int b = blockIdx.x, c = threadIdx.x;
  double s = 0.0;
  for (int m = G.gstart[b]; m < G.gstart[b + 1]; ++m) s += (double)bf2f(H[(size_t)m * kW + c]);
  gp[(size_t)b * kW + c] = f2bf((float)s);
}

// dP3[m] = [H3 > 0] * dg[graph(m)]
__global__ void k_pool_bwd(GraphArgs G, const uint16_t *dg, const uint16_t *H, uint16_t *dP) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)G.Nn * kW) return;
  const int m = (int)(i / kW), c = (int)(i % kW);
  dP[i] = bf2f(H[i]) > 0.0f ? dg[(size_t)G.node_graph[m] * kW + c] : (uint16_t)0;
}

// p[b] = z2[b] . U3 + c3 (FP32, j ascending): one wavefront per graph
__global__ void k_head(const uint16_t *z2, const uint16_t *U3, const float *c3, int B, float *p) {
  const int b = blockIdx.x, lane = threadIdx.x;
  if (b >= B) return;
  float s = 0.0f;
  for (int j = lane; j < kH; j += 64) s += bf2f(z2[(size_t)b * kH + j]) * bf2f(U3[j]);
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) p[b] = s + c3[0];
}

// loss and dL/dp over one minibatch (single work-group, fixed-order sums)
__global__ __launch_bounds__(256) void k_loss(const float *p, const float *y, int B, float lam, float tau,
                                              float *loss_out, float *dp) {
  __shared__ float red[256];
  __shared__ float npairs_s;
  const int t = threadIdx.x;
  float cnt = 0.0f;
  for (int i = t; i < B; i += 256)
    for (int j = 0; j < B; ++j) cnt += y[i] < y[j] ? 1.0f : 0.0f;
  red[t] = cnt;
  __syncthreads();
  if (t == 0) {
    float s = 0.0f;
    for (int k = 0; k < 256; ++k) s += red[k];
    npairs_s = s;
  }
  __syncthreads();
  const float np = npairs_s;
  const float wr = (np > 0.0f && lam != 0.0f) ? lam / np : 0.0f;
  float lsum = 0.0f;
  for (int i = t; i < B; i += 256) {
    const float d = p[i] - y[i];
    float gi = 2.0f * d / B;
    float li = d * d / B;
    if (wr != 0.0f) {
      for (int j = 0; j < B; ++j) {
        if (y[i] < y[j]) {
          const float z = (p[i] - p[j]) / tau;
          li += wr * (fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))));
          gi += wr / tau / (1.0f + expf(-z));
        }
        if (y[j] < y[i]) {
          const float z = (p[j] - p[i]) / tau;
          gi -= wr / tau / (1.0f + expf(-z));
        }
      }
    }
    dp[i] = gi;
    lsum += li;
  }
  red[t] = lsum;
  __syncthreads();
  if (t == 0) {
    float s = 0.0f;
    for (int k = 0; k < 256; ++k) s += red[k];
    *loss_out = s;
  }
}

// head backward: dz2 = [z2 > 0] r(dp U3); dU3 = z2^T dp; dc3 = sum dp
__global__ void k_head_bwd(const uint16_t *z2, const uint16_t *U3, const float *dp, int B, uint16_t *dz2, float *dU3,
                           float *dc3) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < kH) {
    float s = 0.0f;
    for (int b = 0; b < B; ++b) {
      const float z = bf2f(z2[(size_t)b * kH + j]);
      s += z * dp[b];
      dz2[(size_t)b * kH + j] = z > 0.0f ? f2bf(dp[b] * bf2f(U3[j])) : (uint16_t)0;
    }
    dU3[j] = s;
  }
  if (j == 0) {
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += dp[b];
    dc3[0] = s;
  }
}

__global__ void k_adam(float *w, const float *gr, float *m, float *v, size_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t *wbf) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wbf[i] = f2bf(wi);
}

__global__ void k_cast(const float *w, size_t n, uint16_t *wbf) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wbf[i] = f2bf(w[i]);
}

// standardised prediction -> label scale
__global__ void k_unscale(const float *p, int n, float mean, float sd, float *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = mean + sd * p[i];
}


inline unsigned nblk(size_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace
}  // namespace ad

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace ad;

namespace {

struct Offs {
  size_t W[kLayers + 1], b[kLayers + 1], U1, c1, U2, c2, U3, c3, total;
};

Offs make_offs() {
  Offs o;
  size_t p = 0;
  o.W[0] = p;
  p += (size_t)kFeat * kW;
  o.b[0] = p;
  p += kW;
  for (int l = 1; l <= kLayers; ++l) {
    o.W[l] = p;
    p += (size_t)2 * kW * kW;
    o.b[l] = p;
    p += kW;
  }
  o.U1 = p;
  p += (size_t)kW * kH;
  o.c1 = p;
  p += kH;
  o.U2 = p;
  p += (size_t)kH * kH;
  o.c2 = p;
  p += kH;
  o.U3 = p;
  p += kH;
  o.c3 = p;
  p += 1;
  o.total = p;
  return o;
}

}  // namespace

struct ad_prescreen {
  ad_ctx *ctx = nullptr;
  Offs o;
  ad_prescreen_cfg cfg;
  float *w = nullptr, *gr = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wbf = nullptr;
  double mean = 0.0, sd = 1.0;
  int64_t step = 0;
  // grow-only device buffers: activations, and node layouts + labels + losses
  char *work = nullptr;
  size_t work_bytes = 0;
  char *plan = nullptr;
  size_t plan_bytes = 0;
};

namespace {

#define PS_TRY(ctx, expr)                                    \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return (ctx)->hip_fail(_e, #expr); \
  } while (0)

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// one minibatch: node layout (device), activations (device workspace)
struct MB {
  int B = 0, Nn = 0;
  const int *node_atom, *node_g0, *node_graph, *gstart;
  uint16_t *Xmb, *H[kLayers + 1], *M[kLayers + 1], *g, *z1, *z2, *dz1, *dz2, *dg, *dP, *dP2, *dHM;
  float *p, *dp, *part;
  const float *y;   // standardised labels (training)
  float *loss;      // where the loss goes (training)
  size_t part_floats;
};

constexpr int kSplitRows = 2048;   // nodes per split-K chunk of a weight gradient

// Host node layout of minibatches: nodes of graph i of a minibatch are
// [gstart[i], gstart[i+1]) in minibatch numbering; node_atom maps a node to
// its batch atom.  Several minibatches are laid out back to back.
struct Plan {
  std::vector<int> na, ng0, ngr, gst;   // per node (3) and per minibatch (B + 1 each)
  std::vector<int> node_off, nn;        // per minibatch: first node, node count
  std::vector<float> y;                 // labels, B per minibatch
  int B = 0, max_nn = 0;
  void add(const ad_batch *b, const int *sel, int B_, const float *ys) {
    B = B_;
    node_off.push_back((int)na.size());
    int acc = 0;
    for (int i = 0; i < B_; ++i) {
      const LigDesc &d = b->lig_host[sel[i]];
      gst.push_back(acc);
      for (int a = 0; a < d.n_atoms; ++a) {
        na.push_back(d.atom_off + a);
        ng0.push_back(acc);
        ngr.push_back(i);
      }
      acc += d.n_atoms;
    }
    gst.push_back(acc);
    nn.push_back(acc);
    max_nn = std::max(max_nn, acc);
    if (ys) y.insert(y.end(), ys, ys + B_);
  }
  int steps() const { return (int)nn.size(); }
};

// device copy of a plan; returns pointers through `base`
struct PlanDev {
  int *na, *ng0, *ngr, *gst;
  float *y, *loss;
};

int upload_plan(ad_prescreen *ps, const Plan &P, PlanDev *D) {
  ad_ctx *c = ps->ctx;
  const size_t n = P.na.size(), ng = P.gst.size(), ny = P.y.size(), ns = (size_t)P.steps();
  const size_t sz = 3 * al(n * 4 + 4) + al(ng * 4) + al(ny * 4 + 4) + al(ns * 4);
  if (ps->plan_bytes < sz) {
    hipStreamSynchronize(c->stream);
    if (ps->plan) hipFree(ps->plan);
    ps->plan = nullptr;
    ps->plan_bytes = 0;
    if (hipMalloc(&ps->plan, sz) != hipSuccess) return c->fail(AD_E_OOM, "cannot allocate pre-screen batch layout");
    ps->plan_bytes = sz;
  }
  char *q = ps->plan;
  auto take = [&](size_t bytes) {
    char *r = q;
    q += al(bytes);
    return r;
  };
  D->na = (int *)take(n * 4 + 4);
  D->ng0 = (int *)take(n * 4 + 4);
  D->ngr = (int *)take(n * 4 + 4);
  D->gst = (int *)take(ng * 4);
  D->y = (float *)take(ny * 4 + 4);
  D->loss = (float *)take(ns * 4);
  // pageable host memory: the copies complete before the calls return
  PS_TRY(c, hipMemcpy(D->na, P.na.data(), n * 4, hipMemcpyHostToDevice));
  PS_TRY(c, hipMemcpy(D->ng0, P.ng0.data(), n * 4, hipMemcpyHostToDevice));
  PS_TRY(c, hipMemcpy(D->ngr, P.ngr.data(), n * 4, hipMemcpyHostToDevice));
  PS_TRY(c, hipMemcpy(D->gst, P.gst.data(), ng * 4, hipMemcpyHostToDevice));
  if (ny) PS_TRY(c, hipMemcpy(D->y, P.y.data(), ny * 4, hipMemcpyHostToDevice));
  return AD_OK;
}

// activation workspace for B graphs and up to Nn nodes (grow-only)
int alloc_ws(ad_prescreen *ps, int B, int Nn, bool train, MB *mb) {
  ad_ctx *c = ps->ctx;
  // split-K partials: the largest of the node-reduced [(256+1) x 128] and
  // the graph-reduced [(256+1) x 256] weight (+ bias) gradients
  const size_t z_nodes = std::max(1, (Nn + kSplitRows - 1) / kSplitRows);
  const size_t z_graphs = std::max(1, (B + kSplitRows - 1) / kSplitRows);
  const size_t part_floats = std::max(z_nodes * (2 * kW + 1) * kW, z_graphs * (kH + 1) * kH);
  const size_t hsz = al((size_t)Nn * kW * 2);
  size_t sz = al((size_t)Nn * kFeat * 2);
  sz += (kLayers + 1) * hsz + (train ? kLayers * hsz : 0);           // H, M (M: read by the backward pass only)
  sz += al((size_t)B * kW * 2) + 2 * al((size_t)B * kH * 2);        // g z1 z2
  sz += 2 * al((size_t)B * 4);                                       // p dp
  if (train) {
    sz += 2 * al((size_t)B * kH * 2) + al((size_t)B * kW * 2);      // dz1 dz2 dg
    sz += 2 * hsz + al((size_t)Nn * 2 * kW * 2);                     // dP dP2 dHM
    sz += al(part_floats * 4);
  }
  if (ps->work_bytes < sz) {
    hipStreamSynchronize(c->stream);
    if (ps->work) hipFree(ps->work);
    ps->work = nullptr;
    ps->work_bytes = 0;
    if (hipMalloc(&ps->work, sz) != hipSuccess) return c->fail(AD_E_OOM, "cannot allocate pre-screen workspace");
    ps->work_bytes = sz;
  }
  char *q = ps->work;
  auto take = [&](size_t n) {
    char *r = q;
    q += al(n);
    return r;
  };
  mb->Xmb = (uint16_t *)take((size_t)Nn * kFeat * 2);
  for (int l = 0; l <= kLayers; ++l) mb->H[l] = (uint16_t *)take((size_t)Nn * kW * 2);
  mb->M[0] = nullptr;
  for (int l = 1; l <= kLayers; ++l) mb->M[l] = train ? (uint16_t *)take((size_t)Nn * kW * 2) : nullptr;
  mb->g = (uint16_t *)take((size_t)B * kW * 2);
  mb->z1 = (uint16_t *)take((size_t)B * kH * 2);
  mb->z2 = (uint16_t *)take((size_t)B * kH * 2);
  mb->p = (float *)take((size_t)B * 4);
  mb->dp = (float *)take((size_t)B * 4);
  if (train) {
    mb->dz1 = (uint16_t *)take((size_t)B * kH * 2);
    mb->dz2 = (uint16_t *)take((size_t)B * kH * 2);
    mb->dg = (uint16_t *)take((size_t)B * kW * 2);
    mb->dP = (uint16_t *)take((size_t)Nn * kW * 2);
    mb->dP2 = (uint16_t *)take((size_t)Nn * kW * 2);
    mb->dHM = (uint16_t *)take((size_t)Nn * 2 * kW * 2);
    mb->part = (float *)take(part_floats * 4);
    mb->part_floats = part_floats;
  }
  return AD_OK;
}

// minibatch s of an uploaded plan
void bind_step(const Plan &P, const PlanDev &D, int s, MB *mb) {
  mb->B = P.B;
  mb->Nn = P.nn[s];
  const int o = P.node_off[s];
  mb->node_atom = D.na + o;
  mb->node_g0 = D.ng0 + o;
  mb->node_graph = D.ngr + o;
  mb->gstart = D.gst + (size_t)s * (P.B + 1);
  mb->y = D.y + (size_t)s * P.B;
  mb->loss = D.loss + s;
}

GemmArgs gemm_base(int M, int N, int K) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.M = M;
  g.N = N;
  g.K = K;
  g.k_chunk = K;
  g.m_ones = -1;
  return g;
}

hipError_t gemm(const GemmArgs &g, hipStream_t s, int zsplit = 1) {
  dim3 grid(nblk(g.N, BN), nblk(g.M, BM), zsplit);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// weight gradient and bias gradient in one GEMM: out[0..Kin) = A^T . D and
// out[Kin] = 1^T . D (the bias follows its weight matrix in the parameter
// vector), the reduction over R rows split into 2,048-row chunks summed in
// chunk order
hipError_t wgrad(const GemmArgs &gbase, int R, float *part, size_t part_floats, float *out, hipStream_t s) {
  GemmArgs g = gbase;
  g.m_ones = g.M;
  g.M += 1;
  const int Z = std::max(1, (R + kSplitRows - 1) / kSplitRows);
  g.k_chunk = kSplitRows;
  g.part = part;
  if ((size_t)Z * g.M * g.N > part_floats) return hipErrorInvalidValue;
  hipError_t e = gemm(g, s, Z);
  if (e != hipSuccess) return e;
  const size_t MN = (size_t)g.M * g.N;
  hipLaunchKernelGGL(k_reduce_parts, dim3(nblk(MN)), dim3(256), 0, s, part, Z, MN, out);
  return hipGetLastError();
}

int forward(ad_prescreen *ps, const ad_batch *b, MB &mb, bool keep_m) {
  ad_ctx *c = ps->ctx;
  hipStream_t s = c->stream;
  const Offs &o = ps->o;
  GraphArgs G{mb.node_atom, mb.node_g0, mb.node_graph, mb.gstart, b->ps_nbr, mb.Nn, mb.B};
  hipLaunchKernelGGL(k_gather_x, dim3(nblk((size_t)mb.Nn * kFeat)), dim3(256), 0, s, G, b->ps_x, mb.Xmb);
  GemmArgs g = gemm_base(mb.Nn, kW, kFeat);
  g.a_mode = 0;
  g.A1 = mb.Xmb;
  g.lda1 = kFeat;
  g.B = ps->wbf + o.W[0];
  g.ldb = kW;
  g.bias = ps->w + o.b[0];
  g.relu = 1;
  g.C16 = mb.H[0];
  g.ldc16 = kW;
  PS_TRY(c, gemm(g, s));
  for (int l = 1; l <= kLayers; ++l) {
    // one launch per layer: the neighbour gather runs in the GEMM's A loader
    // (M = r(A H) is stored only when a backward pass will read it)
    g = gemm_base(mb.Nn, kW, 2 * kW);
    g.a_mode = 4;
    g.split = kW;
    g.A1 = mb.H[l - 1];
    g.lda1 = kW;
    g.node_atom = mb.node_atom;
    g.node_g0 = mb.node_g0;
    g.nbr = b->ps_nbr;
    g.Mout = keep_m ? mb.M[l] : nullptr;
    g.B = ps->wbf + o.W[l];
    g.ldb = kW;
    g.bias = ps->w + o.b[l];
    g.relu = 1;
    g.C16 = mb.H[l];
    g.ldc16 = kW;
    PS_TRY(c, gemm(g, s));
  }
  hipLaunchKernelGGL(k_pool, dim3(mb.B), dim3(kW), 0, s, G, mb.H[kLayers], mb.g);
  g = gemm_base(mb.B, kH, kW);
  g.A1 = mb.g;
  g.lda1 = kW;
  g.B = ps->wbf + o.U1;
  g.ldb = kH;
  g.bias = ps->w + o.c1;
  g.relu = 1;
  g.C16 = mb.z1;
  g.ldc16 = kH;
  PS_TRY(c, gemm(g, s));
  g = gemm_base(mb.B, kH, kH);
  g.A1 = mb.z1;
  g.lda1 = kH;
  g.B = ps->wbf + o.U2;
  g.ldb = kH;
  g.bias = ps->w + o.c2;
  g.relu = 1;
  g.C16 = mb.z2;
  g.ldc16 = kH;
  PS_TRY(c, gemm(g, s));
  hipLaunchKernelGGL(k_head, dim3(mb.B), dim3(64), 0, s, mb.z2, ps->wbf + o.U3, ps->w + o.c3, mb.B, mb.p);
  PS_TRY(c, hipGetLastError());
  return AD_OK;
}

int backward(ad_prescreen *ps, const ad_batch *b, MB &mb) {
  ad_ctx *c = ps->ctx;
  hipStream_t s = c->stream;
  const Offs &o = ps->o;
  float *gr = ps->gr;
  GraphArgs G{mb.node_atom, mb.node_g0, mb.node_graph, mb.gstart, b->ps_nbr, mb.Nn, mb.B};
  hipLaunchKernelGGL(k_head_bwd, dim3(1), dim3(kH), 0, s, mb.z2, ps->wbf + o.U3, mb.dp, mb.B, mb.dz2, gr + o.U3,
                     gr + o.c3);
  // U2 and c2; dz1
  GemmArgs g = gemm_base(kH, kH, mb.B);
  g.a_mode = 2;
  g.A1 = mb.z1;
  g.lda1 = kH;
  g.B = mb.dz2;
  g.ldb = kH;
  PS_TRY(c, wgrad(g, mb.B, mb.part, mb.part_floats, gr + o.U2, s));
  g = gemm_base(mb.B, kH, kH);
  g.A1 = mb.dz2;
  g.lda1 = kH;
  g.b_mode = 1;
  g.B = ps->wbf + o.U2;
  g.ldb = kH;
  g.mask = mb.z1;
  g.ldm = kH;
  g.C16 = mb.dz1;
  g.ldc16 = kH;
  PS_TRY(c, gemm(g, s));
  // U1 and c1; dg
  g = gemm_base(kW, kH, mb.B);
  g.a_mode = 2;
  g.A1 = mb.g;
  g.lda1 = kW;
  g.B = mb.dz1;
  g.ldb = kH;
  PS_TRY(c, wgrad(g, mb.B, mb.part, mb.part_floats, gr + o.U1, s));
  g = gemm_base(mb.B, kW, kH);
  g.A1 = mb.dz1;
  g.lda1 = kH;
  g.b_mode = 1;
  g.B = ps->wbf + o.U1;
  g.ldb = kH;
  g.C16 = mb.dg;
  g.ldc16 = kW;
  PS_TRY(c, gemm(g, s));
  // pool backward, then the message-passing layers (W_l and b_l together)
  uint16_t *dP = mb.dP, *dPn = mb.dP2;
  hipLaunchKernelGGL(k_pool_bwd, dim3(nblk((size_t)mb.Nn * kW)), dim3(256), 0, s, G, mb.dg, mb.H[kLayers], dP);
  for (int l = kLayers; l >= 1; --l) {
    g = gemm_base(2 * kW, kW, mb.Nn);
    g.a_mode = 3;
    g.split = kW;
    g.A1 = mb.H[l - 1];
    g.lda1 = kW;
    g.A2 = mb.M[l];
    g.lda2 = kW;
    g.B = dP;
    g.ldb = kW;
    PS_TRY(c, wgrad(g, mb.Nn, mb.part, mb.part_floats, gr + o.W[l], s));
    g = gemm_base(mb.Nn, 2 * kW, kW);
    g.A1 = dP;
    g.lda1 = kW;
    g.b_mode = 1;
    g.B = ps->wbf + o.W[l];
    g.ldb = kW;
    g.C16 = mb.dHM;
    g.ldc16 = 2 * kW;
    PS_TRY(c, gemm(g, s));
    hipLaunchKernelGGL(k_neighbour_bwd, dim3(nblk((size_t)mb.Nn * kW)), dim3(256), 0, s, G, mb.dHM, mb.H[l - 1],
                       dPn);
    std::swap(dP, dPn);
  }
  g = gemm_base(kFeat, kW, mb.Nn);
  g.a_mode = 2;
  g.A1 = mb.Xmb;
  g.lda1 = kFeat;
  g.B = dP;
  g.ldb = kW;
  PS_TRY(c, wgrad(g, mb.Nn, mb.part, mb.part_floats, gr + o.W[0], s));
  PS_TRY(c, hipGetLastError());
  return AD_OK;
}

// forward, loss into mb.loss and dL/dp, backward (gradient into ps->gr)
int step_grad(ad_prescreen *ps, const ad_batch *b, MB &mb) {
  ad_ctx *c = ps->ctx;
  int rc = forward(ps, b, mb, true);
  if (rc) return rc;
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, c->stream, mb.p, mb.y, mb.B, (float)ps->cfg.lam,
                     (float)ps->cfg.tau, mb.loss, mb.dp);
  PS_TRY(c, hipGetLastError());
  return backward(ps, b, mb);
}

int check_ps(ad_prescreen *ps, const ad_batch *b, int n, const int *idx) {
  if (!ps || !ps->ctx) return AD_E_INVALID;   // null, or detached by ad_destroy
  ad_ctx *c = ps->ctx;
  if (!b || b->ctx != c) return c->fail(AD_E_INVALID, "bad batch");
  if (!b->ps_ok) return c->fail(AD_E_INVALID, "batch has atoms with more than 8 bonds (pre-screen limit)");
  if (n < 0) return c->fail(AD_E_INVALID, "n < 0");
  if (idx)
    for (int i = 0; i < n; ++i)
      if (idx[i] < 0 || idx[i] >= b->n_lig) return c->fail(AD_E_INVALID, "ligand index out of range");
  return AD_OK;
}

}  // namespace

extern "C" int ad_prescreen_create(ad_ctx *c, const ad_prescreen_cfg *cfg, uint64_t seed, ad_prescreen **out) {
  if (!c || !out) return AD_E_INVALID;
  *out = nullptr;
  ad_prescreen_cfg d;
  d.batch_size = 256;
  d.lr = 1e-3;
  d.lam = 1.0;
  d.tau = 0.5;
  d.beta1 = 0.9;
  d.beta2 = 0.999;
  d.eps = 1e-8;
  d.label_max = HUGE_VAL;
  if (cfg) d = *cfg;
  if (d.batch_size < 2 || d.batch_size > 4096 || !(d.lr > 0) || !(d.tau > 0) || !(d.lam >= 0) ||
      !(d.beta1 >= 0 && d.beta1 < 1) || !(d.beta2 >= 0 && d.beta2 < 1) || !(d.eps > 0) || std::isnan(d.label_max))
    return c->fail(AD_E_INVALID, "bad pre-screen configuration");
  hipSetDevice(c->device);
  ad_prescreen *ps = new ad_prescreen();
  ps->ctx = c;
  ps->cfg = d;
  ps->o = make_offs();
  const size_t P = ps->o.total;
  if (hipMalloc(&ps->w, P * 4) != hipSuccess || hipMalloc(&ps->gr, P * 4) != hipSuccess ||
      hipMalloc(&ps->m, P * 4) != hipSuccess || hipMalloc(&ps->v, P * 4) != hipSuccess ||
      hipMalloc(&ps->wbf, P * 2) != hipSuccess) {
    ad_prescreen_destroy(ps);
    return c->fail(AD_E_OOM, "cannot allocate pre-screen parameters");
  }
  // He-uniform weights, zero biases (host RNG seeded by `seed`)
  std::vector<float> w(P, 0.0f);
  std::mt19937_64 rng(seed);
  auto fill = [&](size_t off, int fan_in, size_t n) {
    std::uniform_real_distribution<double> u(-std::sqrt(6.0 / fan_in), std::sqrt(6.0 / fan_in));
    for (size_t i = 0; i < n; ++i) w[off + i] = (float)u(rng);
  };
  const Offs &o = ps->o;
  fill(o.W[0], kFeat, (size_t)kFeat * kW);
  for (int l = 1; l <= kLayers; ++l) fill(o.W[l], 2 * kW, (size_t)2 * kW * kW);
  fill(o.U1, kW, (size_t)kW * kH);
  fill(o.U2, kH, (size_t)kH * kH);
  fill(o.U3, kH, kH);
  // a small output layer starts the predictions near the label mean
  for (int i = 0; i < kH; ++i) w[o.U3 + i] *= 0.01f;
  int rc = ad_prescreen_set_params(ps, w.data());
  if (rc) {
    ad_prescreen_destroy(ps);
    return rc;
  }
  register_prescreen(c, ps);
  *out = ps;
  return AD_OK;
}

void register_prescreen(ad_ctx *c, ad_prescreen *ps) {
  std::lock_guard<std::mutex> lk(c->child_mu);
  c->prescreens.insert(ps);
}

// Frees the pre-screen's device memory and detaches it from its context
// (called by ad_destroy for pre-screens still alive, under the context lock).
void prescreen_release(ad_prescreen *ps) {
  if (!ps->ctx) return;
  hipSetDevice(ps->ctx->device);
  hipStreamSynchronize(ps->ctx->stream);
  void *bufs[] = {ps->w, ps->gr, ps->m, ps->v, ps->wbf, ps->work, ps->plan};
  for (void *p : bufs)
    if (p) hipFree(p);
  ps->w = ps->gr = ps->m = ps->v = nullptr;
  ps->wbf = nullptr;
  ps->work = ps->plan = nullptr;
  ps->work_bytes = ps->plan_bytes = 0;
  ps->ctx = nullptr;
}

extern "C" void ad_prescreen_destroy(ad_prescreen *ps) {
  if (!ps) return;
  if (ps->ctx) {
    ad_ctx *c = ps->ctx;
    std::lock_guard<std::mutex> lk(c->child_mu);
    c->prescreens.erase(ps);
    prescreen_release(ps);
  }
  delete ps;
}

extern "C" int ad_prescreen_n_params(void) { return (int)make_offs().total; }

extern "C" int ad_prescreen_set_params(ad_prescreen *ps, const float *params) {
  if (!ps || !ps->ctx || !params) return AD_E_INVALID;
  ad_ctx *c = ps->ctx;
  const size_t P = ps->o.total;
  for (size_t i = 0; i < P; ++i)
    if (!std::isfinite(params[i])) return c->fail(AD_E_INVALID, "non-finite parameter");
  hipSetDevice(c->device);
  PS_TRY(c, hipMemcpyAsync(ps->w, params, P * 4, hipMemcpyHostToDevice, c->stream));
  PS_TRY(c, hipMemsetAsync(ps->m, 0, P * 4, c->stream));
  PS_TRY(c, hipMemsetAsync(ps->v, 0, P * 4, c->stream));
  hipLaunchKernelGGL(k_cast, dim3(nblk(P)), dim3(256), 0, c->stream, ps->w, P, ps->wbf);
  PS_TRY(c, hipGetLastError());
  PS_TRY(c, hipStreamSynchronize(c->stream));
  ps->step = 0;
  return AD_OK;
}

extern "C" int ad_prescreen_get_params(ad_prescreen *ps, float *params) {
  if (!ps || !ps->ctx || !params) return AD_E_INVALID;
  ad_ctx *c = ps->ctx;
  hipSetDevice(c->device);
  PS_TRY(c, hipMemcpyAsync(params, ps->w, ps->o.total * 4, hipMemcpyDeviceToHost, c->stream));
  PS_TRY(c, hipStreamSynchronize(c->stream));
  return AD_OK;
}

extern "C" int ad_prescreen_set_scale(ad_prescreen *ps, double mean, double sd) {
  if (!ps || !std::isfinite(mean) || !(sd > 0) || !std::isfinite(sd)) return AD_E_INVALID;
  ps->mean = mean;
  ps->sd = sd;
  return AD_OK;
}

extern "C" int ad_prescreen_get_scale(ad_prescreen *ps, double *mean, double *sd) {
  if (!ps) return AD_E_INVALID;
  if (mean) *mean = ps->mean;
  if (sd) *sd = ps->sd;
  return AD_OK;
}

extern "C" int ad_prescreen_predict(ad_prescreen *ps, const ad_batch *b, int n, const int *lig_idx, float *scores) {
  int rc = check_ps(ps, b, n, lig_idx);
  if (rc) return rc;
  if (n == 0) return AD_OK;
  if (!scores) return ps->ctx->fail(AD_E_INVALID, "null scores");
  ad_ctx *c = ps->ctx;
  hipSetDevice(c->device);
  // all chunks of up to 2,048 graphs in one layout upload
  const int chunk = 2048;
  Plan P;
  std::vector<int> sel(chunk);
  std::vector<int> chunk_n;
  for (int s0 = 0; s0 < n; s0 += chunk) {
    const int B = std::min(chunk, n - s0);
    for (int i = 0; i < B; ++i) sel[i] = lig_idx ? lig_idx[s0 + i] : s0 + i;
    P.add(b, sel.data(), B, nullptr);
    P.gst.resize(P.gst.size() + (size_t)(chunk - B));   // uniform stride of chunk + 1 per step
    chunk_n.push_back(B);
  }
  P.B = chunk;
  PlanDev D;
  rc = upload_plan(ps, P, &D);
  if (rc) return rc;
  MB mb;
  rc = alloc_ws(ps, chunk, P.max_nn, false, &mb);
  if (rc) return rc;
  float *out = mb.dp;   // unused in prediction: holds the rescaled scores
  for (int s = 0; s < P.steps(); ++s) {
    bind_step(P, D, s, &mb);
    mb.B = chunk_n[s];
    rc = forward(ps, b, mb, false);
    if (rc) return rc;
    hipLaunchKernelGGL(k_unscale, dim3(nblk(mb.B)), dim3(256), 0, c->stream, mb.p, mb.B, (float)ps->mean,
                       (float)ps->sd, out);
    PS_TRY(c, hipMemcpyAsync(scores + (size_t)s * chunk, out, (size_t)mb.B * 4, hipMemcpyDeviceToHost, c->stream));
    PS_TRY(c, hipStreamSynchronize(c->stream));
  }
  return AD_OK;
}

extern "C" int ad_prescreen_grad(ad_prescreen *ps, const ad_batch *b, int n, const int *lig_idx, const float *labels,
                                 float *loss, float *grad, float *pred_std) {
  int rc = check_ps(ps, b, n, lig_idx);
  if (rc) return rc;
  ad_ctx *c = ps->ctx;
  if (n < 2 || n > 4096 || !labels) return c->fail(AD_E_INVALID, "need 2..4096 labelled ligands");
  hipSetDevice(c->device);
  std::vector<int> sel(n);
  std::vector<float> ys(n);
  for (int i = 0; i < n; ++i) {
    sel[i] = lig_idx ? lig_idx[i] : i;
    ys[i] = (float)((std::min((double)labels[i], ps->cfg.label_max) - ps->mean) / ps->sd);
  }
  Plan P;
  P.add(b, sel.data(), n, ys.data());
  PlanDev D;
  rc = upload_plan(ps, P, &D);
  if (rc) return rc;
  MB mb;
  rc = alloc_ws(ps, n, P.max_nn, true, &mb);
  if (rc) return rc;
  bind_step(P, D, 0, &mb);
  rc = step_grad(ps, b, mb);
  if (rc) return rc;
  if (loss) PS_TRY(c, hipMemcpyAsync(loss, mb.loss, 4, hipMemcpyDeviceToHost, c->stream));
  if (grad) PS_TRY(c, hipMemcpyAsync(grad, ps->gr, ps->o.total * 4, hipMemcpyDeviceToHost, c->stream));
  if (pred_std) PS_TRY(c, hipMemcpyAsync(pred_std, mb.p, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  PS_TRY(c, hipStreamSynchronize(c->stream));
  return AD_OK;
}

extern "C" int ad_prescreen_train(ad_prescreen *ps, const ad_batch *b, int n, const int *lig_idx,
                                  const float *labels, int epochs, uint64_t seed, float *loss_curve) {
  int rc = check_ps(ps, b, n, lig_idx);
  if (rc) return rc;
  ad_ctx *c = ps->ctx;
  if (n < 2 || epochs < 0 || !labels) return c->fail(AD_E_INVALID, "need >= 2 labelled ligands, epochs >= 0");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(labels[i])) return c->fail(AD_E_INVALID, "non-finite label");
  hipSetDevice(c->device);
  // clip, then standardise the labels
  std::vector<double> yc(n);
  for (int i = 0; i < n; ++i) yc[i] = std::min((double)labels[i], ps->cfg.label_max);
  double mu = 0, var = 0;
  for (int i = 0; i < n; ++i) mu += yc[i];
  mu /= n;
  for (int i = 0; i < n; ++i) var += (yc[i] - mu) * (yc[i] - mu);
  const double sd = std::sqrt(var / n) > 1e-12 ? std::sqrt(var / n) : 1.0;
  ps->mean = mu;
  ps->sd = sd;
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  const int Bsz = std::min(ps->cfg.batch_size, n);
  std::vector<int> sel(Bsz);
  std::vector<float> ys(Bsz);
  std::mt19937_64 rng(seed);
  const size_t Pn = ps->o.total;
  for (int ep = 0; ep < epochs; ++ep) {
    // the epoch's minibatches (full ones only) laid out and uploaded at once;
    // the steps then run back to back on the stream, losses stay on the device
    std::shuffle(order.begin(), order.end(), rng);
    Plan P;
    for (int s0 = 0; s0 + Bsz <= n; s0 += Bsz) {
      for (int i = 0; i < Bsz; ++i) {
        const int k = order[s0 + i];
        sel[i] = lig_idx ? lig_idx[k] : k;
        ys[i] = (float)((yc[k] - mu) / sd);
      }
      P.add(b, sel.data(), Bsz, ys.data());
    }
    const int steps = P.steps();
    if (steps == 0) {
      if (loss_curve) loss_curve[ep] = 0.0f;
      continue;
    }
    PlanDev D;
    rc = upload_plan(ps, P, &D);
    if (rc) return rc;
    MB mb;
    rc = alloc_ws(ps, Bsz, P.max_nn, true, &mb);
    if (rc) return rc;
    for (int s = 0; s < steps; ++s) {
      bind_step(P, D, s, &mb);
      rc = step_grad(ps, b, mb);
      if (rc) return rc;
      ps->step += 1;
      const float c1 = 1.0f - (float)std::pow(ps->cfg.beta1, (double)ps->step);
      const float c2 = 1.0f - (float)std::pow(ps->cfg.beta2, (double)ps->step);
      hipLaunchKernelGGL(k_adam, dim3(nblk(Pn)), dim3(256), 0, c->stream, ps->w, ps->gr, ps->m, ps->v, Pn,
                         (float)ps->cfg.lr, (float)ps->cfg.beta1, (float)ps->cfg.beta2, (float)ps->cfg.eps, c1, c2,
                         ps->wbf);
      PS_TRY(c, hipGetLastError());
    }
    std::vector<float> losses(steps);
    PS_TRY(c, hipMemcpyAsync(losses.data(), D.loss, (size_t)steps * 4, hipMemcpyDeviceToHost, c->stream));
    PS_TRY(c, hipStreamSynchronize(c->stream));
    double lsum = 0;
    for (float l : losses) lsum += l;
    if (loss_curve) loss_curve[ep] = (float)(lsum / steps);
  }
  return AD_OK;
}
