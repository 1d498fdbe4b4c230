// Pointwise warm-start network for CG on (I + tau L_s) u = f: a 4-layer MLP
// (16 -> 64 -> 64 -> 64 -> 1, tanh) evaluated and trained on the matrix cores
// with BF16 operands and FP32 accumulation.
//
// Layers are computed in transposed form, D[unit][node] = sum_k W[unit][k] H[k][node],
// with gfx950's v_mfma_f32_16x16x32_bf16 (A = 16 units x 32 inputs, B = 32
// inputs x 16 nodes).  Lane l holds D[unit = 4 (l/16) + r][node = l%16].  In a
// K-reduction MFMA lane l contributes 8 K values (slots i = 0..7) of row or
// column l%16, and A and B are paired slot by slot, so the assignment of input
// units to (l/16, i) is free as long as both operands use it.  The one chosen,
//   input k = 32 c + 16 (i/4) + 4 (l/16) + i%4   for K chunk c,
// puts in lane l exactly the D values it holds from two 16-unit blocks of the
// previous layer: activations stay in registers from layer to layer, and the
// BF16 weight copies are stored with their columns in that order, so that an
// A operand is one 16-byte load.  The first layer (16 inputs) fills slots
// 0..3 and leaves 4..7 zero.  Backward: the deltas propagate through W^T the
// same way; the weight gradients (K = nodes) take 32-node batches through
// LDS, [row][node] per layer.
//
// BF16 rounding happens exactly at the MFMA operands: W1..W3 (and their
// transposes), the layer inputs X, H1, H2 in the forward pass, the deltas and
// inputs in the backward GEMMs.  Biases, W4, the activations and all sums are
// FP32.  Parameters (FP32 master copy), offsets in floats:
//   W1 [64][16] @0, b1 @1024, W2 [64][64] @1088, b2 @5184, W3 [64][64] @5248,
//   b3 @9344, W4 [64] @9408, b4 @9472; total 9473.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "nfl_internal.h"

namespace nfl {

constexpr int MLP_NF = 16, MLP_H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 1024, OFF_W2 = 1088, OFF_B2 = 5184, OFF_W3 = 5248,
              OFF_B3 = 9344, OFF_W4 = 9408, OFF_B4 = 9472, MLP_NP = 9473;
// BF16 copies with permuted columns: W1 [64][32] (slots 4..7 of each lane
// group zero), W2, W3, W2^T, W3^T [64][64]
constexpr int BF_W1 = 0, BF_W2 = 2048, BF_W3 = 6144, BF_W2T = 10240, BF_W3T = 14336,
              MLP_NBF = 18432;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4m __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 bits, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// Column position of input unit k in a permuted 64-wide weight row: lane
// group g reads positions 32 c + 8 g .. + 7, i.e. units 32 c + 16 (i/4) + 4 g + i%4.
__host__ __device__ __forceinline__ int kpos(int k) {
  return (k & ~31) + 8 * ((k >> 2) & 3) + 4 * ((k >> 4) & 1) + (k & 3);
}

__device__ __forceinline__ float tanh_f(float x) {
  // tanh(x) = 1 - 2 / (e^{2x} + 1) with the hardware exp2 and reciprocal
  // (absolute error below 2^-21); for large |x| e is inf or 0 and the
  // reciprocal 0 or 1, so the result saturates at +-1 without a clamp
  const float e = __builtin_amdgcn_exp2f(x * 2.885390081777927f);   // 2 log2(e)
  return fmaf(-2.f, __builtin_amdgcn_rcpf(e + 1.f), 1.f);
}

__device__ __forceinline__ uint32_t pack2(float a, float b) {
  const bf16x2 r = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, r);
}

// B operand from two D-layout blocks: slots 0..3 from lo, 4..7 from hi
__device__ __forceinline__ bf16x8 pack8(const f32x4m &lo, const f32x4m &hi) {
  const uint4 w = make_uint4(pack2(lo[0], lo[1]), pack2(lo[2], lo[3]), pack2(hi[0], hi[1]),
                             pack2(hi[2], hi[3]));
  return __builtin_bit_cast(bf16x8, w);
}

__device__ __forceinline__ f32x4m mfma32(const bf16x8 &a, const bf16x8 &b, const f32x4m &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// A operand: row 16 ub + l%16, K chunk c of a permuted [rows][ld] bf16 matrix
__device__ __forceinline__ bf16x8 load_a(const uint16_t *__restrict__ w, int ld, int ub, int c,
                                        int lane) {
  const uint16_t *p = w + (16 * ub + (lane & 15)) * ld + 32 * c + 8 * (lane >> 4);
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

// Forward pass of 16 nodes (features in B layout: lane holds the 4 features
// 4*(l/16)..+3 of node l%16 in slots 0..3).  Outputs: the activations h1, h2,
// h3 (D layout, FP32) and the network output (valid in every lane for node l%16).
struct Acts {
  f32x4m h1[4], h2[4], h3[4];
  float out;
};

__device__ __forceinline__ void mlp_forward16(const uint16_t *__restrict__ wbf,
                                              const float *__restrict__ prm, const bf16x8 &xb,
                                              int lane, Acts &A) {
  const int q = lane >> 4;
  const f32x4m zero = {0.f, 0.f, 0.f, 0.f};
  // layer 1
#pragma unroll
  for (int ub = 0; ub < 4; ++ub) {
    f32x4m d = mfma32(load_a(wbf + BF_W1, 32, ub, 0, lane), xb, zero);
#pragma unroll
    for (int r = 0; r < 4; ++r) d[r] = tanh_f(d[r] + prm[OFF_B1 + 16 * ub + 4 * q + r]);
    A.h1[ub] = d;
  }
  // layers 2 and 3
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const f32x4m *hin = layer == 0 ? A.h1 : A.h2;
    f32x4m *hout = layer == 0 ? A.h2 : A.h3;
    const uint16_t *w = wbf + (layer == 0 ? BF_W2 : BF_W3);
    const float *bias = prm + (layer == 0 ? OFF_B2 : OFF_B3);
    const bf16x8 b0 = pack8(hin[0], hin[1]), b1 = pack8(hin[2], hin[3]);
#pragma unroll
    for (int ub = 0; ub < 4; ++ub) {
      f32x4m d = mfma32(load_a(w, 64, ub, 0, lane), b0, zero);
      d = mfma32(load_a(w, 64, ub, 1, lane), b1, d);
#pragma unroll
      for (int r = 0; r < 4; ++r) d[r] = tanh_f(d[r] + bias[16 * ub + 4 * q + r]);
      hout[ub] = d;
    }
  }
  // layer 4 (FP32 dot product over the 64 units)
  float part = 0.f;
#pragma unroll
  for (int ub = 0; ub < 4; ++ub)
#pragma unroll
    for (int r = 0; r < 4; ++r) part = fmaf(prm[OFF_W4 + 16 * ub + 4 * q + r], A.h3[ub][r], part);
  part += __shfl_xor(part, 16);
  part += __shfl_xor(part, 32);
  A.out = part + prm[OFF_B4];
}

// B operand of the first layer: the lane's 4 features, slots 4..7 zero
__device__ __forceinline__ bf16x8 pack_features(const float (&x)[4]) {
  const f32x4m lo = {x[0], x[1], x[2], x[3]}, z = {0.f, 0.f, 0.f, 0.f};
  return pack8(lo, z);
}

// ---------------------------------------------------------------------------
// Features of node i (sorted order): scaled position 4 v~ (|.| <= 1), own
// right-hand side f, degree / mean degree, one-hot class, zero padding.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float node_feature(const float4 &q, int nos, float f, float dn, int cls,
                                              int k) {
  const uint32_t cell = __float_as_uint(q.w);
  if (k < 3) {
    const float c = (float)(k == 0 ? (cell & 1023u) : k == 1 ? ((cell >> 10) & 1023u) : (cell >> 20));
    const float fr = k == 0 ? q.x : k == 1 ? q.y : q.z;
    return 4.f * ((c + fr) / (float)nos - 0.5f);
  }
  if (k == 3) return f;
  if (k == 4) return dn;
  return (k - 5 == cls) ? 1.f : 0.f;
}

// The BF16 weight copies staged in LDS once per block (36 KB; four blocks of
// four waves fit a CU): the A operands are then LDS reads, cheaper than
// re-reading them from the caches and, unlike holding them in registers,
// leaving room for four waves per SIMD to cover the MFMA -> tanh chains.
__device__ __forceinline__ void stage_weights(const uint16_t *__restrict__ wbf, uint4 *wl) {
  const uint4 *src = reinterpret_cast<const uint4 *>(wbf);
  for (int t = threadIdx.x; t < MLP_NBF / 8; t += blockDim.x) wl[t] = src[t];
  __syncthreads();
}

// Inference over all nodes (sorted order): u0[i] = net(features_i).
__global__ __launch_bounds__(256) void k_mlp_infer(const uint16_t *__restrict__ wbf,
                                                   const float *__restrict__ prm,
                                                   const float4 *__restrict__ pts,
                                                   const float *__restrict__ deg, float dinvmean,
                                                   const double *__restrict__ f_sorted, int cls,
                                                   int nos, int d, int64_t n,
                                                   double *__restrict__ u0) {
  __shared__ uint4 wl[MLP_NBF / 8];
  stage_weights(wbf, wl);
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int node = lane & 15, q = lane >> 4;
  for (int64_t b = wave; b * 16 < n; b += nw) {
    const int64_t i = b * 16 + node;
    const bool ok = i < n;
    float4 p = ok ? pts[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    if (d < 3) p.z = 0.f;
    if (d < 2) p.y = 0.f;
    const float f = ok ? (float)f_sorted[i] : 0.f;
    const float dn = ok ? deg[i] * dinvmean : 0.f;
    float x[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = node_feature(p, nos, f, dn, cls, 4 * q + v);
    Acts A;
    // (an opaque offset keeps the operand reads inside the loop)
    int off = 0;
    asm volatile("" : "+s"(off));
    mlp_forward16(reinterpret_cast<const uint16_t *>(wl) + off, prm, pack_features(x), lane, A);
    if (ok && q == 0) u0[i] = (double)A.out;
  }
}

// Forward + backward on explicit features (B x 16, FP32) and targets; each
// wave loops over 32-node batches (two 16-node passes) and accumulates its
// gradient, then writes it (and its loss sum) to part[wave][MLP_NP + 1].
// scale = d loss / d out factor of one node's squared error (2): the deltas
// rounded to bf16 do not depend on the batch size; the reduction applies the
// mean's 1/B.
constexpr int MLP_WB = 32;   // nodes per weight-gradient product (the MFMA's K)

// 8 bf16 of row 16 blk + l%16, nodes 8 (l/16) .. + 7 of a [rows][32] LDS array
__device__ __forceinline__ bf16x8 lds_op(const uint16_t *t, int blk, int lane) {
  return __builtin_bit_cast(
      bf16x8, *reinterpret_cast<const uint4 *>(t + (16 * blk + (lane & 15)) * MLP_WB + 8 * (lane >> 4)));
}

__global__ __launch_bounds__(64) void k_mlp_train(const uint16_t *__restrict__ wbf,
                                                  const float *__restrict__ prm,
                                                  const float *__restrict__ feat,
                                                  const float *__restrict__ target, int64_t B,
                                                  float scale, float *__restrict__ part) {
  // bf16 operands of the weight gradients, [unit or feature][node of the batch]
  __shared__ __align__(16) uint16_t tD3[64 * MLP_WB], tD2[64 * MLP_WB], tD1[64 * MLP_WB],
      tH2[64 * MLP_WB], tH1[64 * MLP_WB], tX[16 * MLP_WB];
  const int lane = threadIdx.x;
  const int node = lane & 15, q = lane >> 4;
  const int64_t wave = blockIdx.x, nw = gridDim.x;
  f32x4m g3[4][4], g2[4][4], g1[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    g1[a] = f32x4m{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 4; ++b) g3[a][b] = g2[a][b] = f32x4m{0.f, 0.f, 0.f, 0.f};
  }
  float gb1[16], gb2[16], gb3[16], gw4[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) gb1[k] = gb2[k] = gb3[k] = gw4[k] = 0.f;
  float gb4 = 0.f, loss = 0.f;

  for (int64_t b = wave; b * MLP_WB < B; b += nw) {
#pragma unroll 1
    for (int h = 0; h < MLP_WB / 16; ++h) {
      // reload the weight operands per pass instead of holding all of them
      // in registers next to the gradient accumulators
      const uint16_t *wb = wbf;
      asm volatile("" : "+s"(wb));
      const int col = 16 * h + node;
      const int64_t i = b * MLP_WB + col;
      const bool ok = i < B;
      float x[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) x[v] = ok ? feat[i * MLP_NF + 4 * q + v] : 0.f;
      Acts A;
      mlp_forward16(wb, prm, pack_features(x), lane, A);
      const float err = ok ? A.out - target[i] : 0.f;
      if (q == 0) loss += err * err;
      const float g = scale * err;  // d loss / d out for this node
      if (q == 0) gb4 += g;
      // layer 4: dW4, delta3 = g W4 (1 - h3^2)
      f32x4m d3[4];
#pragma unroll
      for (int ub = 0; ub < 4; ++ub)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float hv = A.h3[ub][r];
          gw4[4 * ub + r] = fmaf(g, hv, gw4[4 * ub + r]);
          d3[ub][r] = g * prm[OFF_W4 + 16 * ub + 4 * q + r] * (1.f - hv * hv);
        }
      // propagate: delta2 = (W3^T delta3) (1 - h2^2); delta1 = (W2^T delta2) (1 - h1^2)
      f32x4m d2[4], d1[4];
#pragma unroll
      for (int layer = 0; layer < 2; ++layer) {
        const f32x4m *dout = layer == 0 ? d3 : d2;
        f32x4m *din = layer == 0 ? d2 : d1;
        const f32x4m *hin = layer == 0 ? A.h2 : A.h1;
        const uint16_t *wt = wb + (layer == 0 ? BF_W3T : BF_W2T);
        const bf16x8 b0 = pack8(dout[0], dout[1]), b1 = pack8(dout[2], dout[3]);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          f32x4m acc = mfma32(load_a(wt, 64, kb, 0, lane), b0, f32x4m{0.f, 0.f, 0.f, 0.f});
          acc = mfma32(load_a(wt, 64, kb, 1, lane), b1, acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float hv = hin[kb][r];
            din[kb][r] = acc[r] * (1.f - hv * hv);
          }
        }
      }
      // bias gradients (per lane: units 16 ub + 4 q + r of node `node`), and
      // the bf16 operands of the weight gradients in column `col`
#pragma unroll
      for (int ub = 0; ub < 4; ++ub)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          gb3[4 * ub + r] += d3[ub][r];
          gb2[4 * ub + r] += d2[ub][r];
          gb1[4 * ub + r] += d1[ub][r];
          const int row = (16 * ub + 4 * q + r) * MLP_WB + col;
          tD3[row] = f2bf(d3[ub][r]);
          tD2[row] = f2bf(d2[ub][r]);
          tD1[row] = f2bf(d1[ub][r]);
          tH2[row] = f2bf(A.h2[ub][r]);
          tH1[row] = f2bf(A.h1[ub][r]);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) tX[(4 * q + v) * MLP_WB + col] = f2bf(x[v]);
    }
    __syncthreads();
    // dW[u][k] = sum over the batch's nodes of delta[u][node] in[k][node]:
    // A = deltas [u][node], B = inputs [node][k]
    const bf16x8 xo = lds_op(tX, 0, lane);
#pragma unroll
    for (int ub = 0; ub < 4; ++ub) {
      const bf16x8 a3 = lds_op(tD3, ub, lane), a2 = lds_op(tD2, ub, lane);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        g3[ub][kb] = mfma32(a3, lds_op(tH2, kb, lane), g3[ub][kb]);
        g2[ub][kb] = mfma32(a2, lds_op(tH1, kb, lane), g2[ub][kb]);
      }
      g1[ub] = mfma32(lds_op(tD1, ub, lane), xo, g1[ub]);
    }
    __syncthreads();   // the next batch overwrites the operands
  }
  // write the wave's partial gradient.  gacc blocks hold D[u = 4 q + r][k = l%16].
  float *out = part + wave * (MLP_NP + 1);
#pragma unroll
  for (int ub = 0; ub < 4; ++ub)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int u = 16 * ub + 4 * q + r;
      out[OFF_W1 + u * 16 + (lane & 15)] = g1[ub][r];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        out[OFF_W2 + u * 64 + 16 * kb + (lane & 15)] = g2[ub][kb][r];
        out[OFF_W3 + u * 64 + 16 * kb + (lane & 15)] = g3[ub][kb][r];
      }
    }
  // bias / W4 gradients: reduce over the 16 nodes (lanes with the same q)
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    float a1 = gb1[k], a2 = gb2[k], a3 = gb3[k], a4 = gw4[k];
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      a1 += __shfl_xor(a1, o);
      a2 += __shfl_xor(a2, o);
      a3 += __shfl_xor(a3, o);
      a4 += __shfl_xor(a4, o);
    }
    if ((lane & 15) == 0) {
      const int u = 16 * (k >> 2) + 4 * q + (k & 3);
      out[OFF_B1 + u] = a1;
      out[OFF_B2 + u] = a2;
      out[OFF_B3 + u] = a3;
      out[OFF_W4 + u] = a4;
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    gb4 += __shfl_xor(gb4, o);
    loss += __shfl_xor(loss, o);
  }
  if (lane == 0) {
    out[OFF_B4] = gb4;
    out[MLP_NP] = loss;
  }
}

// grad[p] = inv_b * sum over waves, in a fixed order: 8 slices of the waves
// (w = s mod 8) summed per thread, then the slices in order; 32 parameters
// per block.  The loss entry stays a sum.
constexpr int RED_P = 32, RED_S = 8;
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ part, int nwaves,
                                                    float inv_b, float *__restrict__ grad) {
  __shared__ float sl[RED_S][RED_P];
  const int p = blockIdx.x * RED_P + (threadIdx.x % RED_P), sidx = threadIdx.x / RED_P;
  float s = 0.f;
  if (p <= MLP_NP)
    for (int w = sidx; w < nwaves; w += RED_S) s += part[(int64_t)w * (MLP_NP + 1) + p];
  sl[sidx][threadIdx.x % RED_P] = s;
  __syncthreads();
  if (threadIdx.x < RED_P && p <= MLP_NP) {
    float t = 0.f;
    for (int k = 0; k < RED_S; ++k) t += sl[k][threadIdx.x];
    grad[p] = p < MLP_NP ? t * inv_b : t;
  }
}

// Adam step on the FP32 master parameters; refresh the BF16 copies.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ prm,
                                                  const float *__restrict__ grad,
                                                  float *__restrict__ m1, float *__restrict__ m2,
                                                  float lr, float b1, float b2, float eps,
                                                  float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= MLP_NP) return;
  const float g = grad[p];
  const float a = b1 * m1[p] + (1.f - b1) * g;
  const float v = b2 * m2[p] + (1.f - b2) * g * g;
  m1[p] = a;
  m2[p] = v;
  prm[p] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// BF16 copies in the permuted column order of the MFMA operands
__global__ __launch_bounds__(256) void k_mlp_tobf16(const float *__restrict__ prm,
                                                    uint16_t *__restrict__ wbf) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < 2048) {   // W1: row u, slot i of lane group g = feature 4 g + i (i < 4)
    const int u = t >> 5, g = (t >> 3) & 3, i = t & 7;
    wbf[BF_W1 + t] = i < 4 ? f2bf(prm[OFF_W1 + u * 16 + 4 * g + i]) : (uint16_t)0;
  }
  if (t < 4096) {
    const int u = t >> 6, k = t & 63;
    wbf[BF_W2 + u * 64 + kpos(k)] = f2bf(prm[OFF_W2 + t]);
    wbf[BF_W3 + u * 64 + kpos(k)] = f2bf(prm[OFF_W3 + t]);
    wbf[BF_W2T + k * 64 + kpos(u)] = f2bf(prm[OFF_W2 + t]);
    wbf[BF_W3T + k * 64 + kpos(u)] = f2bf(prm[OFF_W3 + t]);
  }
}

// Training features for a sample of nodes (sorted positions idx[s]).
__global__ __launch_bounds__(256) void k_mlp_features(const float4 *__restrict__ pts,
                                                      const int *__restrict__ perm,
                                                      const float *__restrict__ deg,
                                                      float dinvmean,
                                                      const double *__restrict__ f_user,
                                                      const double *__restrict__ u_user, int cls,
                                                      int nos, int d,
                                                      const int *__restrict__ idx, int64_t ns,
                                                      float *__restrict__ feat,
                                                      float *__restrict__ target) {
  const int64_t s = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (s >= ns) return;
  const int i = idx[s];
  float4 p = pts[i];
  if (d < 3) p.z = 0.f;
  if (d < 2) p.y = 0.f;
  const int j = perm[i];
  const float f = (float)f_user[j], dn = deg[i] * dinvmean;
  for (int k = 0; k < MLP_NF; ++k) feat[s * MLP_NF + k] = node_feature(p, nos, f, dn, cls, k);
  target[s] = (float)u_user[j];
}

}  // namespace nfl

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct nfl_mlp {
  hipStream_t stream = nullptr;
  int ncls = 0;
  nfl::DBuf<float> prm, m1, m2, grad, part, feat, target;
  nfl::DBuf<uint16_t> wbf;
  nfl::DBuf<int> idx;
  int64_t step = 0;
  // plans whose nfl_cg_solve(..., NFL_WARM_MLP) reads this network: destroying
  // the network detaches them, destroying a plan removes it from this list
  std::vector<nfl_plan *> attached;
};

namespace nfl {

// Remove plan P from the attachment list of its network (if any).
void mlp_detach_plan(nfl_plan *P) {
  nfl_mlp *M = P->mlp;
  if (!M) return;
  auto &a = M->attached;
  a.erase(std::remove(a.begin(), a.end(), P), a.end());
  P->mlp = nullptr;
  P->mlp_cls = 0;
}

static int mlp_refresh(nfl_mlp *M) {
  hipLaunchKernelGGL(k_mlp_tobf16, dim3(16), dim3(256), 0, M->stream, M->prm.p, M->wbf.p);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

// fwd + bwd + reduce on features already in M->feat / M->target (B rows)
static int mlp_grad(nfl_mlp *M, int64_t B, double *loss_host) {
  const int nw = (int)std::min<int64_t>(512, (B + MLP_WB - 1) / MLP_WB);
  NFL_TRY(M->part.ensure((size_t)nw * (MLP_NP + 1)));
  hipLaunchKernelGGL(k_mlp_train, dim3(nw), dim3(64), 0, M->stream, M->wbf.p, M->prm.p, M->feat.p,
                     M->target.p, B, 2.0f, M->part.p);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NP + 1 + RED_P - 1) / RED_P), dim3(256), 0, M->stream,
                     M->part.p, nw, 1.0f / (float)B, M->grad.p);
  NFL_HIP(hipGetLastError());
  if (loss_host) {
    float l = 0.f;
    NFL_HIP(hipMemcpyAsync(&l, M->grad.p + MLP_NP, sizeof(float), hipMemcpyDeviceToHost, M->stream));
    NFL_HIP(hipStreamSynchronize(M->stream));
    *loss_host = (double)l / (double)B;
  }
  return NFL_OK;
}

static int mlp_adam(nfl_mlp *M, double lr) {
  M->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)M->step), c2 = 1.f - std::pow(b2, (float)M->step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NP + 255) / 256), dim3(256), 0, M->stream, M->prm.p,
                     M->grad.p, M->m1.p, M->m2.p, (float)lr, b1, b2, 1e-8f, c1, c2);
  NFL_HIP(hipGetLastError());
  return mlp_refresh(M);
}

// Mean degree of a plan (host, from the stats computed at set_kernel).
static float plan_dinvmean(nfl_plan *P, DBuf<double> &tmp) {
  (void)tmp;
  return (float)(1.0 / P->dmean);
}

int mlp_predict_sorted(nfl_mlp *M, nfl_plan *P, int cls, const double *f_sorted, double *u0) {
  LBuf<double> tmp;
  const int64_t nb16 = (P->n + 15) / 16;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (nb16 + 3) / 4));
  hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(256), 0, P->stream, M->wbf.p, M->prm.p,
                     P->pts.p, P->deg.p, plan_dinvmean(P, tmp), f_sorted, cls, P->nos, P->d, P->n,
                     u0);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int mlp_warm_start(nfl_plan *P, const double *f_sorted, double *u_sorted) {
  if (!P->mlp) {
    set_error("no warm-start network attached to this plan (nfl_mlp_attach)");
    return NFL_ERR_ORDER;
  }
  if (P->mlp->stream != P->stream) {
    // the network's buffers are read on the plan's stream; order them first
    NFL_HIP(hipStreamSynchronize(P->mlp->stream));
  }
  return mlp_predict_sorted(P->mlp, P, P->mlp_cls, f_sorted, u_sorted);
}

}  // namespace nfl

using namespace nfl;

extern "C" {

int nfl_mlp_create(nfl_mlp_handle *h, int n_classes, uint64_t seed, void *hip_stream) {
  if (!h) { set_error("null handle pointer"); return NFL_ERR_ARG; }
  *h = nullptr;
  if (n_classes < 1 || n_classes > MLP_NF - 5) { set_error("n_classes must be in 1..11"); return NFL_ERR_ARG; }
  nfl_mlp *M = new (std::nothrow) nfl_mlp();
  if (!M) { set_error("host allocation failed"); return NFL_ERR_OOM; }
  M->stream = (hipStream_t)hip_stream;
  M->ncls = n_classes;
  int rc = M->prm.ensure(MLP_NP);
  if (rc == NFL_OK) rc = M->m1.ensure(MLP_NP);
  if (rc == NFL_OK) rc = M->m2.ensure(MLP_NP);
  if (rc == NFL_OK) rc = M->grad.ensure(MLP_NP + 1);
  if (rc == NFL_OK) rc = M->wbf.ensure(MLP_NBF);
  if (rc != NFL_OK) { delete M; return rc; }
  // Glorot-uniform weights from a splitmix64 stream, zero biases
  std::vector<float> p(MLP_NP, 0.f);
  uint64_t st = seed * 0x9e3779b97f4a7c15ULL + 12345;
  auto uni = [&]() {
    st += 0x9e3779b97f4a7c15ULL;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z ^= z >> 31;
    return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  };
  auto init = [&](int off, int fan_out, int fan_in, int fan_in_used) {
    const double a = std::sqrt(6.0 / (fan_in_used + fan_out));
    for (int u = 0; u < fan_out; ++u)
      for (int k = 0; k < fan_in; ++k) p[off + u * fan_in + k] = k < fan_in_used ? (float)(a * uni()) : 0.f;
  };
  init(OFF_W1, 64, 16, 5 + n_classes);
  init(OFF_W2, 64, 64, 64);
  init(OFF_W3, 64, 64, 64);
  init(OFF_W4, 1, 64, 64);
  hipError_t e = hipMemcpyAsync(M->prm.p, p.data(), MLP_NP * 4, hipMemcpyHostToDevice, M->stream);
  if (e == hipSuccess) e = hipMemsetAsync(M->m1.p, 0, MLP_NP * 4, M->stream);
  if (e == hipSuccess) e = hipMemsetAsync(M->m2.p, 0, MLP_NP * 4, M->stream);
  if (e != hipSuccess || mlp_refresh(M) != NFL_OK) {
    set_error("nfl_mlp_create: initialisation failed");
    delete M;
    return NFL_ERR_HIP;
  }
  *h = M;
  return NFL_OK;
}

int nfl_mlp_destroy(nfl_mlp_handle M) {
  if (!M) return NFL_OK;
  (void)hipStreamSynchronize(M->stream);
  // a later warm-started solve on these plans fails with NFL_ERR_ORDER
  // instead of reading freed memory
  for (nfl_plan *P : M->attached) {
    (void)hipStreamSynchronize(P->stream);
    P->mlp = nullptr;
    P->mlp_cls = 0;
  }
  M->attached.clear();
  delete M;   // the device buffers are freed by their destructors
  return NFL_OK;
}

int nfl_mlp_get_params(nfl_mlp_handle M, float *host, int64_t count) {
  if (!M || !host || count < MLP_NP) { set_error("need a network and >= 9473 floats"); return NFL_ERR_ARG; }
  NFL_HIP(hipMemcpyAsync(host, M->prm.p, MLP_NP * 4, hipMemcpyDeviceToHost, M->stream));
  NFL_HIP(hipStreamSynchronize(M->stream));
  return NFL_OK;
}

int nfl_mlp_set_params(nfl_mlp_handle M, const float *host, int64_t count) {
  if (!M || !host || count < MLP_NP) { set_error("need a network and >= 9473 floats"); return NFL_ERR_ARG; }
  NFL_HIP(hipMemcpyAsync(M->prm.p, host, MLP_NP * 4, hipMemcpyHostToDevice, M->stream));
  NFL_HIP(hipMemsetAsync(M->m1.p, 0, MLP_NP * 4, M->stream));
  NFL_HIP(hipMemsetAsync(M->m2.p, 0, MLP_NP * 4, M->stream));
  M->step = 0;
  NFL_TRY(mlp_refresh(M));
  NFL_HIP(hipStreamSynchronize(M->stream));
  return NFL_OK;
}

int nfl_mlp_forward(nfl_mlp_handle M, const float *feat_dev, int64_t B, float *out_dev) {
  if (!M || !feat_dev || !out_dev || B < 1) { set_error("bad arguments"); return NFL_ERR_ARG; }
  NFL_TRY(M->feat.ensure((size_t)B * MLP_NF));
  NFL_HIP(hipMemcpyAsync(M->feat.p, feat_dev, (size_t)B * MLP_NF * 4, hipMemcpyDeviceToDevice, M->stream));
  return mlp_forward_explicit(M, B, out_dev);
}

int nfl_mlp_gradient(nfl_mlp_handle M, const float *feat_dev, const float *target_dev, int64_t B,
                     float *grad_host, int64_t count, double *loss_host) {
  if (!M || !feat_dev || !target_dev || B < 1 || !grad_host || count < MLP_NP) {
    set_error("bad arguments");
    return NFL_ERR_ARG;
  }
  NFL_TRY(M->feat.ensure((size_t)B * MLP_NF));
  NFL_TRY(M->target.ensure((size_t)B));
  NFL_HIP(hipMemcpyAsync(M->feat.p, feat_dev, (size_t)B * MLP_NF * 4, hipMemcpyDeviceToDevice, M->stream));
  NFL_HIP(hipMemcpyAsync(M->target.p, target_dev, (size_t)B * 4, hipMemcpyDeviceToDevice, M->stream));
  NFL_TRY(mlp_grad(M, B, loss_host));
  NFL_HIP(hipMemcpyAsync(grad_host, M->grad.p, MLP_NP * 4, hipMemcpyDeviceToHost, M->stream));
  NFL_HIP(hipStreamSynchronize(M->stream));
  return NFL_OK;
}

int nfl_mlp_train_step(nfl_mlp_handle M, nfl_handle P, const double *f_dev, const double *u_dev,
                       int cls, int64_t nsample, uint64_t seed, double lr, double *loss_host) {
  if (!M || !P || !f_dev || !u_dev || nsample < 1 || !(lr > 0)) { set_error("bad arguments"); return NFL_ERR_ARG; }
  if (!P->have_kernel || P->frame_only) { set_error("plan has no kernel or no degrees"); return NFL_ERR_ORDER; }
  if (cls < 0 || cls >= M->ncls) { set_error("class out of range"); return NFL_ERR_ARG; }
  const int64_t ns = std::min<int64_t>(nsample, P->n);
  // sample without replacement: a random window of a seeded shuffle is not
  // needed for training; stride sampling with a seeded offset is enough
  std::vector<int> idx((size_t)ns);
  uint64_t st = seed * 0x9e3779b97f4a7c15ULL + 7;
  for (int64_t s = 0; s < ns; ++s) {
    st = st * 6364136223846793005ULL + 1442695040888963407ULL;
    idx[(size_t)s] = (int)((st >> 33) % (uint64_t)P->n);
  }
  NFL_TRY(M->idx.ensure((size_t)ns));
  NFL_TRY(M->feat.ensure((size_t)ns * MLP_NF));
  NFL_TRY(M->target.ensure((size_t)ns));
  if (M->stream != P->stream) NFL_HIP(hipStreamSynchronize(P->stream));
  NFL_HIP(hipMemcpyAsync(M->idx.p, idx.data(), ns * 4, hipMemcpyHostToDevice, M->stream));
  LBuf<double> tmp;
  hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, M->stream,
                     P->pts.p, P->perm.p, P->deg.p, plan_dinvmean(P, tmp), f_dev, u_dev, cls, P->nos,
                     P->d, M->idx.p, ns, M->feat.p, M->target.p);
  NFL_HIP(hipGetLastError());
  NFL_TRY(mlp_grad(M, ns, loss_host));
  NFL_TRY(mlp_adam(M, lr));
  NFL_HIP(hipStreamSynchronize(M->stream));
  return NFL_OK;
}

int nfl_mlp_predict(nfl_mlp_handle M, nfl_handle P, const double *f_dev, int cls, double *u_dev) {
  if (!M || !P || !f_dev || !u_dev) { set_error("bad arguments"); return NFL_ERR_ARG; }
  if (!P->have_kernel || P->frame_only) { set_error("plan has no kernel or no degrees"); return NFL_ERR_ORDER; }
  if (cls < 0 || cls >= M->ncls) { set_error("class out of range"); return NFL_ERR_ARG; }
  LBuf<double> fs, us;
  NFL_TRY(fs.ensure(P->n));
  NFL_TRY(us.ensure(P->n));
  NFL_TRY(gather64(P, f_dev, fs.p));
  NFL_TRY(mlp_predict_sorted(M, P, cls, fs.p, us.p));
  NFL_TRY(scatter64(P, us.p, u_dev));
  NFL_HIP(hipStreamSynchronize(P->stream));
  return NFL_OK;
}

int nfl_mlp_attach(nfl_handle P, nfl_mlp_handle M, int cls) {
  if (!P) { set_error("null plan"); return NFL_ERR_ARG; }
  if (M && (cls < 0 || cls >= M->ncls)) { set_error("class out of range"); return NFL_ERR_ARG; }
  mlp_detach_plan(P);
  if (M) {
    P->mlp = M;
    P->mlp_cls = cls;
    M->attached.push_back(P);
  }
  return NFL_OK;
}

int nfl_mlp_save(nfl_mlp_handle M, const char *path) {
  if (!M || !path) { set_error("bad arguments"); return NFL_ERR_ARG; }
  std::vector<float> p(MLP_NP);
  NFL_TRY(nfl_mlp_get_params(M, p.data(), MLP_NP));
  FILE *fp = std::fopen(path, "wb");
  if (!fp) { set_error(std::string("cannot open ") + path); return NFL_ERR_ARG; }
  const char magic[8] = {'N', 'F', 'L', 'M', 'L', 'P', '0', '1'};
  const int32_t hdr[4] = {MLP_NF, MLP_H, MLP_NP, M->ncls};
  bool ok = std::fwrite(magic, 1, 8, fp) == 8 && std::fwrite(hdr, 4, 4, fp) == 4 &&
            std::fwrite(p.data(), 4, MLP_NP, fp) == (size_t)MLP_NP;
  ok = (std::fclose(fp) == 0) && ok;
  if (!ok) { set_error("write failed"); return NFL_ERR_ARG; }
  return NFL_OK;
}

int nfl_mlp_load(nfl_mlp_handle M, const char *path) {
  if (!M || !path) { set_error("bad arguments"); return NFL_ERR_ARG; }
  FILE *fp = std::fopen(path, "rb");
  if (!fp) { set_error(std::string("cannot open ") + path); return NFL_ERR_ARG; }
  char magic[8];
  int32_t hdr[4];
  std::vector<float> p(MLP_NP);
  bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "NFLMLP01", 8) == 0 &&
            std::fread(hdr, 4, 4, fp) == 4 && hdr[0] == MLP_NF && hdr[1] == MLP_H &&
            hdr[2] == MLP_NP && hdr[3] == M->ncls &&
            std::fread(p.data(), 4, MLP_NP, fp) == (size_t)MLP_NP;
  std::fclose(fp);
  if (!ok) { set_error("not a compatible network file"); return NFL_ERR_ARG; }
  return nfl_mlp_set_params(M, p.data(), MLP_NP);
}

}  // extern "C"

namespace nfl {

// Forward on explicit features (M->feat, B rows) -> out (FP32), one wave per
// 16 rows.
__global__ __launch_bounds__(256) void k_mlp_fwd_explicit(const uint16_t *__restrict__ wbf,
                                                          const float *__restrict__ prm,
                                                          const float *__restrict__ feat,
                                                          int64_t B, float *__restrict__ out) {
  __shared__ uint4 wl[MLP_NBF / 8];
  stage_weights(wbf, wl);
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int node = lane & 15, q = lane >> 4;
  for (int64_t b = wave; b * 16 < B; b += nw) {
    const int64_t i = b * 16 + node;
    const bool ok = i < B;
    float x[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = ok ? feat[i * MLP_NF + 4 * q + v] : 0.f;
    Acts A;
    // (an opaque offset keeps the operand reads inside the loop)
    int off = 0;
    asm volatile("" : "+s"(off));
    mlp_forward16(reinterpret_cast<const uint16_t *>(wl) + off, prm, pack_features(x), lane, A);
    if (ok && q == 0) out[i] = A.out;
  }
}

int mlp_forward_explicit(nfl_mlp *M, int64_t B, float *out) {
  const int64_t nb16 = (B + 15) / 16;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (nb16 + 3) / 4));
  hipLaunchKernelGGL(k_mlp_fwd_explicit, dim3(blocks), dim3(256), 0, M->stream, M->wbf.p, M->prm.p,
                     M->feat.p, B, out);
  NFL_HIP(hipGetLastError());
  NFL_HIP(hipStreamSynchronize(M->stream));
  return NFL_OK;
}

}  // namespace nfl
