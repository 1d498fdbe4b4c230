// Device code shared by the single-graph and the batched NFFT kernels:
// window polynomials, input/output operations, the matrix-core spread and
// interpolation bodies (d = 3) and the LDS FFT line transforms.
#pragma once

#include <hip/hip_runtime.h>

#include "nfl_internal.h"

namespace nfl {

// ---------------------------------------------------------------------------
// Window.  The Kaiser-Bessel window psi(t) = sinh(b s)/(s b e^{bm}),
// s = sqrt(m^2 - t^2), t in (-m, m] (grid units), is applied as 2m
// polynomials, one per grid offset c of a node's window:
//   psi(c - (m-1) - f) = sum_k coef[c][k] g^k,  g = 2f - 1,
// where f in [0, 1) is the node's fraction inside its cell.  The host fits the
// coefficients (FP64, rounded to float32) and deconvolves with the exact
// transform of this piecewise polynomial.
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ float win_poly(const float (&cf)[NC], float f) {
  const float g = fmaf(2.f, f, -1.f);
  float p = cf[NC - 1];
#pragma unroll
  for (int k = NC - 2; k >= 0; --k) p = fmaf(p, g, cf[k]);
  return p;
}

__device__ __forceinline__ void load_coef(const float *__restrict__ wcoef, int c, float (&cf)[WIN_NC]) {
#pragma unroll
  for (int k = 0; k < WIN_NC; ++k) cf[k] = wcoef[c * WIN_NC + k];
}

struct KArgs {
  const float *x32;
  float *y32;
  const double *x64;
  double *y64;
  double tau;
  const int *perm;
  const float *dinv;
  float *deg_out;
  float *dinv_out;
  const int *stop;   // null, or a device flag: when nonzero every kernel of the product returns at once
  // deterministic spread (null: float atomics): bits of max |input| written
  // by the product's pre-pass; fx_mult bounds every grid value by
  // max |input| * fx_mult (see fx_scale)
  const unsigned *fx_max;
  float fx_mult;
  // non-null: the tile spread stores the caller-order input in sorted order
  // here (xs[i] = x[perm[i]]), and the tile interpolation's output step reads
  // it back instead of gathering x through the permutation again
  float *xs;
  // non-null (OUT_SORTED_F64_SSL, tile interpolation): one partial sum of
  // x64_i y64_i per workgroup, over its nodes in a fixed order (the CG's p.q)
  double *dot;
};

// Deterministic spread: the plan's grid holds int64 fixed-point values
// round(v * 2^e).  Integer addition is associative, so the sum a cell
// receives does not depend on the order of the work items' atomic additions
// (float atomics make it run-to-run dependent).  The exponent comes from a
// bound b = max |input| * fx_mult >= every |cell sum| (number of nodes times
// the largest window product times the input bound), so that
// |sum| * 2^e < 2^61: no overflow, and a resolution of b 2^-61, far below
// FP32 rounding of the values.  Spread and r2c derive the same e from the
// same bits.
__device__ __forceinline__ double fx_scale(unsigned maxbits, float mult) {
  const double b = (double)__uint_as_float(maxbits) * (double)mult + 1e-300;
  int e;
  (void)frexp(b, &e);   // b < 2^e
  return ldexp(1.0, 61 - e);
}

// add v into grid cell idx: a float atomic, or the fixed-point int64 atomic
__device__ __forceinline__ void grid_add(float *grid, size_t idx, float v, double fx) {
  if (fx != 0.0)
    atomicAdd(reinterpret_cast<unsigned long long *>(grid) + idx,
              (unsigned long long)__double2ll_rn((double)v * fx));
  else
    unsafeAtomicAdd(grid + idx, v);
}

// The bound is kept as FX_WORDS words FX_STRIDE apart: a producer block b
// takes word b mod FX_WORDS for its atomic maximum (atomics on one address
// serialise, ~10 ns each), readers take the maximum of the words.
__device__ __forceinline__ unsigned *fx_word(unsigned *w, int block) {
  return w + (block % FX_WORDS) * FX_STRIDE;
}

__device__ __forceinline__ unsigned fx_bits(const unsigned *w) {
  unsigned v = 0;
#pragma unroll
  for (int k = 0; k < FX_WORDS; ++k) v = max(v, w[k * FX_STRIDE]);
  return v;
}

__device__ __forceinline__ double fx_of(const KArgs &ka) {
  return ka.fx_max ? fx_scale(fx_bits(ka.fx_max), ka.fx_mult) : 0.0;
}

// Uniform early exit of a product's kernels once an iterative solver on the
// device has stopped (its flag is set by the solver's own kernels).
__device__ __forceinline__ bool stopped(const int *stop) { return stop && *stop; }

template <int IN>
__device__ __forceinline__ float load_in(const KArgs &a, int i) {
  if constexpr (IN == IN_USER_F32) return a.x32[a.perm[i]];
  else if constexpr (IN == IN_USER_F32_DINV) return a.dinv[i] * a.x32[a.perm[i]];
  else if constexpr (IN == IN_ONES) return 1.0f;
  else if constexpr (IN == IN_SORTED_F32) return a.x32[i];
  else return (float)((double)a.dinv[i] * a.x64[i]);
}

template <int OUT>
__device__ __forceinline__ void store_out(const KArgs &a, int i, float f) {
  if constexpr (OUT == OUT_USER_RAW) {
    a.y32[a.perm[i]] = f;
  } else if constexpr (OUT == OUT_USER_W) {
    const int j = a.perm[i];
    a.y32[j] = f - a.x32[j];
  } else if constexpr (OUT == OUT_USER_LS) {
    const int j = a.perm[i];
    const float xu = a.x32[j], di = a.dinv[i];
    const float xt = di * xu;
    a.y32[j] = xu - di * (f - xt);
  } else if constexpr (OUT == OUT_USER_A) {
    const int j = a.perm[i];
    const float di = a.dinv[i];
    const float xt = di * a.x32[j];
    a.y32[j] = di * (f - xt);
  } else if constexpr (OUT == OUT_DEGREE) {
    const float dg = f - 1.0f;
    a.deg_out[i] = dg;
    a.dinv_out[i] = dg > 0.f ? 1.0f / __builtin_sqrtf(dg) : 0.f;
  } else if constexpr (OUT == OUT_SORTED_F64_A) {
    const double di = (double)a.dinv[i];
    const float xt = (float)(di * a.x64[i]);
    a.y64[i] = di * ((double)f - (double)xt);
  } else {
    const double di = (double)a.dinv[i];
    const double xv = a.x64[i];
    const float xt = (float)(di * xv);
    const double av = di * ((double)f - (double)xt);
    a.y64[i] = xv + a.tau * (xv - av);
  }
}

// Output-side operands of one node (permutation entry, caller-order input,
// d^{-1/2}), loaded ahead of the node's store: the caller-order input is a
// gather behind the permutation, two dependent loads that would otherwise
// stall the wave right after its matrix-core work.  store_pre computes what
// store_out computes, from these values.
struct OutPre {
  int j;
  float xu, di;
  double xd;
};

template <int OUT>
constexpr bool pre_user() {
  return OUT == OUT_USER_RAW || OUT == OUT_USER_W || OUT == OUT_USER_LS || OUT == OUT_USER_A;
}

template <int OUT>
__device__ __forceinline__ void pre_index(const KArgs &a, int i, bool ok, OutPre &p) {
  p.j = 0;
  p.xu = 0.f;
  p.di = 0.f;
  p.xd = 0.0;
  if (!ok) return;
  if constexpr (pre_user<OUT>()) p.j = a.perm[i];
  if constexpr (OUT == OUT_USER_W || OUT == OUT_USER_LS || OUT == OUT_USER_A)
    if (a.xs) p.xu = a.xs[i];   // coalesced, no dependent gather
  if constexpr (OUT == OUT_USER_LS || OUT == OUT_USER_A || OUT == OUT_SORTED_F64_A ||
                OUT == OUT_SORTED_F64_SSL)
    p.di = a.dinv[i];
  if constexpr (OUT == OUT_SORTED_F64_A || OUT == OUT_SORTED_F64_SSL) p.xd = a.x64[i];
}

template <int OUT>
__device__ __forceinline__ void pre_gather(const KArgs &a, bool ok, OutPre &p) {
  if constexpr (OUT == OUT_USER_W || OUT == OUT_USER_LS || OUT == OUT_USER_A) {
    if (ok && !a.xs) p.xu = a.x32[p.j];
  }
}

// the operands of lane src's node
template <int OUT>
__device__ __forceinline__ OutPre pre_from(const OutPre &p, int src) {
  OutPre q = p;
  if constexpr (pre_user<OUT>()) q.j = __shfl(p.j, src);
  if constexpr (OUT == OUT_USER_W || OUT == OUT_USER_LS || OUT == OUT_USER_A) q.xu = __shfl(p.xu, src);
  if constexpr (OUT == OUT_USER_LS || OUT == OUT_USER_A || OUT == OUT_SORTED_F64_A ||
                OUT == OUT_SORTED_F64_SSL)
    q.di = __shfl(p.di, src);
  if constexpr (OUT == OUT_SORTED_F64_A || OUT == OUT_SORTED_F64_SSL) q.xd = __shfl(p.xd, src);
  return q;
}

// Returns x64_i y64_i for OUT_SORTED_F64_SSL (the term of the CG's p.q),
// else 0.
template <int OUT>
__device__ __forceinline__ double store_pre(const KArgs &a, int i, float f, const OutPre &p) {
  if constexpr (OUT == OUT_USER_RAW) {
    a.y32[p.j] = f;
  } else if constexpr (OUT == OUT_USER_W) {
    a.y32[p.j] = f - p.xu;
  } else if constexpr (OUT == OUT_USER_LS) {
    const float xt = p.di * p.xu;
    a.y32[p.j] = p.xu - p.di * (f - xt);
  } else if constexpr (OUT == OUT_USER_A) {
    const float xt = p.di * p.xu;
    a.y32[p.j] = p.di * (f - xt);
  } else if constexpr (OUT == OUT_DEGREE) {
    const float dg = f - 1.0f;
    a.deg_out[i] = dg;
    a.dinv_out[i] = dg > 0.f ? 1.0f / __builtin_sqrtf(dg) : 0.f;
  } else if constexpr (OUT == OUT_SORTED_F64_A) {
    const double di = (double)p.di;
    const float xt = (float)(di * p.xd);
    a.y64[i] = di * ((double)f - (double)xt);
  } else {
    const double di = (double)p.di;
    const double xv = p.xd;
    const float xt = (float)(di * xv);
    const double av = di * ((double)f - (double)xt);
    const double yv = xv + a.tau * (xv - av);
    a.y64[i] = yv;
    return xv * yv;
  }
  return 0.0;
}

// v[l] + v[l ^ 16] + v[l ^ 32] + v[l ^ 48] on every lane, summed in the
// order (v + v^16) + (v + v^16)^32, with the cross-row lane swaps of the
// vector ALU (no LDS round trip): a swap of a value with itself returns, in
// its two halves, the lane's own value and its partner's.
__device__ __forceinline__ float sum_rows4(float v) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Workgroups are dispatched to the 8 XCDs round-robin by id, and each XCD has
// its own L2.  xcd_block maps workgroup id b of nb to a logical block so that
// each XCD gets one contiguous range of blocks (bijective on [0, nb)): the
// column passes of the FFT, whose neighbouring workgroups read parts of the
// same cache lines, then fetch each line into one L2 instead of several, and
// so do the tile forms' work groups, whose neighbours in the sort share grid
// cells.
constexpr int NUM_XCD = 8;

__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b % NUM_XCD, q = b / NUM_XCD;
  const int per = nb / NUM_XCD, rem = nb % NUM_XCD;
  return x * per + min(x, rem) + q;
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}


// ---------------------------------------------------------------------------
// d = 3 spread and interpolation on the matrix cores.
//
// Nodes are processed in sub-batches of 16.  Per sub-batch each lane l
// evaluates, for node l/4, the window polynomials of the offsets
// 4 (l%4) .. 4 (l%4) + 3 on all three axes (12 Horner evaluations) and writes
// them to a per-wave weight table wt[node][axis][offset] in LDS (the x value
// of the node rides along in wt[node][3][0]).  The matrix-core loop then reads
// its operands from the table with independent broadcast loads.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Weight-table row pitch (floats per node): 80 for the spread, whose reads
// touch 4 node rows x 16 columns (rows 16 banks apart), 65 for the interp,
// whose reads touch 16 node rows in the same column (rows 1 bank apart).
constexpr int WT_SPREAD = 80, WT_INTERP = 65;

// x-pitch of an LDS tile with P^3 logical cells: >= P*P and = 4 (mod 32), so
// that 16 consecutive x-offsets land on distinct bank quadruples.
__host__ __device__ __forceinline__ int tile_px(int P) { return P * P + ((4 - P * P) % 32 + 32) % 32; }

// Fill the weight table for the 16 nodes sub*16 .. sub*16+15 of the current
// 64-node batch held in registers (lane l holds node l of the batch: record
// qb, input value xb); cnt = valid nodes of the sub-batch.  Returns, in every
// lane, the packed cell of sub-batch node (lane % 16).
template <int W, bool WITH_X, int STRIDE>
__device__ __forceinline__ uint32_t fill_weights(const float4 &qb, float xb, int sub, int cnt,
                                                 int lane, const float (&cf)[4][WIN_NC],
                                                 float *wt) {
  // weights: lane l evaluates node l/4 at offsets 4 (l%4) .. 4 (l%4) + 3.  With
  // a row pitch that is a multiple of 4 the four values go out as one 16-byte
  // store; eight consecutive lanes then cover eight distinct 4-bank groups.
  const int node = lane >> 2, part = lane & 3;
  const int src = sub * 16 + min(node, cnt - 1);
  const float qx = __shfl(qb.x, src), qy = __shfl(qb.y, src), qz = __shfl(qb.z, src);
  float *w = wt + node * STRIDE + 4 * part;
  if constexpr (STRIDE % 4 == 0) {
    *reinterpret_cast<float4 *>(w) = make_float4(win_poly(cf[0], qx), win_poly(cf[1], qx),
                                                 win_poly(cf[2], qx), win_poly(cf[3], qx));
    *reinterpret_cast<float4 *>(w + 16) = make_float4(win_poly(cf[0], qy), win_poly(cf[1], qy),
                                                      win_poly(cf[2], qy), win_poly(cf[3], qy));
    *reinterpret_cast<float4 *>(w + 32) = make_float4(win_poly(cf[0], qz), win_poly(cf[1], qz),
                                                      win_poly(cf[2], qz), win_poly(cf[3], qz));
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      w[0 * 16 + u] = win_poly(cf[u], qx);
      w[1 * 16 + u] = win_poly(cf[u], qy);
      w[2 * 16 + u] = win_poly(cf[u], qz);
    }
  }
  if (WITH_X) {
    const float xv = __shfl(xb, src);
    if (part == 0) wt[node * STRIDE + 3 * 16] = xv;
  }
  // cells: lane l returns the packed cell of sub-batch node l % 16
  const int cn = lane & 15;
  const int csrc = sub * 16 + min(cn, cnt - 1);
  const uint32_t cell = (uint32_t)__shfl((int)__float_as_uint(qb.w), csrc);
  return cn < cnt ? cell : 0xffffffffu;
}

// One 64-node batch of sorted records (and, for the spread, input values),
// loaded one per lane; past the end: zero records.
template <int IN, bool WITH_X>
__device__ __forceinline__ void load_batch(const float4 *__restrict__ pts, const KArgs &ka, int i0,
                                           int e, int lane, float4 &qb, float &xb) {
  qb = make_float4(0.f, 0.f, 0.f, 0.f);
  xb = 0.f;
  if (i0 + lane < e) {
    const int i = i0 + lane;
    qb = pts[i];
    if constexpr (WITH_X && (IN == IN_USER_F32 || IN == IN_USER_F32_DINV)) {
      const float raw = ka.x32[ka.perm[i]];
      if (ka.xs) ka.xs[i] = raw;
      xb = IN == IN_USER_F32_DINV ? ka.dinv[i] * raw : raw;
    } else if constexpr (WITH_X) {
      xb = load_in<IN>(ka, i);
    }
  }
}

// Spread: for the nodes p of one grid cell
//   G[ax][ay][az] += sum_p (x_p wx_p[ax]) (wy_p[ay] wz_p[az])
// with v_mfma_f32_16x16x4_f32: rows = x-offsets ax (W of 16 used), K = 4
// nodes, columns = z-offsets (and, for W <= 8, S = 16/WP y-offsets packed
// side by side), NB column blocks, one per y-offset group.  Lane l (node slot
// l/16, column l%16) accumulates D[ax = 4 (l/16) + r][column l%16], r < 4, in
// registers over a run of nodes, then adds it into its wave's PRIVATE copy of
// the padded tile (plain read-add-write: every lane of a flush owns a
// distinct cell, and the LDS operations of one wave are ordered).  At the end
// the NW private tiles (one per wave: NW = 4, or 1 for the one-wave variant
// used on short items) are summed and added into the grid.
//
// ZM ("z-merge", needs T + W - 1 <= 16): the 16 columns cover the whole
// z-extent of the padded tile, so nodes of different cells of one (x, y)
// column of the tile share the accumulators: node p contributes to column c
// with wz_p[c - lz_p] (lz_p = its cell's z inside the tile) and runs, hence
// flushes, are per (x, y) column instead of per cell.
template <int W, bool ZM>
struct SpreadShape {
  static constexpr int WP = ZM ? 16 : (W <= 4 ? 4 : (W <= 8 ? 8 : 16));
  static constexpr int S = 16 / WP;
  static constexpr int NB = (W + S - 1) / S;
};

template <int W, int IN, bool ZM, int NW = 4>
__device__ __forceinline__ void spread3_mfma_body(const Item it, const float4 *__restrict__ pts,
                                                  const KArgs ka, float *__restrict__ grid,
                                                  int nos, int tshift,
                                                  const float *__restrict__ wcoef) {
  constexpr int M = W / 2;
  constexpr int WP = SpreadShape<W, ZM>::WP, S = SpreadShape<W, ZM>::S,
                NB = SpreadShape<W, ZM>::NB;
  extern __shared__ float lds[];
  const int T = 1 << tshift, P = T + W - 1, PX = tile_px(P), P3 = PX * P;
  const int ntd = nos >> tshift;
  const int tz = it.tile % ntd, ty = (it.tile / ntd) % ntd, tx = it.tile / (ntd * ntd);
  const int ox = tx * T, oy = ty * T, oz = tz * T;
  for (int c = threadIdx.x; c < NW * P3; c += 64 * NW) lds[c] = 0.f;
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int c16 = lane & 15, p4 = lane >> 4;
  const int sub = c16 / WP, az = c16 % WP;
  float *tile = lds + wave * P3;
  float *wt = lds + NW * P3 + wave * (16 * WT_SPREAD);
  const int len = it.end - it.start, per = (len + NW - 1) / NW;
  const int s = it.start + min(len, wave * per), e = it.start + min(len, (wave + 1) * per);
  // run key: the cell, or with ZM its (x, y) column
  const uint32_t keymask = ZM ? 0x000fffffu : 0xffffffffu;

  float cf[4][WIN_NC];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int o = 4 * (lane & 3) + u;   // the offsets this lane evaluates in fill_weights
#pragma unroll
    for (int k = 0; k < WIN_NC; ++k) cf[u][k] = wcoef[o * WIN_NC + k];   // rows 2m..15 of the table are 0
  }
  f32x4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint32_t cur = 0xffffffffu;

  // add the accumulators of the run `cell` into the private tile
  auto flush = [&](uint32_t cell) {
    const int lx = (int)(cell & 1023u) - ox, ly = (int)((cell >> 10) & 1023u) - oy;
    const int lz = ZM ? 0 : (int)(cell >> 20) - oz;
    const bool zok = ZM ? (az < P) : (az < W);
    float old[NB][4];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int ay = S * nb + sub;
      const float *base = tile + lx * PX + (ly + ay) * P + lz + az;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ax = 4 * p4 + r;
        old[nb][r] = (zok && ay < W && ax < W) ? base[ax * PX] : 0.f;
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int ay = S * nb + sub;
      float *base = tile + lx * PX + (ly + ay) * P + lz + az;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ax = 4 * p4 + r;
        if (zok && ay < W && ax < W) base[ax * PX] = old[nb][r] + acc[nb][r];
      }
      acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };

  float4 qb, qn;
  float xb, xn;
  load_batch<IN, true>(pts, ka, s, e, lane, qb, xb);
  for (int b0 = s; b0 < e; b0 += 64) {
    load_batch<IN, true>(pts, ka, b0 + 64, e, lane, qn, xn);  // prefetch the next batch
    const int bcnt = min(64, e - b0);
    for (int sb = 0; sb * 16 < bcnt; ++sb) {
      const int cnt = min(16, bcnt - sb * 16);
      const int cellv = (int)fill_weights<W, true, WT_SPREAD>(qb, xb, sb, cnt, lane, cf, wt);
      wave_sync_lds();
      int j = 0;
      while (j < cnt) {
        const uint32_t key = (uint32_t)__builtin_amdgcn_readlane(cellv, j) & keymask;
        if (key != cur) {
          if (cur != 0xffffffffu) flush(cur);
          cur = key;
        }
        int k = 1;
        while (k < 4 && j + k < cnt &&
               ((uint32_t)__builtin_amdgcn_readlane(cellv, j + k) & keymask) == key)
          ++k;
        const int node = j + min(p4, k - 1);
        const float *w = wt + node * WT_SPREAD;
        const float xv = p4 < k ? w[3 * 16] : 0.f;
        const float a = xv * w[c16 & 15];
        float wz;
        if (ZM) {
          const int lzp = (int)((uint32_t)__shfl(cellv, node) >> 20) - oz;
          const int o = az - lzp;
          wz = (o >= 0 && o < W) ? w[2 * 16 + o] : 0.f;
        } else {
          wz = w[2 * 16 + (az & 15)];
        }
        float by[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) by[nb] = w[16 + S * nb + sub];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, by[nb] * wz, acc[nb], 0, 0, 0);
        j += k;
      }
      wave_sync_lds();
    }
    qb = qn;
    xb = xn;
  }
  if (cur != 0xffffffffu) flush(cur);
  __syncthreads();

  // sum the private tiles and add into the grid: each wave takes rows (px, py)
  // of the tile, 64 / ZL rows at a time with ZL >= P lanes along z
  const int mask = nos - 1;
  const double fx = fx_of(ka);
  const int ZL = P <= 16 ? 16 : (P <= 32 ? 32 : 64), RL = 64 / ZL;
  const int pz = lane % ZL, rsub = lane / ZL;
  for (int row0 = wave * RL; row0 < P * P; row0 += NW * RL) {
    const int row = row0 + rsub;
    if (row < P * P && pz < P) {
      const int px = row / P, py = row - px * P;
      const int o = px * PX + py * P + pz;
      float v;
      if constexpr (NW == 4) v = (lds[o] + lds[P3 + o]) + (lds[2 * P3 + o] + lds[3 * P3 + o]);
      else if constexpr (NW == 2) v = lds[o] + lds[P3 + o];
      else v = lds[o];
      if (v != 0.f) {
        const int gx = (ox - (M - 1) + px) & mask, gy = (oy - (M - 1) + py) & mask,
                  gz = (oz - (M - 1) + pz) & mask;
        grid_add(grid, ((size_t)gx * nos + gy) * nos + gz, v, fx);
      }
    }
  }
}

// Interpolation, the transpose of the spread: for up to 16 nodes p of one cell
//   D[ax][p] = sum_ay wy_p[ay] sum_az G[ax][ay][az] wz_p[az],  f_p = sum_ax wx_p[ax] D[ax][p],
// rows = x-offsets, columns = nodes, K over (ay, 4 consecutive az) in W * KZ
// steps (KZ = ceil(W/4)).  The cell's window G, read from the workgroup's
// shared LDS copy of the padded tile, is the register-resident A operand:
// lane l holds G[ax = l%16][ay][4 t + l/16].
template <int W, int IN, int OUT, int NW = 4>
__device__ __forceinline__ void interp3_mfma_body(const Item *__restrict__ items, int item,
                                                  const float4 *__restrict__ pts,
                                                  const KArgs ka,
                                                  const float *__restrict__ grid, int nos,
                                                  int tshift,
                                                  const float *__restrict__ wcoef) {
  constexpr int M = W / 2, KZ = (W + 3) / 4, NQ = W * KZ;
  extern __shared__ float lds[];
  const int T = 1 << tshift, P = T + W - 1, PP = P * P, PX = tile_px(P), P3 = PX * P;
  const Item it = items[item];
  const int ntd = nos >> tshift;
  const int tz = it.tile % ntd, ty = (it.tile / ntd) % ntd, tx = it.tile / (ntd * ntd);
  const int ox = tx * T, oy = ty * T, oz = tz * T;
  const int mask = nos - 1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  {
    // stage the padded tile: each wave takes rows (px, py), 64 / ZL at a time
    const int ZL = P <= 16 ? 16 : (P <= 32 ? 32 : 64), RL = 64 / ZL;
    const int pz = lane % ZL, rsub = lane / ZL;
    for (int row0 = wave * RL; row0 < PP; row0 += NW * RL) {
      const int row = row0 + rsub;
      if (row < PP && pz < P) {
        const int px = row / P, py = row - px * P;
        const int gx = (ox - (M - 1) + px) & mask, gy = (oy - (M - 1) + py) & mask,
                  gz = (oz - (M - 1) + pz) & mask;
        lds[px * PX + py * P + pz] = grid[((size_t)gx * nos + gy) * nos + gz];
      }
    }
  }
  __syncthreads();

  const int c16 = lane & 15, k4 = lane >> 4;
  float *wt = lds + P3 + wave * (16 * WT_INTERP);
  const int len = it.end - it.start, per = (len + NW - 1) / NW;
  const int s = it.start + min(len, wave * per), e = it.start + min(len, (wave + 1) * per);

  float cf[4][WIN_NC];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int o = 4 * (lane & 3) + u;   // the offsets this lane evaluates in fill_weights
#pragma unroll
    for (int k = 0; k < WIN_NC; ++k) cf[u][k] = wcoef[o * WIN_NC + k];   // rows 2m..15 of the table are 0
  }
  float g[NQ];
  uint32_t cur = 0xffffffffu;
  float4 qb, qn;
  float xb, xn;
  load_batch<IN, false>(pts, ka, s, e, lane, qb, xb);
  for (int b0 = s; b0 < e; b0 += 64) {
    load_batch<IN, false>(pts, ka, b0 + 64, e, lane, qn, xn);  // prefetch the next batch
    const int bcnt = min(64, e - b0);
    for (int sb = 0; sb * 16 < bcnt; ++sb) {
      const int cnt = min(16, bcnt - sb * 16);
      const int i0 = b0 + sb * 16;
      const int cellv = (int)fill_weights<W, false, WT_INTERP>(qb, xb, sb, cnt, lane, cf, wt);
      wave_sync_lds();
      int j = 0;
      while (j < cnt) {
        const uint32_t cell = (uint32_t)__builtin_amdgcn_readlane(cellv, j);
        if (cell != cur) {
          cur = cell;
          const int lx = (int)(cell & 1023u) - ox, ly = (int)((cell >> 10) & 1023u) - oy,
                    lz = (int)(cell >> 20) - oz;
          const float *base = lds + (lx + c16) * PX + ly * P + lz;
#pragma unroll
          for (int ay = 0; ay < W; ++ay)
#pragma unroll
            for (int t = 0; t < KZ; ++t) {
              const int zz = 4 * t + k4;
              g[ay * KZ + t] = (c16 < W && zz < W) ? base[ay * P + zz] : 0.f;
            }
        }
        int k = 1;
        while (k < 16 && j + k < cnt && (uint32_t)__builtin_amdgcn_readlane(cellv, j + k) == cell) ++k;
        const float *w = wt + (j + min(c16, k - 1)) * WT_INTERP;
        float wyv[W], wzv[KZ], wxv[4];
#pragma unroll
        for (int ay = 0; ay < W; ++ay) wyv[ay] = w[16 + ay];
#pragma unroll
        for (int t = 0; t < KZ; ++t) wzv[t] = w[32 + ((4 * t + k4) & 15)];
#pragma unroll
        for (int r = 0; r < 4; ++r) wxv[r] = w[(4 * k4 + r) & 15];
        f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ay = 0; ay < W; ++ay)
#pragma unroll
          for (int t = 0; t < KZ; ++t)
            d = __builtin_amdgcn_mfma_f32_16x16x4f32(g[ay * KZ + t], wyv[ay] * wzv[t], d, 0, 0, 0);
        float part = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * k4 + r < W) part = fmaf(wxv[r], d[r], part);
        part = sum_rows4(part);
        if (k4 == 0 && c16 < k) store_out<OUT>(ka, i0 + j + c16, part);
        j += k;
      }
      wave_sync_lds();
    }
    qb = qn;
    xb = xn;
  }
}


// ---------------------------------------------------------------------------
// Tile-stationary spread and interpolation (T + W - 1 <= 16).
//
// All nodes of a work item lie in one T^3 tile, so all their windows lie in
// the padded tile of P = T + W - 1 <= 16 cells per axis, and the 16 x 16 block
// of v_mfma_f32_16x16x4_f32 covers a whole x-by-z slice of it.  With the
// window rows of every node shifted to its cell's place in the padded tile,
// the contraction runs over arbitrary groups of 4 nodes, whatever their cells:
//   spread:  G[ax][ay][az] += sum_p (x_p wx_p[ax]) (wy_p[ay] wz_p[az]),
//            rows ax, K = 4 nodes, columns az, one accumulator per ay (P of
//            them): the wave's whole padded tile stays in registers, so there
//            are no per-cell runs and no per-run flushes; at the end the
//            waves add their tiles into one LDS copy (ds_add_f32), which is
//            added into the grid with global atomics;
//   interp:  D[ax][p] = sum_{ay,az} G[ax][ay][az] wy_p[ay] wz_p[az] with the
//            item's padded tile as the register-resident A operand (loaded
//            once per item), 16 nodes as the columns, K = (ay, az) in 4P
//            steps; f_p = sum_ax wx_p[ax] D[ax][p].
// Weight table per wave: 16 node rows of TS_PITCH words, the shifted x, y and
// z rows at word 0, 32 and 64 (row entries outside the node's window are 0),
// the node's cell y inside the tile at word 96.  In the spread, matrix
// instructions whose y-slice lies outside the windows of all four of their
// nodes (exact zeros) are skipped with a wave-uniform branch.
// The LDS tile is laid out [ax][ay * 16 + az] with row stride TS_XS(P).
// ---------------------------------------------------------------------------
// Row pitches: the spread reads two node rows per half-wave (pitch = 16 mod
// 32 puts them 16 banks apart); the interpolation reads 16 node rows per
// half-wave, including 16-byte reads (pitch/4 odd: eight consecutive rows in
// distinct 4-bank groups).
constexpr int TS_PITCH = 112, TS_PITCH_I = 100;

__host__ __device__ constexpr int ts_xs(int P) { return P * 16 + 4; }   // 4 rows apart = 16 banks

// Fill the shifted weight rows of sub-batch nodes sub*16 .. sub*16+15: lane l
// evaluates node l/4 at offsets U (l%4) .. +U-1, U = ceil(W/4) (the offsets at
// or past W have zero polynomials), and writes them at offset + its cell's
// position in the tile.  The readers use [0, 16) of each 32-float segment: the
// entries there outside the window are zeroed first ([0, T) and [4U, 16)), and
// the window values written after them (one wave's LDS writes execute in
// order).  SPREAD: the x row carries x_p wx_p (x_p = 0 for nodes past cnt).
template <int W>
constexpr int fill_upl() { return (W + 3) / 4; }

// YREL: the y weights stay relative to the node's own window (y' = offset,
// no shift by the cell, no zero padding), for runs of nodes that share their
// cell's y inside the tile.  `first`: batch lane of the run's first node.
template <int T, int W, bool SPREAD, int PITCH, bool YREL = false>
__device__ __forceinline__ void fill_shifted(const float4 &qb, float xb, int first, int cnt,
                                             int lane, const float (&cf)[fill_upl<W>()][WIN_NC],
                                             float *wt, int ox, int oy, int oz) {
  constexpr int U = fill_upl<W>();
  static_assert(T % 4 == 0 && T + 16 <= 32, "row segment layout");
  const int node = lane >> 2, part = lane & 3;
  const int src = first + min(node, cnt - 1);
  const float qx = __shfl(qb.x, src), qy = __shfl(qb.y, src), qz = __shfl(qb.z, src);
  const uint32_t cell = (uint32_t)__shfl((int)__float_as_uint(qb.w), src);
  float xv = 1.f;
  if constexpr (SPREAD) {
    xv = __shfl(xb, src);
    if (node >= cnt) xv = 0.f;
  }
  const int lx = (int)(cell & 1023u) - ox, ly = (int)((cell >> 10) & 1023u) - oy,
            lz = (int)(cell >> 20) - oz;
  float *row = wt + node * PITCH;
  if (part == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (YREL && a == 1) continue;
#pragma unroll
      for (int z = 0; z < T; z += 4)
        *reinterpret_cast<float4 *>(row + 32 * a + z) = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int z = 4 * U; z < 16; z += 4)
        *reinterpret_cast<float4 *>(row + 32 * a + z) = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int o = U * part + u;
    row[lx + o] = xv * win_poly(cf[u], qx);
    row[32 + (YREL ? 0 : ly) + o] = win_poly(cf[u], qy);
    row[64 + lz + o] = win_poly(cf[u], qz);
  }
}

// fill_shifted with the window coefficients read from LDS (cft: WIN_MAXW rows
// of WIN_NC floats) at each use instead of being held in registers.
// ZREL: the z weights stay relative to the node's own window (z' = offset,
// no shift by the cell and no zero padding): for runs of nodes that share
// their cell's z inside the tile.  `first` is the batch lane of the first
// node of the run.
template <int T, int W, bool SPREAD, int PITCH, bool ZREL = false, bool YREL = false>
__device__ __forceinline__ void fill_shifted_lds(const float4 &qb, float xb, int first, int cnt,
                                                 int lane, const float *cft, float *wt, int ox,
                                                 int oy, int oz) {
  constexpr int U = fill_upl<W>();
  static_assert(T % 4 == 0 && T + 16 <= 32, "row segment layout");
  static_assert(WIN_NC % 4 == 0, "coefficient rows are read as float4");
  const int node = lane >> 2, part = lane & 3;
  const int src = first + min(node, cnt - 1);
  const float qx = __shfl(qb.x, src), qy = __shfl(qb.y, src), qz = __shfl(qb.z, src);
  const uint32_t cell = (uint32_t)__shfl((int)__float_as_uint(qb.w), src);
  float xv = 1.f;
  if constexpr (SPREAD) {
    xv = __shfl(xb, src);
    if (node >= cnt) xv = 0.f;
  }
  const int lx = (int)(cell & 1023u) - ox, ly = (int)((cell >> 10) & 1023u) - oy,
            lz = (int)(cell >> 20) - oz;
  float *row = wt + node * PITCH;
  if (part == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if ((ZREL && a == 2) || (YREL && a == 1)) continue;
#pragma unroll
      for (int z = 0; z < T; z += 4)
        *reinterpret_cast<float4 *>(row + 32 * a + z) = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int z = 4 * U; z < 16; z += 4)
        *reinterpret_cast<float4 *>(row + 32 * a + z) = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int o = U * part + u;
    float c[WIN_NC];
    const float4 *cp = reinterpret_cast<const float4 *>(cft + o * WIN_NC);
#pragma unroll
    for (int k = 0; k < WIN_NC / 4; ++k) {
      const float4 t = cp[k];
      c[4 * k] = t.x;
      c[4 * k + 1] = t.y;
      c[4 * k + 2] = t.z;
      c[4 * k + 3] = t.w;
    }
    row[lx + o] = xv * win_poly(c, qx);
    row[32 + (YREL ? 0 : ly) + o] = win_poly(c, qy);
    row[64 + (ZREL ? 0 : lz) + o] = win_poly(c, qz);
  }
}

// Spread tile layout in LDS once the weight tables are free: [ax][az][ay],
// ay fastest, z stride 17 and x stride ts_sxs(P) = 4 mod 8 words.  The
// accumulator stores (16 consecutive ay per row of lanes, four x rows 16
// banks apart) and the flush reads (16 consecutive az, odd stride) are then
// free of bank conflicts.
constexpr int TS_SZS = 17;
__host__ __device__ constexpr int ts_sxs(int P) { return (P * TS_SZS + 3) / 8 * 8 + 4; }

// LDS of the tile spread, in floats: the weight tables of NW waves and the
// window coefficients during the accumulation, then up to two tile copies.
__host__ __device__ constexpr int spread_tile_lds_floats(int P, int NW) {
  const int run = NW * 16 * TS_PITCH + WIN_MAXW * WIN_NC;
  const int sum = (NW >= 2 ? 2 : 1) * 16 * ts_sxs(P);
  return run > sum ? run : sum;
}

// The 4-node steps of one run of the spread (nodes sharing their cell's z
// offset L inside the tile, z rows relative to the window): W z-slices per
// step into accumulators L .. L + W - 1 (x rows by y columns).  Two operand
// sets: the operands of step st + 1 are loaded (always: rows 4 (st + 1) + p4
// < 16 lie in the table) while the matrix instructions of step st issue.
// Steps past nst are skipped whole.
template <int L, int W, int P, int PITCH>
__device__ __forceinline__ void spread_zrun_steps(f32x4 (&acc)[P], const float *wt, int nst,
                                                  int c16, int p4) {
  static_assert(L + W <= P, "the run's window lies in the padded tile");
  constexpr int WQ = (W + 3) / 4;
  float a[2], wy[2], wz[2][4 * WQ];
  auto load_step = [&](int st, float &a_, float &wy_, float (&wz_)[4 * WQ]) {
    const float *w = wt + (4 * st + p4) * PITCH;
    a_ = w[c16];
    wy_ = w[32 + c16];
#pragma unroll
    for (int q = 0; q < WQ; ++q) {
      const float4 v = *reinterpret_cast<const float4 *>(w + 64 + 4 * q);
      wz_[4 * q] = v.x;
      wz_[4 * q + 1] = v.y;
      wz_[4 * q + 2] = v.z;
      wz_[4 * q + 3] = v.w;
    }
  };
  load_step(0, a[0], wy[0], wz[0]);
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int c = st & 1;
    if (st + 1 < 4) load_step(st + 1, a[c ^ 1], wy[c ^ 1], wz[c ^ 1]);
    if (st < nst) {
#pragma unroll
      for (int z = 0; z < W; ++z)
        acc[L + z] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], wz[c][z] * wy[c], acc[L + z], 0, 0, 0);
    }
  }
}

// The nodes of one 64-node batch whose cell has z offset L in the tile (a
// contiguous range of lanes: a tile's nodes are sorted z-major), in runs of
// up to 16.  L is a compile-time constant in each call, so every matrix
// instruction names its accumulator statically and the accumulators stay in
// place across the classes.
template <int L, int T, int W, int P>
__device__ __forceinline__ void spread_zclass(f32x4 (&acc)[P], int lzl, int bcnt, int lane,
                                              const float4 &qb, float xb, const float *cft,
                                              float *wt, int ox, int oy, int oz, int c16, int p4) {
  const unsigned long long m = __ballot(lane < bcnt && lzl == L);
  if (m == 0) return;
  const int p0 = __builtin_ctzll(m), pe = p0 + __popcll(m);
  for (int pos = p0; pos < pe; pos += 16) {
    const int cnt = min(16, pe - pos);
    fill_shifted_lds<T, W, true, TS_PITCH, true>(qb, xb, pos, cnt, lane, cft, wt, ox, oy, oz);
    wave_sync_lds();
    spread_zrun_steps<L, W, P, TS_PITCH>(acc, wt, (cnt + 3) >> 2, c16, p4);
    wave_sync_lds();
  }
}

template <int L, int T, int W, int P>
__device__ __forceinline__ void spread_zclasses(f32x4 (&acc)[P], int lzl, int bcnt, int lane,
                                                const float4 &qb, float xb, const float *cft,
                                                float *wt, int ox, int oy, int oz, int c16,
                                                int p4) {
  if constexpr (L < T) {
    spread_zclass<L, T, W, P>(acc, lzl, bcnt, lane, qb, xb, cft, wt, ox, oy, oz, c16, p4);
    spread_zclasses<L + 1, T, W, P>(acc, lzl, bcnt, lane, qb, xb, cft, wt, ox, oy, oz, c16, p4);
  }
}

template <int W, int T, int IN, int NW = 4>
__device__ __forceinline__ void spread3_tile_body(const Item it, const float4 *__restrict__ pts,
                                                  const KArgs ka, float *__restrict__ grid,
                                                  int nos, const float *__restrict__ wcoef) {
  constexpr int M = W / 2, P = T + W - 1, XS = ts_sxs(P);
  static_assert(P <= 16, "tile-stationary form needs T + W - 1 <= 16");
  static_assert(P - W + 1 == T, "z classes 0 .. T - 1");
  extern __shared__ float lds[];
  const int ntd = nos / T;
  const int tz = it.tile % ntd, ty = (it.tile / ntd) % ntd, tx = it.tile / (ntd * ntd);
  const int ox = tx * T, oy = ty * T, oz = tz * T;

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int c16 = lane & 15, p4 = lane >> 4;
  float *wt = lds + wave * (16 * TS_PITCH);
  const int len = it.end - it.start, per = (len + NW - 1) / NW;
  const int s = it.start + min(len, wave * per), e = it.start + min(len, (wave + 1) * per);

  // the first batch loads while the window coefficients (rows 2m..15 are 0)
  // are staged after the weight tables
  float4 qb, qn;
  float xb, xn;
  load_batch<IN, true>(pts, ka, s, e, lane, qb, xb);
  float *cft = lds + NW * 16 * TS_PITCH;
  for (int q = threadIdx.x; q < WIN_MAXW * WIN_NC; q += NW * 64) cft[q] = wcoef[q];
  __syncthreads();
  f32x4 acc[P];
#pragma unroll
  for (int z = 0; z < P; ++z) acc[z] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int b0 = s; b0 < e; b0 += 64) {
    load_batch<IN, true>(pts, ka, b0 + 64, e, lane, qn, xn);  // prefetch the next batch
    const int bcnt = min(64, e - b0);
    const int lzl = (int)(__float_as_uint(qb.w) >> 20) - oz;
    spread_zclasses<0, T, W, P>(acc, lzl, bcnt, lane, qb, xb, cft, wt, ox, oy, oz, c16, p4);
    qb = qn;
    xb = xn;
  }
  // Sum the waves' tiles without LDS atomics (measured far slower than plain
  // LDS traffic): once every wave is done with its weight table, waves 0 and 1
  // store their tiles into copies C0 and C1 (in the LDS of the tables), then
  // waves 2 and 3 add theirs into C0 and C1; the flush adds C0 + C1.
  constexpr int NC = NW >= 2 ? 2 : 1;
  static_assert(NW == 1 || NW == 2 || NW == 4, "one, two or four waves");
  __syncthreads();
  {
    // copies of 16 x-rows (row 15 and y-columns >= P are written, never read)
    float *cp = lds + (wave % NC) * (16 * XS) + (4 * p4) * XS + c16;
    if (wave < NC) {
#pragma unroll
      for (int z = 0; z < P; ++z)
#pragma unroll
        for (int r = 0; r < 4; ++r) cp[r * XS + z * TS_SZS] = acc[z][r];
    }
    __syncthreads();
    if (NW == 4 && wave >= NC) {
      // read-add-write in groups of 4 z-slices: 16 loads in flight at a time
#pragma unroll
      for (int z0 = 0; z0 < P; z0 += 4) {
        float old[4][4];
#pragma unroll
        for (int z = z0; z < z0 + 4 && z < P; ++z)
#pragma unroll
          for (int r = 0; r < 4; ++r) old[z - z0][r] = cp[r * XS + z * TS_SZS];
#pragma unroll
        for (int z = z0; z < z0 + 4 && z < P; ++z)
#pragma unroll
          for (int r = 0; r < 4; ++r) cp[r * XS + z * TS_SZS] = old[z - z0][r] + acc[z][r];
      }
    }
    __syncthreads();
  }
  // into the grid: each wave takes rows (px, py), four at a time, z along
  // lanes; all its LDS reads are issued before the first global add
  const int mask = nos - 1;
  const double fx = fx_of(ka);
  const int pz = lane & 15, rsub = lane >> 4;
  constexpr int NRG = (P * P + NW * 4 - 1) / (NW * 4);   // row groups per wave
  float fv[NRG];
#pragma unroll
  for (int k = 0; k < NRG; ++k) {
    const int row = wave * 4 + k * (NW * 4) + rsub;
    fv[k] = 0.f;
    if (row < P * P && pz < P) {
      const int px = row / P, py = row - px * P;
      const int o = px * XS + pz * TS_SZS + py;
      fv[k] = NC == 2 ? lds[o] + lds[16 * XS + o] : lds[o];
    }
  }
#pragma unroll
  for (int k = 0; k < NRG; ++k) {
    const int row = wave * 4 + k * (NW * 4) + rsub;
    if (fv[k] != 0.f) {   // (rows past P * P and z past P hold 0)
      const int px = row / P, py = row - px * P;
      const int gx = (ox - (M - 1) + px) & mask, gy = (oy - (M - 1) + py) & mask,
                gz = (oz - (M - 1) + pz) & mask;
      grid_add(grid, ((size_t)gx * nos + gy) * nos + gz, fv[k], fx);
    }
  }
}

template <int W, int T, int IN, int OUT, int NW = 4>
__device__ __forceinline__ void interp3_tile_body(const Item *__restrict__ items, int item,
                                                  const float4 *__restrict__ pts,
                                                  const KArgs ka,
                                                  const float *__restrict__ grid, int nos,
                                                  const float *__restrict__ wcoef,
                                                  double *dot_acc = nullptr) {
  constexpr int M = W / 2, P = T + W - 1, XS = ts_xs(P);
  static_assert(P <= 16, "tile-stationary form needs T + W - 1 <= 16");
  extern __shared__ float lds[];
  float *tile = lds;
  const Item it = items[item];
  const int ntd = nos / T;
  const int tz = it.tile % ntd, ty = (it.tile / ntd) % ntd, tx = it.tile / (ntd * ntd);
  const int ox = tx * T, oy = ty * T, oz = tz * T;
  const int mask = nos - 1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int c16 = lane & 15, p4 = lane >> 4;
  // Stage the padded tile (z padded to 16 with zeros): the wave issues all its
  // loads before its first LDS store, so they wait once, not once per row
  // group, and the first batch's records load before the barrier.
  constexpr int NRG = (P * P + NW * 4 - 1) / (NW * 4);   // row groups per wave
  float stg[NRG];
#pragma unroll
  for (int k = 0; k < NRG; ++k) {
    const int row = wave * 4 + k * (NW * 4) + p4;
    stg[k] = 0.f;
    if (row < P * P && c16 < P) {
      const int px = row / P, py = row - px * P;
      const int gx = (ox - (M - 1) + px) & mask, gy = (oy - (M - 1) + py) & mask,
                gz = (oz - (M - 1) + c16) & mask;
      stg[k] = grid[((size_t)gx * nos + gy) * nos + gz];
    }
  }
  // Nodes are taken in runs of <= 16 that share their cell's z inside the tile
  // (the sort orders a tile's nodes z-major, so a run is usually 16 long):
  // their z windows coincide, so K = (padded y, z window) needs ZQ = W/4
  // quads per y instead of the 4 of the whole padded z extent.
  // A operand for the run's z offset lz: lane (row c16, k = p4) holds
  // G[c16][y][lz + 4 zq + p4] at step y ZQ + zq; reloaded when lz changes.
  constexpr int ZQ = (W + 3) / 4, NK = P * ZQ;
  static_assert(T + 4 * ZQ <= 17, "the shifted z window stays inside a 16-wide tile row");
  float g[NK];
  int cur_lz = -1;

  float *wt = lds + P * XS + wave * (16 * TS_PITCH_I);
  float *cft = lds + P * XS + NW * 16 * TS_PITCH_I;   // window coefficients after the tables
  const int len = it.end - it.start, per = (len + NW - 1) / NW;
  const int s = it.start + min(len, wave * per), e = it.start + min(len, (wave + 1) * per);
  float4 qb, qn;
  float xb, xn;
  OutPre ob, on;
  load_batch<IN, false>(pts, ka, s, e, lane, qb, xb);
  pre_index<OUT>(ka, s + lane, s + lane < e, ob);
#pragma unroll
  for (int k = 0; k < NRG; ++k) {
    const int row = wave * 4 + k * (NW * 4) + p4;
    if (row < P * P) {
      const int px = row / P, py = row - px * P;
      tile[px * XS + py * 16 + c16] = stg[k];
    }
  }
  // (rows 2m..15 of the coefficient table are 0)
  for (int q = threadIdx.x; q < WIN_MAXW * WIN_NC; q += NW * 64) cft[q] = wcoef[q];
  __syncthreads();
  pre_gather<OUT>(ka, s + lane < e, ob);
  for (int b0 = s; b0 < e; b0 += 64) {
    // prefetch the next batch: records, permutation entries, d^{-1/2}
    load_batch<IN, false>(pts, ka, b0 + 64, e, lane, qn, xn);
    pre_index<OUT>(ka, b0 + 64 + lane, b0 + 64 + lane < e, on);
    const int bcnt = min(64, e - b0);
    const int lzl = (int)(__float_as_uint(qb.w) >> 20) - oz;   // this lane's node: z in the tile
    int cnt;
    for (int pos = 0; pos < bcnt; pos += cnt) {
      const int lz0 = __builtin_amdgcn_readlane(lzl, pos);
      const unsigned long long same = __ballot(lane < bcnt && lzl == lz0);
      // run length from pos: the trailing ones of same >> pos (all 64 bits are
      // ones when pos = 0 and the whole batch shares lz: ctz of 0 is undefined)
      const unsigned long long rest = ~(same >> pos);
      const int run = rest ? __builtin_ctzll(rest) : 64;            // >= 1: the node at pos
      cnt = min(16, min(run, bcnt - pos));
      if (lz0 != cur_lz) {
        cur_lz = lz0;
        // rows c16 >= P read row P - 1 and are zeroed by a select (a
        // conditional read per element costs an exec-mask save and restore)
        const float *trow = tile + min(c16, P - 1) * XS + lz0 + p4;
#pragma unroll
        for (int y = 0; y < P; ++y)
#pragma unroll
          for (int zq = 0; zq < ZQ; ++zq) {
            const float v = trow[y * 16 + 4 * zq];
            g[y * ZQ + zq] = c16 < P ? v : 0.f;
          }
      }
      const int i0 = b0 + pos;
      const OutPre op = pre_from<OUT>(ob, pos + c16);
      fill_shifted_lds<T, W, false, TS_PITCH_I, true>(qb, xb, pos, cnt, lane, cft, wt, ox, oy, oz);
      wave_sync_lds();
      const float *w = wt + c16 * TS_PITCH_I;    // column c16 = node c16
      float wzq[ZQ], wy[16];
#pragma unroll
      for (int q = 0; q < ZQ; ++q) wzq[q] = w[64 + 4 * q + p4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = *reinterpret_cast<const float4 *>(w + 32 + 4 * q);
        wy[4 * q] = v.x;
        wy[4 * q + 1] = v.y;
        wy[4 * q + 2] = v.z;
        wy[4 * q + 3] = v.w;
      }
      // two accumulator chains: a chain's next instruction comes two matrix
      // instructions later, past the result latency
      f32x4 d[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) d[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < NK; ++st)
        d[st & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(g[st], wy[st / ZQ] * wzq[st % ZQ],
                                                         d[st & 1], 0, 0, 0);
      float part = 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) part = fmaf(w[4 * p4 + r], d[0][r] + d[1][r], part);
      part = sum_rows4(part);
      if (p4 == 0 && c16 < cnt) {
        const double t = store_pre<OUT>(ka, i0 + c16, part, op);
        if constexpr (OUT == OUT_SORTED_F64_SSL)
          if (dot_acc) *dot_acc += t;   // this lane's nodes, in the order they come
      }
      wave_sync_lds();
    }
    qb = qn;
    xb = xn;
    // the next batch's caller-order gather lands during its first sub-batch
    ob = on;
    pre_gather<OUT>(ka, b0 + 64 + lane < e, ob);
  }
}

// ---------------------------------------------------------------------------
// FFT: Stockham autosort in LDS on `nl` lines of length L = nos (a power of
// 2), radix-4 passes and one radix-2 pass when log2 L is odd.  A pass that
// merges r sub-transforms of length m reads x_t = a[j + t L/r] (t < r),
// multiplies by w^{t k} (w = e^{-2 pi i/(r m)}, k = j mod m), takes the
// r-point DFT over t and writes output u to b[(j/m) r m + u m + k].  The
// twiddles come from an LDS table twl[k] = e^{-2 pi i k/L}, k < L, which each
// kernel fills from the global half table (e^{-2 pi i k/L}, k < L/2) before
// its first barrier.  SIGN = +1 gives the inverse (unnormalised) transform.
// The result is returned in `a` (buffers are swapped).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

constexpr int FFT_THREADS = 256, FFT_ELEMS = 512, FFT_MAXL = 512;

__device__ __forceinline__ void load_twiddles(float2 *twl, const float2 *__restrict__ tw, int L) {
  for (int k = threadIdx.x; k < L / 2; k += FFT_THREADS) {
    const float2 w = tw[k];
    twl[k] = w;
    twl[k + L / 2] = make_float2(-w.x, -w.y);
  }
}

template <int SIGN>
__device__ void lds_fft(float2 *&a, float2 *&b, int L, int logL, int nl,
                        const float2 *__restrict__ twl) {
  int logm = 0;
  while (logm < logL) {
    const int m = 1 << logm;
    if (logL - logm >= 2) {
      const int Lr = L >> 2, sh = logL - 2 - logm;
      for (int idx = threadIdx.x; idx < nl * Lr; idx += FFT_THREADS) {
        const int line = idx >> (logL - 2), j = idx & (Lr - 1);
        const int k = j & (m - 1), g = j >> logm;
        const float2 *src = a + line * L + j;
        const float2 x0 = src[0];
        float2 x1 = src[Lr], x2 = src[2 * Lr], x3 = src[3 * Lr];
        const int st = k << sh;
        float2 w1 = twl[st], w2 = twl[2 * st], w3 = twl[3 * st];
        if (SIGN > 0) {
          w1.y = -w1.y;
          w2.y = -w2.y;
          w3.y = -w3.y;
        }
        x1 = cmul(x1, w1);
        x2 = cmul(x2, w2);
        x3 = cmul(x3, w3);
        const float2 s02 = make_float2(x0.x + x2.x, x0.y + x2.y);
        const float2 d02 = make_float2(x0.x - x2.x, x0.y - x2.y);
        const float2 s13 = make_float2(x1.x + x3.x, x1.y + x3.y);
        const float2 d13 = make_float2(x1.x - x3.x, x1.y - x3.y);
        // -i d13 (forward) or +i d13 (inverse)
        const float2 rd = SIGN < 0 ? make_float2(d13.y, -d13.x) : make_float2(-d13.y, d13.x);
        float2 *dst = b + line * L + (g << (logm + 2)) + k;
        dst[0] = make_float2(s02.x + s13.x, s02.y + s13.y);
        dst[m] = make_float2(d02.x + rd.x, d02.y + rd.y);
        dst[2 * m] = make_float2(s02.x - s13.x, s02.y - s13.y);
        dst[3 * m] = make_float2(d02.x - rd.x, d02.y - rd.y);
      }
      logm += 2;
    } else {
      const int half_n = L >> 1;
      for (int idx = threadIdx.x; idx < nl * half_n; idx += FFT_THREADS) {
        const int line = idx >> (logL - 1), j = idx & (half_n - 1);
        const int k = j & (m - 1), g = j >> logm;
        float2 w = twl[k << (logL - 1 - logm)];
        if (SIGN > 0) w.y = -w.y;
        const float2 x0 = a[line * L + j], x1 = a[line * L + j + half_n];
        const float2 t = cmul(w, x1);
        const int o = line * L + (g << (logm + 1)) + k;
        b[o] = make_float2(x0.x + t.x, x0.y + t.y);
        b[o + m] = make_float2(x0.x - t.x, x0.y - t.y);
      }
      logm += 1;
    }
    __syncthreads();
    float2 *tmp = a;
    a = b;
    b = tmp;
  }
}

// LDS of one FFT workgroup: two buffers of lpb lines and the twiddle table.
__host__ __device__ __forceinline__ size_t fft_lds_bytes(int lpb, int L) {
  return ((size_t)2 * lpb * L + L) * 8;
}

// Lines per workgroup of each pass for lines of length L, N = L/2, with at
// most `elems` complex values per workgroup:
//   z passes (r2c / c2r): elems / L lines;
//   y passes: the Hz = N/2 + 1 columns split into equal groups of at most
//     elems / L;
//   x pass: enough workgroups (>= 1024) for the (N+1)(N/2+1) columns.
// The single-plan product uses FFT_ELEMS_PLAN for lines of up to 128: its
// passes are latency bound and gain from more, smaller workgroups (at the
// benchmark workload 190.6 -> 189.0 us per product with 256 instead of 512;
// 195.6 with 128, 195.6 with 1024; at L = 256 the five passes took 92
// instead of 74 us); the batched launch, whose passes cover hundreds of
// grids, keeps FFT_ELEMS (4.32 ms per batch; 4.92 with 256).
constexpr int FFT_ELEMS_PLAN = 256;
__host__ __device__ __forceinline__ int fft_lpb_z(int L, int elems = FFT_ELEMS) {
  return L >= elems ? 1 : elems / L;
}
// real lines per workgroup of the r2c / c2r passes (two per complex line)
__host__ __device__ __forceinline__ int fft_lpb_zr(int L, int elems = FFT_ELEMS) {
  return 2 * fft_lpb_z(L, elems);
}
__host__ __device__ __forceinline__ int fft_lpb_y(int L, int elems = FFT_ELEMS) {
  const int Hz = L / 4 + 1, mx = fft_lpb_z(L, elems);
  const int groups = (Hz + mx - 1) / mx;
  return (Hz + groups - 1) / groups;
}
__host__ __device__ __forceinline__ int fft_lpb_x(int L, int elems = FFT_ELEMS) {
  const int C = (L / 2 + 1) * (L / 4 + 1);
  int l = C / 1024;
  if (l < 1) l = 1;
  const int mx = fft_lpb_z(L, elems);
  return l > mx ? mx : l;
}

// Real lines along the last (contiguous) axis -> half spectrum lz in [0, Hz).
// Two real lines a, b go through one complex transform of z = a + i b; with
// Z = FFT(z): A[k] = (Z[k] + conj Z[-k]) / 2, B[k] = (Z[k] - conj Z[-k]) / (2i).
// lpb real lines (an even number) per workgroup.  ZERO: each input element is
// set to 0 after it is read (every element is read once, by one thread), which
// leaves the spread grid clear for the next product.
// fx_max non-null: the grid holds the deterministic spread's int64 fixed-point
// values (scaled by fx_scale(*fx_max, fx_mult)), converted here.
// lines non-null: the block's lines are lines[l0 ..] (a list of line
// indices, e.g. the lines some node's window touches) instead of l0 ...
template <bool ZERO = false>
__device__ __forceinline__ void r2c_lines_body(int blk, float *__restrict__ grid,
                                               float2 *__restrict__ H, int nlines, int L,
                                               int logL, int lpb, int Hz,
                                               const float2 *__restrict__ tw,
                                               const unsigned *__restrict__ fx_max = nullptr,
                                               float fx_mult = 0.f,
                                               const int *__restrict__ lines = nullptr) {
  extern __shared__ float2 sm[];
  const int np = lpb >> 1;
  float2 *a = sm, *b = sm + np * L, *twl = sm + 2 * np * L;
  load_twiddles(twl, tw, L);
  const int l0 = blk * lpb;
  const int nl = min(lpb, nlines - l0), npp = (nl + 1) >> 1;
  auto line = [&](int li) { return lines ? lines[l0 + li] : l0 + li; };
  if (fx_max) {
    const double inv = 1.0 / fx_scale(fx_bits(fx_max), fx_mult);   // a power of 2: exact
    for (int idx = threadIdx.x; idx < npp * L; idx += FFT_THREADS) {
      const int pl = idx / L, j = idx - pl * L;
      const bool two = 2 * pl + 1 < nl;
      long long *pa = reinterpret_cast<long long *>(grid) + (size_t)line(2 * pl) * L + j;
      long long *pb = two ? reinterpret_cast<long long *>(grid) + (size_t)line(2 * pl + 1) * L + j : pa;
      const float re = (float)((double)pa[0] * inv);
      const float im = two ? (float)((double)pb[0] * inv) : 0.f;
      a[idx] = make_float2(re, im);
      if (ZERO) {
        pa[0] = 0;
        if (two) pb[0] = 0;
      }
    }
  } else {
    for (int idx = threadIdx.x; idx < npp * L; idx += FFT_THREADS) {
      const int pl = idx / L, j = idx - pl * L;
      const bool two = 2 * pl + 1 < nl;
      float *pa = grid + (size_t)line(2 * pl) * L + j;
      float *pb = two ? grid + (size_t)line(2 * pl + 1) * L + j : pa;
      const float re = *pa;
      const float im = two ? *pb : 0.f;
      a[idx] = make_float2(re, im);
      if (ZERO) {
        *pa = 0.f;
        if (two) *pb = 0.f;
      }
    }
  }
  __syncthreads();
  lds_fft<-1>(a, b, L, logL, npp, twl);
  for (int idx = threadIdx.x; idx < nl * Hz; idx += FFT_THREADS) {
    const int li = idx / Hz, k = idx - li * Hz, pl = li >> 1;
    const float2 zk = a[pl * L + k], zm = a[pl * L + ((L - k) & (L - 1))];
    H[(size_t)line(li) * Hz + k] = (li & 1) == 0
                                       ? make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y))
                                       : make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
  }
}

// Half spectra (lz in [0, Hz), Hermitian in lz, zero beyond) -> real lines,
// two per complex transform: IFFT(A + i B) = a + i b for real a, b.
__device__ __forceinline__ void c2r_lines_body(int blk, const float2 *__restrict__ H,
                                               float *__restrict__ grid, int nlines, int L,
                                               int logL, int lpb, int Hz,
                                               const float2 *__restrict__ tw,
                                               const int *__restrict__ lines = nullptr) {
  extern __shared__ float2 sm[];
  const int np = lpb >> 1;
  float2 *a = sm, *b = sm + np * L, *twl = sm + 2 * np * L;
  load_twiddles(twl, tw, L);
  const int l0 = blk * lpb;
  const int nl = min(lpb, nlines - l0), npp = (nl + 1) >> 1;
  auto line = [&](int li) { return lines ? lines[l0 + li] : l0 + li; };
  for (int idx = threadIdx.x; idx < npp * L; idx += FFT_THREADS) a[idx] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int idx = threadIdx.x; idx < npp * Hz; idx += FFT_THREADS) {
    const int pl = idx / Hz, k = idx - pl * Hz;
    const float2 A = H[(size_t)line(2 * pl) * Hz + k];
    const float2 B = 2 * pl + 1 < nl ? H[(size_t)line(2 * pl + 1) * Hz + k] : make_float2(0.f, 0.f);
    a[pl * L + k] = make_float2(A.x - B.y, A.y + B.x);                  // A + i B
    if (k > 0) a[pl * L + L - k] = make_float2(A.x + B.y, B.x - A.y);   // conj A + i conj B
  }
  __syncthreads();
  lds_fft<+1>(a, b, L, logL, npp, twl);
  for (int idx = threadIdx.x; idx < nl * L; idx += FFT_THREADS) {
    const int li = idx / L, j = idx - li * L;
    const float2 v = a[(li >> 1) * L + j];
    grid[(size_t)line(li) * L + j] = (li & 1) ? v.y : v.x;
  }
}

// d = 3 middle axis (y), forward: H1[(x*L + y)*Hz + lz] -> H2[(x*F + y')*Hz + lz],
// keeping ly = y' - N/2 in [-N/2, N/2]; lpb columns lz per workgroup.
// xs non-null: block row blk / ngroups takes slab x = xs[blk / ngroups].
__device__ __forceinline__ void y_fwd_body(int blk, const float2 *__restrict__ H1,
                                           float2 *__restrict__ H2, int L, int logL, int lpb,
                                           int Hz, int N, const float2 *__restrict__ tw,
                                           const int *__restrict__ xs = nullptr) {
  extern __shared__ float2 sm[];
  float2 *a = sm, *b = sm + lpb * L, *twl = sm + 2 * lpb * L;
  load_twiddles(twl, tw, L);
  const int ngroups = (Hz + lpb - 1) / lpb;
  const int x = xs ? xs[blk / ngroups] : blk / ngroups, lz0 = (blk % ngroups) * lpb;
  const int nl = min(lpb, Hz - lz0);
  const int F = N + 1;
  for (int idx = threadIdx.x; idx < nl * L; idx += FFT_THREADS) {
    const int y = idx / nl, li = idx - y * nl;
    a[li * L + y] = H1[((size_t)x * L + y) * Hz + lz0 + li];
  }
  __syncthreads();
  lds_fft<-1>(a, b, L, logL, nl, twl);
  for (int idx = threadIdx.x; idx < F * nl; idx += FFT_THREADS) {
    const int yp = idx / nl, li = idx - yp * nl;
    const int ly = (yp - N / 2 + L) & (L - 1);
    H2[((size_t)x * F + yp) * Hz + lz0 + li] = a[li * L + ly];
  }
}

// xs non-null: slab x = xs[blk / ngroups]; sup non-null: only the lines
// (x, y) with sup[x L + y] set are written (the others stay as they are).
__device__ __forceinline__ void y_inv_body(int blk, const float2 *__restrict__ H2,
                                           float2 *__restrict__ H1, int L, int logL, int lpb,
                                           int Hz, int N, const float2 *__restrict__ tw,
                                           const int *__restrict__ xs = nullptr,
                                           const uint8_t *__restrict__ sup = nullptr) {
  extern __shared__ float2 sm[];
  float2 *a = sm, *b = sm + lpb * L, *twl = sm + 2 * lpb * L;
  load_twiddles(twl, tw, L);
  const int ngroups = (Hz + lpb - 1) / lpb;
  const int x = xs ? xs[blk / ngroups] : blk / ngroups, lz0 = (blk % ngroups) * lpb;
  const int nl = min(lpb, Hz - lz0);
  const int F = N + 1;
  for (int idx = threadIdx.x; idx < nl * L; idx += FFT_THREADS) a[idx] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int idx = threadIdx.x; idx < F * nl; idx += FFT_THREADS) {
    const int yp = idx / nl, li = idx - yp * nl;
    const int ly = (yp - N / 2 + L) & (L - 1);
    a[li * L + ly] = H2[((size_t)x * F + yp) * Hz + lz0 + li];
  }
  __syncthreads();
  lds_fft<+1>(a, b, L, logL, nl, twl);
  for (int idx = threadIdx.x; idx < nl * L; idx += FFT_THREADS) {
    const int y = idx / nl, li = idx - y * nl;
    if (!sup || sup[x * L + y]) H1[((size_t)x * L + y) * Hz + lz0 + li] = a[li * L + y];
  }
}

// First axis (x): forward FFT, multiply by the filter on lx in [-N/2, N/2]
// (zero elsewhere), inverse FFT.  Hx[x*C + c], filter[(lx + N/2)*C + c].
// xin non-null: only the x with xin[x] set are written back.
__device__ __forceinline__ void x_filter_body(int blk, float2 *__restrict__ Hx,
                                              const float *__restrict__ filt, int C, int L,
                                              int logL, int lpb, int N,
                                              const float2 *__restrict__ tw,
                                              const uint8_t *__restrict__ xin = nullptr) {
  extern __shared__ float2 sm[];
  float2 *a = sm, *b = sm + lpb * L, *twl = sm + 2 * lpb * L;
  load_twiddles(twl, tw, L);
  const int c0 = blk * lpb;
  const int nl = min(lpb, C - c0);
  for (int idx = threadIdx.x; idx < nl * L; idx += FFT_THREADS) {
    const int x = idx / nl, li = idx - x * nl;
    a[li * L + x] = Hx[(size_t)x * C + c0 + li];
  }
  __syncthreads();
  lds_fft<-1>(a, b, L, logL, nl, twl);
  for (int idx = threadIdx.x; idx < nl * L; idx += FFT_THREADS) {
    const int li = idx / L, x = idx - li * L;
    const int lx = x < L / 2 ? x : x - L;
    float f = 0.f;
    if (lx >= -N / 2 && lx <= N / 2) f = filt[(size_t)(lx + N / 2) * C + c0 + li];
    a[idx].x *= f;
    a[idx].y *= f;
  }
  __syncthreads();
  lds_fft<+1>(a, b, L, logL, nl, twl);
  for (int idx = threadIdx.x; idx < nl * L; idx += FFT_THREADS) {
    const int x = idx / nl, li = idx - x * nl;
    if (!xin || xin[x]) Hx[(size_t)x * C + c0 + li] = a[li * L + x];
  }
}

}  // namespace nfl
