// NFFT fast summation on gfx950 (Alg. nfft_fastsum): spread -> FFT ->
// multiply by the filter -> inverse FFT -> interpolate, with the pre- and
// post-operations of Alg. nfft_normalized_matvec fused into the first and
// last kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <unordered_map>

#include "nfft_device.h"
#include "nfl_internal.h"

namespace nfl {

// ---------------------------------------------------------------------------
// d = 3 spread.  One workgroup per work item (a range of sorted nodes inside
// one T^3 tile) owns an LDS copy of the tile padded by the window, (T+W-1)^3.
// Each wave walks a contiguous slice of the item; the nodes of one grid cell
// share the same W^3 window, so a wave accumulates that window in registers
// (lane = one (y, z) pair of the window, W x-values each) across all nodes of
// the cell and adds it to LDS once per cell.  Finally the padded tile is
// added into the grid (halo cells overlap neighbouring tiles).
// ---------------------------------------------------------------------------
template <int W, int IN>
__global__ __launch_bounds__(256) void k_spread3(const Item *__restrict__ items,
                                                 const float4 *__restrict__ pts, KArgs ka,
                                                 float *__restrict__ grid, int nos, int tshift,
                                                 const float *__restrict__ wcoef) {
  constexpr int M = W / 2, R = (W * W + 63) / 64;
  extern __shared__ float lds[];
  if (stopped(ka.stop)) return;
  const int T = 1 << tshift, P = T + W - 1, PP = P * P, P3 = PP * P;
  const Item it = items[blockIdx.x];
  const int ntd = nos >> tshift;
  const int tz = it.tile % ntd, ty = (it.tile / ntd) % ntd, tx = it.tile / (ntd * ntd);
  const int ox = tx * T, oy = ty * T, oz = tz * T;
  for (int c = threadIdx.x; c < P3; c += 256) lds[c] = 0.f;
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int len = it.end - it.start, per = (len + 3) >> 2;
  const int s = it.start + min(len, wave * per), e = it.start + min(len, (wave + 1) * per);

  int pay[R], paz[R];
  bool pv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = lane + 64 * r;
    pv[r] = p < W * W;
    pay[r] = pv[r] ? p / W : 0;
    paz[r] = pv[r] ? p % W : 0;
  }
  const int wdim = lane / W;
  float cf[WIN_NC];
  load_coef(wcoef, min(lane - wdim * W, WIN_MAXW - 1), cf);

  float acc[R][W];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int a = 0; a < W; ++a) acc[r][a] = 0.f;
  uint32_t cur = 0xffffffffu;

  auto flush = [&](uint32_t cell) {
    const int lx = (int)(cell & 1023u) - ox, ly = (int)((cell >> 10) & 1023u) - oy,
              lz = (int)(cell >> 20) - oz;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (pv[r]) {
        float *base = lds + (lx * P + ly + pay[r]) * P + lz + paz[r];
#pragma unroll
        for (int a = 0; a < W; ++a) {
          __hip_atomic_fetch_add(base + a * PP, acc[r][a], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
          acc[r][a] = 0.f;
        }
      }
    }
  };

  // Nodes are fetched 64 at a time (one per lane, coalesced) and walked one
  // by one from registers, so no per-node global-load latency is exposed.
  for (int i0 = s; i0 < e; i0 += 64) {
    const int cnt = min(64, e - i0);
    float4 qb = make_float4(0.f, 0.f, 0.f, 0.f);
    float xb = 0.f;
    if (lane < cnt) {
      qb = pts[i0 + lane];
      xb = load_in<IN>(ka, i0 + lane);
    }
    for (int j = 0; j < cnt; ++j) {
      const uint32_t cell = (uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(qb.w), j);
      const float xv = readlane_f(xb, j);
      if (cell != cur) {
        if (cur != 0xffffffffu) flush(cur);
        cur = cell;
      }
      const float qx = readlane_f(qb.x, j), qy = readlane_f(qb.y, j), qz = readlane_f(qb.z, j);
      const float fr = wdim == 0 ? qx : (wdim == 1 ? qy : qz);
      const float wgt = win_poly(cf, fr);
      float wx[W];
#pragma unroll
      for (int a = 0; a < W; ++a) wx[a] = readlane_f(wgt, a);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float wy = __shfl(wgt, W + pay[r]);
        const float wz = __shfl(wgt, 2 * W + paz[r]);
        const float sy = pv[r] ? xv * wy * wz : 0.f;
#pragma unroll
        for (int a = 0; a < W; ++a) acc[r][a] = fmaf(sy, wx[a], acc[r][a]);
      }
    }
  }
  if (cur != 0xffffffffu) flush(cur);
  __syncthreads();

  const int mask = nos - 1;
  const double fx = fx_of(ka);
  for (int c = threadIdx.x; c < P3; c += 256) {
    const float v = lds[c];
    if (v != 0.f) {
      const int px = c / PP, rem = c - px * PP, py = rem / P, pz = rem - py * P;
      const int gx = (ox - (M - 1) + px) & mask, gy = (oy - (M - 1) + py) & mask,
                gz = (oz - (M - 1) + pz) & mask;
      grid_add(grid, ((size_t)gx * nos + gy) * nos + gz, v, fx);
    }
  }
}

// ---------------------------------------------------------------------------
// d = 3 interpolation, the transpose of k_spread3: the workgroup stages its
// padded tile from the grid into LDS; a wave keeps the window of the current
// cell in registers (same lane layout as the spread) and, for each node,
// forms sum_a wx[a] sum_(y,z) wy wz g and reduces it over the wave.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int W, int IN, int OUT>
__global__ __launch_bounds__(256) void k_interp3(const Item *__restrict__ items,
                                                 const float4 *__restrict__ pts, KArgs ka,
                                                 const float *__restrict__ grid, int nos,
                                                 int tshift, const float *__restrict__ wcoef) {
  constexpr int M = W / 2, R = (W * W + 63) / 64;
  extern __shared__ float lds[];
  if (stopped(ka.stop)) return;
  const int T = 1 << tshift, P = T + W - 1, PP = P * P, P3 = PP * P;
  const Item it = items[blockIdx.x];
  const int ntd = nos >> tshift;
  const int tz = it.tile % ntd, ty = (it.tile / ntd) % ntd, tx = it.tile / (ntd * ntd);
  const int ox = tx * T, oy = ty * T, oz = tz * T;
  const int mask = nos - 1;
  for (int c = threadIdx.x; c < P3; c += 256) {
    const int px = c / PP, rem = c - px * PP, py = rem / P, pz = rem - py * P;
    const int gx = (ox - (M - 1) + px) & mask, gy = (oy - (M - 1) + py) & mask,
              gz = (oz - (M - 1) + pz) & mask;
    lds[c] = grid[((size_t)gx * nos + gy) * nos + gz];
  }
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int len = it.end - it.start, per = (len + 3) >> 2;
  const int s = it.start + min(len, wave * per), e = it.start + min(len, (wave + 1) * per);

  int pay[R], paz[R];
  bool pv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = lane + 64 * r;
    pv[r] = p < W * W;
    pay[r] = pv[r] ? p / W : 0;
    paz[r] = pv[r] ? p % W : 0;
  }
  const int wdim = lane / W;
  float cf[WIN_NC];
  load_coef(wcoef, min(lane - wdim * W, WIN_MAXW - 1), cf);

  float g[R][W];
  uint32_t cur = 0xffffffffu;
  for (int i0 = s; i0 < e; i0 += 64) {
    const int cnt = min(64, e - i0);
    float4 qb = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lane < cnt) qb = pts[i0 + lane];
    float res = 0.f;
    for (int j = 0; j < cnt; ++j) {
      const uint32_t cell = (uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(qb.w), j);
      if (cell != cur) {
        cur = cell;
        const int lx = (int)(cell & 1023u) - ox, ly = (int)((cell >> 10) & 1023u) - oy,
                  lz = (int)(cell >> 20) - oz;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float *base = lds + (lx * P + ly + pay[r]) * P + lz + paz[r];
#pragma unroll
          for (int a = 0; a < W; ++a) g[r][a] = pv[r] ? base[a * PP] : 0.f;
        }
      }
      const float qx = readlane_f(qb.x, j), qy = readlane_f(qb.y, j), qz = readlane_f(qb.z, j);
      const float fr = wdim == 0 ? qx : (wdim == 1 ? qy : qz);
      const float wgt = win_poly(cf, fr);
      float wx[W];
#pragma unroll
      for (int a = 0; a < W; ++a) wx[a] = readlane_f(wgt, a);
      float part = 0.f;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float wy = __shfl(wgt, W + pay[r]);
        const float wz = __shfl(wgt, 2 * W + paz[r]);
        float t = 0.f;
#pragma unroll
        for (int a = 0; a < W; ++a) t = fmaf(wx[a], g[r][a], t);
        part = fmaf(wy * wz, t, part);
      }
      part = wave_sum(part);
      if (lane == j) res = part;
    }
    if (lane < cnt) store_out<OUT>(ka, i0 + lane, res);
  }
}

// Matrix-core spread and interpolation of one plan: one workgroup per item.
template <int W, int IN, bool ZM>
__global__ __launch_bounds__(256) void k_spread3_mfma(const Item *__restrict__ items,
                                                      const float4 *__restrict__ pts, KArgs ka,
                                                      float *__restrict__ grid, int nos,
                                                      int tshift,
                                                      const float *__restrict__ wcoef) {
  if (stopped(ka.stop)) return;
  spread3_mfma_body<W, IN, ZM>(items[blockIdx.x], pts, ka, grid, nos, tshift, wcoef);
}

template <int W, int IN, int OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W <= 8 ? 5 : 1)))
void k_interp3_mfma(const Item *__restrict__ items,
                                                      const float4 *__restrict__ pts, KArgs ka,
                                                      const float *__restrict__ grid, int nos,
                                                      int tshift,
                                                      const float *__restrict__ wcoef) {
  if (stopped(ka.stop)) return;
  interp3_mfma_body<W, IN, OUT>(items, blockIdx.x, pts, ka, grid, nos, tshift, wcoef);
}

// Tile-stationary forms (T + W - 1 <= 16), one workgroup per group of
// segments (the plan's gitems / goff): the segments of a group are taken one
// after the other, each with its own tile staging (interpolation) or flush
// (spread); the barrier between two frees the LDS of the previous one.  The
// groups follow the sort, so neighbouring groups share grid cells; each XCD
// takes one contiguous range of them (xcd_block), which keeps those cells in
// one L2 (a product at the benchmark workload: 194.6 -> 190.5 us).  The
// spread keeps its accumulators in VGPRs without spills within the register
// budget of three waves per SIMD (168 per lane); it uses at most 127 (m = 6),
// so four fit.
template <int W, int T, int IN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void k_spread3_tile(const Item *__restrict__ items, const int *__restrict__ goff,
                    const float4 *__restrict__ pts, KArgs ka, float *__restrict__ grid, int nos,
                    const float *__restrict__ wcoef) {
  if (stopped(ka.stop)) return;
  const int gb = xcd_block(blockIdx.x, gridDim.x);
  const int g0 = goff[gb], g1 = goff[gb + 1];
  for (int it = g0; it < g1; ++it) {
    if (it > g0) __syncthreads();
    spread3_tile_body<W, T, IN>(items[it], pts, ka, grid, nos, wcoef);
  }
}

template <int W, int T, int IN, int OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_interp3_tile(const Item *__restrict__ items, const int *__restrict__ goff,
                    const float4 *__restrict__ pts, KArgs ka, const float *__restrict__ grid,
                    int nos, const float *__restrict__ wcoef) {
  if (stopped(ka.stop)) return;
  const int gb = xcd_block(blockIdx.x, gridDim.x);
  const int g0 = goff[gb], g1 = goff[gb + 1];
  double dsum = 0.0;
  for (int it = g0; it < g1; ++it) {
    if (it > g0) __syncthreads();
    interp3_tile_body<W, T, IN, OUT>(items, it, pts, ka, grid, nos, wcoef, &dsum);
  }
  if constexpr (OUT == OUT_SORTED_F64_SSL) {
    if (ka.dot) {   // the workgroup's partial of x64 . y64, summed in a fixed order
      __shared__ double wsum[4];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) dsum += __shfl_xor(dsum, o);
      if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = dsum;
      __syncthreads();
      if (threadIdx.x == 0) ka.dot[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    }
  }
}

// ---------------------------------------------------------------------------
// d = 1, 2: one thread per node, direct global accumulation / gathering.
// ---------------------------------------------------------------------------
// Spread for d = 1, 2, one work item (nodes of one T^d tile) per workgroup,
// without per-node atomics: batches of 256 nodes stage their window weights
// in LDS, then each thread owns cells of the padded tile ((T + W - 1)^d
// cells) and sums the contributions of the batch's nodes whose windows cover
// them; the padded tile is added into the grid once per item.
template <int IN>
__global__ __launch_bounds__(256) void k_spread12(const Item *__restrict__ items,
                                                  const float4 *__restrict__ pts, KArgs ka,
                                                  float *__restrict__ grid, int d, int nos,
                                                  int m, int tshift,
                                                  const float *__restrict__ wcoef) {
  __shared__ float sc[WIN_MAXW * WIN_NC];
  __shared__ float wxs[256 * (WIN_MAXW + 1)], wys[256 * (WIN_MAXW + 1)];
  __shared__ float xs[256];
  __shared__ int loc[256];                     // local cell offsets lx | ly << 8
  const int t = threadIdx.x;
  if (stopped(ka.stop)) return;
  for (int q = t; q < WIN_MAXW * WIN_NC; q += 256) sc[q] = wcoef[q];
  const Item it = items[blockIdx.x];
  const int W = 2 * m, mask = nos - 1, T = 1 << tshift, Pd = T + W - 1;
  const int ntd = nos >> tshift;
  const int tx0 = (d == 2 ? it.tile / ntd : it.tile) << tshift;
  const int ty0 = d == 2 ? (it.tile % ntd) << tshift : 0;
  const int ncell = d == 2 ? Pd * Pd : Pd;
  constexpr int CPT = (WIN_MAXW + 4 - 1) * (WIN_MAXW + 4 - 1) / 256 + 1;   // cells per thread
  float acc[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) acc[c] = 0.f;
  for (int b0 = it.start; b0 < it.end; b0 += 256) {
    const int cnt = min(256, it.end - b0);
    __syncthreads();
    if (t < cnt) {
      const int i = b0 + t;
      const float4 q = pts[i];
      const uint32_t cell = __float_as_uint(q.w);
      const int cx = cell & 1023u, cy = (cell >> 10) & 1023u;
      xs[t] = load_in<IN>(ka, i);
      loc[t] = (cx - tx0) | ((d == 2 ? cy - ty0 : 0) << 8);
      const float gx0 = fmaf(2.f, q.x, -1.f), gy0 = fmaf(2.f, q.y, -1.f);
      for (int a = 0; a < W; ++a) {
        float px = sc[a * WIN_NC + WIN_NC - 1], py = px;
        for (int k = WIN_NC - 2; k >= 0; --k) {
          px = fmaf(px, gx0, sc[a * WIN_NC + k]);
          py = fmaf(py, gy0, sc[a * WIN_NC + k]);
        }
        wxs[t * (WIN_MAXW + 1) + a] = px;
        wys[t * (WIN_MAXW + 1) + a] = d == 2 ? py : 1.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int e = t + 256 * c;
      if (e >= ncell) break;
      const int px = d == 2 ? e / Pd : e, py = d == 2 ? e % Pd : 0;
      float sacc = acc[c];
      for (int j = 0; j < cnt; ++j) {
        const int l = loc[j];
        const int a = px - (l & 255), bb = py - (l >> 8);
        if (a >= 0 && a < W && bb >= 0 && bb < W)
          sacc = fmaf(xs[j] * wxs[j * (WIN_MAXW + 1) + a], wys[j * (WIN_MAXW + 1) + bb], sacc);
      }
      acc[c] = sacc;
    }
  }
  const double fx = fx_of(ka);
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int e = t + 256 * c;
    if (e >= ncell) break;
    const int px = d == 2 ? e / Pd : e, py = d == 2 ? e % Pd : 0;
    const int gx = (tx0 - (m - 1) + px) & mask;
    if (acc[c] != 0.f) {
      if (d == 1)
        grid_add(grid, gx, acc[c], fx);
      else
        grid_add(grid, (size_t)gx * nos + ((ty0 - (m - 1) + py) & mask), acc[c], fx);
    }
  }
}

// Interpolation for d = 1, 2, the transpose of k_spread12: one work item per
// workgroup; its padded tile is staged in LDS once, then each node sums its
// window from there.
template <int IN, int OUT>
__global__ __launch_bounds__(256) void k_interp12(const Item *__restrict__ items,
                                                  const float4 *__restrict__ pts, KArgs ka,
                                                  const float *__restrict__ grid, int d, int nos,
                                                  int m, int tshift,
                                                  const float *__restrict__ wcoef) {
  __shared__ float sc[WIN_MAXW * WIN_NC];
  __shared__ float tile[(WIN_MAXW + 4 - 1) * (WIN_MAXW + 4 - 1)];
  const int t = threadIdx.x;
  if (stopped(ka.stop)) return;
  for (int q = t; q < WIN_MAXW * WIN_NC; q += 256) sc[q] = wcoef[q];
  const Item it = items[blockIdx.x];
  const int W = 2 * m, mask = nos - 1, T = 1 << tshift, Pd = T + W - 1;
  const int ntd = nos >> tshift;
  const int tx0 = (d == 2 ? it.tile / ntd : it.tile) << tshift;
  const int ty0 = d == 2 ? (it.tile % ntd) << tshift : 0;
  const int ncell = d == 2 ? Pd * Pd : Pd;
  for (int e = t; e < ncell; e += 256) {
    const int px = d == 2 ? e / Pd : e, py = d == 2 ? e % Pd : 0;
    const int gx = (tx0 - (m - 1) + px) & mask;
    tile[e] = d == 1 ? grid[gx] : grid[(size_t)gx * nos + ((ty0 - (m - 1) + py) & mask)];
  }
  __syncthreads();
  for (int i = it.start + t; i < it.end; i += 256) {
    const float4 q = pts[i];
    const uint32_t cell = __float_as_uint(q.w);
    const int lx = (int)(cell & 1023u) - tx0;
    const int ly = d == 2 ? (int)((cell >> 10) & 1023u) - ty0 : 0;
    float wx[WIN_MAXW], wy[WIN_MAXW];
    const float gx0 = fmaf(2.f, q.x, -1.f), gy0 = fmaf(2.f, q.y, -1.f);
    for (int a = 0; a < W; ++a) {
      float px = sc[a * WIN_NC + WIN_NC - 1], py = px;
      for (int k = WIN_NC - 2; k >= 0; --k) {
        px = fmaf(px, gx0, sc[a * WIN_NC + k]);
        py = fmaf(py, gy0, sc[a * WIN_NC + k]);
      }
      wx[a] = px;
      wy[a] = d == 2 ? py : 1.f;
    }
    float f = 0.f;
    for (int a = 0; a < W; ++a) {
      if (d == 1) {
        f = fmaf(wx[a], tile[lx + a], f);
      } else {
        const float *row = tile + (lx + a) * Pd + ly;
        float r = 0.f;
        for (int c = 0; c < W; ++c) r = fmaf(wy[c], row[c], r);
        f = fmaf(wx[a], r, f);
      }
    }
    store_out<OUT>(ka, i, f);
  }
}


// FFT passes of one plan (line layouts in the bodies' comments).
template <bool ZERO>
__global__ __launch_bounds__(FFT_THREADS) void k_r2c_lines(float *__restrict__ grid,
                                                           float2 *__restrict__ H, int nlines,
                                                           int L, int logL, int lpb, int Hz,
                                                           const float2 *__restrict__ tw,
                                                           const int *__restrict__ stop,
                                                           const unsigned *__restrict__ fx_max,
                                                           float fx_mult,
                                                           const int *__restrict__ lines) {
  if (stopped(stop)) return;
  r2c_lines_body<ZERO>(blockIdx.x, grid, H, nlines, L, logL, lpb, Hz, tw, fx_max, fx_mult, lines);
}

__global__ __launch_bounds__(FFT_THREADS) void k_c2r_lines(const float2 *__restrict__ H,
                                                           float *__restrict__ grid, int nlines,
                                                           int L, int logL, int lpb, int Hz,
                                                           const float2 *__restrict__ tw,
                                                           const int *__restrict__ stop,
                                                           unsigned *__restrict__ fx_reset,
                                                           const int *__restrict__ lines) {
  if (stopped(stop)) return;
  // the last pass of a product clears the deterministic spread's input bound
  // for the next product's pre-pass (every reader of it has finished)
  if (fx_reset && blockIdx.x == 0 && threadIdx.x < FX_WORDS) fx_reset[threadIdx.x * FX_STRIDE] = 0u;
  c2r_lines_body(blockIdx.x, H, grid, nlines, L, logL, lpb, Hz, tw, lines);
}

__global__ __launch_bounds__(FFT_THREADS) void k_y_fwd(const float2 *__restrict__ H1,
                                                       float2 *__restrict__ H2, int L, int logL,
                                                       int lpb, int Hz, int N,
                                                       const float2 *__restrict__ tw,
                                                       const int *__restrict__ stop,
                                                       const int *__restrict__ xs) {
  if (stopped(stop)) return;
  y_fwd_body(xcd_block(blockIdx.x, gridDim.x), H1, H2, L, logL, lpb, Hz, N, tw, xs);
}

__global__ __launch_bounds__(FFT_THREADS) void k_y_inv(const float2 *__restrict__ H2,
                                                       float2 *__restrict__ H1, int L, int logL,
                                                       int lpb, int Hz, int N,
                                                       const float2 *__restrict__ tw,
                                                       const int *__restrict__ stop,
                                                       const int *__restrict__ xs,
                                                       const uint8_t *__restrict__ sup) {
  if (stopped(stop)) return;
  y_inv_body(xcd_block(blockIdx.x, gridDim.x), H2, H1, L, logL, lpb, Hz, N, tw, xs, sup);
}

__global__ __launch_bounds__(FFT_THREADS) void k_x_filter(float2 *__restrict__ Hx,
                                                          const float *__restrict__ filt, int C,
                                                          int L, int logL, int lpb, int N,
                                                          const float2 *__restrict__ tw,
                                                          const int *__restrict__ stop,
                                                          const uint8_t *__restrict__ xin) {
  if (stopped(stop)) return;
  x_filter_body(xcd_block(blockIdx.x, gridDim.x), Hx, filt, C, L, logL, lpb, N, tw, xin);
}

__global__ void k_filter1(float2 *__restrict__ H, const float *__restrict__ filt, int Hz,
                          const int *__restrict__ stop) {
  if (stopped(stop)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < Hz) {
    H[i].x *= filt[i];
    H[i].y *= filt[i];
  }
}

// Pre-pass of the deterministic spread: *out = max(*out, bits of max_i |x_i|)
// (non-negative floats order like their bit patterns); x null: |x| = 1.
template <class T>
__global__ __launch_bounds__(1024) void k_fx_max(const T *__restrict__ x, int64_t n,
                                                 unsigned *__restrict__ out,
                                                 const int *__restrict__ stop) {
  if (stopped(stop)) return;
  __shared__ float wm[16];
  float m = x ? 0.f : 1.f;
  if (x) {
    // 16-byte loads where the base is aligned (torch tensors are), scalar tail
    constexpr int V = 16 / sizeof(T);
    const bool vec = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    const int64_t nv = vec ? n / V : 0;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, nt = (int64_t)gridDim.x * blockDim.x;
#pragma unroll 4
    for (int64_t i = tid; i < nv; i += nt) {
      const float4 q = reinterpret_cast<const float4 *>(x)[i];
      const T *e = reinterpret_cast<const T *>(&q);
#pragma unroll
      for (int k = 0; k < V; ++k) m = fmaxf(m, (float)fabs((double)e[k]));
    }
    for (int64_t i = nv * V + tid; i < n; i += nt) m = fmaxf(m, (float)fabs((double)x[i]));
    m *= 1.f + 1e-6f;   // round up past the float rounding of double inputs
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  // one atomic per block, on word blockIdx mod FX_WORDS (at most 256 blocks of
  // 1024 threads; 512 blocks of 256 on one word took ~8 us at n = 1e6)
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, wm[w]);
    atomicMax(fx_word(out, blockIdx.x), __float_as_uint(m));
  }
}

__global__ __launch_bounds__(256) void k_fill(float *__restrict__ p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

__global__ __launch_bounds__(256) void k_scatter32(const float *__restrict__ src,
                                                   const int *__restrict__ perm, int64_t n,
                                                   float *__restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[perm[i]] = src[i];
}

int scatter_f32(nfl_plan *P, const float *src, float *dst) {
  const int nb = (int)std::min<int64_t>(4096, (P->n + 255) / 256);
  hipLaunchKernelGGL(k_scatter32, dim3(nb), dim3(256), 0, P->stream, src, P->perm.p, P->n, dst);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int fill_f32(float *p, int64_t n, float v, hipStream_t s) {
  const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_fill, dim3(std::max(nb, 1)), dim3(256), 0, s, p, n, v);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static KArgs make_kargs(nfl_plan *P, const VecArgs &a) {
  KArgs k;
  k.x32 = a.x32;
  k.y32 = a.y32;
  k.x64 = a.x64;
  k.y64 = a.y64;
  k.tau = a.tau;
  k.perm = P->perm.p;
  k.dinv = P->dinv.p;
  k.deg_out = P->deg.p;
  k.dinv_out = P->dinv.p;
  k.stop = P->stop;
  k.fx_max = nullptr;
  k.fx_mult = 0.f;
  k.xs = a.xs;
  k.dot = a.dot;
  return k;
}

static size_t tile_lds_bytes(const nfl_plan *P) {
  const int T = 1 << P->tshift, Pd = T + 2 * P->m - 1;
  return (size_t)Pd * Pd * Pd * sizeof(float);
}

// Raise a kernel's dynamic LDS limit once per process (per size): launches
// recorded into a HIP graph then make no attribute calls.
template <class K>
static int set_lds(K kern, size_t lds) {
  if (lds <= 65536) return NFL_OK;
  static std::mutex mu;
  static std::unordered_map<const void *, size_t> done;
  std::lock_guard<std::mutex> lock(mu);
  size_t &cur = done[(const void *)kern];
  if (cur >= lds) return NFL_OK;
  NFL_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  cur = lds;
  return NFL_OK;
}

template <int W, int IN, bool ZM>
static int launch_spread3_mfma(nfl_plan *P, const KArgs &k, float *grid) {
  const int Pd = (1 << P->tshift) + W - 1;
  const size_t lds = (4 * (size_t)tile_px(Pd) * Pd + 4 * 16 * WT_SPREAD) * sizeof(float);
  NFL_TRY(set_lds(k_spread3_mfma<W, IN, ZM>, lds));
  hipLaunchKernelGGL((k_spread3_mfma<W, IN, ZM>), dim3(P->nitems), dim3(256), lds, P->stream,
                     P->items.p, P->pts.p, k, grid, P->nos, P->tshift, P->wcoef.p);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

static size_t tile_form_lds(int W, int T, bool spread) {
  const int Pd = T + W - 1;
  if (spread) return (size_t)spread_tile_lds_floats(Pd, 4) * sizeof(float);
  // the window coefficients stay in LDS after the tables
  return ((size_t)Pd * ts_xs(Pd) + (size_t)4 * 16 * TS_PITCH_I + WIN_MAXW * WIN_NC) * sizeof(float);
}

template <int W, int T, int IN>
static int launch_spread3_tile(nfl_plan *P, const KArgs &k, float *grid) {
  if (P->ngroups <= 0) {
    set_error("spread: the plan has no work groups for the tile-stationary form");
    return NFL_ERR_ORDER;
  }
  const size_t lds = tile_form_lds(W, T, true);
  NFL_TRY(set_lds(k_spread3_tile<W, T, IN>, lds));
  hipLaunchKernelGGL((k_spread3_tile<W, T, IN>), dim3(P->ngroups), dim3(256), lds, P->stream,
                     P->gitems.p, P->goff.p, P->pts.p, k, grid, P->nos, P->wcoef.p);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

template <int W, int T, int IN, int OUT>
static int launch_interp3_tile(nfl_plan *P, const KArgs &k, const float *grid) {
  if (P->ngroups <= 0) {
    set_error("interp: the plan has no work groups for the tile-stationary form");
    return NFL_ERR_ORDER;
  }
  const size_t lds = tile_form_lds(W, T, false);
  NFL_TRY(set_lds(k_interp3_tile<W, T, IN, OUT>, lds));
  hipLaunchKernelGGL((k_interp3_tile<W, T, IN, OUT>), dim3(P->ngroups), dim3(256), lds,
                     P->stream, P->gitems.p, P->goff.p, P->pts.p, k, grid, P->nos, P->wcoef.p);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

// Workgroups of both tile-stationary kernels (window W, tile T) that one CU
// holds at once (the smaller of the two), times the CUs.
// (One per CU if the occupancy query fails: correct, with fewer groups.)
template <int W, int T>
static int tile_slots_wt(int cus) {
  int a = 0, b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_spread3_tile<W, T, IN_USER_F32_DINV>, 256,
                                                   tile_form_lds(W, T, true)) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_interp3_tile<W, T, IN_USER_F32, OUT_USER_LS>,
                                                   256, tile_form_lds(W, T, false)) != hipSuccess) {
    (void)hipGetLastError();
    return cus;
  }
  return cus * std::max(1, std::min(a, b));
}

int tile_group_slots(const nfl_plan *P) {
  if (P->d != 3) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    cus = 1;
  }
  const int T = 1 << P->tshift;
  switch (T * 100 + 2 * P->m) {
    case 404: return tile_slots_wt<4, 4>(cus);
    case 406: return tile_slots_wt<6, 4>(cus);
    case 408: return tile_slots_wt<8, 4>(cus);
    case 410: return tile_slots_wt<10, 4>(cus);
    case 412: return tile_slots_wt<12, 4>(cus);
    case 804: return tile_slots_wt<4, 8>(cus);
    case 806: return tile_slots_wt<6, 8>(cus);
    case 808: return tile_slots_wt<8, 8>(cus);
    default: return 0;
  }
}

template <int W, int IN>
static int launch_spread3(nfl_plan *P, const KArgs &k, float *grid) {
  if (P->opt_kernel == 0) {
    const int T = 1 << P->tshift;
    if constexpr (W + 3 <= 16) {
      if (T == 4) return launch_spread3_tile<W, 4, IN>(P, k, grid);
    }
    if constexpr (W + 7 <= 16) {
      if (T == 8) return launch_spread3_tile<W, 8, IN>(P, k, grid);
    }
  }
  if (P->opt_kernel != 1) {
    const int T = 1 << P->tshift;
    if constexpr (W >= 9) {
      if (T + W - 1 <= 16) return launch_spread3_mfma<W, IN, true>(P, k, grid);
    }
    return launch_spread3_mfma<W, IN, false>(P, k, grid);
  }
  const size_t lds = tile_lds_bytes(P);
  NFL_TRY(set_lds(k_spread3<W, IN>, lds));
  hipLaunchKernelGGL((k_spread3<W, IN>), dim3(P->nitems), dim3(256), lds, P->stream, P->items.p,
                     P->pts.p, k, grid, P->nos, P->tshift, P->wcoef.p);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

template <int W, int IN, int OUT>
static int launch_interp3(nfl_plan *P, const KArgs &k, const float *grid) {
  if (P->opt_kernel == 0) {
    const int T = 1 << P->tshift;
    if constexpr (W + 3 <= 16) {
      if (T == 4) return launch_interp3_tile<W, 4, IN, OUT>(P, k, grid);
    }
    if constexpr (W + 7 <= 16) {
      if (T == 8) return launch_interp3_tile<W, 8, IN, OUT>(P, k, grid);
    }
  }
  if (P->opt_kernel != 1) {
    const int Pd = (1 << P->tshift) + W - 1;
    const size_t lds = ((size_t)tile_px(Pd) * Pd + 4 * 16 * WT_INTERP) * sizeof(float);
    NFL_TRY(set_lds(k_interp3_mfma<W, IN, OUT>, lds));
    hipLaunchKernelGGL((k_interp3_mfma<W, IN, OUT>), dim3(P->nitems), dim3(256), lds, P->stream,
                       P->items.p, P->pts.p, k, grid, P->nos, P->tshift, P->wcoef.p);
  } else {
    const size_t lds = tile_lds_bytes(P);
    NFL_TRY(set_lds(k_interp3<W, IN, OUT>, lds));
    hipLaunchKernelGGL((k_interp3<W, IN, OUT>), dim3(P->nitems), dim3(256), lds, P->stream,
                       P->items.p, P->pts.p, k, grid, P->nos, P->tshift, P->wcoef.p);
  }
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

template <int IN>
static int spread_in(nfl_plan *P, const KArgs &k, float *grid) {
  if (P->d == 3) {
    switch (P->m) {
      case 2: return launch_spread3<4, IN>(P, k, grid);
      case 3: return launch_spread3<6, IN>(P, k, grid);
      case 4: return launch_spread3<8, IN>(P, k, grid);
      case 5: return launch_spread3<10, IN>(P, k, grid);
      case 6: return launch_spread3<12, IN>(P, k, grid);
      case 7: return launch_spread3<14, IN>(P, k, grid);
      case 8: return launch_spread3<16, IN>(P, k, grid);
      default: set_error("spread: m out of range"); return NFL_ERR_UNSUPPORTED;
    }
  }
  if ((1 << P->tshift) + 2 * P->m - 1 > WIN_MAXW + 4 - 1) {
    set_error("spread: tile too large for the d <= 2 kernel (tile + 2m - 1 must be <= 19)");
    return NFL_ERR_UNSUPPORTED;
  }
  if (P->nitems == 0) return NFL_OK;
  hipLaunchKernelGGL((k_spread12<IN>), dim3(P->nitems), dim3(256), 0, P->stream, P->items.p,
                     P->pts.p, k, grid, P->d, P->nos, P->m, P->tshift, P->wcoef.p);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

// The bound of the deterministic spread's grid values: every cell sums at
// most n terms x~_i psi psi psi, |x~_i| <= max |input| * (d^{-1/2} bound for
// the normalised inputs), psi <= psi(0); with margins for rounding.
static int fx_prepass(nfl_plan *P, int in_mode, const VecArgs &a) {
  double factor = 1.0;
  if (in_mode == IN_USER_F32_DINV || in_mode == IN_SORTED_F64_DINV)
    factor = 1.01 / std::sqrt(std::max(P->dmin, 1e-300));
  P->fx_mult = (float)(1.0625 * factor * (double)P->n * std::pow(1.01 * P->win_max, P->d));
  if (a.fx_ready) return NFL_OK;   // the producer of the input wrote its bound
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(256, (P->n + 4095) / 4096));
  if (in_mode == IN_ONES) {
    hipLaunchKernelGGL(k_fx_max<float>, dim3(1), dim3(64), 0, P->stream, (const float *)nullptr,
                       (int64_t)0, P->fx_max.p, P->stop);
  } else if (in_mode == IN_SORTED_F64_DINV) {
    hipLaunchKernelGGL(k_fx_max<double>, dim3(nb), dim3(1024), 0, P->stream, a.x64, P->n,
                       P->fx_max.p, P->stop);
  } else {
    hipLaunchKernelGGL(k_fx_max<float>, dim3(nb), dim3(1024), 0, P->stream, a.x32, P->n,
                       P->fx_max.p, P->stop);
  }
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int spread(nfl_plan *P, int in_mode, const VecArgs &a, float *grid, bool clear) {
  int64_t gsz = 1;
  for (int t = 0; t < P->d; ++t) gsz *= P->nos;
  const bool fx = P->opt_det && grid == P->grid.p;
  if (clear) NFL_TRY(fill_f32(grid, fx ? 2 * gsz : gsz, 0.f, P->stream));
  if (fx) NFL_TRY(fx_prepass(P, in_mode, a));
  if (P->prof_ev) NFL_HIP(hipEventRecord(P->prof_ev[1], P->stream));
  KArgs k = make_kargs(P, a);
  if (fx) {
    k.fx_max = P->fx_max.p;
    k.fx_mult = P->fx_mult;
  }
  switch (in_mode) {
    case IN_USER_F32: return spread_in<IN_USER_F32>(P, k, grid);
    case IN_USER_F32_DINV: return spread_in<IN_USER_F32_DINV>(P, k, grid);
    case IN_ONES: return spread_in<IN_ONES>(P, k, grid);
    case IN_SORTED_F64_DINV: return spread_in<IN_SORTED_F64_DINV>(P, k, grid);
    default: set_error("spread: bad input mode"); return NFL_ERR_ARG;
  }
}

template <int IN, int OUT>
static int interp_io(nfl_plan *P, const KArgs &k, const float *grid) {
  if (P->d == 3) {
    switch (P->m) {
      case 2: return launch_interp3<4, IN, OUT>(P, k, grid);
      case 3: return launch_interp3<6, IN, OUT>(P, k, grid);
      case 4: return launch_interp3<8, IN, OUT>(P, k, grid);
      case 5: return launch_interp3<10, IN, OUT>(P, k, grid);
      case 6: return launch_interp3<12, IN, OUT>(P, k, grid);
      case 7: return launch_interp3<14, IN, OUT>(P, k, grid);
      case 8: return launch_interp3<16, IN, OUT>(P, k, grid);
      default: set_error("interp: m out of range"); return NFL_ERR_UNSUPPORTED;
    }
  }
  if ((1 << P->tshift) + 2 * P->m - 1 > WIN_MAXW + 4 - 1) {
    set_error("interp: tile too large for the d <= 2 kernel (tile + 2m - 1 must be <= 19)");
    return NFL_ERR_UNSUPPORTED;
  }
  if (P->nitems == 0) return NFL_OK;
  hipLaunchKernelGGL((k_interp12<IN, OUT>), dim3(P->nitems), dim3(256), 0, P->stream,
                     P->items.p, P->pts.p, k, grid, P->d, P->nos, P->m, P->tshift, P->wcoef.p);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int interp(nfl_plan *P, const float *grid, int in_mode, int out_mode, const VecArgs &a) {
  const KArgs k = make_kargs(P, a);
  // (input mode only matters through the post-operation; pairs in use)
  if (out_mode == OUT_USER_RAW) return interp_io<IN_USER_F32, OUT_USER_RAW>(P, k, grid);
  if (out_mode == OUT_USER_W) return interp_io<IN_USER_F32, OUT_USER_W>(P, k, grid);
  if (out_mode == OUT_USER_LS) return interp_io<IN_USER_F32, OUT_USER_LS>(P, k, grid);
  if (out_mode == OUT_USER_A) return interp_io<IN_USER_F32, OUT_USER_A>(P, k, grid);
  if (out_mode == OUT_DEGREE) return interp_io<IN_ONES, OUT_DEGREE>(P, k, grid);
  if (out_mode == OUT_SORTED_F64_A) return interp_io<IN_SORTED_F64_DINV, OUT_SORTED_F64_A>(P, k, grid);
  if (out_mode == OUT_SORTED_F64_SSL)
    return interp_io<IN_SORTED_F64_DINV, OUT_SORTED_F64_SSL>(P, k, grid);
  (void)in_mode;
  set_error("interp: bad output mode");
  return NFL_ERR_ARG;
}

int convolve(nfl_plan *P, const float *gin_c, float *gout, bool zero_in, bool support) {
  // the input is written only when zero_in (then it is the plan's own grid)
  float *gin = const_cast<float *>(gin_c);
  auto r2c = zero_in ? k_r2c_lines<true> : k_r2c_lines<false>;
  const bool fx = P->opt_det && gin_c == P->grid.p;   // the spread used the fixed-point grid
  const unsigned *fxm = fx ? P->fx_max.p : nullptr;
  unsigned *fxr = fx ? P->fx_max.p : nullptr;
  const float fxu = P->fx_mult;
  const int L = P->nos, N = P->N, Hz = N / 2 + 1, F = N + 1;
  int logL = 0;
  while ((1 << logL) < L) ++logL;
  // values per workgroup: FFT_ELEMS_PLAN up to L = 128 (longer lines: two per
  // workgroup at least, as with FFT_ELEMS)
  const int fe = L <= 128 ? FFT_ELEMS_PLAN : FFT_ELEMS;
  const int lpz = fft_lpb_zr(L, fe);   // real lines per workgroup, two per FFT
  const size_t ldz = fft_lds_bytes(lpz / 2, L);
  const float2 *tw = P->tw.p;
  if (P->d == 1) {
    hipLaunchKernelGGL(r2c, dim3(1), dim3(FFT_THREADS), ldz, P->stream, gin, P->spec1.p,
                       1, L, logL, lpz, Hz, tw, P->stop, fxm, fxu, (const int *)nullptr);
    hipLaunchKernelGGL(k_filter1, dim3(1), dim3(256), 0, P->stream, P->spec1.p, P->filt.p, Hz, P->stop);
    hipLaunchKernelGGL(k_c2r_lines, dim3(1), dim3(FFT_THREADS), ldz, P->stream, P->spec1.p, gout,
                       1, L, logL, lpz, Hz, tw, P->stop, fxr, (const int *)nullptr);
  } else if (P->d == 2) {
    const int nlines = L;
    const int nb = (nlines + lpz - 1) / lpz;
    hipLaunchKernelGGL(r2c, dim3(nb), dim3(FFT_THREADS), ldz, P->stream, gin, P->spec1.p,
                       nlines, L, logL, lpz, Hz, tw, P->stop, fxm, fxu, (const int *)nullptr);
    hipLaunchKernelGGL(k_x_filter, dim3(Hz), dim3(FFT_THREADS), fft_lds_bytes(1, L), P->stream,
                       P->spec1.p, P->filt.p, Hz, L, logL, 1, N, tw, P->stop,
                       (const uint8_t *)nullptr);
    hipLaunchKernelGGL(k_c2r_lines, dim3(nb), dim3(FFT_THREADS), ldz, P->stream, P->spec1.p, gout,
                       nlines, L, logL, lpz, Hz, tw, P->stop, fxr, (const int *)nullptr);
  } else {
    // On the plan's own grids the passes take only the support: the z-lines
    // some node's window touches, the x-slabs holding them; the spectrum
    // entries off the support are zero from the last clear and stay zero.
    const bool sup = support && P->zs_nlines > 0;
    if (sup && !P->spec_clean) {
      NFL_TRY(fill_f32(reinterpret_cast<float *>(P->spec1.p), (int64_t)2 * L * L * Hz, 0.f, P->stream));
      NFL_TRY(fill_f32(reinterpret_cast<float *>(P->spec2.p), (int64_t)2 * L * F * Hz, 0.f, P->stream));
      P->spec_clean = true;
    }
    if (!sup) P->spec_clean = false;   // the full passes write every entry
    const int *zl = sup ? P->zs_lines.p : nullptr, *zx = sup ? P->zs_x.p : nullptr;
    const uint8_t *zmap = sup ? P->zs_map.p : nullptr, *zxin = sup ? P->zs_map.p + (size_t)L * L : nullptr;
    const int nlines = sup ? P->zs_nlines : L * L, nxs = sup ? P->zs_nx : L;
    const int nb = (nlines + lpz - 1) / lpz;
    hipLaunchKernelGGL(r2c, dim3(nb), dim3(FFT_THREADS), ldz, P->stream, gin, P->spec1.p,
                       nlines, L, logL, lpz, Hz, tw, P->stop, fxm, fxu, zl);
    const int lpy = fft_lpb_y(L, fe), ngroups = (Hz + lpy - 1) / lpy;
    const size_t ldy = fft_lds_bytes(lpy, L);
    hipLaunchKernelGGL(k_y_fwd, dim3(nxs * ngroups), dim3(FFT_THREADS), ldy, P->stream, P->spec1.p,
                       P->spec2.p, L, logL, lpy, Hz, N, tw, P->stop, zx);
    const int C = F * Hz, lpx = fft_lpb_x(L, fe);
    hipLaunchKernelGGL(k_x_filter, dim3((C + lpx - 1) / lpx), dim3(FFT_THREADS),
                       fft_lds_bytes(lpx, L), P->stream, P->spec2.p, P->filt.p, C, L, logL, lpx,
                       N, tw, P->stop, zxin);
    hipLaunchKernelGGL(k_y_inv, dim3(nxs * ngroups), dim3(FFT_THREADS), ldy, P->stream, P->spec2.p,
                       P->spec1.p, L, logL, lpy, Hz, N, tw, P->stop, zx, zmap);
    hipLaunchKernelGGL(k_c2r_lines, dim3(nb), dim3(FFT_THREADS), ldz, P->stream, P->spec1.p, gout,
                       nlines, L, logL, lpz, Hz, tw, P->stop, fxr, zl);
  }
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

// Two grids: the spread accumulates into `grid`, which the r2c pass reads and
// leaves zero for the next product (so no separate clear once it is clean);
// the c2r pass writes `grid2`, which the interpolation reads.
// Both tile-stationary forms run (d = 3, default kernels, T + 2m - 1 <= 16).
static bool tile_forms(const nfl_plan *P) {
  const int T = 1 << P->tshift, W = 2 * P->m;
  return P->d == 3 && P->opt_kernel == 0 && ((T == 4 && W + 3 <= 16) || (T == 8 && W + 7 <= 16));
}

int product_dot_parts(const nfl_plan *P) {
  return P->prec == 32 && tile_forms(P) && P->ngroups > 0 && P->ngroups <= DOT_PARTS_MAX
             ? P->ngroups
             : 0;
}

int fastsum(nfl_plan *P, int in_mode, int out_mode, const VecArgs &a_in) {
  if (P->prec == 64) return fastsum64(P, in_mode, out_mode, a_in);
  VecArgs a = a_in;
  // the output step needs the caller-order input: the tile spread leaves a
  // sorted copy of it for the tile interpolation
  if ((in_mode == IN_USER_F32 || in_mode == IN_USER_F32_DINV) && a.x32 &&
      (out_mode == OUT_USER_W || out_mode == OUT_USER_LS || out_mode == OUT_USER_A) &&
      tile_forms(P) && P->xs32.p)
    a.xs = P->xs32.p;
  if (P->prof_ev) NFL_HIP(hipEventRecord(P->prof_ev[0], P->stream));
  const bool clear = !P->grid_clean;
  P->grid_clean = false;
  NFL_TRY(spread(P, in_mode, a, P->grid.p, clear));
  if (P->prof_ev) NFL_HIP(hipEventRecord(P->prof_ev[2], P->stream));
  NFL_TRY(convolve(P, P->grid.p, P->grid2.p, true, true));
  P->grid_clean = true;
  if (P->prof_ev) NFL_HIP(hipEventRecord(P->prof_ev[3], P->stream));
  NFL_TRY(interp(P, P->grid2.p, in_mode, out_mode, a));
  NFL_TRY(near_field(P, in_mode, out_mode, a));   // Laplacian RBF kernel only
  if (P->prof_ev) NFL_HIP(hipEventRecord(P->prof_ev[4], P->stream));
  return NFL_OK;
}

}  // namespace nfl
