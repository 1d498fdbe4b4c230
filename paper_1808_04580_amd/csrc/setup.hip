// Setup of a plan: node statistics, grid keys, radix sort, work items and
// the FP64 filter (steps 1-3 of Alg. nfft_normalized_matvec).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "nfl_internal.h"
#include "workdiv.h"

namespace nfl {

// ---------------------------------------------------------------------------
// Node statistics: bounding-box midpoint c and R = max ||v - c|| (FP64).
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

__global__ __launch_bounds__(RED_THREADS) void k_bbox_partial(const float *__restrict__ v,
                                                              int64_t n, int d,
                                                              double *__restrict__ part) {
  __shared__ float smin[3][RED_THREADS], smax[3][RED_THREADS];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * RED_THREADS) {
    for (int t = 0; t < d; ++t) {
      float x = v[i * d + t];
      lo[t] = fminf(lo[t], x);
      hi[t] = fmaxf(hi[t], x);
    }
  }
  for (int t = 0; t < 3; ++t) {
    smin[t][threadIdx.x] = lo[t];
    smax[t][threadIdx.x] = hi[t];
  }
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int t = 0; t < 3; ++t) {
        smin[t][threadIdx.x] = fminf(smin[t][threadIdx.x], smin[t][threadIdx.x + s]);
        smax[t][threadIdx.x] = fmaxf(smax[t][threadIdx.x], smax[t][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    part[blockIdx.x * 6 + threadIdx.x] = smin[threadIdx.x][0];
    part[blockIdx.x * 6 + 3 + threadIdx.x] = smax[threadIdx.x][0];
  }
}

// One block: reduce the partial boxes, write the midpoint to part[0..2].
__global__ __launch_bounds__(64) void k_bbox_final(double *part, int nparts, int d) {
  if (threadIdx.x == 0) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nparts; ++b)
      for (int t = 0; t < 3; ++t) {
        lo[t] = fmin(lo[t], part[b * 6 + t]);
        hi[t] = fmax(hi[t], part[b * 6 + 3 + t]);
      }
    for (int t = 0; t < 3; ++t) part[t] = t < d ? 0.5 * (lo[t] + hi[t]) : 0.0;
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_radius_partial(const float *__restrict__ v,
                                                                int64_t n, int d,
                                                                const double *__restrict__ c,
                                                                double *__restrict__ part) {
  __shared__ double s[RED_THREADS];
  double r2 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * RED_THREADS) {
    double a = 0.0;
    for (int t = 0; t < d; ++t) {
      double x = (double)v[i * d + t] - c[t];
      a += x * x;
    }
    r2 = a == a ? fmax(r2, a) : INFINITY;   // a NaN coordinate makes the radius infinite
  }
  s[threadIdx.x] = r2;
  __syncthreads();
  for (int k = RED_THREADS / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(64) void k_radius_final(double *part, int nparts, double *out) {
  if (threadIdx.x == 0) {
    double r2 = 0.0;
    for (int b = 0; b < nparts; ++b) r2 = fmax(r2, part[b]);
    out[0] = sqrt(r2);
  }
}

int radius_about(nfl_plan *P, const double *centre, double *radius) {
  const int nb = (int)std::min<int64_t>(1024, (P->n + RED_THREADS - 1) / RED_THREADS);
  NFL_TRY(P->red.ensure((size_t)nb * 6 + 8));
  double *part = P->red.p;
  double *res = P->red.p + (size_t)nb * 6;
  NFL_HIP(hipMemcpyAsync(res, centre, 3 * sizeof(double), hipMemcpyHostToDevice, P->stream));
  hipLaunchKernelGGL(k_radius_partial, dim3(nb), dim3(RED_THREADS), 0, P->stream, P->pts_user.p,
                     P->n, P->d, res, part);
  hipLaunchKernelGGL(k_radius_final, dim3(1), dim3(64), 0, P->stream, part, nb, res + 3);
  NFL_HIP(hipGetLastError());
  NFL_HIP(hipMemcpyAsync(radius, res + 3, sizeof(double), hipMemcpyDeviceToHost, P->stream));
  NFL_HIP(hipStreamSynchronize(P->stream));
  return NFL_OK;
}

int bbox_and_radius(nfl_plan *P) {
  const int nb = (int)std::min<int64_t>(1024, (P->n + RED_THREADS - 1) / RED_THREADS);
  NFL_TRY(P->red.ensure((size_t)nb * 6 + 8));
  double *part = P->red.p;
  double *res = P->red.p + (size_t)nb * 6;  // centre (3) + radius (1)
  hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(RED_THREADS), 0, P->stream, P->pts_user.p,
                     P->n, P->d, part);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, P->stream, part, nb, P->d);
  NFL_HIP(hipMemcpyAsync(res, part, 3 * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
  hipLaunchKernelGGL(k_radius_partial, dim3(nb), dim3(RED_THREADS), 0, P->stream, P->pts_user.p,
                     P->n, P->d, res, part);
  hipLaunchKernelGGL(k_radius_final, dim3(1), dim3(64), 0, P->stream, part, nb, res + 3);
  NFL_HIP(hipGetLastError());
  double h[4];
  NFL_HIP(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, P->stream));
  NFL_HIP(hipStreamSynchronize(P->stream));
  for (int t = 0; t < 3; ++t) P->centre[t] = h[t];
  P->radius = h[3];
  return NFL_OK;
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 (1024 elements per block, recursive on block sums).
// ---------------------------------------------------------------------------
constexpr int SCAN_THREADS = 256, SCAN_PER = 4, SCAN_TILE = SCAN_THREADS * SCAN_PER;

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_block(const uint32_t *__restrict__ in,
                                                             uint32_t *__restrict__ out,
                                                             int64_t len,
                                                             uint32_t *__restrict__ bsum) {
  __shared__ uint32_t s[SCAN_THREADS];
  const int64_t base = blockIdx.x * (int64_t)SCAN_TILE + threadIdx.x * SCAN_PER;
  uint32_t v[SCAN_PER], tot = 0;
  for (int k = 0; k < SCAN_PER; ++k) {
    v[k] = (base + k < len) ? in[base + k] : 0u;
    tot += v[k];
  }
  s[threadIdx.x] = tot;
  __syncthreads();
  // Hillis-Steele inclusive scan over the thread totals
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    uint32_t add = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - tot;
  for (int k = 0; k < SCAN_PER; ++k) {
    if (base + k < len) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == SCAN_THREADS - 1 && bsum) bsum[blockIdx.x] = s[threadIdx.x];
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(uint32_t *__restrict__ out, int64_t len,
                                                           const uint32_t *__restrict__ bsum) {
  const int64_t base = blockIdx.x * (int64_t)SCAN_TILE + threadIdx.x * SCAN_PER;
  const uint32_t a = bsum[blockIdx.x];
  for (int k = 0; k < SCAN_PER; ++k)
    if (base + k < len) out[base + k] += a;
}

static int scan_rec(const uint32_t *in, uint32_t *out, int64_t len, hipStream_t s,
                    uint32_t *scratch) {
  const int64_t nb = (len + SCAN_TILE - 1) / SCAN_TILE;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(SCAN_THREADS), 0, s, in, out, len,
                       (uint32_t *)nullptr);
    return NFL_OK;
  }
  uint32_t *bs = scratch, *bss = scratch + nb;
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, out, len,
                     bs);
  NFL_TRY(scan_rec(bs, bss, nb, s, scratch + 2 * nb));
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, out, len, bss);
  return NFL_OK;
}

// scratch must hold >= 2*len/1024 + 64 entries (geometric series).
static size_t scan_scratch_count(int64_t len) { return (size_t)(2 * (len / SCAN_TILE + 2) + 64); }

// ---------------------------------------------------------------------------
// LSD radix sort of (key, value) pairs, 8-bit digits, stable.
// Each block ranks its 4096 elements in 16 rounds of 256: inside a wave the
// elements with equal digit are found with 8 ballots; across the 4 waves by
// per-wave digit counts in LDS.  The per-digit block offsets come from an
// exclusive scan of the digit-major histogram, which makes the sort stable.
// ---------------------------------------------------------------------------
constexpr int RS_THREADS = 256, RS_ROUNDS = 16, RS_TILE = RS_THREADS * RS_ROUNDS;

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t *__restrict__ keys,
                                                        int64_t n, int shift,
                                                        uint32_t *__restrict__ hist, int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * (int64_t)RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t i = base + r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, int64_t n, int shift,
    const uint32_t *__restrict__ offs, int nblocks, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[RS_THREADS / 64][256];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  run[t] = offs[(int64_t)t * nblocks + blockIdx.x];
  for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = blockIdx.x * (int64_t)RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + r * RS_THREADS + t;
    const bool valid = i < n;
    uint32_t key = valid ? kin[i] : 0u, val = valid ? vin[i] : 0u;
    uint32_t dg = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t bb = __ballot(valid && bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[wave][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dg] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dg];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int w = 0; w < RS_THREADS / 64; ++w) {
      tot += wcnt[w][t];
      wcnt[w][t] = 0;
    }
    run[t] += tot;
    __syncthreads();
  }
}

int radix_sort_pairs(uint32_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s,
                     DBuf<unsigned char> &tmp) {
  if (n <= 1 || bits <= 0) return NFL_OK;
  const int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
  const int64_t hlen = 256LL * nblocks;
  const size_t need = (size_t)n * 8 + (size_t)hlen * 8 + scan_scratch_count(hlen) * 4 + 256;
  NFL_TRY(tmp.ensure(need));
  uint32_t *k2 = (uint32_t *)tmp.p;
  uint32_t *v2 = k2 + n;
  uint32_t *hist = v2 + n;
  uint32_t *offs = hist + hlen;
  uint32_t *scr = offs + hlen;
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  const int passes = (bits + 7) / 8;
  for (int ps = 0; ps < passes; ++ps) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(RS_THREADS), 0, s, ka, n, ps * 8, hist,
                       nblocks);
    NFL_TRY(scan_rec(hist, offs, hlen, s, scr));
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(RS_THREADS), 0, s, ka, va, n, ps * 8,
                       offs, nblocks, kb, vb);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    NFL_HIP(hipMemcpyAsync(keys, ka, n * 4, hipMemcpyDeviceToDevice, s));
    NFL_HIP(hipMemcpyAsync(vals, va, n * 4, hipMemcpyDeviceToDevice, s));
  }
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t len, hipStream_t s,
                       DBuf<uint32_t> &scratch, size_t off) {
  NFL_TRY(scratch.ensure(off + scan_scratch_count(len)));
  return scan_rec(in, out, len, s, scratch.p + off);
}

// ---------------------------------------------------------------------------
// Grid coordinates and keys.  u = nos (rho (v - c) + 1/2) in FP64, split into
// the integer cell and a float32 fraction in [0, 1).  Key = tile-major cell
// index; the packed cell (10 bits per axis) rides along in the node record.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_keys(const float *__restrict__ v, int64_t n, int d,
                                              double c0, double c1, double c2, double rho,
                                              int nos, int tshift, uint32_t *__restrict__ keys,
                                              uint32_t *__restrict__ idx,
                                              float4 *__restrict__ rec) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const double c[3] = {c0, c1, c2};
  int cell[3] = {0, 0, 0};
  float fr[3] = {0.f, 0.f, 0.f};
  for (int t = 0; t < d; ++t) {
    double u = (double)nos * (rho * ((double)v[i * d + t] - c[t]) + 0.5);
    double f = floor(u);
    int ci = (int)f;
    double fr64 = u - f;
    if (ci < 0) { ci = 0; fr64 = 0.0; }
    if (ci > nos - 1) { ci = nos - 1; fr64 = 0.0; }
    float ff = (float)fr64;
    if (ff >= 1.0f) ff = 0x1.fffffep-1f;  // keep the fraction below 1 after rounding
    cell[t] = ci;
    fr[t] = ff;
  }
  const uint32_t T = 1u << tshift, ntd = (uint32_t)nos >> tshift;
  uint32_t tile = 0, local = 0;
  for (int t = 0; t < d; ++t) tile = tile * ntd + ((uint32_t)cell[t] >> tshift);
  // inside a tile the last axis is the slowest: nodes of one z-offset (of one
  // y-offset, then one cell) are consecutive, which the interpolation's runs use
  for (int t = d - 1; t >= 0; --t) local = local * T + ((uint32_t)cell[t] & (T - 1));
  keys[i] = (tile << (d * tshift)) | local;
  idx[i] = (uint32_t)i;
  const uint32_t packed = (uint32_t)cell[0] | ((uint32_t)cell[1] << 10) | ((uint32_t)cell[2] << 20);
  rec[i] = make_float4(fr[0], fr[1], fr[2], __uint_as_float(packed));
}

__global__ __launch_bounds__(256) void k_gather_nodes(const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ idx, int64_t n,
                                                      float4 *__restrict__ pts,
                                                      int *__restrict__ perm) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = idx[i];
  pts[i] = rec[j];
  perm[i] = (int)j;
}

// Sorted keys: the nodes of a tile are contiguous.  end[tile] = one past its
// last node (tiles without nodes keep 0).
__global__ __launch_bounds__(256) void k_tile_ends(const uint32_t *__restrict__ keys, int64_t n,
                                                   int shift, uint32_t *__restrict__ end) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = keys[i] >> shift;
  if (i + 1 == n || (keys[i + 1] >> shift) != t) end[t] = (uint32_t)(i + 1);
}

int build_sorted_nodes(nfl_plan *P) {
  const int64_t n = P->n;
  const int d = P->d;
  int T = std::min(P->opt_tile, P->nos);
  if (d == 3) {
    // the matrix-core spread keeps four private copies of the padded tile in LDS
    const int W = 2 * P->m;
    auto lds_need = [&](int t) {
      const int p = t + W - 1, px = p * p + ((4 - p * p) % 32 + 32) % 32;
      return (size_t)4 * px * p * 4 + 4 * 16 * 80 * 4;
    };
    while (T > 4 && lds_need(T) > 160 * 1024) T >>= 1;
  } else {
    // the d <= 2 spread sums one padded tile of T + 2m - 1 <= 19 cells per axis
    while (T > 1 && T + 2 * P->m - 1 > 19) T >>= 1;
  }
  int tshift = 0;
  while ((1 << tshift) < T) ++tshift;
  P->tshift = tshift;
  int lognos = 0;
  while ((1 << lognos) < P->nos) ++lognos;
  const int bits = d * lognos;
  const int64_t ntiles = 1LL << (d * (lognos - tshift));

  // temporaries: keys, idx, records, tile counts
  LBuf<unsigned char> work;
  const size_t need = (size_t)n * 4 * 2 + (size_t)n * 16 + (size_t)ntiles * 4 + 64;
  NFL_TRY(work.ensure(need));
  uint32_t *keys = (uint32_t *)work.p;
  uint32_t *idx = keys + n;
  const size_t rec_off = ((size_t)2 * n + 3) & ~(size_t)3;  // 16-byte aligned
  float4 *rec = (float4 *)(keys + rec_off);
  uint32_t *cnt = (uint32_t *)(rec + n);

  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_keys, dim3(nb), dim3(256), 0, P->stream, P->pts_user.p, n, d, P->centre[0],
                     P->centre[1], P->centre[2], P->rho, P->nos, tshift, keys, idx, rec);
  int rc = radix_sort_pairs(keys, idx, n, bits, P->stream, P->tmp);
  if (rc < 0) { work.release(); return rc; }
  rc = P->pts.ensure(n);
  if (rc == NFL_OK) rc = P->perm.ensure(n);
  if (rc < 0) { work.release(); return rc; }
  hipLaunchKernelGGL(k_gather_nodes, dim3(nb), dim3(256), 0, P->stream, rec, idx, n, P->pts.p,
                     P->perm.p);
  hipError_t e = hipMemsetAsync(cnt, 0, (size_t)ntiles * 4, P->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_tile_ends, dim3(nb), dim3(256), 0, P->stream, keys, n, d * tshift, cnt);
    e = hipGetLastError();
  }
  std::vector<uint32_t> hc((size_t)ntiles);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hc.data(), cnt, (size_t)ntiles * 4, hipMemcpyDeviceToHost, P->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
  work.release();
  if (e != hipSuccess) {
    set_error(std::string("build_sorted_nodes: ") + hipGetErrorString(e));
    return NFL_ERR_HIP;
  }
  // tile sizes from the run ends (tiles are in sorted order)
  {
    uint32_t prev = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
      if (hc[(size_t)t] == 0) continue;
      const uint32_t e_t = hc[(size_t)t];
      hc[(size_t)t] = e_t - prev;
      prev = e_t;
    }
  }
  // Work items: each occupied tile split into near-equal chunks of at most
  // opt_chunk nodes (at most 64 for d <= 2, whose spread loops over every
  // node of an item for each cell of the padded tile: short items keep that
  // loop short and give more workgroups to small clustered problems).
  const int64_t chunk = d == 3 ? P->opt_chunk : std::min(P->opt_chunk, 64);
  std::vector<Item> items;
  int64_t start = 0;
  int maxlen = 0;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t c = hc[(size_t)t];
    if (c == 0) continue;
    const int64_t nch = (c + chunk - 1) / chunk;
    for (int64_t k = 0; k < nch; ++k) {
      Item it;
      it.tile = (int)t;
      it.start = (int)(start + c * k / nch);
      it.end = (int)(start + c * (k + 1) / nch);
      it.pad = (int)k;
      maxlen = std::max(maxlen, it.end - it.start);
      items.push_back(it);
    }
    start += c;
  }
  // First chunks of all tiles, then second chunks, ...: chunks of one tile
  // then run apart in time, so their tile flushes (atomic adds to the same
  // grid cells) do not queue on the same addresses.
  std::stable_sort(items.begin(), items.end(),
                   [](const Item &a, const Item &b) { return a.pad < b.pad; });
  for (Item &it : items) it.pad = 0;
  P->nitems = (int)items.size();
  P->max_item_len = maxlen;
  // sorted-node offset of every tile (the near-field sum walks neighbour tiles)
  {
    std::vector<int> ts((size_t)ntiles + 1);
    int64_t acc = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
      ts[(size_t)t] = (int)acc;
      acc += hc[(size_t)t];
    }
    ts[(size_t)ntiles] = (int)acc;
    P->ntiles = ntiles;
    NFL_TRY(P->tile_start.ensure(ts.size()));
    NFL_HIP(hipMemcpyAsync(P->tile_start.p, ts.data(), ts.size() * sizeof(int),
                           hipMemcpyHostToDevice, P->stream));
    NFL_HIP(hipStreamSynchronize(P->stream));
  }
  NFL_TRY(P->items.ensure(items.size()));
  NFL_HIP(hipMemcpyAsync(P->items.p, items.data(), items.size() * sizeof(Item),
                         hipMemcpyHostToDevice, P->stream));
  P->ngroups = 0;
  if (const int slots = tile_group_slots(P); slots > 0 && n > 0) {
    std::vector<GroupSeg> segs;
    std::vector<int> goff;
    cost_groups(hc, n, slots, segs, goff);
    std::vector<Item> gi(segs.size());
    for (size_t k = 0; k < segs.size(); ++k) gi[k] = Item{segs[k].tile, segs[k].start, segs[k].end, 0};
    NFL_TRY(P->gitems.ensure(gi.size()));
    NFL_TRY(P->goff.ensure(goff.size()));
    NFL_HIP(hipMemcpyAsync(P->gitems.p, gi.data(), gi.size() * sizeof(Item),
                           hipMemcpyHostToDevice, P->stream));
    NFL_HIP(hipMemcpyAsync(P->goff.p, goff.data(), goff.size() * sizeof(int),
                           hipMemcpyHostToDevice, P->stream));
    NFL_HIP(hipStreamSynchronize(P->stream));   // the host vectors go out of scope
    P->ngroups = (int)goff.size() - 1;
  }
  // d = 3: the z-lines some node's window touches.  A node of cell c spreads
  // into cells c - m + 1 .. c + m (mod nos) along each axis, so the lines of an
  // occupied tile with origin o lie in [o - m + 1, o + T + m) along x and y.
  P->zs_nlines = P->zs_nx = 0;
  P->spec_clean = false;
  if (d == 3) {
    const int nos = P->nos, T = 1 << tshift, ntd = nos >> tshift, m = P->m;
    std::vector<uint8_t> map((size_t)nos * nos + nos, 0);
    for (int64_t t = 0; t < ntiles; ++t) {
      if (hc[(size_t)t] == 0) continue;
      const int tx = (int)(t / ((int64_t)ntd * ntd)), ty = (int)((t / ntd) % ntd);
      for (int x = tx * T - m + 1; x < tx * T + T + m; ++x)
        for (int y = ty * T - m + 1; y < ty * T + T + m; ++y)
          map[(size_t)(x & (nos - 1)) * nos + (y & (nos - 1))] = 1;
    }
    std::vector<int> lines, xs;
    for (int x = 0; x < nos; ++x) {
      bool any = false;
      for (int y = 0; y < nos; ++y)
        if (map[(size_t)x * nos + y]) {
          lines.push_back(x * nos + y);
          any = true;
        }
      if (any) {
        xs.push_back(x);
        map[(size_t)nos * nos + x] = 1;
      }
    }
    if (!lines.empty()) {
      NFL_TRY(P->zs_lines.ensure(lines.size()));
      NFL_TRY(P->zs_x.ensure(xs.size()));
      NFL_TRY(P->zs_map.ensure(map.size()));
      NFL_HIP(hipMemcpyAsync(P->zs_lines.p, lines.data(), lines.size() * sizeof(int),
                             hipMemcpyHostToDevice, P->stream));
      NFL_HIP(hipMemcpyAsync(P->zs_x.p, xs.data(), xs.size() * sizeof(int),
                             hipMemcpyHostToDevice, P->stream));
      NFL_HIP(hipMemcpyAsync(P->zs_map.p, map.data(), map.size(), hipMemcpyHostToDevice,
                             P->stream));
      P->zs_nlines = (int)lines.size();
      P->zs_nx = (int)xs.size();
    }
  }
  NFL_HIP(hipStreamSynchronize(P->stream));
  return NFL_OK;
}

// ---------------------------------------------------------------------------
// Filter (host, FP64).  The kernel's Fourier coefficients b_l of eq.
// b_l::K_RF (normalised by N^d), the Nyquist coefficients split evenly
// between +l and -l (real part of Alg. nfft_fastsum), divided by the square
// of the window transform per axis (deconvolution before the FFT of step 1
// and after the inverse FFT of step 3).
// ---------------------------------------------------------------------------

// Radial derivatives K^{(k)}(r), k < p, of exp(-r^2/s^2) via the Hermite
// recurrence H_{k+1}(x) = 2x H_k(x) - 2k H_{k-1}(x).
static void gauss_derivs(double r, double s, int p, double *out) {
  const double x = r / s, e = std::exp(-x * x);
  double hm = 1.0, h = 2.0 * x;
  out[0] = e;
  double f = -1.0 / s;
  if (p > 1) out[1] = f * h * e;
  double fk = f;
  for (int k = 1; k + 1 < p; ++k) {
    const double hn = 2.0 * x * h - 2.0 * k * hm;
    hm = h;
    h = hn;
    fk *= f;
    out[k + 1] = fk * h * e;
  }
}

// Radial derivatives K^{(k)}(r0), k < p, of (1 + r^2/c^2)^alpha: the
// multiquadric (alpha = 1/2) or inverse multiquadric (alpha = -1/2) kernel of
// eq. W_general divided by its value at 0.  With u(h) = 1 + (r0 + h)^2/c^2
// (a quadratic in h), the Taylor coefficients w_k of u^alpha follow from
// u w' = alpha u' w (J. C. P. Miller's recurrence for powers of a power
// series): w_k = (1 / (k u_0)) sum_{j=1}^{min(k, 2)} ((alpha + 1) j - k) u_j w_{k-j};
// K^{(k)}(r0) = k! w_k.
static void power_derivs(double r0, double c, double alpha, int p, double *out) {
  const double u[3] = {1.0 + r0 * r0 / (c * c), 2.0 * r0 / (c * c), 1.0 / (c * c)};
  std::vector<double> w((size_t)p);
  w[0] = std::pow(u[0], alpha);
  for (int k = 1; k < p; ++k) {
    double acc = 0.0;
    for (int j = 1; j <= std::min(k, 2); ++j) acc += ((alpha + 1.0) * j - k) * u[j] * w[k - j];
    w[k] = acc / (k * u[0]);
  }
  double f = 1.0;
  for (int k = 0; k < p; ++k) {
    if (k > 0) f *= k;
    out[k] = f * w[k];
  }
}

static double binom(int a, int b) {
  double r = 1.0;
  for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
  return r;
}

// Two-point Taylor interpolant of degree 2p-1 on [a, b] from the derivative
// values fa[k], fb[k], k < p (closed form of the two-point Hermite basis).
static double two_point_taylor(double x, double a, double b, const double *fa, const double *fb,
                               int p) {
  const double ua = (x - a) / (b - a), ub = (x - b) / (a - b);
  double sum = 0.0, kf = 1.0;
  for (int k = 0; k < p; ++k) {
    if (k > 0) kf *= k;
    double sa = 0.0, sb = 0.0;
    for (int j = 0; j + k < p; ++j) {
      const double c = binom(p - 1 + j, j);
      sa += c * std::pow(ua, j);
      sb += c * std::pow(ub, j);
    }
    sum += fa[k] / kf * std::pow(x - a, k) * std::pow(ub, p) * sa;
    sum += fb[k] / kf * std::pow(x - b, k) * std::pow(ua, p) * sb;
  }
  return sum;
}

// In-place radix-2 complex FFT (FP64, forward sign -1) of length L (power of 2).
static void fft64(std::complex<double> *a, int L, int stride) {
  for (int i = 1, j = 0; i < L; ++i) {
    int bit = L >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[(size_t)i * stride], a[(size_t)j * stride]);
  }
  for (int len = 2; len <= L; len <<= 1) {
    const double ang = -2.0 * M_PI / len;
    for (int i = 0; i < L; i += len)
      for (int k = 0; k < len / 2; ++k) {
        const std::complex<double> w(std::cos(ang * k), std::sin(ang * k));
        std::complex<double> &u = a[(size_t)(i + k) * stride];
        std::complex<double> &v = a[(size_t)(i + k + len / 2) * stride];
        const std::complex<double> t = w * v;
        v = u - t;
        u = u + t;
      }
  }
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the three-term
// recurrence of the Legendre polynomials).
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      const double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// The Kaiser-Bessel window in grid units,
//   psi(t) = sinh(b s) / (s b e^{bm}),  s = sqrt(m^2 - t^2),  |t| <= m,
// with b = pi (2 - 1/sigma_os), sigma_os = 2 (the oversampling factor).
static double kb_psi(double t, int m, double b) {
  const double s = std::sqrt(std::max(0.0, (double)m * m - t * t));
  return (s > 0 ? std::sinh(b * s) / s : b) / (b * std::exp(b * m));
}

// The kernels evaluate the window as 2m polynomials, one per grid offset c of
// a node's window: psi(c - (m-1) - f) ~= sum_k coef[c][k] g^k, g = 2f - 1, for
// the cell fraction f in [0, 1).  Degree WIN_NC-1 interpolation at Chebyshev
// nodes in FP64, coefficients rounded to float32 (FP32 rounding level).
static void window_poly(int m, double b, std::vector<float> &coef) {
  const int W = 2 * m, D = WIN_NC;
  coef.assign((size_t)WIN_MAXW * D, 0.f);
  std::vector<double> V((size_t)D * D), y(D);
  for (int c = 0; c < W; ++c) {
    for (int k = 0; k < D; ++k) {
      const double g = std::cos(M_PI * (k + 0.5) / D), f = 0.5 * (g + 1.0);
      y[k] = kb_psi(c - (m - 1) - f, m, b);
      double pw = 1.0;
      for (int q = 0; q < D; ++q, pw *= g) V[(size_t)k * D + q] = pw;
    }
    // Gaussian elimination with partial pivoting on the D x D Vandermonde system
    for (int col = 0; col < D; ++col) {
      int piv = col;
      for (int r = col + 1; r < D; ++r)
        if (std::fabs(V[(size_t)r * D + col]) > std::fabs(V[(size_t)piv * D + col])) piv = r;
      for (int q = 0; q < D; ++q) std::swap(V[(size_t)col * D + q], V[(size_t)piv * D + q]);
      std::swap(y[col], y[piv]);
      for (int r = col + 1; r < D; ++r) {
        const double fct = V[(size_t)r * D + col] / V[(size_t)col * D + col];
        for (int q = col; q < D; ++q) V[(size_t)r * D + q] -= fct * V[(size_t)col * D + q];
        y[r] -= fct * y[col];
      }
    }
    for (int r = D - 1; r >= 0; --r) {
      double acc = y[r];
      for (int q = r + 1; q < D; ++q) acc -= V[(size_t)r * D + q] * y[q];
      y[r] = acc / V[(size_t)r * D + r];
    }
    for (int k = 0; k < D; ++k) coef[(size_t)c * D + k] = (float)y[k];
  }
}

// Fourier transform, at frequency xi, of the window the kernels apply (the
// piecewise polynomial with float32 coefficients), by 32-point Gauss-Legendre
// quadrature on each unit interval.
static double window_hat(double xi, int m, const std::vector<float> &coef) {
  static thread_local std::vector<double> gx, gw;
  if (gx.empty()) gauss_legendre(32, gx, gw);
  double acc = 0.0;
  for (int c = 0; c < 2 * m; ++c)
    for (size_t k = 0; k < gx.size(); ++k) {
      const double f = 0.5 * (gx[k] + 1.0), g = gx[k];
      double p = 0.0;
      for (int q = WIN_NC - 1; q >= 0; --q) p = p * g + (double)coef[(size_t)c * WIN_NC + q];
      const double t = c - (m - 1) - f;
      acc += 0.5 * gw[k] * p * std::cos(2.0 * M_PI * xi * t);
    }
  return acc;
}

int window_coefficients(int m, std::vector<float> &coef) {
  if (m < 1 || 2 * m > WIN_MAXW) return NFL_ERR_ARG;
  window_poly(m, M_PI * (2.0 - 0.5), coef);
  return NFL_OK;
}

// Radial derivatives of exp(-r/s): (-1/s)^k exp(-r/s), k < p.
static void laplace_derivs(double r, double s, int p, double *out) {
  double f = std::exp(-r / s);
  for (int k = 0; k < p; ++k) {
    out[k] = f;
    f *= -1.0 / s;
  }
}

// The inner polynomial T_I of the Laplacian RBF kernel exp(-r/s): the
// two-point Taylor interpolant on [-eps_I, eps_I] of the even extension of the
// kernel (p conditions at each end), which is even of degree <= 2p - 2; its
// coefficients c_k in (r / eps_I)^(2k), k < p, by interpolation at p points
// in (0, 1] (exact for such a polynomial up to rounding).
int inner_poly(double s, double eps_I, int p, std::vector<double> &c) {
  if (!(eps_I > 0) || p < 1 || p > 16) return NFL_ERR_ARG;
  std::vector<double> fb(p), fa(p);
  laplace_derivs(eps_I, s, p, fb.data());
  for (int k = 0; k < p; ++k) fa[k] = (k & 1) ? -fb[k] : fb[k];
  std::vector<double> A((size_t)p * p), rhs(p);
  for (int i = 0; i < p; ++i) {
    const double u = std::cos(M_PI * (i + 0.5) / (2 * p));   // u = r / eps_I in (0, 1)
    rhs[i] = two_point_taylor(u * eps_I, -eps_I, eps_I, fa.data(), fb.data(), p);
    double w = 1.0;
    for (int k = 0; k < p; ++k) {
      A[(size_t)i * p + k] = w;
      w *= u * u;
    }
  }
  // Gaussian elimination with partial pivoting
  for (int col = 0; col < p; ++col) {
    int piv = col;
    for (int r = col + 1; r < p; ++r)
      if (std::fabs(A[(size_t)r * p + col]) > std::fabs(A[(size_t)piv * p + col])) piv = r;
    if (A[(size_t)piv * p + col] == 0.0) return NFL_ERR_ARG;
    for (int k = 0; k < p; ++k) std::swap(A[(size_t)col * p + k], A[(size_t)piv * p + k]);
    std::swap(rhs[col], rhs[piv]);
    for (int r = col + 1; r < p; ++r) {
      const double f = A[(size_t)r * p + col] / A[(size_t)col * p + col];
      for (int k = col; k < p; ++k) A[(size_t)r * p + k] -= f * A[(size_t)col * p + k];
      rhs[r] -= f * rhs[col];
    }
  }
  c.assign(p, 0.0);
  for (int r = p - 1; r >= 0; --r) {
    double t = rhs[r];
    for (int k = r + 1; k < p; ++k) t -= A[(size_t)r * p + k] * c[k];
    c[r] = t / A[(size_t)r * p + r];
  }
  return NFL_OK;
}

// The regularised kernel K_R of the fast summation in the scaled coordinates,
// divided by K(0) (sigma_t is the scaled width or the scaled multiquadric
// parameter c): K on r <= 1/2 - eps_B (and, for the Laplacian RBF kernel, the
// inner polynomial T_I on r <= eps_I), the two-point Taylor transition to the
// constant K(1/2) on (1/2 - eps_B, 1/2], that constant beyond 1/2.
RegKernel::RegKernel(int kind_, double sigma_t_, double eps_B_, double eps_I_, int p_)
    : kind(kind_), sigma_t(sigma_t_), eps_B(eps_B_), eps_I(eps_I_), p(p_), r0(0.5 - eps_B_),
      alpha(kind_ == NFL_KERNEL_MULTIQUADRIC ? 0.5 : -0.5), fa(p_), fb(p_, 0.0), ia(p_), ib(p_) {
  if (kind == NFL_KERNEL_GAUSSIAN)
    gauss_derivs(r0, sigma_t, p, fa.data());
  else if (kind == NFL_KERNEL_LAPLACIAN_RBF)
    laplace_derivs(r0, sigma_t, p, fa.data());
  else
    power_derivs(r0, sigma_t, alpha, p, fa.data());
  fb[0] = K(0.5);
  k_half = fb[0];
  if (kind == NFL_KERNEL_LAPLACIAN_RBF) {
    laplace_derivs(eps_I, sigma_t, p, ib.data());
    for (int k = 0; k < p; ++k) ia[k] = (k & 1) ? -ib[k] : ib[k];
  }
}

double RegKernel::K(double r) const {
  if (kind == NFL_KERNEL_GAUSSIAN) return std::exp(-(r * r) / (sigma_t * sigma_t));
  if (kind == NFL_KERNEL_LAPLACIAN_RBF) return std::exp(-r / sigma_t);
  return std::pow(1.0 + (r * r) / (sigma_t * sigma_t), alpha);
}

double RegKernel::operator()(double r) const {
  if (kind == NFL_KERNEL_LAPLACIAN_RBF && r <= eps_I)
    return two_point_taylor(r, -eps_I, eps_I, ia.data(), ib.data(), p);
  if (r <= r0) return K(r);
  if (eps_B <= 0.0) return k_half;  // no transition region
  if (r <= 0.5) return two_point_taylor(r, r0, 0.5, fa.data(), fb.data(), p);
  return two_point_taylor(0.5, r0, 0.5, fa.data(), fb.data(), p);
}

// b_l of eq. b_l::K_RF for l in I_N^d, normalised by N^d: the DFT of the
// samples K_R(j/N), j in I_N^d, each axis stored at index j mod N (so b_l sits
// at l mod N).  K_R is even, so b_l is real.
void kernel_bhat(int d, int N, const RegKernel &KR, std::vector<double> &bhat) {
  size_t tot = 1;
  for (int t = 0; t < d; ++t) tot *= (size_t)N;
  std::vector<std::complex<double>> S(tot);
  for (size_t q = 0; q < tot; ++q) {
    size_t r = q;
    double rr = 0.0;
    for (int t = d - 1; t >= 0; --t) {
      int jm = (int)(r % N);
      r /= N;
      int j = jm < N / 2 ? jm : jm - N;  // j in I_N
      rr += (double)j * j;
    }
    S[q] = KR(std::sqrt(rr) / N);
  }
  size_t stride = 1;
  for (int t = d - 1; t >= 0; --t) {
    const size_t outer = tot / ((size_t)N * stride);
    for (size_t o = 0; o < outer; ++o)
      for (size_t in = 0; in < stride; ++in) fft64(&S[o * N * stride + in], N, (int)stride);
    stride *= N;
  }
  const double norm = std::pow((double)N, -d);
  bhat.resize(tot);
  for (size_t q = 0; q < tot; ++q) bhat[q] = S[q].real() * norm;
}

int compute_filter(int d, int N, int m, int p, double eps_B, double sigma_t,
                   std::vector<double> &out, int kind, double eps_I, bool exact_window) {
  if (d < 1 || d > 3 || N < 2 || (N & 1) || m < 1 || p < 1 || 2 * m > WIN_MAXW) return NFL_ERR_ARG;
  if (kind < NFL_KERNEL_GAUSSIAN || kind > NFL_KERNEL_LAPLACIAN_RBF) return NFL_ERR_ARG;
  if (kind == NFL_KERNEL_LAPLACIAN_RBF && !(eps_I > 0 && eps_I + eps_B < 0.5)) return NFL_ERR_ARG;
  const int nos = 2 * N;
  std::vector<float> wcoef;
  window_poly(m, M_PI * (2.0 - 0.5), wcoef);
  const RegKernel KR(kind, sigma_t, eps_B, eps_I, p);
  std::vector<double> S;
  kernel_bhat(d, N, KR, S);
  // ---- window transform at l = -N/2..N/2
  std::vector<double> wh(N + 1);
  // (the FP64 path applies the Kaiser-Bessel function itself: its exact transform)
  for (int l = -N / 2; l <= N / 2; ++l)
    wh[l + N / 2] = exact_window ? kb_hat_exact((double)l / nos, m)
                                 : window_hat((double)l / nos, m, wcoef);
  // ---- half-spectrum filter: first d-1 axes l in [-N/2, N/2], last in [0, N/2]
  const int H = N / 2 + 1, F = N + 1;
  size_t cnt = (size_t)H;
  for (int t = 0; t < d - 1; ++t) cnt *= (size_t)F;
  out.assign(cnt, 0.0);
  for (size_t q = 0; q < cnt; ++q) {
    int l[3];
    size_t r = q;
    l[d - 1] = (int)(r % H);
    r /= H;
    for (int t = d - 2; t >= 0; --t) {
      l[t] = (int)(r % F) - N / 2;
      r /= F;
    }
    bool has_pos = false, has_neg = false;
    size_t si = 0;
    double den = 1.0;
    for (int t = 0; t < d; ++t) {
      has_pos |= (l[t] == N / 2);
      has_neg |= (l[t] == -N / 2);
      const int lm = ((l[t] % N) + N) % N;
      si = si * N + lm;
      const double w = wh[l[t] + N / 2];
      den *= w * w;
    }
    const double share = 0.5 * ((has_pos ? 0.0 : 1.0) + (has_neg ? 0.0 : 1.0));
    out[q] = share * S[si] / den;
  }
  return NFL_OK;
}

int build_filter_host(nfl_plan *P) {
  return compute_filter(P->d, P->N, P->m, P->p, P->eps_B, P->sigma_t, P->filt_host, P->kind,
                        P->eps_I);
}

}  // namespace nfl
