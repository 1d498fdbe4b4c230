// Near-field correction of the fast summation for the Laplacian RBF kernel
// exp(-r / sigma) (eq. W_laplacian_rbf).  The kernel is not smooth at 0, so the
// regularised kernel K_R is the even polynomial T_I on r <= eps_I (the
// near-origin regularisation of the fast summation); the trigonometric sum then
// misses sum_{||v~_i - v~_j|| <= eps_I} x~_j (K - T_I)(||v~_i - v~_j||) for every
// node i (the node itself included), which this kernel adds directly.
//
// One work item (the nodes of one grid tile) per workgroup: the item's nodes
// are the targets, and the nodes of every tile within eps_I, taken as one
// list (node ranges of the tiles and their prefix sums in LDS), are staged in
// LDS 256 at a time with their input values.  Items shorter than the
// workgroup give each target several thread groups, each taking every G-th
// staged source; the groups' sums are added at the end.  Distances are
// formed in grid-cell units from exact integer cell differences plus the
// differences of the float fractions.  Every output mode is affine in the fast
// sum f (y = alpha x + beta f), so the correction adds beta * delta to the
// output the interpolation already wrote; the degree pass also recomputes
// d^{-1/2}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "nfl_internal.h"
#include "nfft_device.h"

namespace nfl {

namespace {

constexpr int NT = 256;
constexpr int NF_MAXP = 16;
constexpr int NF_MAXTILES = 1024;   // neighbour tiles per item, (2R + 1)^d

// Adds one workgroup's part of the correction: every output mode is affine in
// the fast sum, so the parts of several workgroups add up.  The degree pass
// adds into the degree only; d^{-1/2} is recomputed afterwards (k_near_dinv).
template <int OUT>
__device__ __forceinline__ void add_out(const KArgs &a, int i, float d) {
  if constexpr (OUT == OUT_USER_RAW || OUT == OUT_USER_W) {
    unsafeAtomicAdd(&a.y32[a.perm[i]], d);
  } else if constexpr (OUT == OUT_USER_LS) {
    unsafeAtomicAdd(&a.y32[a.perm[i]], -(a.dinv[i] * d));
  } else if constexpr (OUT == OUT_USER_A) {
    unsafeAtomicAdd(&a.y32[a.perm[i]], a.dinv[i] * d);
  } else if constexpr (OUT == OUT_DEGREE) {
    unsafeAtomicAdd(&a.deg_out[i], d);
  } else if constexpr (OUT == OUT_SORTED_F64_A) {
    unsafeAtomicAdd(&a.y64[i], (double)a.dinv[i] * (double)d);
  } else {  // OUT_SORTED_F64_SSL
    unsafeAtomicAdd(&a.y64[i], -(a.tau * (double)a.dinv[i] * (double)d));
  }
}

// d^{-1/2} from the corrected degrees (the formula of the degree pass).
__global__ __launch_bounds__(256) void k_near_dinv(const float *__restrict__ deg,
                                                   float *__restrict__ dinv, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float dg = deg[i];
    dinv[i] = dg > 0.f ? 1.0f / __builtin_sqrtf(dg) : 0.f;
  }
}

// Node coordinates relative to the item's tile origin, in grid cells: the
// integer cell difference exactly, plus the float fraction, rounded once
// (by at most 2^-19 of a cell while |coordinate| < 64 cells; candidate
// sources lie within R + 1 tiles of the origin).
__device__ __forceinline__ float3 rel_cells(const float4 &q, const int (&org)[3], int d) {
  const uint32_t c = __float_as_uint(q.w);
  float3 r;
  r.x = (float)((int)(c & 1023u) - org[0]) + q.x;
  r.y = d > 1 ? (float)((int)((c >> 10) & 1023u) - org[1]) + q.y : 0.f;
  r.z = d > 2 ? (float)((int)((c >> 20) & 1023u) - org[2]) + q.z : 0.f;
  return r;
}

// PC: number of polynomial coefficients evaluated (>= p; the ones past p are
// zero), a compile-time constant so that the coefficients stay in registers.
template <int IN, int OUT, int PC>
__global__ __launch_bounds__(NT) void k_near(const Item *__restrict__ items,
                                             const float4 *__restrict__ pts,
                                             const int *__restrict__ tile_start, KArgs ka, int d,
                                             int ntd, int tsize, int R, float eps_cells2,
                                             float kexp, float ku2,
                                             const float *__restrict__ coef, int p) {
  __shared__ float4 ssrc[NT];              // staged sources: tile-relative cells, value
  __shared__ int ns0[NF_MAXTILES];         // first node of each neighbour tile
  __shared__ int pref[NF_MAXTILES + 1];    // prefix sums of their node counts
  __shared__ int bsum[NT + 1];
  __shared__ float part[NT];
  if (stopped(ka.stop)) return;
  const int t = threadIdx.x;
  float cf[PC];
#pragma unroll
  for (int c = 0; c < PC; ++c) cf[c] = c < p ? coef[c] : 0.f;
  const Item it = items[blockIdx.x];
  int tc[3] = {0, 0, 0};
  {
    int r = it.tile;
    for (int a = d - 1; a >= 0; --a) {
      tc[a] = r % ntd;
      r /= ntd;
    }
  }
  const int org[3] = {tc[0] * tsize, tc[1] * tsize, tc[2] * tsize};
  // neighbour tiles: the (2R + 1)^d cube around the item's tile, without the
  // tiles whose nearest cell is farther than eps_I from the item's tile and
  // those outside the grid
  const int side = 2 * R + 1;
  const int nnb = d == 3 ? side * side * side : (d == 2 ? side * side : side);
  constexpr int PER = NF_MAXTILES / NT;    // tiles per thread in the scan
  int cnts[PER], run = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = t * PER + u;
    int a0 = 0, a1 = 0;
    if (q < nnb) {
      int o[3] = {0, 0, 0};
      int r = q;
      for (int a = d - 1; a >= 0; --a) {
        o[a] = r % side - R;
        r /= side;
      }
      int tt[3], gap2 = 0;
      bool in = true;
      for (int a = 0; a < 3; ++a) {
        tt[a] = tc[a] + o[a];
        if (a < d && (tt[a] < 0 || tt[a] >= ntd)) in = false;
        const int g = max(0, abs(o[a]) - 1) * tsize;
        gap2 += g * g;
      }
      if (in && (float)gap2 <= eps_cells2) {
        const int tile = d == 3 ? (tt[0] * ntd + tt[1]) * ntd + tt[2] : (d == 2 ? tt[0] * ntd + tt[1] : tt[0]);
        a0 = tile_start[tile];
        a1 = tile_start[tile + 1];
      }
      ns0[q] = a0;
    }
    cnts[u] = a1 - a0;
    run += a1 - a0;
  }
  // exclusive scan of the per-thread totals (Hillis-Steele over NT threads)
  bsum[t] = run;
  __syncthreads();
  for (int o = 1; o < NT; o <<= 1) {
    const int v = t >= o ? bsum[t - o] : 0;
    __syncthreads();
    bsum[t] += v;
    __syncthreads();
  }
  {
    int acc = bsum[t] - run;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = t * PER + u;
      if (q < nnb) pref[q] = acc;
      acc += cnts[u];
    }
    if (t == NT - 1) pref[nnb] = bsum[NT - 1];   // all nodes of the neighbour tiles
  }
  __syncthreads();
  const int total = pref[nnb];
  // Batches of targets: a full batch takes one target per thread; the last,
  // partial batch gives each of its rem targets G thread groups, group g
  // taking every G-th staged source, so that no batch leaves threads idle.
  for (int b0 = it.start; b0 < it.end;) {
    const int rem = it.end - b0;
    const int G = rem >= NT ? 1 : min(NT / rem, 32);
    const int TB = NT / G;
    const int ti = t % TB, gi = t / TB;
    const int i = b0 + ti;
    const bool act = gi < G && i < it.end;
    float3 tp3 = make_float3(0.f, 0.f, 0.f);
    if (act) tp3 = rel_cells(pts[i], org, d);
    float acc = 0.f;
    // the neighbour tiles' nodes as one list, staged NT at a time; slice
    // blockIdx.y of gridDim.y takes every gridDim.y-th chunk
    for (int c0 = blockIdx.y * NT; c0 < total; c0 += gridDim.y * NT) {
      const int cnt = min(NT, total - c0);
      __syncthreads();
      if (t < cnt) {
        const int v = c0 + t;
        int lo = 0, hi = nnb;   // the last q with pref[q] <= v
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (pref[mid] <= v) lo = mid;
          else hi = mid;
        }
        const int j = ns0[lo] + (v - pref[lo]);
        const float3 sr = rel_cells(pts[j], org, d);
        ssrc[t] = make_float4(sr.x, sr.y, sr.z, load_in<IN>(ka, j));
      }
      __syncthreads();
      if (act) {
        // branch-free: pairs past eps_I contribute an exact 0
#pragma unroll 4
        for (int k = gi; k < cnt; k += G) {
          const float4 sq = ssrc[k];
          const float dx = tp3.x - sq.x, dy = tp3.y - sq.y, dz = tp3.z - sq.z;
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          // K(r): hardware square root and exp2 (about 1 ulp each)
          const float e = __builtin_amdgcn_exp2f(__builtin_amdgcn_sqrtf(r2) * kexp);
          const float u2 = fminf(r2 * ku2, 1.f);   // (r / eps_I)^2, clamped: finite past eps_I
          float tp = cf[PC - 1];
#pragma unroll
          for (int c = PC - 2; c >= 0; --c) tp = fmaf(tp, u2, cf[c]);
          acc = fmaf(r2 <= eps_cells2 ? sq.w : 0.f, e - tp, acc);
        }
      }
    }
    // the groups' partial sums of each target, added in group order
    part[t] = acc;
    __syncthreads();
    if (gi == 0 && act) {
      float s = part[ti];
      for (int g = 1; g < G; ++g) s += part[g * TB + ti];
      if (s != 0.f) add_out<OUT>(ka, i, s);
    }
    __syncthreads();   // part is rewritten by the next batch of targets
    b0 += min(TB, rem);
  }
}

template <int IN, int OUT>
int launch_near(nfl_plan *P, const KArgs &k) {
  const int T = 1 << P->tshift;
  const double eps_cells = P->eps_I * P->nos;
  // a source within eps_I of a node of tile tc lies in a tile at most
  // ceil(eps_I / T) tiles away along every axis
  const int R = (int)std::ceil(eps_cells / T);
  int nnb = 1;
  for (int a = 0; a < P->d; ++a) nnb *= 2 * R + 1;
  if (nnb > NF_MAXTILES) {
    set_error("near field: eps_I spans too many tiles (raise the tile size or lower eps_I)");
    return NFL_ERR_UNSUPPORTED;
  }
  const int ntd = P->nos >> P->tshift;
  // slices per item: enough workgroups (~8192) to fill the chip when the
  // items are few and their neighbourhoods large
  const int slices = std::min(64, std::max(1, (8192 + P->nitems - 1) / P->nitems));
  // K(r) = 2^(r_cells * kexp), (r / eps_I)^2 = r_cells^2 * ku2 (r_cells in grid cells)
  const float kexp = (float)(-1.0 / (P->nos * P->sigma_t * std::log(2.0)));
  const float ku2 = (float)(1.0 / (eps_cells * eps_cells));
  auto kern = P->p <= 4   ? k_near<IN, OUT, 4>
              : P->p <= 6 ? k_near<IN, OUT, 6>
              : P->p <= 8 ? k_near<IN, OUT, 8>
                          : k_near<IN, OUT, NF_MAXP>;
  hipLaunchKernelGGL(kern, dim3(P->nitems, slices), dim3(NT), 0, P->stream, P->items.p, P->pts.p,
                     P->tile_start.p, k, P->d, ntd, T, R, (float)(eps_cells * eps_cells), kexp, ku2,
                     P->ti_coef.p, P->p);
  NFL_HIP(hipGetLastError());
  if constexpr (OUT == OUT_DEGREE) {
    const int nb = (int)std::min<int64_t>(4096, (P->n + 255) / 256);
    hipLaunchKernelGGL(k_near_dinv, dim3(nb), dim3(256), 0, P->stream, P->deg.p, P->dinv.p, P->n);
    NFL_HIP(hipGetLastError());
  }
  return NFL_OK;
}

}  // namespace

int near_field(nfl_plan *P, int in_mode, int out_mode, const VecArgs &a) {
  if (P->kind != NFL_KERNEL_LAPLACIAN_RBF || P->nitems == 0) return NFL_OK;
  if (P->p > NF_MAXP) {
    set_error("near field: p above 16 is not supported");
    return NFL_ERR_UNSUPPORTED;
  }
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
  k.xs = nullptr;
  if (in_mode == IN_USER_F32 && out_mode == OUT_USER_RAW) return launch_near<IN_USER_F32, OUT_USER_RAW>(P, k);
  if (in_mode == IN_USER_F32 && out_mode == OUT_USER_W) return launch_near<IN_USER_F32, OUT_USER_W>(P, k);
  if (in_mode == IN_USER_F32_DINV && out_mode == OUT_USER_LS) return launch_near<IN_USER_F32_DINV, OUT_USER_LS>(P, k);
  if (in_mode == IN_USER_F32_DINV && out_mode == OUT_USER_A) return launch_near<IN_USER_F32_DINV, OUT_USER_A>(P, k);
  if (in_mode == IN_ONES && out_mode == OUT_DEGREE) return launch_near<IN_ONES, OUT_DEGREE>(P, k);
  if (in_mode == IN_SORTED_F64_DINV && out_mode == OUT_SORTED_F64_A)
    return launch_near<IN_SORTED_F64_DINV, OUT_SORTED_F64_A>(P, k);
  if (in_mode == IN_SORTED_F64_DINV && out_mode == OUT_SORTED_F64_SSL)
    return launch_near<IN_SORTED_F64_DINV, OUT_SORTED_F64_SSL>(P, k);
  set_error("near field: this pair of input and output modes is not supported");
  return NFL_ERR_UNSUPPORTED;
}

}  // namespace nfl
