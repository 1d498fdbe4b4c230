// Many graphs, each with a block of vectors, through one captured launch
// sequence: y_{g,j} = L_s(g) x_{g,j} (Alg. nfft_normalized_matvec, step 5)
// for every graph g of the batch and every vector j of its block.
//
// A job is one (graph, vector) pair with its own grid and spectra.  Each
// stage of the fast summation (Alg. nfft_fastsum) is one kernel over the
// work of all jobs: the spread and interpolation kernels walk a flattened
// list of (job, item) pairs -- one launch per window width, since the width
// is a compile-time shape of the matrix-core loops -- and the FFT passes map
// each workgroup to a job by a search over per-job workgroup offsets.  The
// sequence (spreads, five FFT passes, interpolations) is captured once into a
// HIP graph; an apply is one graph launch.  Each job has two grids: the spread
// grid, which the r2c pass leaves zero for the next replay, and the grid the
// c2r pass writes and the interpolation reads.  The input
// and output base pointers live in a small device record that a one-thread
// kernel rewrites when they change, so the captured graph never changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "nfft_device.h"
#include "nfl_internal.h"

namespace nfl {

struct BJob {
  const float4 *pts;
  const Item *items;
  const int *perm;
  const float *dinv;
  const float *wcoef;
  const float *filt;
  const float2 *tw;
  float *grid;    // spread output, left zero by the r2c pass
  float *grid2;   // c2r output, interpolation input
  float2 *spec1;
  float2 *spec2;
  int64_t xoff;   // offset of this job's vector in the packed x / y
  int nos, N, tshift, logL;
  int lpz, lpy, lpx, pad;   // FFT lines per workgroup: z (real lines), y and x passes
  // the plan's z-line support (null: every line): lines, x-slabs, flags
  const int *zl;
  const int *zx;
  const uint8_t *zmap;
  int nzl, nzx;
};

struct BItem {
  int job;
  int item;
};

struct BIO {
  const float *x;
  float *y;
};

__global__ void k_batch_set_io(BIO *io, const float *x, float *y) {
  io->x = x;
  io->y = y;
}

// Items of at most SHORT_ITEM nodes run on one-wave workgroups (NW = 1):
// a quarter of the LDS of the four-wave form, so several times more of these
// short items are in flight per compute unit, and one private tile to clear
// and flush instead of four.
constexpr int SHORT_ITEM = 128;

template <int W, bool ZM, int NW>
__global__ __launch_bounds__(64 * NW) void kb_spread(const BItem *__restrict__ list,
                                                     const BJob *__restrict__ jobs,
                                                     const BIO *__restrict__ io) {
  const BItem b = list[blockIdx.x];
  const BJob &J = jobs[b.job];
  KArgs ka{};
  ka.x32 = io->x + J.xoff;
  ka.perm = J.perm;
  ka.dinv = J.dinv;
  spread3_mfma_body<W, IN_USER_F32_DINV, ZM, NW>(J.items[b.item], J.pts, ka, J.grid, J.nos,
                                                 J.tshift, J.wcoef);
}

template <int W, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(W <= 8 ? 5 : 1)))
void kb_interp(const BItem *__restrict__ list, const BJob *__restrict__ jobs,
               const BIO *__restrict__ io) {
  const BItem b = list[blockIdx.x];
  const BJob &J = jobs[b.job];
  KArgs ka{};
  ka.x32 = io->x + J.xoff;
  ka.y32 = io->y + J.xoff;
  ka.perm = J.perm;
  ka.dinv = J.dinv;
  interp3_mfma_body<W, IN_USER_F32_DINV, OUT_USER_LS, NW>(J.items, b.item, J.pts, ka, J.grid2,
                                                          J.nos, J.tshift, J.wcoef);
}

// the tile-stationary kernels run three waves per SIMD, as the single-plan ones
template <int W, int T, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) void kb_spread_tile(const BItem *__restrict__ list,
                                                          const BJob *__restrict__ jobs,
                                                          const BIO *__restrict__ io) {
  const BItem b = list[blockIdx.x];
  const BJob &J = jobs[b.job];
  KArgs ka{};
  ka.x32 = io->x + J.xoff;
  ka.perm = J.perm;
  ka.dinv = J.dinv;
  spread3_tile_body<W, T, IN_USER_F32_DINV, NW>(J.items[b.item], J.pts, ka, J.grid, J.nos,
                                                J.wcoef);
}

template <int W, int T, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) void kb_interp_tile(const BItem *__restrict__ list,
                                                          const BJob *__restrict__ jobs,
                                                          const BIO *__restrict__ io) {
  const BItem b = list[blockIdx.x];
  const BJob &J = jobs[b.job];
  KArgs ka{};
  ka.x32 = io->x + J.xoff;
  ka.y32 = io->y + J.xoff;
  ka.perm = J.perm;
  ka.dinv = J.dinv;
  interp3_tile_body<W, T, IN_USER_F32_DINV, OUT_USER_LS, NW>(J.items, b.item, J.pts, ka, J.grid2,
                                                             J.nos, J.wcoef);
}

// Job of workgroup `blk`: the largest j with first[j] <= blk (first[0] = 0).
__device__ __forceinline__ int find_job(const int *__restrict__ first, int njobs, int blk) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int f = __builtin_amdgcn_readfirstlane(first[mid]);
    if (f <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

enum { FFT_R2C = 0, FFT_YF = 1, FFT_XF = 2, FFT_YI = 3, FFT_C2R = 4, FFT_STAGES = 5 };

// Workgroups one job needs in each FFT pass.  As the single-plan convolution,
// except for the x pass: with many jobs in flight, its workgroups take full
// FFT_ELEMS / L columns instead of splitting one grid finely.
static int fft_blocks(int stage, int L, int N, int nzl, int nzx) {
  const int Hz = N / 2 + 1, F = N + 1;
  switch (stage) {
    case FFT_R2C:
    case FFT_C2R: return (nzl + fft_lpb_zr(L) - 1) / fft_lpb_zr(L);
    case FFT_YF:
    case FFT_YI: return nzx * ((Hz + fft_lpb_y(L) - 1) / fft_lpb_y(L));
    default: return (F * Hz + fft_lpb_z(L) - 1) / fft_lpb_z(L);
  }
}

template <int STAGE>
__global__ __launch_bounds__(FFT_THREADS) void kb_fft(const int *__restrict__ first, int njobs,
                                                      const BJob *__restrict__ jobs) {
  // the column passes take their blocks XCD-contiguous, as in the single-plan FFT
  const int blk = (STAGE == FFT_YF || STAGE == FFT_XF || STAGE == FFT_YI)
                      ? xcd_block(blockIdx.x, gridDim.x)
                      : (int)blockIdx.x;
  const int j = find_job(first, njobs, blk);
  const BJob &J = jobs[j];
  const int lb = blk - __builtin_amdgcn_readfirstlane(first[j]);
  const int L = J.nos, N = J.N, Hz = N / 2 + 1;
  // passes on the plan's z-line support (the spectra are zero off it)
  if constexpr (STAGE == FFT_R2C)
    r2c_lines_body<true>(lb, J.grid, J.spec1, J.nzl, L, J.logL, J.lpz, Hz, J.tw, nullptr, 0.f, J.zl);
  else if constexpr (STAGE == FFT_YF)
    y_fwd_body(lb, J.spec1, J.spec2, L, J.logL, J.lpy, Hz, N, J.tw, J.zx);
  else if constexpr (STAGE == FFT_XF)
    x_filter_body(lb, J.spec2, J.filt, (N + 1) * Hz, L, J.logL, J.lpx, N, J.tw,
                  J.zmap ? J.zmap + (size_t)L * L : nullptr);
  else if constexpr (STAGE == FFT_YI)
    y_inv_body(lb, J.spec2, J.spec1, L, J.logL, J.lpy, Hz, N, J.tw, J.zx, J.zmap);
  else
    c2r_lines_body(lb, J.spec1, J.grid2, J.nzl, L, J.logL, J.lpz, Hz, J.tw, J.zl);
}

// The spread or interpolation launches of all jobs of one window width W and
// kernel form (per-cell runs, z-merged per-cell runs, or tile-stationary with
// tile T): [0] four-wave workgroups, [1] one-wave workgroups for short items.
enum { FORM_RUNS = 0, FORM_ZMERGE = 1, FORM_TILE4 = 4, FORM_TILE8 = 8 };
struct BGroup {
  int W = 0;
  int form = FORM_RUNS;
  int begin[2] = {0, 0}, count[2] = {0, 0};   // ranges in the item list
  size_t lds_spread[2] = {0, 0}, lds_interp[2] = {0, 0};
};

static int kernel_form(int W, int T) {
  if (T + W - 1 <= 16 && (T == 4 || T == 8)) return T == 4 ? FORM_TILE4 : FORM_TILE8;
  return (W >= 9 && T + W - 1 <= 16) ? FORM_ZMERGE : FORM_RUNS;
}

template <class K>
static int set_max_lds(K kern, size_t lds) {
  if (lds > 65536)
    NFL_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
  return NFL_OK;
}

template <int W, int NW>
static int launch_group_wn(const BGroup &g, int v, const BItem *list, const BJob *jobs,
                           const BIO *io, hipStream_t s, bool spread_pass, bool prepare) {
  if (!prepare && g.count[v] == 0) return NFL_OK;
  if constexpr (W + 3 <= 16) {
    if (g.form == FORM_TILE4) {
      if (spread_pass) {
        if (prepare) return set_max_lds(kb_spread_tile<W, 4, NW>, g.lds_spread[v]);
        hipLaunchKernelGGL((kb_spread_tile<W, 4, NW>), dim3(g.count[v]), dim3(64 * NW),
                           g.lds_spread[v], s, list + g.begin[v], jobs, io);
      } else {
        if (prepare) return set_max_lds(kb_interp_tile<W, 4, NW>, g.lds_interp[v]);
        hipLaunchKernelGGL((kb_interp_tile<W, 4, NW>), dim3(g.count[v]), dim3(64 * NW),
                           g.lds_interp[v], s, list + g.begin[v], jobs, io);
      }
      NFL_HIP(hipGetLastError());
      return NFL_OK;
    }
  }
  if constexpr (W + 7 <= 16) {
    if (g.form == FORM_TILE8) {
      if (spread_pass) {
        if (prepare) return set_max_lds(kb_spread_tile<W, 8, NW>, g.lds_spread[v]);
        hipLaunchKernelGGL((kb_spread_tile<W, 8, NW>), dim3(g.count[v]), dim3(64 * NW),
                           g.lds_spread[v], s, list + g.begin[v], jobs, io);
      } else {
        if (prepare) return set_max_lds(kb_interp_tile<W, 8, NW>, g.lds_interp[v]);
        hipLaunchKernelGGL((kb_interp_tile<W, 8, NW>), dim3(g.count[v]), dim3(64 * NW),
                           g.lds_interp[v], s, list + g.begin[v], jobs, io);
      }
      NFL_HIP(hipGetLastError());
      return NFL_OK;
    }
  }
  if (spread_pass) {
    if constexpr (W >= 9) {
      if (g.form == FORM_ZMERGE) {
        if (prepare) return set_max_lds(kb_spread<W, true, NW>, g.lds_spread[v]);
        hipLaunchKernelGGL((kb_spread<W, true, NW>), dim3(g.count[v]), dim3(64 * NW),
                           g.lds_spread[v], s, list + g.begin[v], jobs, io);
        NFL_HIP(hipGetLastError());
        return NFL_OK;
      }
    }
    if (prepare) return set_max_lds(kb_spread<W, false, NW>, g.lds_spread[v]);
    hipLaunchKernelGGL((kb_spread<W, false, NW>), dim3(g.count[v]), dim3(64 * NW),
                       g.lds_spread[v], s, list + g.begin[v], jobs, io);
  } else {
    if (prepare) return set_max_lds(kb_interp<W, NW>, g.lds_interp[v]);
    hipLaunchKernelGGL((kb_interp<W, NW>), dim3(g.count[v]), dim3(64 * NW), g.lds_interp[v], s,
                       list + g.begin[v], jobs, io);
  }
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

template <int W>
static int launch_group_w(const BGroup &g, const BItem *list, const BJob *jobs, const BIO *io,
                          hipStream_t s, bool spread_pass, bool prepare) {
  const int rc = launch_group_wn<W, 4>(g, 0, list, jobs, io, s, spread_pass, prepare);
  if (rc < 0) return rc;
  return launch_group_wn<W, 1>(g, 1, list, jobs, io, s, spread_pass, prepare);
}

static int launch_group(const BGroup &g, const BItem *list, const BJob *jobs, const BIO *io,
                        hipStream_t s, bool spread_pass, bool prepare = false) {
  switch (g.W) {
    case 4: return launch_group_w<4>(g, list, jobs, io, s, spread_pass, prepare);
    case 6: return launch_group_w<6>(g, list, jobs, io, s, spread_pass, prepare);
    case 8: return launch_group_w<8>(g, list, jobs, io, s, spread_pass, prepare);
    case 10: return launch_group_w<10>(g, list, jobs, io, s, spread_pass, prepare);
    case 12: return launch_group_w<12>(g, list, jobs, io, s, spread_pass, prepare);
    case 14: return launch_group_w<14>(g, list, jobs, io, s, spread_pass, prepare);
    case 16: return launch_group_w<16>(g, list, jobs, io, s, spread_pass, prepare);
    default: set_error("batch: window width out of range"); return NFL_ERR_UNSUPPORTED;
  }
}

template <int STAGE>
static int launch_fft(const int *first, int njobs, int nblocks, const BJob *jobs, hipStream_t s) {
  constexpr size_t lds = ((size_t)2 * FFT_ELEMS + FFT_MAXL) * sizeof(float2);
  hipLaunchKernelGGL((kb_fft<STAGE>), dim3(nblocks), dim3(FFT_THREADS), lds, s, first, njobs,
                     jobs);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

}  // namespace nfl

using namespace nfl;

struct nfl_batch_s {
  int device = 0;
  hipStream_t stream = nullptr;   // caller's stream: graph launches
  hipStream_t cap = nullptr;      // library stream used only to record the graph
  int nvec = 0;
  std::vector<nfl_plan *> plans;
  std::vector<uint64_t> gens;
  std::vector<int64_t> off;       // node offsets, nplans + 1
  int njobs = 0;
  std::vector<BGroup> groups;
  int fft_nblocks[FFT_STAGES] = {0, 0, 0, 0, 0};
  DBuf<BJob> jobs;
  DBuf<BItem> list;
  DBuf<int> first;                // FFT_STAGES x (njobs + 1)
  DBuf<BIO> io;
  DBuf<float> grids;
  DBuf<float2> spec1, spec2;
  int64_t grid_elems = 0;
  int64_t arena_bytes = 0;
  int nkernels = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const float *last_x = nullptr;
  float *last_y = nullptr;
};

namespace nfl {

// The launch sequence of one batched product, enqueued on stream s.
static int batch_sequence(nfl_batch_s *B, hipStream_t s) {
  for (const BGroup &g : B->groups)
    NFL_TRY(launch_group(g, B->list.p, B->jobs.p, B->io.p, s, true));
  const int nj = B->njobs;
  const int *f = B->first.p;
  NFL_TRY(launch_fft<FFT_R2C>(f + 0 * (nj + 1), nj, B->fft_nblocks[FFT_R2C], B->jobs.p, s));
  NFL_TRY(launch_fft<FFT_YF>(f + 1 * (nj + 1), nj, B->fft_nblocks[FFT_YF], B->jobs.p, s));
  NFL_TRY(launch_fft<FFT_XF>(f + 2 * (nj + 1), nj, B->fft_nblocks[FFT_XF], B->jobs.p, s));
  NFL_TRY(launch_fft<FFT_YI>(f + 3 * (nj + 1), nj, B->fft_nblocks[FFT_YI], B->jobs.p, s));
  NFL_TRY(launch_fft<FFT_C2R>(f + 4 * (nj + 1), nj, B->fft_nblocks[FFT_C2R], B->jobs.p, s));
  for (const BGroup &g : B->groups)
    NFL_TRY(launch_group(g, B->list.p, B->jobs.p, B->io.p, s, false));
  return NFL_OK;
}

static void batch_release(nfl_batch_s *B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  B->jobs.release();
  B->list.release();
  B->first.release();
  B->io.release();
  B->grids.release();
  B->spec1.release();
  B->spec2.release();
}

static int batch_build(nfl_batch_s *B) {
  const int np = (int)B->plans.size(), nv = B->nvec;
  B->off.assign(np + 1, 0);
  for (int g = 0; g < np; ++g) B->off[g + 1] = B->off[g] + B->plans[g]->n;

  // per-job descriptors; arena offsets
  B->njobs = np * nv;
  std::vector<BJob> hj((size_t)B->njobs);
  int64_t gsum = 0, s1sum = 0, s2sum = 0;
  std::vector<int64_t> goff(B->njobs), s1off(B->njobs), s2off(B->njobs);
  for (int g = 0; g < np; ++g) {
    const nfl_plan *P = B->plans[g];
    const int L = P->nos, N = P->N, Hz = N / 2 + 1, F = N + 1;
    for (int j = 0; j < nv; ++j) {
      const int q = g * nv + j;
      goff[q] = gsum;
      s1off[q] = s1sum;
      s2off[q] = s2sum;
      gsum += (int64_t)L * L * L;
      s1sum += (int64_t)L * L * Hz;
      s2sum += (int64_t)L * F * Hz;
    }
  }
  NFL_TRY(B->grids.ensure((size_t)2 * gsum));
  NFL_TRY(B->spec1.ensure((size_t)s1sum));
  NFL_TRY(B->spec2.ensure((size_t)s2sum));
  B->grid_elems = gsum;
  B->arena_bytes = 2 * gsum * 4 + (s1sum + s2sum) * 8;
  // the spread grids start clear; every replay leaves them clear again.  The
  // spectra are zero off each plan's z-line support, which no pass writes.
  NFL_TRY(fill_f32(B->grids.p, gsum, 0.f, B->stream));
  NFL_TRY(fill_f32(reinterpret_cast<float *>(B->spec1.p), 2 * s1sum, 0.f, B->stream));
  NFL_TRY(fill_f32(reinterpret_cast<float *>(B->spec2.p), 2 * s2sum, 0.f, B->stream));
  NFL_HIP(hipStreamSynchronize(B->stream));

  for (int g = 0; g < np; ++g) {
    const nfl_plan *P = B->plans[g];
    int logL = 0;
    while ((1 << logL) < P->nos) ++logL;
    for (int j = 0; j < nv; ++j) {
      const int q = g * nv + j;
      BJob &J = hj[q];
      std::memset(&J, 0, sizeof(J));
      J.pts = P->pts.p;
      J.items = P->items.p;
      J.perm = P->perm.p;
      J.dinv = P->dinv.p;
      J.wcoef = P->wcoef.p;
      J.filt = P->filt.p;
      J.tw = P->tw.p;
      J.grid = B->grids.p + goff[q];
      J.grid2 = B->grids.p + gsum + goff[q];
      J.spec1 = B->spec1.p + s1off[q];
      J.spec2 = B->spec2.p + s2off[q];
      J.xoff = (int64_t)nv * B->off[g] + (int64_t)j * P->n;
      J.nos = P->nos;
      J.N = P->N;
      J.tshift = P->tshift;
      J.logL = logL;
      J.lpz = fft_lpb_zr(P->nos);
      J.lpy = fft_lpb_y(P->nos);
      J.lpx = fft_lpb_z(P->nos);
      const bool sup = P->zs_nlines > 0;
      J.zl = sup ? P->zs_lines.p : nullptr;
      J.zx = sup ? P->zs_x.p : nullptr;
      J.zmap = sup ? P->zs_map.p : nullptr;
      J.nzl = sup ? P->zs_nlines : P->nos * P->nos;
      J.nzx = sup ? P->zs_nx : P->nos;
    }
  }

  // spread / interpolation groups: jobs of equal window width and z-merge
  // mode; inside a group the items run longest first
  struct Key {
    int W;
    int form;
  };
  std::vector<Key> keys;
  std::vector<std::vector<BItem>> glists;
  std::vector<std::vector<int>> glens;
  for (int g = 0; g < np; ++g) {
    nfl_plan *P = B->plans[g];
    std::vector<Item> its((size_t)P->nitems);
    NFL_HIP(hipMemcpy(its.data(), P->items.p, its.size() * sizeof(Item), hipMemcpyDeviceToHost));
    const int W = 2 * P->m;
    const int form = kernel_form(W, 1 << P->tshift);
    size_t k = 0;
    while (k < keys.size() && !(keys[k].W == W && keys[k].form == form)) ++k;
    if (k == keys.size()) {
      keys.push_back({W, form});
      glists.emplace_back();
      glens.emplace_back();
      B->groups.emplace_back();
      B->groups.back().W = W;
      B->groups.back().form = form;
    }
    const int Pd = (1 << P->tshift) + W - 1;
    const size_t p3 = (size_t)tile_px(Pd) * Pd;
    for (int v = 0; v < 2; ++v) {
      const size_t nw = v == 0 ? 4 : 1;
      size_t ls = (nw * p3 + nw * 16 * WT_SPREAD) * sizeof(float);
      size_t li = (p3 + nw * 16 * WT_INTERP) * sizeof(float);
      if (form == FORM_TILE4 || form == FORM_TILE8) {
        const size_t tile = (size_t)Pd * ts_xs(Pd);
        // the spread's tables, coefficient table and tile copies
        ls = (size_t)spread_tile_lds_floats(Pd, (int)nw) * sizeof(float);
        // + the window coefficient table the tile forms keep after the weight tables
        li = (tile + nw * 16 * TS_PITCH_I + WIN_MAXW * WIN_NC) * sizeof(float);
      }
      B->groups[k].lds_spread[v] = std::max(B->groups[k].lds_spread[v], ls);
      B->groups[k].lds_interp[v] = std::max(B->groups[k].lds_interp[v], li);
    }
    for (int j = 0; j < nv; ++j)
      for (int t = 0; t < P->nitems; ++t) {
        glists[k].push_back({g * nv + j, t});
        glens[k].push_back(its[t].end - its[t].start);
      }
  }
  std::vector<BItem> all;
  for (size_t k = 0; k < keys.size(); ++k) {
    std::vector<int> ord(glists[k].size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int a, int b) { return glens[k][a] > glens[k][b]; });
    // longest first; the short tail goes to the one-wave launch
    size_t nlong = 0;
    while (nlong < ord.size() && glens[k][ord[nlong]] > SHORT_ITEM) ++nlong;
    B->groups[k].begin[0] = (int)all.size();
    B->groups[k].count[0] = (int)nlong;
    B->groups[k].begin[1] = (int)(all.size() + nlong);
    B->groups[k].count[1] = (int)(ord.size() - nlong);
    for (int i : ord) all.push_back(glists[k][i]);
  }
  if (all.size() > (size_t)0x7fffffff) { set_error("batch: too many work items"); return NFL_ERR_UNSUPPORTED; }

  // FFT workgroup offsets per stage
  std::vector<int> hf((size_t)FFT_STAGES * (B->njobs + 1));
  for (int st = 0; st < FFT_STAGES; ++st) {
    int64_t acc = 0;
    for (int q = 0; q < B->njobs; ++q) {
      hf[(size_t)st * (B->njobs + 1) + q] = (int)acc;
      acc += fft_blocks(st, hj[q].nos, hj[q].N, hj[q].nzl, hj[q].nzx);
    }
    if (acc > 0x7fffffff) { set_error("batch: FFT grid too large"); return NFL_ERR_UNSUPPORTED; }
    hf[(size_t)st * (B->njobs + 1) + B->njobs] = (int)acc;
    B->fft_nblocks[st] = (int)acc;
  }

  NFL_TRY(B->jobs.ensure(hj.size()));
  NFL_TRY(B->list.ensure(all.size()));
  NFL_TRY(B->first.ensure(hf.size()));
  NFL_TRY(B->io.ensure(1));
  NFL_HIP(hipMemcpy(B->jobs.p, hj.data(), hj.size() * sizeof(BJob), hipMemcpyHostToDevice));
  NFL_HIP(hipMemcpy(B->list.p, all.data(), all.size() * sizeof(BItem), hipMemcpyHostToDevice));
  NFL_HIP(hipMemcpy(B->first.p, hf.data(), hf.size() * sizeof(int), hipMemcpyHostToDevice));
  const BIO zero{nullptr, nullptr};
  NFL_HIP(hipMemcpy(B->io.p, &zero, sizeof(BIO), hipMemcpyHostToDevice));

  // kernel attributes are set before capture
  for (const BGroup &g : B->groups) {
    NFL_TRY(launch_group(g, nullptr, nullptr, nullptr, nullptr, true, true));
    NFL_TRY(launch_group(g, nullptr, nullptr, nullptr, nullptr, false, true));
  }
  B->nkernels = FFT_STAGES;
  for (const BGroup &g : B->groups) B->nkernels += 2 * ((g.count[0] > 0) + (g.count[1] > 0));

  // record the sequence once
  NFL_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
  NFL_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
  const int rc = batch_sequence(B, B->cap);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(B->cap, &gr);
  if (rc < 0) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  NFL_HIP(e);
  B->graph = gr;
  NFL_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  return NFL_OK;
}

}  // namespace nfl

extern "C" {

int nfl_batch_create(nfl_batch *b, const nfl_handle *plans, int nplans, int nvec,
                     void *hip_stream) {
  if (!b) { set_error("null batch pointer"); return NFL_ERR_ARG; }
  *b = nullptr;
  if (!plans || nplans < 1) { set_error("need at least one plan"); return NFL_ERR_ARG; }
  if (nvec < 1 || nvec > 64) { set_error("nvec must be in [1, 64]"); return NFL_ERR_ARG; }
  int dev = 0;
  NFL_HIP(hipGetDevice(&dev));
  for (int g = 0; g < nplans; ++g) {
    const nfl_plan *P = plans[g];
    if (!P) { set_error("null plan in batch"); return NFL_ERR_ARG; }
    if (!P->have_kernel) { set_error("batch: plan without a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
    if (P->frame_only) { set_error("batch: plan of target nodes"); return NFL_ERR_ORDER; }
    if (P->kind == NFL_KERNEL_LAPLACIAN_RBF) { set_error("batch: the Laplacian RBF kernel's near-field sum is not part of the batched launch"); return NFL_ERR_UNSUPPORTED; }
    if (P->d != 3) { set_error("batch: plans must have d = 3"); return NFL_ERR_UNSUPPORTED; }
    if (P->opt_kernel != 0) { set_error("batch: plans must use the matrix-core kernels"); return NFL_ERR_UNSUPPORTED; }
    if (P->prec != 32) { set_error("batch: plans must use the FP32 path"); return NFL_ERR_UNSUPPORTED; }
    if (P->device != dev) { set_error("batch: plans on another device"); return NFL_ERR_ARG; }
    if (P->nos > FFT_MAXL) { set_error("batch: grid too large"); return NFL_ERR_UNSUPPORTED; }
  }
  nfl_batch_s *B = new (std::nothrow) nfl_batch_s();
  if (!B) { set_error("host allocation failed"); return NFL_ERR_OOM; }
  B->device = dev;
  B->stream = (hipStream_t)hip_stream;
  B->nvec = nvec;
  B->plans.assign(plans, plans + nplans);
  for (const nfl_plan *P : B->plans) B->gens.push_back(P->gen);
  // the plans' setup work must be complete before their buffers are read
  for (const nfl_plan *P : B->plans) {
    if (hipStreamSynchronize(P->stream) != hipSuccess) {
      set_error("batch: plan stream failed");
      delete B;
      return NFL_ERR_HIP;
    }
  }
  const int rc = batch_build(B);
  if (rc < 0) {
    batch_release(B);
    delete B;
    return rc;
  }
  *b = B;
  return NFL_OK;
}

int nfl_batch_offsets(nfl_batch b, int64_t *offsets_host, int64_t count) {
  if (!b) { set_error("null batch"); return NFL_ERR_ARG; }
  if (!offsets_host || count < (int64_t)b->off.size()) { set_error("offsets: count < nplans + 1"); return NFL_ERR_ARG; }
  for (size_t g = 0; g < b->off.size(); ++g) offsets_host[g] = b->off[g];
  return NFL_OK;
}

int nfl_batch_info(nfl_batch b, int64_t *total_n, int *njobs, int *nkernels,
                   int64_t *arena_bytes) {
  if (!b) { set_error("null batch"); return NFL_ERR_ARG; }
  if (total_n) *total_n = b->off.back();
  if (njobs) *njobs = b->njobs;
  if (nkernels) *nkernels = b->nkernels;
  if (arena_bytes) *arena_bytes = b->arena_bytes;
  return NFL_OK;
}

int nfl_batch_apply_Ls(nfl_batch b, const float *x_dev, float *y_dev) {
  if (!b) { set_error("null batch"); return NFL_ERR_ARG; }
  if (!x_dev || !y_dev) { set_error("null vector pointer"); return NFL_ERR_ARG; }
  for (size_t g = 0; g < b->plans.size(); ++g)
    if (b->plans[g]->gen != b->gens[g] || !b->plans[g]->have_kernel) {
      set_error("batch: a plan changed after nfl_batch_create");
      return NFL_ERR_ORDER;
    }
  if (x_dev != b->last_x || y_dev != b->last_y) {
    hipLaunchKernelGGL(k_batch_set_io, dim3(1), dim3(1), 0, b->stream, b->io.p, x_dev, y_dev);
    NFL_HIP(hipGetLastError());
    b->last_x = x_dev;
    b->last_y = y_dev;
  }
  NFL_HIP(hipGraphLaunch(b->exec, b->stream));
  return NFL_OK;
}

int nfl_batch_destroy(nfl_batch b) {
  if (!b) return NFL_OK;
  (void)hipStreamSynchronize(b->stream);
  batch_release(b);
  delete b;
  return NFL_OK;
}

}  // extern "C"
