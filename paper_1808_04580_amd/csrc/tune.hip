// Parameter choice for the NFFT fast summation (the paper fixes N, m, eps_B
// and p by hand, Section 3.2; here they are searched per graph).
//
// Accuracy is judged against the exact sums on sampled rows, computed on the
// GPU by a direct FP64 kernel over all n points: for a row j,
//   (W x)_j = sum_{i != j} exp(-||v_j - v_i||^2 / sigma^2) x_i   (Section 2),
//   d_j     = sum_{i != j} exp(-||v_j - v_i||^2 / sigma^2).
// The error of a configuration is max(rel_inf(d), rel_inf(W x)) over the
// sampled rows, x uniform in [-1, 1).  The search:
//   1. kernel approximation: for eps_B in {0, 1/16, 1/8} the smallest
//      power-of-2 N whose error at the widest window (m = min(8, N/2)) is
//      below 0.3 x target; the smallest such N wins;
//   2. window: the smallest m at that N and eps_B with error <= 0.7 x target;
//   3. tile: the fastest of T = 4, 8, 16 (d = 3), timed as a captured HIP
//      graph of products (GPU time, without host launch overhead).
// Results are kept in a text cache keyed by (d, size class of n, band of
// sigma~, target).  A cached configuration is verified on the graph at hand
// with the same probe and tuned afresh if it misses the target.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "nfl_internal.h"

namespace nfl {

constexpr int DIRECT_THREADS = 256;
constexpr int64_t DIRECT_CHUNK = 32768;

__global__ __launch_bounds__(DIRECT_THREADS) void k_direct_rows(
    const float *__restrict__ v, int64_t n, int d, const float *__restrict__ x,
    const int64_t *__restrict__ rows, double inv_s2, int nchunks, double *__restrict__ part) {
  __shared__ double sh[2][DIRECT_THREADS];
  const int r = blockIdx.y, c = blockIdx.x;
  const int64_t j = rows[r];
  double vj[3] = {0.0, 0.0, 0.0};
  for (int t = 0; t < d; ++t) vj[t] = (double)v[j * d + t];
  double sd = 0.0, sw = 0.0;
  const int64_t i0 = (int64_t)c * DIRECT_CHUNK;
  const int64_t i1 = i0 + DIRECT_CHUNK < n ? i0 + DIRECT_CHUNK : n;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += DIRECT_THREADS) {
    if (i == j) continue;
    double r2 = 0.0;
    for (int t = 0; t < d; ++t) {
      const double df = (double)v[i * d + t] - vj[t];
      r2 += df * df;
    }
    const double k = exp(-r2 * inv_s2);
    sd += k;
    if (x) sw += k * (double)x[i];
  }
  sh[0][threadIdx.x] = sd;
  sh[1][threadIdx.x] = sw;
  __syncthreads();
  for (int s = DIRECT_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)r * nchunks + c) * 2 + 0] = sh[0][0];
    part[((size_t)r * nchunks + c) * 2 + 1] = sh[1][0];
  }
}

__global__ void k_gather_rows(const float *__restrict__ a, const float *__restrict__ b,
                              const int64_t *__restrict__ rows, int S, float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S) {
    out[i] = a[rows[i]];
    out[S + i] = b[rows[i]];
  }
}

// Exact W x and d on the given rows (user order); x may be null.
static int direct_rows(nfl_plan *P, double sigma, const float *x_dev, const int64_t *rows_host,
                       int S, double *wx, double *deg) {
  DBuf<int64_t> rows;
  DBuf<double> part;
  const int nchunks = (int)((P->n + DIRECT_CHUNK - 1) / DIRECT_CHUNK);
  NFL_TRY(rows.ensure(S));
  int rc = part.ensure((size_t)S * nchunks * 2);
  if (rc < 0) { rows.release(); return rc; }
  std::vector<double> hp((size_t)S * nchunks * 2);
  hipError_t e = hipMemcpyAsync(rows.p, rows_host, (size_t)S * sizeof(int64_t),
                                hipMemcpyHostToDevice, P->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_direct_rows, dim3(nchunks, S), dim3(DIRECT_THREADS), 0, P->stream,
                       P->pts_user.p, P->n, P->d, x_dev, rows.p, 1.0 / (sigma * sigma), nchunks,
                       part.p);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(hp.data(), part.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost,
                       P->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
  rows.release();
  part.release();
  if (e != hipSuccess) {
    set_error(std::string("direct rows: ") + hipGetErrorString(e));
    return NFL_ERR_HIP;
  }
  for (int r = 0; r < S; ++r) {
    double sd = 0.0, sw = 0.0;
    for (int c = 0; c < nchunks; ++c) {
      sd += hp[((size_t)r * nchunks + c) * 2 + 0];
      sw += hp[((size_t)r * nchunks + c) * 2 + 1];
    }
    if (deg) deg[r] = sd;
    if (wx) wx[r] = sw;
  }
  return NFL_OK;
}

static uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

struct Probe {
  int S = 0;
  std::vector<int64_t> rows;
  std::vector<double> refW, refd;
  DBuf<int64_t> rows_dev;
  DBuf<float> x, y, t, g;
  void release() {
    rows_dev.release();
    x.release();
    y.release();
    t.release();
    g.release();
  }
};

static int probe_init(nfl_plan *P, double sigma, int S, uint64_t seed, Probe &pr) {
  const int64_t n = P->n;
  S = (int)std::min<int64_t>(S, n);
  pr.S = S;
  // S distinct rows: a seeded partial shuffle for small n, rejection otherwise
  uint64_t st = seed;
  if (n <= 4 * (int64_t)S) {
    std::vector<int64_t> all((size_t)n);
    for (int64_t i = 0; i < n; ++i) all[i] = i;
    for (int k = 0; k < S; ++k) {
      const int64_t r = k + (int64_t)(splitmix(st) % (uint64_t)(n - k));
      std::swap(all[k], all[r]);
    }
    pr.rows.assign(all.begin(), all.begin() + S);
  } else {
    std::vector<char> used((size_t)n, 0);
    while ((int)pr.rows.size() < S) {
      const int64_t r = (int64_t)(splitmix(st) % (uint64_t)n);
      if (!used[r]) {
        used[r] = 1;
        pr.rows.push_back(r);
      }
    }
  }
  std::sort(pr.rows.begin(), pr.rows.end());
  std::vector<float> hx((size_t)n);
  for (int64_t i = 0; i < n; ++i)
    hx[i] = (float)((double)(splitmix(st) >> 11) * (2.0 / 9007199254740992.0) - 1.0);
  NFL_TRY(pr.x.ensure(n));
  NFL_TRY(pr.y.ensure(n));
  NFL_TRY(pr.t.ensure(n));
  NFL_TRY(pr.g.ensure((size_t)2 * S));
  NFL_TRY(pr.rows_dev.ensure(S));
  NFL_HIP(hipMemcpyAsync(pr.x.p, hx.data(), (size_t)n * sizeof(float), hipMemcpyHostToDevice,
                         P->stream));
  NFL_HIP(hipMemcpyAsync(pr.rows_dev.p, pr.rows.data(), (size_t)S * sizeof(int64_t),
                         hipMemcpyHostToDevice, P->stream));
  pr.refW.resize(S);
  pr.refd.resize(S);
  return direct_rows(P, sigma, pr.x.p, pr.rows.data(), S, pr.refW.data(), pr.refd.data());
}

// max(rel_inf(d), rel_inf(W x)) of the plan's current configuration.
static int probe_error(nfl_plan *P, Probe &pr, double *err) {
  VecArgs a;
  a.x32 = pr.x.p;
  a.y32 = pr.y.p;
  NFL_TRY(fastsum(P, IN_USER_F32, OUT_USER_W, a));
  NFL_TRY(scatter_f32(P, P->deg.p, pr.t.p));
  hipLaunchKernelGGL(k_gather_rows, dim3((pr.S + 255) / 256), dim3(256), 0, P->stream, pr.y.p,
                     pr.t.p, pr.rows_dev.p, pr.S, pr.g.p);
  NFL_HIP(hipGetLastError());
  std::vector<float> h((size_t)2 * pr.S);
  NFL_HIP(hipMemcpyAsync(h.data(), pr.g.p, h.size() * sizeof(float), hipMemcpyDeviceToHost,
                         P->stream));
  NFL_HIP(hipStreamSynchronize(P->stream));
  double ew = 0, nw = 0, ed = 0, nd = 0;
  for (int r = 0; r < pr.S; ++r) {
    ew = std::max(ew, std::fabs((double)h[r] - pr.refW[r]));
    nw = std::max(nw, std::fabs(pr.refW[r]));
    ed = std::max(ed, std::fabs((double)h[pr.S + r] - pr.refd[r]));
    nd = std::max(nd, std::fabs(pr.refd[r]));
  }
  const double rw = nw > 0 ? ew / nw : ew, rd = nd > 0 ? ed / nd : ed;
  *err = std::isfinite(rw) && std::isfinite(rd) ? std::max(rw, rd) : INFINITY;
  return NFL_OK;
}

// Average milliseconds of one L_s product on the GPU: `reps` products are
// captured into a HIP graph (on a private stream, with the plan's stream
// swapped out during the capture) and the graph launch is timed with HIP
// events on the plan's stream, so small graphs are timed without the host's
// launch overhead.  The product path records no memset nodes.
static int probe_time(nfl_plan *P, Probe &pr, int reps, double *ms) {
  VecArgs a;
  a.x32 = pr.x.p;
  a.y32 = pr.y.p;
  NFL_TRY(fastsum(P, IN_USER_F32_DINV, OUT_USER_LS, a));   // kernel attributes set outside capture
  hipStream_t cap = nullptr, user = P->stream;
  NFL_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  int rc = NFL_OK;
  P->stream = cap;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = NFL_ERR_HIP;
  for (int r = 0; r < reps && rc == NFL_OK; ++r) rc = fastsum(P, IN_USER_F32_DINV, OUT_USER_LS, a);
  const hipError_t ec = hipStreamEndCapture(cap, &g);
  P->stream = user;
  if (rc == NFL_OK && ec != hipSuccess) rc = NFL_ERR_HIP;
  if (rc == NFL_OK && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) rc = NFL_ERR_HIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float t = 0.f;
  if (rc == NFL_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = NFL_ERR_HIP;
  if (rc == NFL_OK && (hipGraphLaunch(ge, user) != hipSuccess ||      // warm
                       hipEventRecord(e0, user) != hipSuccess ||
                       hipGraphLaunch(ge, user) != hipSuccess ||
                       hipEventRecord(e1, user) != hipSuccess ||
                       hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    rc = NFL_ERR_HIP;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  if (rc != NFL_OK) {
    set_error("autotune: graph timing failed");
    return rc;
  }
  *ms = t / reps;
  return NFL_OK;
}

// ---- cache ------------------------------------------------------------------
struct TuneKey {
  int d, size_class, sigma_band, target_code;
  bool operator==(const TuneKey &o) const {
    return d == o.d && size_class == o.size_class && sigma_band == o.sigma_band &&
           target_code == o.target_code;
  }
};

struct TuneEntry {
  TuneKey key;
  int N, m, tile;
  double eps_B, err, ms;
};

static TuneKey make_key(const nfl_plan *P, double sigma, double target) {
  TuneKey k;
  k.d = P->d;
  k.size_class = (int)std::floor(std::log2((double)P->n) / 2.0);          // factors of 4 in n
  const double st0 = P->radius > 0 ? sigma * 0.25 / P->radius : sigma;    // sigma~ at eps_B = 0
  k.sigma_band = (int)std::floor(2.0 * std::log2(st0));                  // factors of sqrt(2)
  k.target_code = (int)std::lround(-4.0 * std::log10(target));
  return k;
}

static std::vector<TuneEntry> cache_read(const char *path) {
  std::vector<TuneEntry> out;
  if (!path) return out;
  FILE *f = std::fopen(path, "r");
  if (!f) return out;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    TuneEntry e;
    if (std::sscanf(line, "%d %d %d %d %d %d %lf %d %lf %lf", &e.key.d, &e.key.size_class,
                    &e.key.sigma_band, &e.key.target_code, &e.N, &e.m, &e.eps_B, &e.tile, &e.err,
                    &e.ms) == 10)
      out.push_back(e);
  }
  std::fclose(f);
  return out;
}

static int cache_write(const char *path, const TuneEntry &ne) {
  std::vector<TuneEntry> all = cache_read(path);
  bool found = false;
  for (auto &e : all)
    if (e.key == ne.key) {
      e = ne;
      found = true;
    }
  if (!found) all.push_back(ne);
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) { set_error("autotune: cannot write the cache file"); return NFL_ERR_ARG; }
  std::fprintf(f, "# NFFT autotune cache: d size_class(floor(log4 n)) sigma_band(floor(2 log2 "
                  "sigma~)) target_code(round(-4 log10 target)) N m eps_B tile err ms\n");
  for (const auto &e : all)
    std::fprintf(f, "%d %d %d %d %d %d %.17g %d %.6g %.6g\n", e.key.d, e.key.size_class,
                 e.key.sigma_band, e.key.target_code, e.N, e.m, e.eps_B, e.tile, e.err, e.ms);
  std::fclose(f);
  if (std::rename(tmp.c_str(), path) != 0) { set_error("autotune: cannot replace the cache file"); return NFL_ERR_ARG; }
  return NFL_OK;
}

// Set (tile, N, m, eps_B) on the plan; a degree failure is reported as a soft
// outcome (*ok = false) so the search can move on.
static int try_config(nfl_plan *P, double sigma, int N, int m, double eps_B, int tile, bool *ok) {
  if (P->d == 3) NFL_TRY(nfl_set_option(P, NFL_OPT_TILE, tile));
  const int rc = nfl_set_kernel(P, sigma, N, m, eps_B);
  *ok = rc == NFL_OK;
  if (rc == NFL_ERR_DEGREE) return NFL_OK;
  return rc;
}

static int autotune(nfl_plan *P, double sigma, double target, int S, uint64_t seed,
                    const char *cache_path, int *N_out, int *m_out, double *eps_out,
                    int *tile_out, double *err_out, double *ms_out, int *cached_out) {
  Probe pr;
  int rc = probe_init(P, sigma, S, seed, pr);
  if (rc < 0) { pr.release(); return rc; }
  const TuneKey key = make_key(P, sigma, target);
  const int tile0 = P->opt_tile;
  auto finish = [&](int N, int m, double eps, int tile, double err, double ms, int cached) {
    if (N_out) *N_out = N;
    if (m_out) *m_out = m;
    if (eps_out) *eps_out = eps;
    if (tile_out) *tile_out = tile;
    if (err_out) *err_out = err;
    if (ms_out) *ms_out = ms;
    if (cached_out) *cached_out = cached;
  };

  // cached configuration for this class, verified here
  for (const TuneEntry &e : cache_read(cache_path)) {
    if (!(e.key == key)) continue;
    bool ok = false;
    rc = try_config(P, sigma, e.N, e.m, e.eps_B, e.tile, &ok);
    if (rc < 0) { pr.release(); return rc; }
    if (!ok) break;
    double err = 0, ms = 0;
    rc = probe_error(P, pr, &err);
    if (rc == NFL_OK && err <= target) rc = probe_time(P, pr, 5, &ms);
    if (rc < 0) { pr.release(); return rc; }
    if (err <= target) {
      finish(e.N, e.m, e.eps_B, e.tile, err, ms, 1);
      pr.release();
      return NFL_OK;
    }
    break;
  }

  // 1. kernel approximation: smallest N per eps_B at the widest window
  const double st0 = P->radius > 0 ? sigma * 0.25 / P->radius : sigma;
  const double eps_list[3] = {0.0, 1.0 / 16, 1.0 / 8};
  int bestN = 0;
  double bestEps = 0, bestErr = INFINITY;
  int fbN = 0, fbm = 0;            // most accurate configuration seen (fallback)
  double fbEps = 0, fbErr = INFINITY;
  for (double eps : eps_list) {
    for (int N = 8; N <= 256; N *= 2) {
      if (bestN && N > bestN) break;
      if (st0 * N < 1.0) continue;   // the Gaussian's spectrum is cut far above 1e-2
      const int m = std::min(8, N / 2);
      bool ok = false;
      rc = try_config(P, sigma, N, m, eps, tile0, &ok);
      if (rc < 0) { pr.release(); return rc; }
      if (!ok) continue;
      double err = 0;
      rc = probe_error(P, pr, &err);
      if (rc < 0) { pr.release(); return rc; }
      if (err < fbErr) {
        fbErr = err;
        fbN = N;
        fbm = m;
        fbEps = eps;
      }
      if (err <= 0.3 * target) {
        if (!bestN || N < bestN || (N == bestN && err < bestErr)) {
          bestN = N;
          bestEps = eps;
          bestErr = err;
        }
        break;
      }
    }
  }
  if (!bestN) {
    // nothing reaches the target: leave the most accurate configuration set
    if (fbN) {
      bool ok = false;
      rc = try_config(P, sigma, fbN, fbm, fbEps, tile0, &ok);
      if (rc < 0) { pr.release(); return rc; }
    }
    finish(fbN, fbm, fbEps, tile0, fbErr, 0.0, 0);
    pr.release();
    set_error("autotune: no configuration reaches the target error");
    return fbN ? NFL_NOT_CONVERGED : NFL_ERR_DEGREE;
  }

  // 2. window: smallest m at (N, eps_B) within 0.7 x target
  int bestM = std::min(8, bestN / 2);
  for (int m = bestM - 1; m >= 2; --m) {
    bool ok = false;
    rc = try_config(P, sigma, bestN, m, bestEps, tile0, &ok);
    if (rc < 0) { pr.release(); return rc; }
    if (!ok) break;
    double err = 0;
    rc = probe_error(P, pr, &err);
    if (rc < 0) { pr.release(); return rc; }
    if (err > 0.7 * target) break;
    bestM = m;
  }

  // 3. tile: fastest product
  int bestT = tile0;
  double bestMs = INFINITY;
  const int tiles_d3[3] = {4, 8, 16};
  const int ntiles = P->d == 3 ? 3 : 1;
  int last_shift = -1;
  for (int k = 0; k < ntiles; ++k) {
    const int T = P->d == 3 ? tiles_d3[k] : tile0;
    bool ok = false;
    rc = try_config(P, sigma, bestN, bestM, bestEps, T, &ok);
    if (rc < 0) { pr.release(); return rc; }
    if (!ok) continue;
    if (P->tshift == last_shift) continue;   // clamped to a tile already timed
    last_shift = P->tshift;
    double ms = 0;
    rc = probe_time(P, pr, 10, &ms);
    if (rc < 0) { pr.release(); return rc; }
    if (ms < bestMs) {
      bestMs = ms;
      bestT = T;
    }
  }

  bool ok = false;
  rc = try_config(P, sigma, bestN, bestM, bestEps, bestT, &ok);
  double err = INFINITY, ms = 0;
  if (rc == NFL_OK && ok) rc = probe_error(P, pr, &err);
  if (rc == NFL_OK && ok) rc = probe_time(P, pr, 5, &ms);
  pr.release();
  if (rc < 0) return rc;
  if (!ok) { set_error("autotune: chosen configuration failed to set"); return NFL_ERR_DEGREE; }
  finish(bestN, bestM, bestEps, bestT, err, ms, 0);
  if (cache_path && err <= target) {
    TuneEntry e{key, bestN, bestM, bestT, bestEps, err, ms};
    NFL_TRY(cache_write(cache_path, e));
  }
  return err <= target ? NFL_OK : NFL_NOT_CONVERGED;
}

}  // namespace nfl

using namespace nfl;

extern "C" {

int nfl_direct_rows(nfl_handle P, double sigma, const float *x_dev, const int64_t *rows_host,
                    int nrows, double *wx_host, double *deg_host) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_points) { set_error("direct rows before set_points"); return NFL_ERR_ORDER; }
  if (!(sigma > 0) || nrows < 1 || !rows_host || (!wx_host && !deg_host) ||
      (wx_host && !x_dev)) {
    set_error("need sigma > 0, rows, an output, and x when W x is asked for");
    return NFL_ERR_ARG;
  }
  if (nrows > 65535) { set_error("at most 65535 rows"); return NFL_ERR_ARG; }
  for (int r = 0; r < nrows; ++r)
    if (rows_host[r] < 0 || rows_host[r] >= P->n) { set_error("row index out of range"); return NFL_ERR_ARG; }
  return direct_rows(P, sigma, wx_host ? x_dev : nullptr, rows_host, nrows, wx_host, deg_host);
}

int nfl_autotune(nfl_handle P, double sigma, double target, int nrows, uint64_t seed,
                 const char *cache_path, int *N, int *m, double *eps_B, int *tile, double *err,
                 double *ms, int *cached) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_points) { set_error("autotune before set_points"); return NFL_ERR_ORDER; }
  if (!(sigma > 0) || !std::isfinite(sigma)) { set_error("sigma must be > 0"); return NFL_ERR_ARG; }
  if (!(target > 0) || !(target < 1)) { set_error("target must be in (0, 1)"); return NFL_ERR_ARG; }
  if (nrows < 1 || nrows > 65535) { set_error("nrows must be in [1, 65535]"); return NFL_ERR_ARG; }
  return autotune(P, sigma, target, nrows, seed, cache_path, N, m, eps_B, tile, err, ms, cached);
}

}  // extern "C"
