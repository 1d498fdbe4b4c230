// All-FP64 NFFT fast summation (NFL_OPT_PRECISION = 64): spread, FFT, filter
// and interpolation in double precision, for error studies against the FP32
// path.  Tab. fastsum_param notes that with the cut-off m = 8 the NFFT
// reaches about IEEE double precision; the FP32 path cannot show that, this
// one can.
//
// Differences from the FP32 path (which stays the production path):
// * the window is the Kaiser-Bessel function itself, evaluated per node in
//   FP64 (no polynomial fit), and the filter divides by the Fourier
//   transform of that truncated window (quadrature to rounding);
// * node fractions are recomputed in FP64 from the caller's coordinates (the
//   FP32 path stores them as float32, ~1e-8 relative position error);
// * degrees and d^{-1/2} are FP64;
// * the FFT is a plain complex FP64 transform of the whole oversampled grid
//   (radix-2 in LDS, one pass per axis, the filter applied between the
//   forward and inverse transforms of the last pass), not pruned;
// * grid accumulation uses FP64 atomics (not bitwise reproducible run to run,
//   at the 1e-16 level).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "nfft_device.h"
#include "nfl_internal.h"

namespace nfl {

namespace {

constexpr double KB_B = M_PI * 1.5;   // b = pi (2 - 1/sigma_os), sigma_os = 2

// psi(t) = sinh(b s) / (s b e^{bm}), s = sqrt(m^2 - t^2), |t| <= m; 0 outside
__device__ __forceinline__ double kb_psi64(double t, int m) {
  const double s2 = (double)m * m - t * t;
  if (s2 < 0.0) return 0.0;
  const double s = sqrt(s2);
  const double bm = KB_B * m;
  // sinh(b s) e^{-bm} = (e^{b(s - m)} - e^{-b(s + m)}) / 2
  const double num = s > 1e-8 ? 0.5 * (exp(KB_B * s - bm) - exp(-KB_B * s - bm)) / s
                              : KB_B * exp(-bm);
  return num / KB_B;
}

struct K64 {
  const float *x32;
  float *y32;
  const double *x64;
  double *y64;
  double tau;
  const int *perm;
  const double *dinv;     // d^{-1/2} in FP64 (sorted order)
  double *deg_out;        // OUT_DEGREE: FP64 degrees and d^{-1/2}
  double *dinv_out;
  float *deg32;           // and their float copies
  float *dinv32;
  const int *stop;
};

template <int IN>
__device__ __forceinline__ double load64(const K64 &a, int i) {
  if constexpr (IN == IN_USER_F32) return (double)a.x32[a.perm[i]];
  else if constexpr (IN == IN_USER_F32_DINV) return a.dinv[i] * (double)a.x32[a.perm[i]];
  else if constexpr (IN == IN_ONES) return 1.0;
  else if constexpr (IN == IN_SORTED_F32) return (double)a.x32[i];
  else return a.dinv[i] * a.x64[i];
}

// the post-operations of Alg. nfft_normalized_matvec (K(0) = 1 subtracted)
template <int OUT>
__device__ __forceinline__ void store64(const K64 &a, int i, double f) {
  if constexpr (OUT == OUT_USER_RAW) {
    a.y32[a.perm[i]] = (float)f;
  } else if constexpr (OUT == OUT_USER_W) {
    const int j = a.perm[i];
    a.y32[j] = (float)(f - (double)a.x32[j]);
  } else if constexpr (OUT == OUT_USER_LS) {
    const int j = a.perm[i];
    const double xu = a.x32[j], di = a.dinv[i];
    a.y32[j] = (float)(xu - di * (f - di * xu));
  } else if constexpr (OUT == OUT_USER_A) {
    const int j = a.perm[i];
    const double xu = a.x32[j], di = a.dinv[i];
    a.y32[j] = (float)(di * (f - di * xu));
  } else if constexpr (OUT == OUT_DEGREE) {
    const double dg = f - 1.0;
    const double di = dg > 0.0 ? 1.0 / sqrt(dg) : 0.0;
    a.deg_out[i] = dg;
    a.dinv_out[i] = di;
    a.deg32[i] = (float)dg;
    a.dinv32[i] = (float)di;
  } else if constexpr (OUT == OUT_SORTED_F64_A) {
    const double di = a.dinv[i];
    a.y64[i] = di * (f - di * a.x64[i]);
  } else {   // OUT_SORTED_F64_SSL
    const double di = a.dinv[i], x = a.x64[i];
    a.y64[i] = x + a.tau * (x - di * (f - di * x));
  }
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// FP64 node fractions (sorted order): u = nos (rho (v - c) + 1/2) per axis,
// minus the cell the sort used (the same FP64 formula, so they agree).
__global__ __launch_bounds__(256) void k_frac64(const float *__restrict__ v, const int *__restrict__ perm,
                                                const float4 *__restrict__ pts, int64_t n, int d,
                                                double c0, double c1, double c2, double rho, int nos,
                                                double4 *__restrict__ fr) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  const uint32_t cell = __float_as_uint(pts[i].w);
  const double c[3] = {c0, c1, c2};
  double f[3] = {0.0, 0.0, 0.0};
  for (int t = 0; t < d; ++t) {
    const int ci = (int)((cell >> (10 * t)) & 1023u);
    f[t] = (double)nos * (rho * ((double)v[(int64_t)j * d + t] - c[t]) + 0.5) - ci;
  }
  fr[i] = make_double4(f[0], f[1], f[2], 0.0);
}

// ---------------------------------------------------------------------------
// d = 3 spread: one workgroup per work item (nodes of one T^3 tile), the
// padded tile ((T + W - 1)^3 doubles) in LDS.  A wave walks its slice of the
// item node by node; lanes hold (y, z) pairs of the window with all W x
// values in registers, accumulated while consecutive nodes share a cell and
// added to LDS when the cell changes; finally the tile is added to the grid.
// ---------------------------------------------------------------------------
template <int W, int IN>
__global__ __launch_bounds__(256) void k_spread64_3(const Item *__restrict__ items,
                                                    const float4 *__restrict__ pts,
                                                    const double4 *__restrict__ fr, K64 ka,
                                                    double *__restrict__ grid, int nos,
                                                    int tshift) {
  constexpr int M = W / 2, R = (W * W + 63) / 64;
  extern __shared__ double lds64[];
  if (stopped(ka.stop)) return;
  const int T = 1 << tshift, P = T + W - 1, PP = P * P, P3 = PP * P;
  const Item it = items[blockIdx.x];
  const int ntd = nos >> tshift;
  const int tz = it.tile % ntd, ty = (it.tile / ntd) % ntd, tx = it.tile / (ntd * ntd);
  const int ox = tx * T, oy = ty * T, oz = tz * T;
  for (int c = threadIdx.x; c < P3; c += 256) lds64[c] = 0.0;
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
  const int wdim = lane / W, woff = lane - wdim * W;   // lanes < 3W evaluate a weight
  double acc[R][W];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int a = 0; a < W; ++a) acc[r][a] = 0.0;
  uint32_t cur = 0xffffffffu;
  auto flush = [&](uint32_t cell) {
    const int lx = (int)(cell & 1023u) - ox, ly = (int)((cell >> 10) & 1023u) - oy,
              lz = (int)(cell >> 20) - oz;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (pv[r]) {
        double *base = lds64 + (lx * P + ly + pay[r]) * P + lz + paz[r];
#pragma unroll
        for (int a = 0; a < W; ++a) {
          atomicAdd(base + a * PP, acc[r][a]);
          acc[r][a] = 0.0;
        }
      }
    }
  };
  for (int i0 = s; i0 < e; i0 += 64) {
    const int cnt = min(64, e - i0);
    uint32_t cb = 0;
    double fxb = 0.0, fyb = 0.0, fzb = 0.0, xb = 0.0;
    if (lane < cnt) {
      cb = __float_as_uint(pts[i0 + lane].w);
      const double4 q = fr[i0 + lane];
      fxb = q.x;
      fyb = q.y;
      fzb = q.z;
      xb = load64<IN>(ka, i0 + lane);
    }
    for (int j = 0; j < cnt; ++j) {
      const uint32_t cell = (uint32_t)__builtin_amdgcn_readlane((int)cb, j);
      const double xv = readlane_d(xb, j);
      if (cell != cur) {
        if (cur != 0xffffffffu) flush(cur);
        cur = cell;
      }
      const double f = wdim == 0 ? readlane_d(fxb, j) : (wdim == 1 ? readlane_d(fyb, j) : readlane_d(fzb, j));
      const double wgt = wdim < 3 ? kb_psi64((double)(woff - (M - 1)) - f, M) : 0.0;
      double wx[W];
#pragma unroll
      for (int a = 0; a < W; ++a) wx[a] = readlane_d(wgt, a);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double wy = __shfl(wgt, W + pay[r]);
        const double wz = __shfl(wgt, 2 * W + paz[r]);
        const double sy = pv[r] ? xv * wy * wz : 0.0;
#pragma unroll
        for (int a = 0; a < W; ++a) acc[r][a] = fma(sy, wx[a], acc[r][a]);
      }
    }
  }
  if (cur != 0xffffffffu) flush(cur);
  __syncthreads();
  const int mask = nos - 1;
  for (int c = threadIdx.x; c < P3; c += 256) {
    const double v = lds64[c];
    if (v != 0.0) {
      const int px = c / PP, rem = c - px * PP, py = rem / P, pz = rem - py * P;
      const int gx = (ox - (M - 1) + px) & mask, gy = (oy - (M - 1) + py) & mask,
                gz = (oz - (M - 1) + pz) & mask;
      unsafeAtomicAdd(&grid[((size_t)gx * nos + gy) * nos + gz], v);
    }
  }
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// d = 3 interpolation, the transpose: the padded tile of the real part of
// the complex grid (stride 2 doubles) staged in LDS; per node the wave forms
// sum_x wx sum_(y,z) wy wz g.
template <int W, int IN, int OUT>
__global__ __launch_bounds__(256) void k_interp64_3(const Item *__restrict__ items,
                                                    const float4 *__restrict__ pts,
                                                    const double4 *__restrict__ fr, K64 ka,
                                                    const double2 *__restrict__ grid, int nos,
                                                    int tshift) {
  constexpr int M = W / 2, R = (W * W + 63) / 64;
  extern __shared__ double lds64[];
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
    lds64[c] = grid[((size_t)gx * nos + gy) * nos + gz].x;
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
  const int wdim = lane / W, woff = lane - wdim * W;
  double g[R][W];
  uint32_t cur = 0xffffffffu;
  for (int i0 = s; i0 < e; i0 += 64) {
    const int cnt = min(64, e - i0);
    uint32_t cb = 0;
    double fxb = 0.0, fyb = 0.0, fzb = 0.0;
    if (lane < cnt) {
      cb = __float_as_uint(pts[i0 + lane].w);
      const double4 q = fr[i0 + lane];
      fxb = q.x;
      fyb = q.y;
      fzb = q.z;
    }
    double res = 0.0;
    for (int j = 0; j < cnt; ++j) {
      const uint32_t cell = (uint32_t)__builtin_amdgcn_readlane((int)cb, j);
      if (cell != cur) {
        cur = cell;
        const int lx = (int)(cell & 1023u) - ox, ly = (int)((cell >> 10) & 1023u) - oy,
                  lz = (int)(cell >> 20) - oz;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double *base = lds64 + (lx * P + ly + pay[r]) * P + lz + paz[r];
#pragma unroll
          for (int a = 0; a < W; ++a) g[r][a] = pv[r] ? base[a * PP] : 0.0;
        }
      }
      const double f = wdim == 0 ? readlane_d(fxb, j) : (wdim == 1 ? readlane_d(fyb, j) : readlane_d(fzb, j));
      const double wgt = wdim < 3 ? kb_psi64((double)(woff - (M - 1)) - f, M) : 0.0;
      double wx[W];
#pragma unroll
      for (int a = 0; a < W; ++a) wx[a] = readlane_d(wgt, a);
      double part = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double wy = __shfl(wgt, W + pay[r]);
        const double wz = __shfl(wgt, 2 * W + paz[r]);
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < W; ++a) t = fma(wx[a], g[r][a], t);
        part = fma(wy * wz, t, part);
      }
      part = wave_sum_d(part);
      if (lane == j) res = part;
    }
    if (lane < cnt) store64<OUT>(ka, i0 + lane, res);
  }
}

// d = 1, 2: one thread per node, the window summed directly in the grid
// (FP64 atomics for the spread).
template <int IN>
__global__ __launch_bounds__(256) void k_spread64_12(const float4 *__restrict__ pts,
                                                     const double4 *__restrict__ fr, K64 ka,
                                                     int64_t n, int d, int m, int nos,
                                                     double *__restrict__ grid) {
  if (stopped(ka.stop)) return;
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t cell = __float_as_uint(pts[i].w);
  const double4 q = fr[i];
  const double x = load64<IN>(ka, (int)i);
  const int W = 2 * m, mask = nos - 1;
  const int cx = (int)(cell & 1023u), cy = (int)((cell >> 10) & 1023u);
  double wy[WIN_MAXW];
  for (int b = 0; b < W; ++b) wy[b] = d == 2 ? kb_psi64((double)(b - (m - 1)) - q.y, m) : 1.0;
  for (int a = 0; a < W; ++a) {
    const double wa = x * kb_psi64((double)(a - (m - 1)) - q.x, m);
    const int gx = (cx - (m - 1) + a) & mask;
    if (d == 1) {
      unsafeAtomicAdd(&grid[gx], wa);
    } else {
      for (int b = 0; b < W; ++b)
        unsafeAtomicAdd(&grid[(size_t)gx * nos + ((cy - (m - 1) + b) & mask)], wa * wy[b]);
    }
  }
}

template <int IN, int OUT>
__global__ __launch_bounds__(256) void k_interp64_12(const float4 *__restrict__ pts,
                                                     const double4 *__restrict__ fr, K64 ka,
                                                     int64_t n, int d, int m, int nos,
                                                     const double2 *__restrict__ grid) {
  if (stopped(ka.stop)) return;
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t cell = __float_as_uint(pts[i].w);
  const double4 q = fr[i];
  const int W = 2 * m, mask = nos - 1;
  const int cx = (int)(cell & 1023u), cy = (int)((cell >> 10) & 1023u);
  double wy[WIN_MAXW];
  for (int b = 0; b < W; ++b) wy[b] = d == 2 ? kb_psi64((double)(b - (m - 1)) - q.y, m) : 1.0;
  double f = 0.0;
  for (int a = 0; a < W; ++a) {
    const double wa = kb_psi64((double)(a - (m - 1)) - q.x, m);
    const int gx = (cx - (m - 1) + a) & mask;
    if (d == 1) {
      f = fma(wa, grid[gx].x, f);
    } else {
      double t = 0.0;
      for (int b = 0; b < W; ++b) t = fma(wy[b], grid[(size_t)gx * nos + ((cy - (m - 1) + b) & mask)].x, t);
      f = fma(wa, t, f);
    }
  }
  store64<OUT>(ka, (int)i, f);
}

// ---------------------------------------------------------------------------
// FFT: complex FP64 transforms of whole lines of length L = nos (a power of
// 2) along one axis, G lines per workgroup.  Element j of line q sits at
// base(q) + j es; the G lines of a workgroup are consecutive in q with
// base(q) = (q / inner) outer_stride + (q % inner) inner_stride.  In LDS the
// lines are bit-reversed on load and transformed in place by radix-2
// butterflies (decimation in time), twiddles w_k = e^{-2 pi i k / L} from a
// table.  Modes: REAL_IN reads the real grid (and clears it) instead of the
// complex one; FILTER multiplies each line by the filter after the forward
// transform and transforms back (the last axis of the forward pass).
// ---------------------------------------------------------------------------
struct LineMap {
  int64_t es, outer_stride, inner_stride;
  int inner, nlines;
};

__device__ __forceinline__ int64_t line_base(const LineMap &mp, int q) {
  return (int64_t)(q / mp.inner) * mp.outer_stride + (int64_t)(q % mp.inner) * mp.inner_stride;
}

__device__ __forceinline__ double2 cmul64(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int SIGN>
__device__ void fft64_lds(double2 *buf, int L, int logL, int G, const double2 *__restrict__ tw) {
  for (int half = 1, st = 0; st < logL; half <<= 1, ++st) {
    const int tstride = L / (2 * half);
    for (int p = threadIdx.x; p < G * (L / 2); p += blockDim.x) {
      const int line = p / (L / 2), b = p - line * (L / 2);
      const int grp = b >> st, k = b & (half - 1);
      const int i0 = line * L + grp * 2 * half + k, i1 = i0 + half;
      double2 w = tw[k * tstride];
      if (SIGN > 0) w.y = -w.y;
      const double2 u = buf[i0], v = cmul64(buf[i1], w);
      buf[i0] = make_double2(u.x + v.x, u.y + v.y);
      buf[i1] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int j, int logL) { return (int)(__brev((unsigned)j) >> (32 - logL)); }

// Full-spectrum value of the half-spectrum filter at FFT indices k (d axes,
// the last fastest): zero outside |l_t| <= N/2, mirrored for l_last < 0 (the
// filter is real and even, so the output of a real input stays real).
__device__ __forceinline__ double filter_full(const double *__restrict__ filt, const int *k, int d,
                                              int L, int N) {
  int l[3];
  for (int t = 0; t < d; ++t) {
    l[t] = k[t] <= L / 2 ? k[t] : k[t] - L;
    if (l[t] > N / 2 || l[t] < -N / 2) return 0.0;
  }
  if (l[d - 1] < 0)
    for (int t = 0; t < d; ++t) l[t] = -l[t];
  const int H = N / 2 + 1, F = N + 1;
  int64_t q = 0;
  for (int t = 0; t < d - 1; ++t) q = q * F + (l[t] + N / 2);
  return filt[q * H + l[d - 1]];
}

template <bool REAL_IN, bool FILTER, int SIGN>
__global__ __launch_bounds__(256) void k_fft64_pass(double2 *__restrict__ data,
                                                    double *__restrict__ rgrid, LineMap mp, int L,
                                                    int logL, int G,
                                                    const double2 *__restrict__ tw,
                                                    const double *__restrict__ filt, int d, int N,
                                                    int axis, const int *__restrict__ stop) {
  extern __shared__ double2 sbuf[];
  if (stopped(stop)) return;
  const int q0 = blockIdx.x * G;
  const int g = min(G, mp.nlines - q0);
  const bool rows = mp.es == 1;   // contiguous lines: threads along j, else across lines
  for (int t = threadIdx.x; t < g * L; t += blockDim.x) {
    int line, j;
    if (rows) { line = t / L; j = t - line * L; } else { j = t / g; line = t - j * g; }
    const int64_t idx = line_base(mp, q0 + line) + (int64_t)j * mp.es;
    double2 v;
    if (REAL_IN) {
      v = make_double2(rgrid[idx], 0.0);
      rgrid[idx] = 0.0;
    } else {
      v = data[idx];
    }
    sbuf[line * L + bitrev(j, logL)] = v;
  }
  __syncthreads();
  if (FILTER) {
    fft64_lds<-1>(sbuf, L, logL, g, tw);
    for (int t = threadIdx.x; t < g * L; t += blockDim.x) {
      const int line = t / L, j = t - line * L;
      // FFT indices of this element: decompose the line's base
      const int64_t b = line_base(mp, q0 + line) + (int64_t)j * mp.es;
      int k[3];
      int64_t r = b;
      for (int a = d - 1; a >= 0; --a) {
        k[a] = (int)(r % L);
        r /= L;
      }
      const double h = filter_full(filt, k, d, L, N);
      const double2 v = sbuf[t];
      sbuf[t] = make_double2(v.x * h, v.y * h);
    }
    __syncthreads();
    // inverse: bit-reverse in LDS (swap pairs), then the butterflies
    for (int t = threadIdx.x; t < g * L; t += blockDim.x) {
      const int line = t / L, j = t - line * L, jr = bitrev(j, logL);
      if (j < jr) {
        const double2 a = sbuf[line * L + j];
        sbuf[line * L + j] = sbuf[line * L + jr];
        sbuf[line * L + jr] = a;
      }
    }
    __syncthreads();
    fft64_lds<+1>(sbuf, L, logL, g, tw);
  } else {
    fft64_lds<SIGN>(sbuf, L, logL, g, tw);
  }
  for (int t = threadIdx.x; t < g * L; t += blockDim.x) {
    int line, j;
    if (rows) { line = t / L; j = t - line * L; } else { j = t / g; line = t - j * g; }
    const int64_t idx = line_base(mp, q0 + line) + (int64_t)j * mp.es;
    data[idx] = sbuf[line * L + j];
  }
  (void)axis;
}

K64 make_k64(nfl_plan *P, const VecArgs &a) {
  K64 k;
  k.x32 = a.x32;
  k.y32 = a.y32;
  k.x64 = a.x64;
  k.y64 = a.y64;
  k.tau = a.tau;
  k.perm = P->perm.p;
  k.dinv = P->dinv64.p;
  k.deg_out = P->deg64.p;
  k.dinv_out = P->dinv64.p;
  k.deg32 = P->deg.p;
  k.dinv32 = P->dinv.p;
  k.stop = P->stop;
  return k;
}

template <int W, int IN>
int launch_spread64_3(nfl_plan *P, const K64 &k) {
  const int T = 1 << P->tshift, Pd = T + W - 1;
  const size_t lds = (size_t)Pd * Pd * Pd * sizeof(double);
  if (lds > 65536) {
    static bool done = false;
    if (!done) {
      NFL_HIP(hipFuncSetAttribute((const void *)k_spread64_3<W, IN>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      done = true;
    }
  }
  hipLaunchKernelGGL((k_spread64_3<W, IN>), dim3(P->nitems), dim3(256), lds, P->stream,
                     P->items.p, P->pts.p, P->frac64.p, k, P->grid64.p, P->nos, P->tshift);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

template <int W, int IN, int OUT>
int launch_interp64_3(nfl_plan *P, const K64 &k) {
  const int T = 1 << P->tshift, Pd = T + W - 1;
  const size_t lds = (size_t)Pd * Pd * Pd * sizeof(double);
  if (lds > 65536) {
    static bool done = false;
    if (!done) {
      NFL_HIP(hipFuncSetAttribute((const void *)k_interp64_3<W, IN, OUT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      done = true;
    }
  }
  hipLaunchKernelGGL((k_interp64_3<W, IN, OUT>), dim3(P->nitems), dim3(256), lds, P->stream,
                     P->items.p, P->pts.p, P->frac64.p, k, P->spec64.p, P->nos, P->tshift);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

template <int IN>
int spread64_in(nfl_plan *P, const K64 &k) {
  if (P->nitems == 0) return NFL_OK;
  if (P->d != 3) {
    const int nb = (int)((P->n + 255) / 256);
    hipLaunchKernelGGL(k_spread64_12<IN>, dim3(nb), dim3(256), 0, P->stream, P->pts.p,
                       P->frac64.p, k, P->n, P->d, P->m, P->nos, P->grid64.p);
    NFL_HIP(hipGetLastError());
    return NFL_OK;
  }
  switch (P->m) {
    case 2: return launch_spread64_3<4, IN>(P, k);
    case 3: return launch_spread64_3<6, IN>(P, k);
    case 4: return launch_spread64_3<8, IN>(P, k);
    case 5: return launch_spread64_3<10, IN>(P, k);
    case 6: return launch_spread64_3<12, IN>(P, k);
    case 7: return launch_spread64_3<14, IN>(P, k);
    case 8: return launch_spread64_3<16, IN>(P, k);
    default: set_error("FP64 spread: m out of range"); return NFL_ERR_UNSUPPORTED;
  }
}

template <int IN, int OUT>
int interp64_io(nfl_plan *P, const K64 &k) {
  if (P->nitems == 0) return NFL_OK;
  if (P->d != 3) {
    const int nb = (int)((P->n + 255) / 256);
    hipLaunchKernelGGL((k_interp64_12<IN, OUT>), dim3(nb), dim3(256), 0, P->stream, P->pts.p,
                       P->frac64.p, k, P->n, P->d, P->m, P->nos, P->spec64.p);
    NFL_HIP(hipGetLastError());
    return NFL_OK;
  }
  switch (P->m) {
    case 2: return launch_interp64_3<4, IN, OUT>(P, k);
    case 3: return launch_interp64_3<6, IN, OUT>(P, k);
    case 4: return launch_interp64_3<8, IN, OUT>(P, k);
    case 5: return launch_interp64_3<10, IN, OUT>(P, k);
    case 6: return launch_interp64_3<12, IN, OUT>(P, k);
    case 7: return launch_interp64_3<14, IN, OUT>(P, k);
    case 8: return launch_interp64_3<16, IN, OUT>(P, k);
    default: set_error("FP64 interp: m out of range"); return NFL_ERR_UNSUPPORTED;
  }
}

// One pass along axis `ax` of the d-dimensional L^d grid.
template <bool REAL_IN, bool FILTER, int SIGN>
int fft64_axis(nfl_plan *P, int ax) {
  const int L = P->nos, d = P->d;
  int logL = 0;
  while ((1 << logL) < L) ++logL;
  LineMap mp;
  int64_t stride = 1;
  for (int t = d - 1; t > ax; --t) stride *= L;   // element stride along the axis
  mp.es = stride;
  int64_t total = 1;
  for (int t = 0; t < d; ++t) total *= L;
  mp.nlines = (int)(total / L);
  if (stride == 1) {          // last axis: lines are rows
    mp.inner = mp.nlines;
    mp.inner_stride = L;
    mp.outer_stride = 0;
  } else {                    // lines indexed by (outer, inner): inner = the axes after ax
    mp.inner = (int)stride;
    mp.inner_stride = 1;
    mp.outer_stride = stride * L;
  }
  const int G = std::max(1, std::min(16, 2048 / L));
  const size_t lds = (size_t)G * L * sizeof(double2);
  const int nb = (mp.nlines + G - 1) / G;
  hipLaunchKernelGGL((k_fft64_pass<REAL_IN, FILTER, SIGN>), dim3(nb), dim3(256), lds, P->stream,
                     P->spec64.p, P->grid64.p, mp, L, logL, G, P->tw64.p, P->filt64.p, d, P->N, ax,
                     P->stop);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int convolve64(nfl_plan *P) {
  const int d = P->d;
  if (d == 1) return fft64_axis<true, true, -1>(P, 0);
  if (d == 2) {
    NFL_TRY((fft64_axis<true, false, -1>(P, 1)));
    NFL_TRY((fft64_axis<false, true, -1>(P, 0)));
    return fft64_axis<false, false, +1>(P, 1);
  }
  NFL_TRY((fft64_axis<true, false, -1>(P, 2)));
  NFL_TRY((fft64_axis<false, false, -1>(P, 1)));
  NFL_TRY((fft64_axis<false, true, -1>(P, 0)));
  NFL_TRY((fft64_axis<false, false, +1>(P, 1)));
  return fft64_axis<false, false, +1>(P, 2);
}

}  // namespace

// Fourier transform at xi of the truncated Kaiser-Bessel window psi on
// (-m, m]: 32-point Gauss-Legendre quadrature on each unit interval (psi is
// analytic there, so this is exact to rounding).  The closed form
// pi I_0(m sqrt(b^2 - (2 pi xi)^2)) / (b e^{bm}) is the transform of the
// untruncated function: ~1e-13 off at m = 6, 4e-5 at m = 2.
static double kb_psi_host(double t, int m) {
  const double s2 = (double)m * m - t * t;
  if (s2 <= 0.0) return s2 == 0.0 ? std::exp(-KB_B * m) : 0.0;
  const double s = std::sqrt(s2), bm = KB_B * m;
  const double sh = s > 1e-4 ? 0.5 * (std::exp(KB_B * s - bm) - std::exp(-KB_B * s - bm)) / s
                             : KB_B * std::exp(-bm) * (1.0 + KB_B * KB_B * s2 / 6.0);
  return sh / KB_B;
}

double kb_hat_exact(double xi, int m) {
  static thread_local std::vector<double> gx, gw;
  if (gx.empty()) {   // Gauss-Legendre nodes and weights on [-1, 1] by Newton on P_32
    const int q = 32;
    gx.resize(q);
    gw.resize(q);
    for (int i = 0; i < (q + 1) / 2; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (q + 0.5)), pp = 0.0;
      for (int it = 0; it < 100; ++it) {
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= q; ++j) {
          const double p3 = p2;
          p2 = p1;
          p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        pp = q * (z * p1 - p2) / (z * z - 1.0);
        const double dz = p1 / pp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      gx[i] = -z;
      gx[q - 1 - i] = z;
      gw[i] = gw[q - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
  }
  double acc = 0.0;
  for (int c = -m; c < m; ++c)
    for (size_t k = 0; k < gx.size(); ++k) {
      const double t = c + 0.5 * (gx[k] + 1.0);
      acc += 0.5 * gw[k] * kb_psi_host(t, m) * std::cos(2.0 * M_PI * xi * t);
    }
  return acc;
}

// Buffers, FP64 fractions, FP64 filter and twiddles of the all-FP64 path.
int setup64(nfl_plan *P) {
  if (P->kind == NFL_KERNEL_LAPLACIAN_RBF) {
    set_error("the FP64 NFFT path does not cover the Laplacian RBF near field");
    return NFL_ERR_UNSUPPORTED;
  }
  int64_t gsz = 1;
  for (int t = 0; t < P->d; ++t) gsz *= P->nos;
  NFL_TRY(P->grid64.ensure(gsz));
  NFL_TRY(P->spec64.ensure(gsz));
  NFL_TRY(P->frac64.ensure(P->n));
  NFL_TRY(P->deg64.ensure(P->n));
  NFL_TRY(P->dinv64.ensure(P->n));
  NFL_HIP(hipMemsetAsync(P->grid64.p, 0, gsz * sizeof(double), P->stream));
  const int nb = (int)((P->n + 255) / 256);
  hipLaunchKernelGGL(k_frac64, dim3(std::max(nb, 1)), dim3(256), 0, P->stream, P->pts_user.p,
                     P->perm.p, P->pts.p, P->n, P->d, P->centre[0], P->centre[1], P->centre[2],
                     P->rho, P->nos, P->frac64.p);
  NFL_HIP(hipGetLastError());
  std::vector<double> filt;
  NFL_TRY(compute_filter(P->d, P->N, P->m, P->p, P->eps_B, P->sigma_t, filt, P->kind, P->eps_I,
                         true));
  NFL_TRY(P->filt64.ensure(filt.size()));
  NFL_HIP(hipMemcpyAsync(P->filt64.p, filt.data(), filt.size() * sizeof(double),
                         hipMemcpyHostToDevice, P->stream));
  std::vector<double2> tw((size_t)P->nos / 2);
  for (int k = 0; k < P->nos / 2; ++k) {
    const double a = -2.0 * M_PI * k / P->nos;
    tw[k] = make_double2(std::cos(a), std::sin(a));
  }
  NFL_TRY(P->tw64.ensure(tw.size()));
  NFL_HIP(hipMemcpyAsync(P->tw64.p, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice,
                         P->stream));
  NFL_HIP(hipStreamSynchronize(P->stream));
  return NFL_OK;
}

int fastsum64(nfl_plan *P, int in_mode, int out_mode, const VecArgs &a) {
  const K64 k = make_k64(P, a);
  if (P->prof_ev) {   // stage events as on the FP32 path (no separate clear)
    NFL_HIP(hipEventRecord(P->prof_ev[0], P->stream));
    NFL_HIP(hipEventRecord(P->prof_ev[1], P->stream));
  }
  // spread into the real FP64 grid (left zero by the first FFT pass)
  switch (in_mode) {
    case IN_USER_F32: NFL_TRY(spread64_in<IN_USER_F32>(P, k)); break;
    case IN_USER_F32_DINV: NFL_TRY(spread64_in<IN_USER_F32_DINV>(P, k)); break;
    case IN_ONES: NFL_TRY(spread64_in<IN_ONES>(P, k)); break;
    case IN_SORTED_F32: NFL_TRY(spread64_in<IN_SORTED_F32>(P, k)); break;
    case IN_SORTED_F64_DINV: NFL_TRY(spread64_in<IN_SORTED_F64_DINV>(P, k)); break;
    default: set_error("FP64 spread: bad input mode"); return NFL_ERR_ARG;
  }
  if (P->prof_ev) NFL_HIP(hipEventRecord(P->prof_ev[2], P->stream));
  NFL_TRY(convolve64(P));
  if (P->prof_ev) NFL_HIP(hipEventRecord(P->prof_ev[3], P->stream));
  int rc;
  switch (out_mode) {
    case OUT_USER_RAW: rc = interp64_io<IN_USER_F32, OUT_USER_RAW>(P, k); break;
    case OUT_USER_W: rc = interp64_io<IN_USER_F32, OUT_USER_W>(P, k); break;
    case OUT_USER_LS: rc = interp64_io<IN_USER_F32, OUT_USER_LS>(P, k); break;
    case OUT_USER_A: rc = interp64_io<IN_USER_F32, OUT_USER_A>(P, k); break;
    case OUT_DEGREE: rc = interp64_io<IN_ONES, OUT_DEGREE>(P, k); break;
    case OUT_SORTED_F64_A: rc = interp64_io<IN_SORTED_F64_DINV, OUT_SORTED_F64_A>(P, k); break;
    case OUT_SORTED_F64_SSL: rc = interp64_io<IN_SORTED_F64_DINV, OUT_SORTED_F64_SSL>(P, k); break;
    default: set_error("FP64 interp: bad output mode"); return NFL_ERR_ARG;
  }
  if (rc == NFL_OK && P->prof_ev) NFL_HIP(hipEventRecord(P->prof_ev[4], P->stream));
  return rc;
}

}  // namespace nfl
