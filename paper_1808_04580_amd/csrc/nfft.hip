// NFFT fast summation on gfx950 (Alg. nfft_fastsum): spread -> FFT ->
// multiply by the filter -> inverse FFT -> interpolate, with the pre- and
// post-operations of Alg. nfft_normalized_matvec fused into the first and
// last kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "nfl_internal.h"

namespace nfl {

// ---------------------------------------------------------------------------
// Kaiser-Bessel window in grid units, normalised as
//   psi(t) = sinh(b s) / (s b e^{bm}),  s = sqrt(m^2 - t^2),  |t| <= m,
// evaluated as e^{-b t^2/(s+m)} (1 - e^{-2bs}) / (2bs): the exponent is never
// positive and the only cancellation happens where psi is ~e^{-bm} small.
// Its transform is pi I_0(m sqrt(b^2 - 4 pi^2 xi^2)) / (b e^{bm}) (host side).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float kb_window(float t, float m, float b) {
  const float t2 = t * t;
  const float s = __builtin_sqrtf(fmaxf(fmaf(-t, t, m * m), 0.f));
  const float e1 = __expf(-b * t2 / (s + m));
  const float x = 2.f * b * s;
  float h;
  if (x < 0.25f)
    h = fmaf(x, fmaf(x, fmaf(x, fmaf(x, 1.f / 120.f, -1.f / 24.f), 1.f / 6.f), -0.5f), 1.f);
  else
    h = (1.f - __expf(-x)) / x;
  return e1 * h;
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
};

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

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

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
                                                 float b) {
  constexpr int M = W / 2, R = (W * W + 63) / 64;
  extern __shared__ float lds[];
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
  const float toff = (float)(lane - wdim * W - (M - 1));

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

  for (int i = s; i < e; ++i) {
    const float4 q = pts[i];
    const uint32_t cell = __float_as_uint(q.w);
    const float xv = load_in<IN>(ka, i);
    if (cell != cur) {
      if (cur != 0xffffffffu) flush(cur);
      cur = cell;
    }
    const float fr = wdim == 0 ? q.x : (wdim == 1 ? q.y : q.z);
    const float wgt = kb_window(toff - fr, (float)M, b);
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
  if (cur != 0xffffffffu) flush(cur);
  __syncthreads();

  const int mask = nos - 1;
  for (int c = threadIdx.x; c < P3; c += 256) {
    const float v = lds[c];
    if (v != 0.f) {
      const int px = c / PP, rem = c - px * PP, py = rem / P, pz = rem - py * P;
      const int gx = (ox - (M - 1) + px) & mask, gy = (oy - (M - 1) + py) & mask,
                gz = (oz - (M - 1) + pz) & mask;
      unsafeAtomicAdd(&grid[((size_t)gx * nos + gy) * nos + gz], v);
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
                                                 int tshift, float b) {
  constexpr int M = W / 2, R = (W * W + 63) / 64;
  extern __shared__ float lds[];
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
  const float toff = (float)(lane - wdim * W - (M - 1));

  float g[R][W];
  uint32_t cur = 0xffffffffu;
  for (int i = s; i < e; ++i) {
    const float4 q = pts[i];
    const uint32_t cell = __float_as_uint(q.w);
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
    const float fr = wdim == 0 ? q.x : (wdim == 1 ? q.y : q.z);
    const float wgt = kb_window(toff - fr, (float)M, b);
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
    if (lane == 0) store_out<OUT>(ka, i, part);
  }
}

// ---------------------------------------------------------------------------
// d = 1, 2: one thread per node, direct global accumulation / gathering.
// ---------------------------------------------------------------------------
template <int IN>
__global__ __launch_bounds__(256) void k_spread12(const float4 *__restrict__ pts, int n, KArgs ka,
                                                  float *__restrict__ grid, int d, int nos,
                                                  int m, float b) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float4 q = pts[i];
  const uint32_t cell = __float_as_uint(q.w);
  const int cx = cell & 1023u, cy = (cell >> 10) & 1023u;
  const float xv = load_in<IN>(ka, i);
  const int W = 2 * m, mask = nos - 1;
  float wx[16], wy[16];
  for (int a = 0; a < W; ++a) {
    wx[a] = kb_window((float)(a - (m - 1)) - q.x, (float)m, b);
    wy[a] = d == 2 ? kb_window((float)(a - (m - 1)) - q.y, (float)m, b) : 1.f;
  }
  for (int a = 0; a < W; ++a) {
    const int gx = (cx - (m - 1) + a) & mask;
    if (d == 1) {
      unsafeAtomicAdd(&grid[gx], xv * wx[a]);
    } else {
      for (int c = 0; c < W; ++c) {
        const int gy = (cy - (m - 1) + c) & mask;
        unsafeAtomicAdd(&grid[(size_t)gx * nos + gy], xv * wx[a] * wy[c]);
      }
    }
  }
}

template <int IN, int OUT>
__global__ __launch_bounds__(256) void k_interp12(const float4 *__restrict__ pts, int n, KArgs ka,
                                                  const float *__restrict__ grid, int d, int nos,
                                                  int m, float b) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float4 q = pts[i];
  const uint32_t cell = __float_as_uint(q.w);
  const int cx = cell & 1023u, cy = (cell >> 10) & 1023u;
  const int W = 2 * m, mask = nos - 1;
  float wx[16], wy[16];
  for (int a = 0; a < W; ++a) {
    wx[a] = kb_window((float)(a - (m - 1)) - q.x, (float)m, b);
    wy[a] = d == 2 ? kb_window((float)(a - (m - 1)) - q.y, (float)m, b) : 1.f;
  }
  float f = 0.f;
  for (int a = 0; a < W; ++a) {
    const int gx = (cx - (m - 1) + a) & mask;
    if (d == 1) {
      f = fmaf(wx[a], grid[gx], f);
    } else {
      float t = 0.f;
      for (int c = 0; c < W; ++c) {
        const int gy = (cy - (m - 1) + c) & mask;
        t = fmaf(wy[c], grid[(size_t)gx * nos + gy], t);
      }
      f = fmaf(wx[a], t, f);
    }
  }
  store_out<OUT>(ka, i, f);
}

// ---------------------------------------------------------------------------
// FFT: radix-2 Stockham in LDS on `nl` lines of length L = nos.  The twiddle
// table holds e^{-2 pi i k/L}, k < L/2; SIGN = +1 gives the inverse
// (unnormalised) transform.  Result returned in `a` (buffers are swapped).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int SIGN>
__device__ void lds_fft(float2 *&a, float2 *&b, int L, int logL, int nl,
                        const float2 *__restrict__ tw) {
  const int half_n = L >> 1;
  for (int s = 0; s < logL; ++s) {
    const int half = 1 << s;
    for (int idx = threadIdx.x; idx < nl * half_n; idx += blockDim.x) {
      const int line = idx >> (logL - 1), j = idx & (half_n - 1);
      const int k = j & (half - 1), g = j >> s;
      float2 w = tw[k << (logL - 1 - s)];
      if (SIGN > 0) w.y = -w.y;
      const float2 x0 = a[line * L + j], x1 = a[line * L + j + half_n];
      const float2 t = cmul(w, x1);
      const int o = line * L + (g << (s + 1)) + k;
      b[o] = make_float2(x0.x + t.x, x0.y + t.y);
      b[o + half] = make_float2(x0.x - t.x, x0.y - t.y);
    }
    __syncthreads();
    float2 *tmp = a;
    a = b;
    b = tmp;
  }
}

constexpr int FFT_THREADS = 256, FFT_ELEMS = 2048;

// Real lines along the last (contiguous) axis -> half spectrum lz in [0, Hz).
__global__ __launch_bounds__(FFT_THREADS) void k_r2c_lines(const float *__restrict__ grid,
                                                           float2 *__restrict__ H, int nlines,
                                                           int L, int logL, int lpb, int Hz,
                                                           const float2 *__restrict__ tw) {
  extern __shared__ float2 sm[];
  float2 *a = sm, *b = sm + lpb * L;
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - l0);
  for (int idx = threadIdx.x; idx < lpb * L; idx += FFT_THREADS) {
    const int li = idx / L;
    a[idx] = make_float2(li < nl ? grid[(size_t)l0 * L + idx] : 0.f, 0.f);
  }
  __syncthreads();
  lds_fft<-1>(a, b, L, logL, lpb, tw);
  for (int idx = threadIdx.x; idx < nl * Hz; idx += FFT_THREADS) {
    const int li = idx / Hz, lz = idx - li * Hz;
    H[(size_t)(l0 + li) * Hz + lz] = a[li * L + lz];
  }
}

// Half spectrum (lz in [0, Hz), Hermitian in lz) -> real lines.
__global__ __launch_bounds__(FFT_THREADS) void k_c2r_lines(const float2 *__restrict__ H,
                                                           float *__restrict__ grid, int nlines,
                                                           int L, int logL, int lpb, int Hz,
                                                           const float2 *__restrict__ tw) {
  extern __shared__ float2 sm[];
  float2 *a = sm, *b = sm + lpb * L;
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - l0);
  for (int idx = threadIdx.x; idx < lpb * L; idx += FFT_THREADS) a[idx] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int idx = threadIdx.x; idx < nl * Hz; idx += FFT_THREADS) {
    const int li = idx / Hz, lz = idx - li * Hz;
    const float2 h = H[(size_t)(l0 + li) * Hz + lz];
    a[li * L + lz] = h;
    if (lz > 0) a[li * L + L - lz] = make_float2(h.x, -h.y);
  }
  __syncthreads();
  lds_fft<+1>(a, b, L, logL, lpb, tw);
  for (int idx = threadIdx.x; idx < nl * L; idx += FFT_THREADS)
    grid[(size_t)l0 * L + idx] = a[idx].x;
}

// d = 3 middle axis (y), forward: H1[(x*L + y)*Hz + lz] -> H2[(x*F + y')*Hz + lz],
// keeping ly = y' - N/2 in [-N/2, N/2].
__global__ __launch_bounds__(FFT_THREADS) void k_y_fwd(const float2 *__restrict__ H1,
                                                       float2 *__restrict__ H2, int L, int logL,
                                                       int lpb, int Hz, int N,
                                                       const float2 *__restrict__ tw) {
  extern __shared__ float2 sm[];
  float2 *a = sm, *b = sm + lpb * L;
  const int ngroups = (Hz + lpb - 1) / lpb;
  const int x = blockIdx.x / ngroups, lz0 = (blockIdx.x % ngroups) * lpb;
  const int nl = min(lpb, Hz - lz0);
  const int F = N + 1;
  for (int idx = threadIdx.x; idx < lpb * L; idx += FFT_THREADS) {
    const int y = idx / lpb, li = idx - y * lpb;
    a[li * L + y] = li < nl ? H1[((size_t)x * L + y) * Hz + lz0 + li] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft<-1>(a, b, L, logL, lpb, tw);
  for (int idx = threadIdx.x; idx < F * nl; idx += FFT_THREADS) {
    const int yp = idx / nl, li = idx - yp * nl;
    const int ly = (yp - N / 2 + L) & (L - 1);
    H2[((size_t)x * F + yp) * Hz + lz0 + li] = a[li * L + ly];
  }
}

__global__ __launch_bounds__(FFT_THREADS) void k_y_inv(const float2 *__restrict__ H2,
                                                       float2 *__restrict__ H1, int L, int logL,
                                                       int lpb, int Hz, int N,
                                                       const float2 *__restrict__ tw) {
  extern __shared__ float2 sm[];
  float2 *a = sm, *b = sm + lpb * L;
  const int ngroups = (Hz + lpb - 1) / lpb;
  const int x = blockIdx.x / ngroups, lz0 = (blockIdx.x % ngroups) * lpb;
  const int nl = min(lpb, Hz - lz0);
  const int F = N + 1;
  for (int idx = threadIdx.x; idx < lpb * L; idx += FFT_THREADS) a[idx] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int idx = threadIdx.x; idx < F * nl; idx += FFT_THREADS) {
    const int yp = idx / nl, li = idx - yp * nl;
    const int ly = (yp - N / 2 + L) & (L - 1);
    a[li * L + ly] = H2[((size_t)x * F + yp) * Hz + lz0 + li];
  }
  __syncthreads();
  lds_fft<+1>(a, b, L, logL, lpb, tw);
  for (int idx = threadIdx.x; idx < lpb * L; idx += FFT_THREADS) {
    const int y = idx / lpb, li = idx - y * lpb;
    if (li < nl) H1[((size_t)x * L + y) * Hz + lz0 + li] = a[li * L + y];
  }
}

// First axis (x): forward FFT, multiply by the filter on lx in [-N/2, N/2]
// (zero elsewhere), inverse FFT.  Hx[x*C + c], filter[(lx + N/2)*C + c].
__global__ __launch_bounds__(FFT_THREADS) void k_x_filter(float2 *__restrict__ Hx,
                                                          const float *__restrict__ filt, int C,
                                                          int L, int logL, int lpb, int N,
                                                          const float2 *__restrict__ tw) {
  extern __shared__ float2 sm[];
  float2 *a = sm, *b = sm + lpb * L;
  const int c0 = blockIdx.x * lpb;
  const int nl = min(lpb, C - c0);
  for (int idx = threadIdx.x; idx < lpb * L; idx += FFT_THREADS) {
    const int x = idx / lpb, li = idx - x * lpb;
    a[li * L + x] = li < nl ? Hx[(size_t)x * C + c0 + li] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft<-1>(a, b, L, logL, lpb, tw);
  for (int idx = threadIdx.x; idx < lpb * L; idx += FFT_THREADS) {
    const int li = idx / L, x = idx - li * L;
    const int lx = x < L / 2 ? x : x - L;
    float f = 0.f;
    if (li < nl && lx >= -N / 2 && lx <= N / 2) f = filt[(size_t)(lx + N / 2) * C + c0 + li];
    a[idx].x *= f;
    a[idx].y *= f;
  }
  __syncthreads();
  lds_fft<+1>(a, b, L, logL, lpb, tw);
  for (int idx = threadIdx.x; idx < lpb * L; idx += FFT_THREADS) {
    const int x = idx / lpb, li = idx - x * lpb;
    if (li < nl) Hx[(size_t)x * C + c0 + li] = a[li * L + x];
  }
}

__global__ void k_filter1(float2 *__restrict__ H, const float *__restrict__ filt, int Hz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < Hz) {
    H[i].x *= filt[i];
    H[i].y *= filt[i];
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
  return k;
}

static size_t tile_lds_bytes(const nfl_plan *P) {
  const int T = 1 << P->tshift, Pd = T + 2 * P->m - 1;
  return (size_t)Pd * Pd * Pd * sizeof(float);
}

template <int W, int IN>
static int launch_spread3(nfl_plan *P, const KArgs &k, float *grid) {
  const size_t lds = tile_lds_bytes(P);
  if (lds > 65536)
    NFL_HIP(hipFuncSetAttribute((const void *)k_spread3<W, IN>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_spread3<W, IN>), dim3(P->nitems), dim3(256), lds, P->stream, P->items.p,
                     P->pts.p, k, grid, P->nos, P->tshift, P->win.b);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

template <int W, int IN, int OUT>
static int launch_interp3(nfl_plan *P, const KArgs &k, const float *grid) {
  const size_t lds = tile_lds_bytes(P);
  if (lds > 65536)
    NFL_HIP(hipFuncSetAttribute((const void *)k_interp3<W, IN, OUT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_interp3<W, IN, OUT>), dim3(P->nitems), dim3(256), lds, P->stream,
                     P->items.p, P->pts.p, k, grid, P->nos, P->tshift, P->win.b);
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
  const int nb = (int)((P->n + 255) / 256);
  hipLaunchKernelGGL((k_spread12<IN>), dim3(nb), dim3(256), 0, P->stream, P->pts.p, (int)P->n, k,
                     grid, P->d, P->nos, P->m, P->win.b);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int spread(nfl_plan *P, int in_mode, const VecArgs &a, float *grid) {
  int64_t gsz = 1;
  for (int t = 0; t < P->d; ++t) gsz *= P->nos;
  NFL_TRY(fill_f32(grid, gsz, 0.f, P->stream));
  const KArgs k = make_kargs(P, a);
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
  const int nb = (int)((P->n + 255) / 256);
  hipLaunchKernelGGL((k_interp12<IN, OUT>), dim3(nb), dim3(256), 0, P->stream, P->pts.p,
                     (int)P->n, k, grid, P->d, P->nos, P->m, P->win.b);
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

int convolve(nfl_plan *P, const float *gin, float *gout) {
  const int L = P->nos, N = P->N, Hz = N / 2 + 1, F = N + 1;
  int logL = 0;
  while ((1 << logL) < L) ++logL;
  const int lpb = std::max(1, FFT_ELEMS / L);
  const size_t lds = (size_t)2 * lpb * L * sizeof(float2);
  const float2 *tw = P->tw.p;
  if (P->d == 1) {
    hipLaunchKernelGGL(k_r2c_lines, dim3(1), dim3(FFT_THREADS), lds, P->stream, gin, P->spec1.p,
                       1, L, logL, lpb, Hz, tw);
    hipLaunchKernelGGL(k_filter1, dim3(1), dim3(256), 0, P->stream, P->spec1.p, P->filt.p, Hz);
    hipLaunchKernelGGL(k_c2r_lines, dim3(1), dim3(FFT_THREADS), lds, P->stream, P->spec1.p, gout,
                       1, L, logL, lpb, Hz, tw);
  } else if (P->d == 2) {
    const int nlines = L;
    const int nb = (nlines + lpb - 1) / lpb;
    hipLaunchKernelGGL(k_r2c_lines, dim3(nb), dim3(FFT_THREADS), lds, P->stream, gin, P->spec1.p,
                       nlines, L, logL, lpb, Hz, tw);
    const int nbx = (Hz + lpb - 1) / lpb;
    hipLaunchKernelGGL(k_x_filter, dim3(nbx), dim3(FFT_THREADS), lds, P->stream, P->spec1.p,
                       P->filt.p, Hz, L, logL, lpb, N, tw);
    hipLaunchKernelGGL(k_c2r_lines, dim3(nb), dim3(FFT_THREADS), lds, P->stream, P->spec1.p, gout,
                       nlines, L, logL, lpb, Hz, tw);
  } else {
    const int nlines = L * L;
    const int nb = (nlines + lpb - 1) / lpb;
    hipLaunchKernelGGL(k_r2c_lines, dim3(nb), dim3(FFT_THREADS), lds, P->stream, gin, P->spec1.p,
                       nlines, L, logL, lpb, Hz, tw);
    const int ngroups = (Hz + lpb - 1) / lpb;
    hipLaunchKernelGGL(k_y_fwd, dim3(L * ngroups), dim3(FFT_THREADS), lds, P->stream, P->spec1.p,
                       P->spec2.p, L, logL, lpb, Hz, N, tw);
    const int C = F * Hz;
    const int nbx = (C + lpb - 1) / lpb;
    hipLaunchKernelGGL(k_x_filter, dim3(nbx), dim3(FFT_THREADS), lds, P->stream, P->spec2.p,
                       P->filt.p, C, L, logL, lpb, N, tw);
    hipLaunchKernelGGL(k_y_inv, dim3(L * ngroups), dim3(FFT_THREADS), lds, P->stream, P->spec2.p,
                       P->spec1.p, L, logL, lpb, Hz, N, tw);
    hipLaunchKernelGGL(k_c2r_lines, dim3(nb), dim3(FFT_THREADS), lds, P->stream, P->spec1.p, gout,
                       nlines, L, logL, lpb, Hz, tw);
  }
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int fastsum(nfl_plan *P, int in_mode, int out_mode, const VecArgs &a) {
  NFL_TRY(spread(P, in_mode, a, P->grid.p));
  NFL_TRY(convolve(P, P->grid.p, P->grid.p));
  return interp(P, P->grid.p, in_mode, out_mode, a);
}

}  // namespace nfl
