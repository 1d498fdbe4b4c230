// Krylov solvers on top of the NFFT operator (Section 4): Lanczos with full
// reorthogonalisation for the largest eigenvalues of A_E (= 1 - smallest of
// L_s) and CG for the kernel-SSL system (I + tau L_s) u = f.  Vectors live in
// the plan's sorted node order in FP64; the operator runs in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <numeric>
#include <vector>

#include "nfl_internal.h"

namespace nfl {

constexpr int VT = 256;        // threads per block for vector kernels
constexpr int VBLOCKS = 1024;  // row blocks for reductions

__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  return t;  // valid in thread 0
}

__global__ __launch_bounds__(VT) void k_dot_partial(const double *__restrict__ x,
                                                    const double *__restrict__ y, int64_t n,
                                                    double *__restrict__ part) {
  __shared__ double sh[VT / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    s += x[i] * y[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[0] = sum of part (op 0) or its square root (op 1); fixed order -> deterministic.
__global__ __launch_bounds__(VT) void k_reduce_final(const double *__restrict__ part, int nb,
                                                     double *__restrict__ out, int op) {
  __shared__ double sh[VT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += VT) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = op == 1 ? sqrt(s) : s;
}

__global__ __launch_bounds__(VT) void k_gather64(const double *__restrict__ src,
                                                 const int *__restrict__ perm, int64_t n,
                                                 double *__restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    dst[i] = src[perm[i]];
}

__global__ __launch_bounds__(VT) void k_scatter64(const double *__restrict__ src,
                                                  const int *__restrict__ perm, int64_t n,
                                                  double *__restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    dst[perm[i]] = src[i];
}

__global__ __launch_bounds__(VT) void k_fill64(double *__restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    p[i] = v;
}

// Deterministic start vector: splitmix64 counter hash -> two uniforms -> Box-Muller.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(VT) void k_start_vector(double *__restrict__ q,
                                                     const int *__restrict__ perm, int64_t n,
                                                     uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    // keyed by the caller's index so the start vector does not depend on the sort
    const uint64_t key = (uint64_t)perm[i] * 2ull + seed * 0x100000001b3ull;
    const double u1 = ((splitmix64(key) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((splitmix64(key + 1) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    q[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

// q = w * (1 / s[0])
__global__ __launch_bounds__(VT) void k_scale_inv(const double *__restrict__ w,
                                                  const double *__restrict__ s, int64_t n,
                                                  double *__restrict__ q) {
  const double f = 1.0 / s[0];
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    q[i] = w[i] * f;
}

// w -= alpha[0] * q + beta[0] * qp (qp may be null)
__global__ __launch_bounds__(VT) void k_lanczos_sub(double *__restrict__ w,
                                                    const double *__restrict__ q,
                                                    const double *__restrict__ qp,
                                                    const double *__restrict__ alpha,
                                                    const double *__restrict__ beta, int64_t n) {
  const double a = alpha[0], b = qp ? beta[0] : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    w[i] -= a * q[i] + (qp ? b * qp[i] : 0.0);
}

// part[b*J + j] = sum over this block's rows of Q[j*ld + i] w[i].  The columns
// are taken GT_COLS at a time, so that one load of w[i] serves all of them;
// each column still sums its rows in the grid-stride order.
constexpr int GT_COLS = 8;

__global__ __launch_bounds__(VT) void k_gemv_t_partial(const double *__restrict__ Q, int64_t ld,
                                                       int J, const double *__restrict__ w,
                                                       int64_t n, double *__restrict__ part) {
  __shared__ double sh[VT / 64];
  for (int j0 = 0; j0 < J; j0 += GT_COLS) {
    const int cnt = min(GT_COLS, J - j0);
    const double *Qj = Q + (int64_t)j0 * ld;
    double s[GT_COLS];
#pragma unroll
    for (int q = 0; q < GT_COLS; ++q) s[q] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VT) {
      const double wi = w[i];
      double qv[GT_COLS];
#pragma unroll
      for (int q = 0; q < GT_COLS; ++q) qv[q] = q < cnt ? Qj[q * ld + i] : 0.0;
#pragma unroll
      for (int q = 0; q < GT_COLS; ++q) s[q] += qv[q] * wi;
    }
#pragma unroll
    for (int q = 0; q < GT_COLS; ++q) {
      if (q < cnt) {   // cnt is the same in every thread: the barriers below match
        const double t = block_sum(s[q], sh);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * J + j0 + q] = t;
      }
    }
  }
}

// out[e] = sum over w < nb of part[w * width + e], e < width (the column sums
// of an nb x width row-major array of partial results).  A workgroup takes 16
// consecutive columns; its 16 thread rows sum interleaved slices of w, which
// are then added in slice order (fixed order -> deterministic).
constexpr int CS_E = 16, CS_S = VT / CS_E;

__global__ __launch_bounds__(VT) void k_colsum(const double *__restrict__ part, int nb, int width,
                                               double *__restrict__ out) {
  __shared__ double sh[CS_S][CS_E + 1];
  const int el = threadIdx.x % CS_E, sl = threadIdx.x / CS_E;
  const int e = blockIdx.x * CS_E + el;
  double s = 0.0;
  if (e < width) {
#pragma unroll 8
    for (int w = sl; w < nb; w += CS_S) s += part[(int64_t)w * width + e];
  }
  sh[sl][el] = s;
  __syncthreads();
  if (sl == 0 && e < width) {
    double t = 0.0;
    for (int k = 0; k < CS_S; ++k) t += sh[k][el];
    out[e] = t;
  }
}

// w[i] -= sum_j Q[j*ld + i] c[j], the terms added in the order of j; the
// loads of GT_COLS columns are issued before their products are added.
__global__ __launch_bounds__(VT) void k_gemv_n_sub(const double *__restrict__ Q, int64_t ld,
                                                   int J, const double *__restrict__ c,
                                                   double *__restrict__ w, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    double s = 0.0;
    for (int j0 = 0; j0 < J; j0 += GT_COLS) {
      const int cnt = min(GT_COLS, J - j0);
      double qv[GT_COLS];
#pragma unroll
      for (int q = 0; q < GT_COLS; ++q)
        qv[q] = q < cnt ? Q[(int64_t)(j0 + q) * ld + i] : 0.0;
#pragma unroll
      for (int q = 0; q < GT_COLS; ++q)
        if (q < cnt) s += qv[q] * c[j0 + q];
    }
    w[i] -= s;
  }
}

// Block forms of the two kernels above for nb <= BT_VECS vectors w_c = W[c*ldw
// + i]: one pass over the rows of GT_COLS basis columns serves all nb vectors.
// part[b*(J*nb) + c*J + j] = sum over this block's rows of Q[j*ld + i] w_c[i];
// each (j, c) sums its rows in the grid-stride order, as k_gemv_t_partial.
constexpr int BT_VECS = 4;

__global__ __launch_bounds__(VT) void k_gemm_tn_partial(const double *__restrict__ Q, int64_t ld,
                                                        int J, const double *__restrict__ W,
                                                        int64_t ldw, int nb, int64_t n,
                                                        double *__restrict__ part) {
  constexpr int NS = GT_COLS * BT_VECS;
  static_assert(NS == 32, "the halving exchanges below take 32 values to one per lane pair");
  __shared__ double sh[VT / 64][NS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j0 = 0; j0 < J; j0 += GT_COLS) {
    const int cnt = min(GT_COLS, J - j0);
    const double *Qj = Q + (int64_t)j0 * ld;
    double s[GT_COLS][BT_VECS];
#pragma unroll
    for (int q = 0; q < GT_COLS; ++q)
#pragma unroll
      for (int c = 0; c < BT_VECS; ++c) s[q][c] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VT) {
      double wv[BT_VECS], qv[GT_COLS];
#pragma unroll
      for (int c = 0; c < BT_VECS; ++c) wv[c] = c < nb ? W[c * ldw + i] : 0.0;
#pragma unroll
      for (int q = 0; q < GT_COLS; ++q) qv[q] = q < cnt ? Qj[q * ld + i] : 0.0;
#pragma unroll
      for (int q = 0; q < GT_COLS; ++q)
#pragma unroll
        for (int c = 0; c < BT_VECS; ++c) s[q][c] += qv[q] * wv[c];
    }
    // wave sums of the NS = 32 values by halving exchanges: at offset o
    // (32, 16, .., 2) a lane keeps the half of its values selected by lane
    // bit o and adds the partner's copy of it, so after five steps lane l
    // holds value l >> 1 summed over its 32 partners; offset 1 adds the pair.
    // 32 shuffles per lane instead of 6 per value.
    double v[NS];
#pragma unroll
    for (int q = 0; q < GT_COLS; ++q)
#pragma unroll
      for (int c = 0; c < BT_VECS; ++c) v[q * BT_VECS + c] = s[q][c];
#pragma unroll
    for (int h = NS / 2, o = 32; h >= 1; h >>= 1, o >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const double mine = up ? v[h + k] : v[k];
        const double give = up ? v[k] : v[h + k];
        v[k] = mine + __shfl_xor(give, o);
      }
    }
    v[0] += __shfl_xor(v[0], 1);
    __syncthreads();   // the previous group's sums have been read
    if ((lane & 1) == 0) sh[wave][lane >> 1] = v[0];
    __syncthreads();
    if (threadIdx.x < NS) {
      const int q = threadIdx.x / BT_VECS, c = threadIdx.x % BT_VECS;
      if (q < cnt && c < nb) {
        double t = 0.0;
        for (int k = 0; k < VT / 64; ++k) t += sh[k][threadIdx.x];
        part[(int64_t)blockIdx.x * J * nb + (int64_t)c * J + j0 + q] = t;
      }
    }
  }
}

// w_c[i] -= sum_j Q[j*ld + i] C[c*ldc + j] for c < nb <= BT_VECS, the terms of
// each vector added in the order of j, as k_gemv_n_sub.
__global__ __launch_bounds__(VT) void k_gemm_n_sub(const double *__restrict__ Q, int64_t ld,
                                                   int J, const double *__restrict__ C, int ldc,
                                                   double *__restrict__ W, int64_t ldw, int nb,
                                                   int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    double s[BT_VECS];
#pragma unroll
    for (int c = 0; c < BT_VECS; ++c) s[c] = 0.0;
    for (int j0 = 0; j0 < J; j0 += GT_COLS) {
      const int cnt = min(GT_COLS, J - j0);
      double qv[GT_COLS];
#pragma unroll
      for (int q = 0; q < GT_COLS; ++q)
        qv[q] = q < cnt ? Q[(int64_t)(j0 + q) * ld + i] : 0.0;
#pragma unroll
      for (int q = 0; q < GT_COLS; ++q)
        if (q < cnt) {
#pragma unroll
          for (int c = 0; c < BT_VECS; ++c)
            if (c < nb) s[c] += qv[q] * C[c * ldc + j0 + q];
        }
    }
#pragma unroll
    for (int c = 0; c < BT_VECS; ++c)
      if (c < nb) W[c * ldw + i] -= s[c];
  }
}

// out[c*n + i] = sum_j Q[j*ld + i] Z[sel[c]*J + j]   (Ritz vectors, sorted order)
__global__ __launch_bounds__(VT) void k_ritz(const double *__restrict__ Q, int64_t ld, int J,
                                             const double *__restrict__ Z,
                                             const int *__restrict__ sel, int k, int64_t n,
                                             double *__restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    for (int c = 0; c < k; ++c) {
      const double *z = Z + (int64_t)sel[c] * J;
      double s = 0.0;
      for (int j = 0; j < J; ++j) s += Q[j * ld + i] * z[j];
      out[(int64_t)c * n + i] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Symmetric tridiagonal eigensolver on the device: implicit QL with shifts
// (the tql2 algorithm of Bowdler, Martin, Reinsch and Wilkinson).
// k_tridiag_ql: one thread runs the QL sweeps on (diag, off) held in LDS and
// records every plane rotation (i, c, s) in order.  k_tridiag_apply: each
// thread owns one row of the identity and applies the whole rotation sequence
// to it, which yields that row of the eigenvector matrix.  Output: eval[J]
// (unsorted), Z[col*J + row] = row-th component of the col-th eigenvector.
// status[0] = 0 on success, 1 if the iteration limit or the rotation buffer
// was exceeded.
// ---------------------------------------------------------------------------
constexpr int QL_MAXJ = 1024;

__global__ __launch_bounds__(64) void k_tridiag_ql(const double *__restrict__ alpha,
                                                   const double *__restrict__ beta, int J,
                                                   double *__restrict__ rot, int64_t max_rot,
                                                   int64_t *__restrict__ nrot_out,
                                                   double *__restrict__ eval,
                                                   int *__restrict__ status) {
  __shared__ double d[QL_MAXJ], e[QL_MAXJ];
  for (int i = threadIdx.x; i < J; i += 64) {
    d[i] = alpha[i];
    e[i] = (i + 1 < J) ? beta[i + 1] : 0.0;  // beta[i+1] couples i and i+1
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int64_t nr = 0;
  int st = 0;
  for (int l = 0; l < J && !st; ++l) {
    int iter = 0;
    int m;
    do {
      for (m = l; m < J - 1; ++m) {
        const double dd = fabs(d[m]) + fabs(d[m + 1]);
        if (fabs(e[m]) <= 2.220446049250313e-16 * dd) break;
      }
      if (m != l) {
        if (++iter > 60) { st = 1; break; }
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = hypot(g, 1.0);
        g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
        double s = 1.0, c = 1.0, p = 0.0;
        bool early = false;
        for (int i = m - 1; i >= l; --i) {
          const double f = s * e[i];
          const double b = c * e[i];
          r = hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] -= p;
            e[m] = 0.0;
            early = true;
            break;
          }
          s = f / r;
          c = g / r;
          g = d[i + 1] - p;
          r = (d[i] - g) * s + 2.0 * c * b;
          p = s * r;
          d[i + 1] = g + p;
          g = c * r - b;
          if (nr < max_rot) {
            rot[3 * nr] = (double)i;
            rot[3 * nr + 1] = c;
            rot[3 * nr + 2] = s;
            ++nr;
          } else {
            st = 1;
          }
        }
        if (early) continue;
        d[l] -= p;
        e[l] = g;
        e[m] = 0.0;
      }
    } while (m != l);
  }
  for (int i = 0; i < J; ++i) eval[i] = d[i];
  nrot_out[0] = nr;
  status[0] = st;
}

constexpr int QL_CHUNK = 512;

// rows [blockIdx.x*rb, +rb), one thread per row; LDS: rb*J doubles + chunk of rotations
__global__ __launch_bounds__(64) void k_tridiag_apply(const double *__restrict__ rot,
                                                      const int64_t *__restrict__ nrot_in, int J,
                                                      int rb, double *__restrict__ Z) {
  extern __shared__ double sm[];
  double *z = sm;                 // z[col*rb + r]
  double *rc = sm + (size_t)rb * J;  // 3*QL_CHUNK
  const int r = threadIdx.x;
  const int row = blockIdx.x * rb + r;
  const bool act = r < rb && row < J;
  if (act)
    for (int col = 0; col < J; ++col) z[col * rb + r] = (col == row) ? 1.0 : 0.0;
  const int64_t nr = nrot_in[0];
  for (int64_t t0 = 0; t0 < nr; t0 += QL_CHUNK) {
    const int cnt = (int)min((int64_t)QL_CHUNK, nr - t0);
    __syncthreads();
    for (int q = threadIdx.x; q < 3 * cnt; q += blockDim.x) rc[q] = rot[3 * t0 + q];
    __syncthreads();
    if (act) {
      for (int t = 0; t < cnt; ++t) {
        const int i = (int)rc[3 * t];
        const double c = rc[3 * t + 1], s = rc[3 * t + 2];
        const double f = z[(i + 1) * rb + r];
        const double zi = z[i * rb + r];
        z[(i + 1) * rb + r] = s * zi + c * f;
        z[i * rb + r] = c * zi - s * f;
      }
    }
  }
  if (act)
    for (int col = 0; col < J; ++col) Z[(int64_t)col * J + row] = z[col * rb + r];
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
struct Reducer {
  LBuf<double> part;
  int nb = 0;
  int init(int64_t n) {
    nb = (int)std::max<int64_t>(1, std::min<int64_t>(VBLOCKS, (n + VT - 1) / VT));
    return part.ensure((size_t)nb * 512 + 16);
  }
};

static int dot(nfl_plan *P, Reducer &R, const double *x, const double *y, double *out,
               int op = 0) {
  hipLaunchKernelGGL(k_dot_partial, dim3(R.nb), dim3(VT), 0, P->stream, x, y, P->n, R.part.p);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(VT), 0, P->stream, R.part.p, R.nb, out, op);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + VT - 1) / VT)); }

// w = A_E q (sorted order, FP64 in/out, FP32 NFFT)
static int apply_A64(nfl_plan *P, const double *q, double *w) {
  VecArgs a;
  a.x64 = q;
  a.y64 = w;
  return fastsum(P, IN_SORTED_F64_DINV, OUT_SORTED_F64_A, a);
}

// w = (I + tau L_s) q; fx_ready: q's bound for the deterministic spread is in
// the plan's fx_max word already (the CG direction kernels write it)
static int apply_SSL64(nfl_plan *P, double tau, const double *q, double *w,
                       bool fx_ready = false, double *dot = nullptr) {
  VecArgs a;
  a.x64 = q;
  a.y64 = w;
  a.tau = tau;
  a.fx_ready = fx_ready;
  a.dot = dot;
  return fastsum(P, IN_SORTED_F64_DINV, OUT_SORTED_F64_SSL, a);
}

// ---------------------------------------------------------------------------
// Symmetric eigensolver for the block projection: cyclic Jacobi with the
// round-robin (circle) pairing of the indices, one workgroup.  In each round
// the m/2 disjoint rotations are computed from the current matrix and then
// applied at once, first to the rows, then to the columns and to V.  The
// matrix is A = (H + H^T)/2 of the leading m x m part of H (column-major,
// leading dimension ldH); the sweeps stop when the off-diagonal Frobenius norm
// is below 1e-15 of the whole norm.  eval[m] unsorted, V[col*m + row];
// status[0] = 1 if 40 sweeps did not converge.
// ---------------------------------------------------------------------------
constexpr int JAC_THREADS = 1024, JAC_MAXM = 1024;

__device__ double jac_block_sum(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < JAC_THREADS / 64; ++k) t += sh[k];
  __syncthreads();
  return t;  // valid in every thread
}

// KSC > 0 (m <= KSC): A and V live in dynamic LDS (2 m^2 doubles) during the
// sweeps and V is copied to Vg at the end; KSC = 0: both are the global work
// arrays.  The LDS forms: KSC = 64, and KSC = 96 (144 KiB of the 160 KiB of
// LDS a workgroup may hold).
constexpr int JAC_LDS_MAXM = 64, JAC_LDS_MAXM2 = 96;

template <int KSC>
__global__ __launch_bounds__(JAC_THREADS) void k_sym_jacobi(const double *__restrict__ H,
                                                            int64_t ldH, int m,
                                                            double *__restrict__ Ag,
                                                            double *__restrict__ Vg,
                                                            double *__restrict__ eval,
                                                            int *__restrict__ status) {
  constexpr bool IN_LDS = KSC > 0;
  extern __shared__ double jac_dyn[];
  double *A = IN_LDS ? jac_dyn : Ag;
  double *V = IN_LDS ? jac_dyn + (size_t)m * m : Vg;
  __shared__ double sh[JAC_THREADS / 64];
  __shared__ double rc[JAC_MAXM / 2], rs[JAC_MAXM / 2];
  __shared__ int rp[JAC_MAXM / 2], rq[JAC_MAXM / 2];
  const int tid = threadIdx.x;
  for (int64_t idx = tid; idx < (int64_t)m * m; idx += JAC_THREADS) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    A[idx] = 0.5 * (H[(int64_t)j * ldH + i] + H[(int64_t)i * ldH + j]);
    V[idx] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  double nn = 0.0;
  for (int64_t idx = tid; idx < (int64_t)m * m; idx += JAC_THREADS) nn += A[idx] * A[idx];
  const double nrm = sqrt(jac_block_sum(nn, sh));
  const int M = m + (m & 1), npair = M / 2;
  // (pair or row, column) index spaces use the stride KS; in the LDS forms it
  // is a constant, so that splitting an index needs no division
  const int KS = IN_LDS ? KSC : m;
  int st = 1;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0;
    for (int64_t idx = tid; idx < (int64_t)KS * KS; idx += JAC_THREADS) {
      const int r = (int)(idx / KS), c = (int)(idx % KS);
      if (r < m && c < m && r != c) off += A[(int64_t)c * m + r] * A[(int64_t)c * m + r];
    }
    off = sqrt(jac_block_sum(off, sh));
    if (off <= 1e-15 * nrm) {
      st = 0;
      break;
    }
    for (int r = 0; r < M - 1; ++r) {
      for (int i = tid; i < npair; i += JAC_THREADS) {
        const int a = i == 0 ? 0 : ((i - 1 + r) % (M - 1)) + 1;
        const int bb = M - 1 - i == 0 ? 0 : ((M - 2 - i + r) % (M - 1)) + 1;
        const int p = min(a, bb), q = max(a, bb);
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = A[(int64_t)q * m + p];
          if (fabs(apq) > 1e-300) {
            const double tau = (A[(int64_t)q * m + q] - A[(int64_t)p * m + p]) / (2.0 * apq);
            const double t = fabs(tau) > 1e150
                                 ? 0.5 / tau
                                 : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        rp[i] = p;
        rq[i] = q < m ? q : -1;
        rc[i] = c;
        rs[i] = s;
      }
      __syncthreads();
      // rows p, q of A
      for (int64_t idx = tid; idx < (int64_t)npair * KS; idx += JAC_THREADS) {
        const int i = (int)(idx / KS), k = (int)(idx % KS);
        const int q = rq[i];
        if (q < 0 || k >= m) continue;
        const int p = rp[i];
        const double c = rc[i], s = rs[i];
        const double ap = A[(int64_t)k * m + p], aq = A[(int64_t)k * m + q];
        A[(int64_t)k * m + p] = c * ap - s * aq;
        A[(int64_t)k * m + q] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of A and of V
      for (int64_t idx = tid; idx < (int64_t)npair * KS; idx += JAC_THREADS) {
        const int i = (int)(idx / KS), k = (int)(idx % KS);
        const int q = rq[i];
        if (q < 0 || k >= m) continue;
        const int p = rp[i];
        const double c = rc[i], s = rs[i];
        const double ap = A[(int64_t)p * m + k], aq = A[(int64_t)q * m + k];
        A[(int64_t)p * m + k] = c * ap - s * aq;
        A[(int64_t)q * m + k] = s * ap + c * aq;
        const double vp = V[(int64_t)p * m + k], vq = V[(int64_t)q * m + k];
        V[(int64_t)p * m + k] = c * vp - s * vq;
        V[(int64_t)q * m + k] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < m; i += JAC_THREADS) eval[i] = A[(int64_t)i * m + i];
  if (IN_LDS)
    for (int64_t idx = tid; idx < (int64_t)m * m; idx += JAC_THREADS) Vg[idx] = V[idx];
  if (tid == 0) status[0] = st;
}

// ---- out = X C (X: n x a, C: a x b row-major with row length ldc >= the
// column count rounded up to TILE, zero-padded) -------------------------------
// One thread per row of X; the coefficient row C[k][j0 .. j0 + TILE) is the
// same for the whole workgroup and is read through scalar loads.
template <int TILE>
__global__ __launch_bounds__(VT) void k_rowmul(const double *__restrict__ X, int64_t ldx, int a,
                                               const double *__restrict__ C, int ldc, int b,
                                               int64_t n, double *__restrict__ out,
                                               int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x;
  if (i >= n) return;
  for (int j0 = 0; j0 < b; j0 += TILE) {
    double acc[TILE];
#pragma unroll
    for (int jj = 0; jj < TILE; ++jj) acc[jj] = 0.0;
#pragma unroll 4
    for (int k = 0; k < a; ++k) {
      const double x = X[(int64_t)k * ldx + i];
      const double *c = C + (int64_t)k * ldc + j0;
#pragma unroll
      for (int jj = 0; jj < TILE; ++jj) acc[jj] += x * c[jj];
    }
#pragma unroll
    for (int jj = 0; jj < TILE; ++jj)
      if (j0 + jj < b) out[(int64_t)(j0 + jj) * ldo + i] = acc[jj];
  }
}

int rowmul_dev(hipStream_t s, const double *X, int64_t ldx, int a, const double *C, int ldc, int b,
               int64_t n, double *out, int64_t ldo) {
  const dim3 grid((unsigned)((n + VT - 1) / VT));
  for (int c0 = 0; c0 < b; c0 += 32) {
    const int bc = std::min(32, b - c0);
    if (bc <= 16)
      hipLaunchKernelGGL(k_rowmul<16>, grid, dim3(VT), 0, s, X, ldx, a, C + c0, ldc, bc, n,
                         out + (int64_t)c0 * ldo, ldo);
    else
      hipLaunchKernelGGL(k_rowmul<32>, grid, dim3(VT), 0, s, X, ldx, a, C + c0, ldc, bc, n,
                         out + (int64_t)c0 * ldo, ldo);
  }
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int colsum(hipStream_t s, const double *part, int nb, int width, double *out) {
  hipLaunchKernelGGL(k_colsum, dim3((width + CS_E - 1) / CS_E), dim3(VT), 0, s, part, nb, width,
                     out);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int sym_eig(hipStream_t s, const double *H, int64_t ldH, int m, double *A_work, double *V,
            double *eval, int *status) {
  if (m < 1 || m > JAC_MAXM) {
    set_error("symmetric eigensolver: order outside 1..1024");
    return NFL_ERR_UNSUPPORTED;
  }
  // the larger LDS form only where the device grants its LDS (else the
  // global form)
  static const bool lds96 = [] {
    const bool ok = hipFuncSetAttribute((const void *)k_sym_jacobi<JAC_LDS_MAXM2>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        2 * JAC_LDS_MAXM2 * JAC_LDS_MAXM2 *
                                            (int)sizeof(double)) == hipSuccess;
    if (!ok) (void)hipGetLastError();
    return ok;
  }();
  const size_t dyn = (size_t)2 * m * m * sizeof(double);
  if (m <= JAC_LDS_MAXM) {
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_sym_jacobi<JAC_LDS_MAXM>, hipFuncAttributeMaxDynamicSharedMemorySize,
        2 * JAC_LDS_MAXM * JAC_LDS_MAXM * (int)sizeof(double));
    NFL_HIP(attr);
    hipLaunchKernelGGL(k_sym_jacobi<JAC_LDS_MAXM>, dim3(1), dim3(JAC_THREADS), dyn, s, H, ldH, m,
                       A_work, V, eval, status);
  } else if (m <= JAC_LDS_MAXM2 && lds96) {
    hipLaunchKernelGGL(k_sym_jacobi<JAC_LDS_MAXM2>, dim3(1), dim3(JAC_THREADS), dyn, s, H, ldH,
                       m, A_work, V, eval, status);
  } else {
    hipLaunchKernelGGL(k_sym_jacobi<0>, dim3(1), dim3(JAC_THREADS), 0, s, H, ldH, m, A_work, V,
                       eval, status);
  }
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

// h[i] += c[i], i < J (one column of the projection)
__global__ __launch_bounds__(VT) void k_add_col(double *__restrict__ h,
                                                const double *__restrict__ c, int J) {
  for (int i = blockIdx.x * VT + threadIdx.x; i < J; i += gridDim.x * VT) h[i] += c[i];
}

// Block Lanczos with full reorthogonalisation for the k largest eigenvalues of
// A_E (Section 4 with blocks of b vectors).  Column J0 + c of the basis is
// multiplied by A_E; the block's products are orthogonalised together, twice,
// against every column built so far, then each twice against the block's
// earlier new columns, and normalised into the next column (which also forms
// the QR factor of the new block).  H holds the coefficients: column J0 + c
// gets the projections in rows < J0 + b + c and the norm in row J0 + b + c,
// so the leading J x J part of H is the projection Q^T A_E Q and the b x b
// block below it the R factor of the next block.  Ritz residual of (theta, s):
// || R s_last || with s_last the last b components of s.
//
// Thick restart (restarts > 0; Wu and Simon, "Thick-restart Lanczos method for
// large symmetric eigenvalue problems", SIAM J. Matrix Anal. Appl. 2000, in its
// block form): when the basis is full and the wanted pairs have not
// converged, the l = min(J - b, max(k + b, J / 2)) leading Ritz vectors
// Q S_l replace the basis, the already orthonormalised next block follows
// them, and the projection becomes diag(theta_l) with the coupling rows
// R s_last (b x l) to that block; the iteration then continues from it.
// `maxit` is then the basis size, and products may reach
// maxit + restarts (maxit - l).
static int block_lanczos(nfl_plan *P, int k, int b, double tol, int maxit, int restarts,
                         double *evals_host, double *evecs_dev, int *iters, double *max_resid) {
  const int64_t n = P->n;
  maxit = (int)std::min<int64_t>(maxit, n - b);
  const int maxblk = maxit / b;
  if (maxblk < 1 || k > maxblk * b) {
    set_error("block lanczos: need k <= maxit and room for one block");
    return NFL_ERR_ARG;
  }
  if (restarts > 0 && maxblk * b < k + 2 * b) {
    set_error("restarted lanczos: the basis (maxit) must hold k + 2 blocks");
    return NFL_ERR_ARG;
  }
  const int mcols = maxblk * b;          // columns whose products are formed
  if (mcols > JAC_MAXM) {
    set_error("block lanczos: maxit above 1024 is not supported");
    return NFL_ERR_UNSUPPORTED;
  }
  const int64_t ld = n, ldH = mcols + b;
  LBuf<double> Q, W, H, cvec, part, Aw, Vw, ev;
  LBuf<int> st, sel;
  NFL_TRY(Q.ensure((size_t)ld * (mcols + b)));
  NFL_TRY(W.ensure((size_t)n * b));
  NFL_TRY(H.ensure((size_t)ldH * ldH));
  NFL_TRY(cvec.ensure((size_t)BT_VECS * (mcols + b)));
  Reducer R;
  NFL_TRY(R.init(n));
  NFL_TRY(part.ensure((size_t)R.nb * BT_VECS * (mcols + b)));
  NFL_TRY(Aw.ensure((size_t)mcols * mcols));
  NFL_TRY(Vw.ensure((size_t)mcols * mcols));
  NFL_TRY(ev.ensure(mcols));
  NFL_TRY(st.ensure(1));
  NFL_TRY(sel.ensure(k));
  const int ldc = (mcols + 31) & ~31;     // row length of the restart coefficients
  LBuf<double> Cr, Qt;
  if (restarts > 0) {
    NFL_TRY(Cr.ensure((size_t)mcols * ldc));
    NFL_TRY(Qt.ensure((size_t)n * mcols));
  }
  const int gb = grid_for(n);
  hipStream_t s = P->stream;
  hipLaunchKernelGGL(k_fill64, dim3(256), dim3(VT), 0, s, H.p, (int64_t)(ldH * ldH), 0.0);

  // orthogonalise w twice against the cnt columns from column `first` on,
  // adding the coefficients to hcol[first..] (hcol may be null); then
  // normalise into column first + cnt, its norm written to *nrm_dev
  auto orth_next = [&](double *w, int first, int cnt, double *hcol, double *nrm_dev) -> int {
    const double *Qf = Q.p + (int64_t)first * ld;
    for (int pass = 0; pass < 2 && cnt > 0; ++pass) {
      hipLaunchKernelGGL(k_gemv_t_partial, dim3(R.nb), dim3(VT), 0, s, Qf, ld, cnt, w, n,
                         part.p);
      hipLaunchKernelGGL(k_colsum, dim3((cnt + CS_E - 1) / CS_E), dim3(VT), 0, s, part.p, R.nb,
                         cnt, cvec.p);
      if (hcol)
        hipLaunchKernelGGL(k_add_col, dim3((cnt + VT - 1) / VT), dim3(VT), 0, s, hcol + first,
                           cvec.p, cnt);
      hipLaunchKernelGGL(k_gemv_n_sub, dim3(gb), dim3(VT), 0, s, Qf, ld, cnt, cvec.p, w, n);
    }
    NFL_TRY(dot(P, R, w, w, nrm_dev, 1));
    hipLaunchKernelGGL(k_scale_inv, dim3(gb), dim3(VT), 0, s, w, nrm_dev, n,
                       Q.p + (int64_t)(first + cnt) * ld);
    NFL_HIP(hipGetLastError());
    return NFL_OK;
  };

  // orthogonalise the products W[:, c0..c0+nv) twice against the first ncol
  // columns, BT_VECS vectors per pass over the basis, adding the coefficients
  // of vector c to column hfirst + c of H
  auto orth_block = [&](int c0, int nv, int ncol, int hfirst) -> int {
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_gemm_tn_partial, dim3(R.nb), dim3(VT), 0, s, Q.p, ld, ncol,
                         W.p + (int64_t)c0 * n, (int64_t)n, nv, n, part.p);
      hipLaunchKernelGGL(k_colsum, dim3((ncol * nv + CS_E - 1) / CS_E), dim3(VT), 0, s, part.p,
                         R.nb, ncol * nv, cvec.p);
      for (int c = 0; c < nv; ++c)
        hipLaunchKernelGGL(k_add_col, dim3((ncol + VT - 1) / VT), dim3(VT), 0, s,
                           H.p + (int64_t)(hfirst + c) * ldH, cvec.p + (int64_t)c * ncol, ncol);
      hipLaunchKernelGGL(k_gemm_n_sub, dim3(gb), dim3(VT), 0, s, Q.p, ld, ncol, cvec.p, ncol,
                         W.p + (int64_t)c0 * n, (int64_t)n, nv, n);
    }
    NFL_HIP(hipGetLastError());
    return NFL_OK;
  };

  // start block: b seeded vectors, orthonormalised
  for (int c = 0; c < b; ++c) {
    hipLaunchKernelGGL(k_start_vector, dim3(gb), dim3(VT), 0, s, W.p, P->perm.p, n,
                       (uint64_t)(c + 1));
    NFL_TRY(orth_next(W.p, 0, c, nullptr, cvec.p + (size_t)BT_VECS * (mcols + b) - 1));
  }

  std::vector<double> h_eval, h_V, h_R((size_t)b * b);
  std::vector<int> h_sel(k), order;
  int Jc = 0, since = 0, done_restarts = 0;
  int64_t nprod = 0;
  bool converged = false;
  double worst = INFINITY;
  while (Jc + b <= mcols) {
    const int J0 = Jc;
    for (int c = 0; c < b; ++c) NFL_TRY(apply_A64(P, Q.p + (int64_t)(J0 + c) * ld, W.p + (int64_t)c * n));
    // against the basis so far (the current block included), then within
    // the new block: together the two give the new block's QR factor
    for (int c0 = 0; c0 < b; c0 += BT_VECS)
      NFL_TRY(orth_block(c0, std::min(BT_VECS, b - c0), J0 + b, J0 + c0));
    for (int c = 0; c < b; ++c) {
      double *hcol = H.p + (int64_t)(J0 + c) * ldH;
      NFL_TRY(orth_next(W.p + (int64_t)c * n, J0 + b, c, hcol, hcol + J0 + b + c));
    }
    nprod += b;
    ++since;
    Jc = J0 + b;
    const bool full = Jc + b > mcols;
    const int every = Jc <= 100 ? std::max(1, 8 / b) : std::max(1, 16 / b);
    if (Jc >= k && (since % every == 0 || full)) {
      NFL_TRY(sym_eig(s, H.p, ldH, Jc, Aw.p, Vw.p, ev.p, st.p));
      h_eval.resize(Jc);
      h_V.resize((size_t)Jc * Jc);
      int h_st = 0;
      NFL_HIP(hipMemcpyAsync(h_eval.data(), ev.p, Jc * sizeof(double), hipMemcpyDeviceToHost, s));
      NFL_HIP(hipMemcpyAsync(h_V.data(), Vw.p, (size_t)Jc * Jc * sizeof(double),
                             hipMemcpyDeviceToHost, s));
      for (int c = 0; c < b; ++c)   // R: rows Jc..Jc+b-1 of columns Jc-b+c
        NFL_HIP(hipMemcpyAsync(h_R.data() + (size_t)c * b, H.p + (int64_t)(Jc - b + c) * ldH + Jc,
                               b * sizeof(double), hipMemcpyDeviceToHost, s));
      NFL_HIP(hipMemcpyAsync(&h_st, st.p, sizeof(int), hipMemcpyDeviceToHost, s));
      NFL_HIP(hipStreamSynchronize(s));
      if (h_st != 0) {
        set_error("block lanczos: Jacobi eigensolver did not converge");
        return NFL_ERR_HIP;
      }
      order.resize(Jc);
      std::iota(order.begin(), order.end(), 0);
      std::sort(order.begin(), order.end(), [&](int a, int bb) { return h_eval[a] > h_eval[bb]; });
      // coupling of Ritz vector `col` to the next block: R s_last
      auto coupling = [&](int col, int r) {
        const double *sv = h_V.data() + (size_t)col * Jc;
        double t = 0.0;
        for (int q = 0; q < b; ++q) t += h_R[(size_t)q * b + r] * sv[Jc - b + q];
        return t;
      };
      worst = 0.0;
      for (int c = 0; c < k; ++c) {
        h_sel[c] = order[c];
        double r2 = 0.0;
        for (int r = 0; r < b; ++r) {
          const double t = coupling(order[c], r);
          r2 += t * t;
        }
        worst = std::max(worst, std::sqrt(r2));
      }
      if (worst <= tol) {
        converged = true;
        break;
      }
      if (full && done_restarts < restarts) {
        // thick restart: Q[:, :l] = Q[:, :Jc] S_l, next block to columns l..l+b-1
        const int l = std::min(Jc - b, std::max(k + b, Jc / 2));
        std::vector<double> hC((size_t)Jc * ldc, 0.0);
        for (int c = 0; c < l; ++c)
          for (int j = 0; j < Jc; ++j) hC[(size_t)j * ldc + c] = h_V[(size_t)order[c] * Jc + j];
        NFL_HIP(hipMemcpyAsync(Cr.p, hC.data(), hC.size() * sizeof(double), hipMemcpyHostToDevice, s));
        NFL_TRY(rowmul_dev(s, Q.p, ld, Jc, Cr.p, ldc, l, n, Qt.p, n));
        NFL_HIP(hipMemcpyAsync(Q.p, Qt.p, (size_t)n * l * sizeof(double), hipMemcpyDeviceToDevice, s));
        NFL_HIP(hipMemcpyAsync(Q.p + (int64_t)l * ld, Q.p + (int64_t)Jc * ld,
                               (size_t)n * b * sizeof(double), hipMemcpyDeviceToDevice, s));
        // projection: diag(theta_l), coupling rows l..l+b-1 (and, by symmetry,
        // the next block's projections onto the Ritz vectors, formed anew
        // when its products are orthogonalised)
        std::vector<double> hH((size_t)ldH * l, 0.0);
        for (int c = 0; c < l; ++c) {
          hH[(size_t)c * ldH + c] = h_eval[order[c]];
          for (int r = 0; r < b; ++r) hH[(size_t)c * ldH + l + r] = coupling(order[c], r);
        }
        hipLaunchKernelGGL(k_fill64, dim3(256), dim3(VT), 0, s, H.p, (int64_t)(ldH * ldH), 0.0);
        NFL_HIP(hipMemcpyAsync(H.p, hH.data(), hH.size() * sizeof(double), hipMemcpyHostToDevice, s));
        NFL_HIP(hipGetLastError());
        NFL_HIP(hipStreamSynchronize(s));   // host arrays go out of scope
        ++done_restarts;
        since = 0;
        Jc = l;
      }
    }
  }
  for (int c = 0; c < k; ++c) evals_host[c] = 1.0 - h_eval[h_sel[c]];
  if (evecs_dev) {
    LBuf<double> Vout;
    NFL_TRY(Vout.ensure((size_t)n * k));
    NFL_HIP(hipMemcpyAsync(sel.p, h_sel.data(), k * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ritz, dim3(gb), dim3(VT), 0, s, Q.p, ld, Jc, Vw.p, sel.p, k, n, Vout.p);
    for (int c = 0; c < k; ++c)
      hipLaunchKernelGGL(k_scatter64, dim3(gb), dim3(VT), 0, s, Vout.p + (int64_t)c * n,
                         P->perm.p, n, evecs_dev + (int64_t)c * n);
    NFL_HIP(hipGetLastError());
    NFL_HIP(hipStreamSynchronize(s));
  }
  if (iters) *iters = (int)nprod;
  if (max_resid) *max_resid = worst;
  return converged ? NFL_OK : NFL_NOT_CONVERGED;
}

int lanczos(nfl_plan *P, int k, int block, double tol, int maxit, double *evals_host,
            double *evecs_dev, int *iters, double *max_resid) {
  if (block > 1 || P->opt_restarts > 0)
    return block_lanczos(P, k, block, tol, maxit, P->opt_restarts, evals_host, evecs_dev, iters,
                         max_resid);
  const int64_t n = P->n;
  maxit = (int)std::min<int64_t>(maxit, n);
  if (k < 1 || k > maxit) {
    set_error("lanczos: need 1 <= k <= min(maxit, n)");
    return NFL_ERR_ARG;
  }
  const int64_t ld = n;
  LBuf<double> Q, w, sc, cvec, part, rot, ev, Z;
  LBuf<int64_t> nrot;
  LBuf<int> st, sel;
  NFL_TRY(Q.ensure((size_t)ld * (maxit + 1)));
  NFL_TRY(w.ensure(n));
  NFL_TRY(sc.ensure(2 * (size_t)maxit + 8));  // alpha[0..maxit), beta[0..maxit]
  NFL_TRY(cvec.ensure(maxit + 1));
  Reducer R;
  NFL_TRY(R.init(n));
  NFL_TRY(part.ensure((size_t)R.nb * (maxit + 1)));
  const int64_t max_rot = (int64_t)8 * (maxit + 1) * (maxit + 1) + 4096;
  NFL_TRY(rot.ensure((size_t)(3 * max_rot)));
  NFL_TRY(ev.ensure(maxit + 1));
  NFL_TRY(Z.ensure((size_t)(maxit + 1) * (maxit + 1)));
  NFL_TRY(nrot.ensure(1));
  NFL_TRY(st.ensure(1));
  NFL_TRY(sel.ensure(k));
  double *alpha = sc.p, *beta = sc.p + maxit;  // beta[j] couples q_{j-1}, q_j
  const int gb = grid_for(n);
  hipStream_t s = P->stream;

  hipLaunchKernelGGL(k_fill64, dim3(1), dim3(VT), 0, s, sc.p, (int64_t)(2 * maxit + 8), 0.0);
  hipLaunchKernelGGL(k_start_vector, dim3(gb), dim3(VT), 0, s, w.p, P->perm.p, n, (uint64_t)1);
  NFL_TRY(dot(P, R, w.p, w.p, beta, 1));  // beta[0] = ||r|| (used only to normalise)
  hipLaunchKernelGGL(k_scale_inv, dim3(gb), dim3(VT), 0, s, w.p, beta, n, Q.p);
  hipLaunchKernelGGL(k_fill64, dim3(1), dim3(VT), 0, s, beta, (int64_t)1, 0.0);

  std::vector<double> h_eval, h_Z, h_beta(1);
  std::vector<int> h_sel(k);
  int J = 0;
  bool converged = false;
  double worst = 0.0;
  if (maxit > QL_MAXJ) {
    set_error("lanczos: maxit above 1024 is not supported");
    return NFL_ERR_UNSUPPORTED;
  }
  for (int j = 0; j < maxit; ++j) {
    const double *qj = Q.p + (int64_t)j * ld;
    NFL_TRY(apply_A64(P, qj, w.p));
    NFL_TRY(dot(P, R, qj, w.p, alpha + j));
    hipLaunchKernelGGL(k_lanczos_sub, dim3(gb), dim3(VT), 0, s, w.p, qj,
                       j > 0 ? Q.p + (int64_t)(j - 1) * ld : (const double *)nullptr, alpha + j,
                       beta + j, n);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_gemv_t_partial, dim3(R.nb), dim3(VT), 0, s, Q.p, ld, j + 1, w.p, n,
                         part.p);
      hipLaunchKernelGGL(k_colsum, dim3((j + 1 + CS_E - 1) / CS_E), dim3(VT), 0, s, part.p, R.nb,
                         j + 1, cvec.p);
      hipLaunchKernelGGL(k_gemv_n_sub, dim3(gb), dim3(VT), 0, s, Q.p, ld, j + 1, cvec.p, w.p, n);
    }
    NFL_TRY(dot(P, R, w.p, w.p, beta + j + 1, 1));
    hipLaunchKernelGGL(k_scale_inv, dim3(gb), dim3(VT), 0, s, w.p, beta + j + 1, n,
                       Q.p + (int64_t)(j + 1) * ld);
    NFL_HIP(hipGetLastError());
    J = j + 1;
    const bool last = (J == maxit);
    const int check_every = J <= 100 ? 5 : 10;
    if (J >= k && (J % check_every == 0 || last || J == k)) {
      hipLaunchKernelGGL(k_tridiag_ql, dim3(1), dim3(64), 0, s, alpha, beta, J, rot.p, max_rot,
                         nrot.p, ev.p, st.p);
      const int rb = std::max(1, std::min(64, (int)(48000 / (8 * J))));
      const size_t zl = ((size_t)rb * J + 3 * QL_CHUNK) * sizeof(double);
      hipLaunchKernelGGL(k_tridiag_apply, dim3((J + rb - 1) / rb), dim3(64), zl, s, rot.p,
                         nrot.p, J, rb, Z.p);
      NFL_HIP(hipGetLastError());
      h_eval.resize(J);
      h_Z.resize((size_t)J * J);
      int h_st = 0;
      NFL_HIP(hipMemcpyAsync(h_eval.data(), ev.p, J * sizeof(double), hipMemcpyDeviceToHost, s));
      NFL_HIP(hipMemcpyAsync(h_Z.data(), Z.p, (size_t)J * J * sizeof(double),
                             hipMemcpyDeviceToHost, s));
      NFL_HIP(hipMemcpyAsync(h_beta.data(), beta + J, sizeof(double), hipMemcpyDeviceToHost, s));
      NFL_HIP(hipMemcpyAsync(&h_st, st.p, sizeof(int), hipMemcpyDeviceToHost, s));
      NFL_HIP(hipStreamSynchronize(s));
      if (h_st != 0) {
        set_error("lanczos: tridiagonal QL did not converge");
        return NFL_ERR_HIP;
      }
      std::vector<int> order(J);
      std::iota(order.begin(), order.end(), 0);
      std::sort(order.begin(), order.end(), [&](int a, int b) { return h_eval[a] > h_eval[b]; });
      worst = 0.0;
      for (int c = 0; c < k; ++c) {
        h_sel[c] = order[c];
        const double res = std::fabs(h_beta[0] * h_Z[(size_t)order[c] * J + (J - 1)]);
        worst = std::max(worst, res);
      }
      if (worst <= tol || h_beta[0] <= 1e-300) {
        converged = true;
        break;
      }
      if (last) break;
    }
  }
  for (int c = 0; c < k; ++c) evals_host[c] = 1.0 - h_eval[h_sel[c]];  // ascending lambda
  if (evecs_dev) {
    LBuf<double> V;
    NFL_TRY(V.ensure((size_t)n * k));
    NFL_HIP(hipMemcpyAsync(sel.p, h_sel.data(), k * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ritz, dim3(gb), dim3(VT), 0, s, Q.p, ld, J, Z.p, sel.p, k, n, V.p);
    for (int c = 0; c < k; ++c)
      hipLaunchKernelGGL(k_scatter64, dim3(gb), dim3(VT), 0, s, V.p + (int64_t)c * n, P->perm.p,
                         n, evecs_dev + (int64_t)c * n);
    NFL_HIP(hipGetLastError());
    NFL_HIP(hipStreamSynchronize(s));
  }
  if (iters) *iters = J;
  if (max_resid) *max_resid = worst;
  return converged ? NFL_OK : NFL_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// CG (Section 4; the kernel-SSL system eq. ssl::system and the KRR system)
//
// The iteration runs on the device without a host round trip per step: every
// kernel of an iteration, the product's included, returns at once when the
// solve's stop flag is set, and the scalars alpha, beta and the convergence
// test are formed by the vector kernels themselves.  Reductions are fixed
// order: each block writes one partial sum; the kernel that needs the total
// sums the partials in the same tree in every block, so all blocks agree on
// the scalar and the result does not depend on scheduling.
//
// Device state: sc[0], sc[1] hold r.r by iteration parity, sc[2] = ||f||_2,
// sc[3] = (tol ||f||)^2, sc[4] the true residual norm; st[0] the stop flag
// (1 converged, 2 breakdown p.q <= 0), st[1] the iterations done.
// ---------------------------------------------------------------------------
constexpr int CG_NB = 1024;    // reduction blocks of the CG vector kernels (partials per sum)

// sum of the nb partials in a fixed tree, valid in every thread of the block
// (each thread adds its partials i, i + VT, ... in order; their loads are
// issued four at a time, so a thread waits once per four, not once per load)
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int nb,
                                               double *sh) {
  double v = 0.0;
  for (int i0 = threadIdx.x; i0 < nb; i0 += 4 * VT) {
    double t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = i0 + u * VT < nb ? part[i0 + u * VT] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) v += t[u];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < VT / 64; ++k) t += sh[k];
  return t;
}

// r = f - q (q null: r = f); p = r; partials of r.r and f.f
// The deterministic spread's input bound for the next product: max |p| over
// the block as float bits (rounded up), one atomic max per block.  The word
// was reset by the last FFT pass of the previous product.
__device__ __forceinline__ void block_absmax_to(float m, unsigned *fx_max) {
  __shared__ float wm[VT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < VT / 64; ++w) m = fmaxf(m, wm[w]);
    atomicMax(fx_max + (blockIdx.x % FX_WORDS) * FX_STRIDE, __float_as_uint(m * (1.f + 1e-6f)));
  }
}

__global__ __launch_bounds__(VT) void k_cg_start(const double *__restrict__ f,
                                                 const double *__restrict__ q, int64_t n,
                                                 double *__restrict__ r, double *__restrict__ p,
                                                 double *__restrict__ part,
                                                 unsigned *__restrict__ fx_max) {
  __shared__ double sh[VT / 64];
  double rr = 0.0, ff = 0.0;
  float mx = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    const double fi = f[i], ri = q ? fi - q[i] : fi;
    r[i] = ri;
    p[i] = ri;
    rr += ri * ri;
    ff += fi * fi;
    mx = fmaxf(mx, (float)fabs(ri));
  }
  rr = block_sum(rr, sh);
  ff = block_sum(ff, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rr;
    part[CG_NB + blockIdx.x] = ff;
  }
  if (fx_max) block_absmax_to(mx, fx_max);
}

// one block: r.r, ||f||, the tolerance, and the stop flag before the first step
__global__ __launch_bounds__(VT) void k_cg_init(const double *__restrict__ part, int nb,
                                                double tol, double *__restrict__ sc,
                                                int *__restrict__ st) {
  __shared__ double sh[VT / 64];
  const double rr = sum_partials(part, nb, sh);
  const double ff = sum_partials(part + CG_NB, nb, sh);
  if (threadIdx.x == 0) {
    const double nf = sqrt(ff), lim = (tol * nf) * (tol * nf);
    sc[0] = rr;
    sc[1] = rr;
    sc[2] = nf;
    sc[3] = lim;
    st[0] = (nf == 0.0 || rr <= lim) ? 1 : 0;
    st[1] = 0;
  }
}

// The solve's stop flag as one value for the whole block: block 0 of k_cg_dir
// (and of k_cg_step on a breakdown) writes it while other blocks of the same
// kernel may be starting, so the waves of a block read it once, together.
__device__ __forceinline__ bool cg_stopped(const int *st) {
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return s_stop != 0;
}

// partials of p.q
__global__ __launch_bounds__(VT) void k_cg_pq(const double *__restrict__ p,
                                              const double *__restrict__ q, int64_t n,
                                              const int *__restrict__ st,
                                              double *__restrict__ part) {
  if (cg_stopped(st)) return;
  __shared__ double sh[VT / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    s += p[i] * q[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// step k: alpha = r.r / p.q; u += alpha p; r -= alpha q; partials of the new r.r
// p.q is the sum of the npq partials pqp (of k_cg_pq, or of the product's
// interpolation)
__global__ __launch_bounds__(VT) void k_cg_step(double *__restrict__ u, double *__restrict__ r,
                                                const double *__restrict__ p,
                                                const double *__restrict__ q, int64_t n, int k,
                                                const double *__restrict__ sc,
                                                int *__restrict__ st,
                                                const double *__restrict__ pqp, int npq,
                                                double *__restrict__ part) {
  if (cg_stopped(st)) return;
  __shared__ double sh[VT / 64];
  const double pq = sum_partials(pqp, npq, sh);
  if (!(pq > 0.0) || !isfinite(pq)) {   // M is not positive definite on p: stop
    if (blockIdx.x == 0 && threadIdx.x == 0) st[0] = 2;
    return;
  }
  const double a = sc[k & 1] / pq;
  double s = 0.0;
  // four elements per thread at a time (stride apart, in the order a plain
  // grid-stride loop takes them), their loads issued together
  const int64_t stride = (int64_t)gridDim.x * VT;
  for (int64_t i0 = blockIdx.x * (int64_t)VT + threadIdx.x; i0 < n; i0 += 4 * stride) {
    double uu[4], pp[4], rr[4], qq[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + v * stride;
      const bool ok = i < n;
      uu[v] = ok ? u[i] : 0.0;
      pp[v] = ok ? p[i] : 0.0;
      rr[v] = ok ? r[i] : 0.0;
      qq[v] = ok ? q[i] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + v * stride;
      if (i < n) {
        u[i] = uu[v] + a * pp[v];
        const double ri = rr[v] - a * qq[v];
        r[i] = ri;
        s += ri * ri;
      }
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[CG_NB + blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) st[1] = k + 1;
}

// step k: beta = r.r_new / r.r; p = r + beta p; the new r.r and the stop test.
// Block 0 writes the flag; blocks that start after it skip the direction
// update, which no later kernel reads once the flag is set.
__global__ __launch_bounds__(VT) void k_cg_dir(double *__restrict__ p,
                                               const double *__restrict__ r, int64_t n, int k,
                                               double *__restrict__ sc, int *__restrict__ st,
                                               const double *__restrict__ part,
                                               int *__restrict__ host_st,
                                               unsigned *__restrict__ fx_max) {
  if (cg_stopped(st)) return;
  __shared__ double sh[VT / 64];
  const double rn = sum_partials(part + CG_NB, (int)gridDim.x, sh);
  const double b = rn / sc[k & 1];
  float mx = 0.f;
  // four elements per thread at a time, loads issued together (as in k_cg_step)
  const int64_t stride = (int64_t)gridDim.x * VT;
  for (int64_t i0 = blockIdx.x * (int64_t)VT + threadIdx.x; i0 < n; i0 += 4 * stride) {
    double rr[4], pp[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + v * stride;
      rr[v] = i < n ? r[i] : 0.0;
      pp[v] = i < n ? p[i] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + v * stride;
      if (i < n) {
        const double pi = rr[v] + b * pp[v];
        p[i] = pi;
        mx = fmaxf(mx, (float)fabs(pi));
      }
    }
  }
  if (fx_max) block_absmax_to(mx, fx_max);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[(k + 1) & 1] = rn;
    const int done = rn <= sc[3] ? 1 : 0;
    if (done) st[0] = 1;
    if (host_st) {
      __hip_atomic_store(host_st, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(host_st + 1, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// r = f - q with partials of r.r (true residual after the solve)
__global__ __launch_bounds__(VT) void k_cg_resid(const double *__restrict__ f,
                                                 const double *__restrict__ q, int64_t n,
                                                 double *__restrict__ part) {
  __shared__ double sh[VT / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    const double ri = f[i] - q[i];
    s += ri * ri;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(VT) void k_cg_final(const double *__restrict__ part, int nb,
                                                 double *__restrict__ sc) {
  __shared__ double sh[VT / 64];
  const double s = sum_partials(part, nb, sh);
  if (threadIdx.x == 0) sc[4] = sqrt(s);
}

// nfl_apply_A64: y = A_E x for one FP64 vector in caller order
int apply_A64_user(nfl_plan *P, const double *x, double *y) {
  const int64_t n = P->n;
  NFL_TRY(P->v64.ensure(2 * (size_t)n));
  NFL_TRY(gather64(P, x, P->v64.p));
  NFL_TRY(apply_A64(P, P->v64.p, P->v64.p + n));
  return scatter64(P, P->v64.p + n, y);
}

__global__ __launch_bounds__(VT) void k_promote(const float *__restrict__ a, int64_t n,
                                                double *__restrict__ b) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    b[i] = (double)a[i];
}

// nfl_degree64: the FP64 degrees (FP64 path) or the float ones promoted, caller order
int degree64_user(nfl_plan *P, double *d) {
  const int64_t n = P->n;
  if (P->prec == 64) return scatter64(P, P->deg64.p, d);
  NFL_TRY(P->v64.ensure(2 * (size_t)n));
  hipLaunchKernelGGL(k_promote, dim3(grid_for(n)), dim3(VT), 0, P->stream, P->deg.p, n, P->v64.p);
  NFL_HIP(hipGetLastError());
  return scatter64(P, P->v64.p, d);
}

int gather64(nfl_plan *P, const double *src, double *dst) {
  hipLaunchKernelGGL(k_gather64, dim3(grid_for(P->n)), dim3(VT), 0, P->stream, src, P->perm.p,
                     P->n, dst);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

int scatter64(nfl_plan *P, const double *src, double *dst) {
  hipLaunchKernelGGL(k_scatter64, dim3(grid_for(P->n)), dim3(VT), 0, P->stream, src, P->perm.p,
                     P->n, dst);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

// ---------------------------------------------------------------------------
// Kernel ridge regression (Section 6.3): CG on (K + beta I) alpha = f with the
// Gram matrix K = W + K(0) I of the plan's kernel.  The vectors stay in the
// caller's order: the product converts p to FP32, runs the fast summation
// with raw sums out (the kernel over K(0), diagonal included) and forms
// q = K(0) * sums + beta p in FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(VT) void k_to_f32(const double *__restrict__ x, int64_t n,
                                               float *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    y[i] = (float)x[i];
}

__global__ __launch_bounds__(VT) void k_krr_combine(const float *__restrict__ t,
                                                    const double *__restrict__ x, double s,
                                                    double beta, int64_t n,
                                                    double *__restrict__ q) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    q[i] = s * (double)t[i] + beta * x[i];
}

struct KrrOp {
  static constexpr bool fx_feed = false;
  static constexpr bool dot_feed = false;
  nfl_plan *P;
  double beta;
  float *x32, *t32;
  int operator()(const double *x, double *q, bool = false, double * = nullptr) const {
    const int gb = grid_for(P->n);
    hipLaunchKernelGGL(k_to_f32, dim3(gb), dim3(VT), 0, P->stream, x, P->n, x32);
    VecArgs a;
    a.x32 = x32;
    a.y32 = t32;
    NFL_TRY(fastsum(P, IN_USER_F32, OUT_USER_RAW, a));
    hipLaunchKernelGGL(k_krr_combine, dim3(gb), dim3(VT), 0, P->stream, t32, x, P->wscale, beta,
                       P->n, q);
    NFL_HIP(hipGetLastError());
    return NFL_OK;
  }
};

struct SslOp {
  static constexpr bool fx_feed = true;   // products take the input bound from the CG kernels
  static constexpr bool dot_feed = true;  // products can form the partials of x . Mx
  nfl_plan *P;
  double tau;
  int operator()(const double *x, double *q, bool fx_ready = false, double *dot = nullptr) const {
    return apply_SSL64(P, tau, x, q, fx_ready, dot);
  }
};

// CG iterations for M u = f on vectors f, u (u holds the start) of the plan's
// length, any fixed node order; M applied by op.  W holds the work vectors and
// device scalars (plan-owned, or carved out of a caller-free static area).
// Iterations are enqueued without waiting; the host looks at the status
// either through the plan's pinned status words one iteration behind the
// device (W.host_st set: the device never waits for the host), or, without
// them, by a copy every `check` iterations.  Iterations enqueued after the
// stop flag is set return at once in every kernel.
struct CgWork {
  double *r, *p, *q;   // n each
  double *part;        // 2 * CG_NB
  double *dot;         // DOT_PARTS_MAX: the product's partials of p.q
  double *sc;          // 8
  int *st;             // 2
  int *host_st = nullptr;          // pinned status words (iterations, converged), device-visible
  hipEvent_t *ev = nullptr;        // two events for the one-behind host check
};

static int cg_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(CG_NB, (n + VT - 1) / VT));
}

template <class Op>
static int cg_core(nfl_plan *P, const Op &op, const CgWork &W, const double *f, double *u,
                   bool u_zero, double tol, int maxit, int *iters, double *relres) {
  const int64_t n = P->n;
  hipStream_t s = P->stream;
  const int nb = cg_blocks(n);
  if (!u_zero) NFL_TRY(op(u, W.q));   // r = f - M u0 (M 0 = 0: no product for a zero start)
  // the direction kernels also write the bound of the next product's input
  // for the deterministic spread (its pre-pass is then skipped)
  unsigned *fxw = (Op::fx_feed && P->opt_det && P->prec == 32) ? P->fx_max.p : nullptr;
  hipLaunchKernelGGL(k_cg_start, dim3(nb), dim3(VT), 0, s, f, u_zero ? nullptr : W.q, n, W.r,
                     W.p, W.part, fxw);
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(VT), 0, s, W.part, nb, tol, W.sc, W.st);
  NFL_HIP(hipGetLastError());
  if (W.host_st) {
    W.host_st[0] = 0;
    W.host_st[1] = 0;
  }
  struct StopGuard {
    nfl_plan *P;
    ~StopGuard() { P->stop = nullptr; }
  } guard{P};
  P->stop = W.st;   // every product kernel of the loop returns once the flag is set
  // the product's interpolation forms the partials of p.q where it can (one
  // kernel fewer per iteration), else k_cg_pq does
  int ndot = 0;
  if constexpr (Op::dot_feed) ndot = product_dot_parts(P);
  constexpr int check = 4;
  for (int k = 0; k < maxit; ++k) {
    if (ndot > 0) {
      NFL_TRY(op(W.p, W.q, fxw != nullptr, W.dot));
    } else {
      NFL_TRY(op(W.p, W.q, fxw != nullptr));
      hipLaunchKernelGGL(k_cg_pq, dim3(nb), dim3(VT), 0, s, W.p, W.q, n, W.st, W.part);
    }
    hipLaunchKernelGGL(k_cg_step, dim3(nb), dim3(VT), 0, s, u, W.r, W.p, W.q, n, k, W.sc, W.st,
                       ndot > 0 ? (const double *)W.dot : (const double *)W.part,
                       ndot > 0 ? ndot : nb, W.part);
    hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(VT), 0, s, W.p, W.r, n, k, W.sc, W.st, W.part,
                       W.host_st, fxw);
    NFL_HIP(hipGetLastError());
    if (W.host_st) {
      // wait for step k - 1 while step k is queued behind it
      NFL_HIP(hipEventRecord(W.ev[k & 1], s));
      if (k > 0) {
        NFL_HIP(hipEventSynchronize(W.ev[(k - 1) & 1]));
        if (__hip_atomic_load(&W.host_st[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
      }
    } else if ((k + 1) % check == 0 && k + 1 < maxit) {
      int h[2];
      NFL_HIP(hipMemcpyAsync(h, W.st, sizeof(h), hipMemcpyDeviceToHost, s));
      NFL_HIP(hipStreamSynchronize(s));
      if (h[0]) break;
    }
  }
  P->stop = nullptr;
  // The last direction kernel (or the start kernel, when the loop never ran a
  // product) may have left a bound for a product that was skipped; the word
  // must start from zero for the next pre-pass.
  if (fxw) NFL_TRY(fill_f32(reinterpret_cast<float *>(fxw), FX_WORDS * FX_STRIDE, 0.f, s));
  // the true residual with the same operator, when the caller asks for it
  // (one more product: a verification, not part of the iteration)
  if (relres) {
    NFL_TRY(op(u, W.q));
    hipLaunchKernelGGL(k_cg_resid, dim3(nb), dim3(VT), 0, s, f, W.q, n, W.part);
    hipLaunchKernelGGL(k_cg_final, dim3(1), dim3(VT), 0, s, W.part, nb, W.sc);
    NFL_HIP(hipGetLastError());
  }
  double h[8];
  int st[2];
  NFL_HIP(hipMemcpyAsync(h, W.sc, sizeof(h), hipMemcpyDeviceToHost, s));
  NFL_HIP(hipMemcpyAsync(st, W.st, sizeof(st), hipMemcpyDeviceToHost, s));
  NFL_HIP(hipStreamSynchronize(s));
  const double nf = h[2];
  const int it = st[1];
  const double rel = nf > 0 ? std::sqrt(h[it & 1]) / nf : 0.0;
  if (iters) *iters = it;
  if (relres) *relres = nf > 0 ? h[4] / nf : 0.0;
  if (st[0] == 2) {
    set_error("CG breakdown: p.Mp <= 0 (the system matrix is not positive definite here)");
    return NFL_NOT_CONVERGED;
  }
  return (rel <= tol || nf == 0) ? NFL_OK : NFL_NOT_CONVERGED;
}

// The plan's CG work space: r, p, q, and the sorted f and u of the SSL
// system (5 n FP64), reduction partials, scalars, the stop flag and the
// pinned status words; allocated by the first solve and kept with the plan.
static int plan_cg_work(nfl_plan *P, CgWork &W, double **f_sorted, double **u_sorted) {
  const size_t n = (size_t)P->n;
  NFL_TRY(P->cg_vec.ensure(5 * n + 2 * CG_NB + 8 + DOT_PARTS_MAX));
  NFL_TRY(P->cg_st.ensure(2));
  if (!P->cg_host) {
    void *h = nullptr;
    NFL_HIP(hipHostMalloc(&h, 64, hipHostMallocDefault));
    P->cg_host = (int *)h;
    for (int e = 0; e < 2; ++e)
      NFL_HIP(hipEventCreateWithFlags(&P->cg_ev[e], hipEventDisableTiming));
  }
  double *b = P->cg_vec.p;
  W.r = b;
  W.p = b + n;
  W.q = b + 2 * n;
  W.part = b + 5 * n;
  W.sc = W.part + 2 * CG_NB;
  W.dot = W.sc + 8;
  W.st = P->cg_st.p;
  W.host_st = P->cg_host;
  W.ev = P->cg_ev;
  if (f_sorted) *f_sorted = b + 3 * n;
  if (u_sorted) *u_sorted = b + 4 * n;
  return NFL_OK;
}

int krr_solve(nfl_plan *P, double beta, const double *f_dev, double *alpha_dev, int warm,
              double tol, int maxit, int *iters, double *relres) {
  const int64_t n = P->n;
  NFL_TRY(P->krr_x32.ensure(n));
  NFL_TRY(P->krr_t32.ensure(n));
  CgWork W;
  NFL_TRY(plan_cg_work(P, W, nullptr, nullptr));
  if (warm != NFL_WARM_USER)
    hipLaunchKernelGGL(k_fill64, dim3(grid_for(n)), dim3(VT), 0, P->stream, alpha_dev, n, 0.0);
  KrrOp op{P, beta, P->krr_x32.p, P->krr_t32.p};
  return cg_core(P, op, W, f_dev, alpha_dev, warm != NFL_WARM_USER, tol, maxit, iters, relres);
}

// The SSL system in the plan's sorted order: f and u are gathered into the
// work space, solved there, and u is scattered back to the caller's order.
static int cg_sorted(nfl_plan *P, const CgWork &W, double tau, const double *f_dev,
                     double *u_dev, double *f, double *u, int warm, double tol, int maxit,
                     int *iters, double *relres) {
  const int64_t n = P->n;
  hipStream_t s = P->stream;
  const int gb = grid_for(n);
  hipLaunchKernelGGL(k_gather64, dim3(gb), dim3(VT), 0, s, f_dev, P->perm.p, n, f);
  if (warm == NFL_WARM_USER) {
    hipLaunchKernelGGL(k_gather64, dim3(gb), dim3(VT), 0, s, u_dev, P->perm.p, n, u);
  } else if (warm == NFL_WARM_MLP) {
    NFL_TRY(mlp_warm_start(P, f, u));
  } else {
    hipLaunchKernelGGL(k_fill64, dim3(gb), dim3(VT), 0, s, u, n, 0.0);
  }
  SslOp op{P, tau};
  const int rc = cg_core(P, op, W, f, u, warm == NFL_WARM_ZERO, tol, maxit, iters, relres);
  if (rc < 0) return rc;
  hipLaunchKernelGGL(k_scatter64, dim3(gb), dim3(VT), 0, s, u, P->perm.p, n, u_dev);
  NFL_HIP(hipGetLastError());
  NFL_HIP(hipStreamSynchronize(s));
  return rc;
}

// ---------------------------------------------------------------------------
// CG without allocation: the work space of the SSL solve lives in one static
// device array, `scratch`, sized for up to NFL_CG_NOALLOC_MAX_N nodes (each
// GPU the library runs on holds its own copy until the process ends).  Host
// code never uses the array's name as an address: its device address is
// taken once per device with hipGetSymbolAddress and kept here.  All calls
// on one GPU share that GPU's array, so calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr size_t CG_SCRATCH_DOUBLES =
    5 * (size_t)NFL_CG_NOALLOC_MAX_N + 2 * CG_NB + 8 + 2 + DOT_PARTS_MAX;
static __device__ __align__(256) double scratch[CG_SCRATCH_DOUBLES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// device address of `scratch` on `dev` (looked up once per device, with that
// device current)
static int scratch_address(int dev, double **out) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
    set_error("device ordinal out of range for the static work space");
    return NFL_ERR_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    NFL_HIP(hipGetDevice(&cur));
    if (cur != dev) NFL_HIP(hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return NFL_ERR_HIP;
    }
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return NFL_OK;
}

int cg_noalloc(nfl_plan *P, double tau, const double *f_dev, double *u_dev, int warm, double tol,
               int maxit, int *iters, double *relres) {
  if (P->n > NFL_CG_NOALLOC_MAX_N) {
    set_error("nfl_cg_solve_noalloc: n exceeds NFL_CG_NOALLOC_MAX_N (the static work space)");
    return NFL_ERR_ARG;
  }
  double *b = nullptr;
  NFL_TRY(scratch_address(P->device, &b));
  const size_t n = (size_t)P->n;
  CgWork W;
  W.r = b;
  W.p = b + n;
  W.q = b + 2 * n;
  W.part = b + 5 * n;
  W.sc = W.part + 2 * CG_NB;
  W.st = reinterpret_cast<int *>(W.sc + 8);
  W.dot = W.sc + 10;
  W.host_st = nullptr;   // status read by a copy every few iterations
  W.ev = nullptr;
  return cg_sorted(P, W, tau, f_dev, u_dev, b + 3 * n, b + 4 * n, warm, tol, maxit, iters,
                   relres);
}

int cg(nfl_plan *P, double tau, const double *f_dev, double *u_dev, int warm, double tol,
       int maxit, int *iters, double *relres) {
  CgWork W;
  double *f = nullptr, *u = nullptr;
  NFL_TRY(plan_cg_work(P, W, &f, &u));
  return cg_sorted(P, W, tau, f_dev, u_dev, f, u, warm, tol, maxit, iters, relres);
}

}  // namespace nfl
