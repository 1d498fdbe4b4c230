// Nystrom-Gaussian-NFFT eigenvalue approximation (Alg. nystrom_hybrid,
// Section 5.2): the k largest eigenpairs of A_E = D_E^{-1/2} W_E D_E^{-1/2}
// from 2L NFFT products and tall-skinny FP64 linear algebra on n x L blocks.
//
//   step 3  Y = A_E G, Q = orth(Y)
//   step 4  B1 = A_E Q, B2 = Q^T B1
//   step 5  Sigma_M, U_M: the M largest positive eigenvalues of B2
//   step 6  Qh Rh = B1 U_M
//   step 7  Uh Lambda Uh^T = Rh Sigma_M^{-1} Rh^T, V = Qh Uh
//   step 8  the k largest eigenvalues and their columns of V
//
// Blocks are column-major n x L (leading dimension n) in the plan's sorted
// node order.  QR factorisations use shifted CholeskyQR3 (Fukaya, Kannan,
// Nakatsukasa, Zhang, Yamamoto, "Shifted Cholesky QR for computing the QR
// factorization of ill-conditioned matrices", SIAM J. Sci. Comput. 2020): a
// Cholesky QR pass on the Gram matrix shifted by 11 (n L + L (L + 1)) u
// ||Y||_F^2, then two plain passes; R is the product of the three factors
// and has a positive diagonal.  Each pass is one Gram kernel (X^T X), one
// single-workgroup Cholesky with triangular inverse, and one row kernel
// X R^{-1}: three reads and one write of the block, where Householder QR
// would sweep it L times.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "nfl_internal.h"

namespace nfl {

namespace {

constexpr int NYS_MAXL = 64;     // largest L (columns of G) this build supports
constexpr int NYS_LDC = 64;      // padded row length of the small coefficient matrices
constexpr int NT = 256;

// "Positive" eigenvalue of B2 in step 5: above this fraction of the largest
// absolute eigenvalue, so that rounding noise around zero is never inverted.
constexpr double POS_REL = 1e-10;

// ---- Gram matrix C = X^T Y (X: n x a, Y: n x b, a, b <= 64) ------------------
// Each workgroup stages GR_ROWS rows of X and Y in LDS and accumulates a 4 x 4
// block of C per thread over its share of the row chunks; the partial sums
// of the workgroups are added in a fixed order by colsum (deterministic).
constexpr int GR_ROWS = 32;
constexpr int GR_PITCH = NYS_MAXL + 1;   // odd pitch: conflict-free column stores
constexpr int GR_MAXB = 1024;

__global__ __launch_bounds__(NT) void k_gram_partial(const double *__restrict__ X, int64_t ldx,
                                                     int a, const double *__restrict__ Y,
                                                     int64_t ldy, int b, int64_t n,
                                                     double *__restrict__ part) {
  __shared__ double xs[GR_ROWS * GR_PITCH];
  __shared__ double ys[GR_ROWS * GR_PITCH];
  const int t = threadIdx.x;
  const int i0 = (t & 15) * 4, j0 = (t >> 4) * 4;
  const bool active = i0 < a && j0 < b;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  const int64_t nchunks = (n + GR_ROWS - 1) / GR_ROWS;
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int64_t r0 = c * GR_ROWS;
    __syncthreads();
    for (int e = t; e < GR_ROWS * NYS_MAXL; e += NT) {
      const int r = e % GR_ROWS, col = e / GR_ROWS;
      const int64_t row = r0 + r;
      xs[r * GR_PITCH + col] = (col < a && row < n) ? X[col * ldx + row] : 0.0;
      ys[r * GR_PITCH + col] = (col < b && row < n) ? Y[col * ldy + row] : 0.0;
    }
    __syncthreads();
    if (active) {
      for (int r = 0; r < GR_ROWS; ++r) {
        double x[4], y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[q] = xs[r * GR_PITCH + i0 + q];
          y[q] = ys[r * GR_PITCH + j0 + q];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] += x[p] * y[q];
      }
    }
  }
  if (!active) return;
  double *out = part + (int64_t)blockIdx.x * a * b;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (i0 + p < a && j0 + q < b) out[(int64_t)(j0 + q) * a + i0 + p] = acc[p][q];
}

// ---- small dense kernels (one workgroup) -------------------------------------
constexpr int SM_PITCH = NYS_MAXL + 1;

// Upper Cholesky factor R (G + s I = R^T R) of the a x a Gram matrix G
// (column-major), with s = 11 (shift_rows a + a (a + 1)) 2^-53 trace(G) when
// shift_rows > 0, else s = 0.  Outputs R column-major (zero below the
// diagonal) and R^{-1} row-major with row length ldc (zero below the diagonal
// and in columns >= a).  status[0] = 0, or j + 1 if pivot j was not positive
// (then both outputs are zero).
__global__ __launch_bounds__(NT) void k_chol(const double *__restrict__ Gm, int a,
                                             int64_t shift_rows, double *__restrict__ Rcm,
                                             double *__restrict__ Rinv, int ldc,
                                             int *__restrict__ status) {
  __shared__ double S[NYS_MAXL * SM_PITCH];   // S[r * SM_PITCH + c]
  __shared__ double rd[NYS_MAXL];             // diagonal of R
  __shared__ double shift;
  const int t = threadIdx.x;
  const int col = t & 63, rgrp = t >> 6;      // column and row group of this thread
  for (int e = t; e < a * a; e += NT) {
    const int r = e % a, c = e / a;
    S[r * SM_PITCH + c] = Gm[e];
  }
  __syncthreads();
  if (t == 0) {
    double sh = 0.0;
    if (shift_rows > 0) {
      double tr = 0.0;
      for (int i = 0; i < a; ++i) tr += S[i * SM_PITCH + i];
      sh = 11.0 * ((double)shift_rows * a + (double)a * (a + 1)) * 0x1p-53 * tr;
    }
    shift = sh;
  }
  __syncthreads();
  for (int i = t; i < a; i += NT) S[i * SM_PITCH + i] += shift;
  __syncthreads();
  // Step j reads the pivot d = S[j][j] (the same value in every thread, so a
  // failure is seen by all), updates the trailing block with the unscaled row
  // j (S[r][c] -= S[j][r] S[j][c] / d, j < r <= c) and, in the same phase,
  // scales the previous row into row j-1 of R; one barrier per step.
  int fail = 0;
  for (int j = 0; j < a; ++j) {
    const double d = S[j * SM_PITCH + j];
    if (!(d > 0.0) || !isfinite(d)) {
      fail = j + 1;
      break;
    }
    if (t == 0) rd[j] = sqrt(d);
    if (j > 0 && rgrp == 0 && col > j - 1 && col < a)
      S[(j - 1) * SM_PITCH + col] /= sqrt(S[(j - 1) * SM_PITCH + (j - 1)]);
    if (col > j && col < a) {
      const double sjc = S[j * SM_PITCH + col] / d;
      for (int r = j + 1 + rgrp; r <= col; r += NT / 64)
        S[r * SM_PITCH + col] -= S[j * SM_PITCH + r] * sjc;
    }
    __syncthreads();
  }
  if (fail) {
    for (int e = t; e < a * a; e += NT) Rcm[e] = 0.0;
    for (int e = t; e < a * ldc; e += NT) Rinv[e] = 0.0;
    if (t == 0) status[0] = fail;
    return;
  }
  // R[r][c] = S[r][c] (r < c), rd[r] (r == c)
  for (int e = t; e < a * a; e += NT) {
    const int r = e % a, c = e / a;
    Rcm[e] = r < c ? S[r * SM_PITCH + c] : (r == c ? rd[r] : 0.0);
  }
  // column c of R^{-1} by back substitution, bottom row first, kept in LDS:
  // X[r][c] (r < c) at S[c][r] (the lower triangle, unused by R), X[c][c] in xd
  __shared__ double xd[NYS_MAXL];
  for (int c = t; c < a; c += NT) {
    const double xc = 1.0 / rd[c];
    xd[c] = xc;
    for (int r = c - 1; r >= 0; --r) {
      double sum = S[r * SM_PITCH + c] * xc;
      for (int k = r + 1; k < c; ++k) sum += S[r * SM_PITCH + k] * S[c * SM_PITCH + k];
      S[c * SM_PITCH + r] = -sum / rd[r];
    }
  }
  __syncthreads();
  for (int e = t; e < a * ldc; e += NT) {
    const int r = e / ldc, c = e % ldc;
    double v = 0.0;
    if (c < a) v = r < c ? S[c * SM_PITCH + r] : (r == c ? xd[c] : 0.0);
    Rinv[e] = v;
  }
  if (t == 0) status[0] = 0;
}

// Rout = R Rin for upper-triangular a x a matrices (column-major).
__global__ __launch_bounds__(NT) void k_trmul(const double *__restrict__ R,
                                              const double *__restrict__ Rin, int a,
                                              double *__restrict__ Rout) {
  for (int e = threadIdx.x; e < a * a; e += NT) {
    const int r = e % a, c = e / a;
    double s = 0.0;
    for (int k = r; k <= c; ++k) s += R[(int64_t)k * a + r] * Rin[(int64_t)c * a + k];
    Rout[e] = s;
  }
}

// C[k * ldc + c] = V[sel[c] * m + k] for c < nsel (the selected eigenvectors
// of an m x m problem as coefficient columns), 0 for nsel <= c < ldc.
__global__ __launch_bounds__(NT) void k_select_cols(const double *__restrict__ V, int m,
                                                    const int *__restrict__ sel, int nsel,
                                                    double *__restrict__ C, int ldc) {
  for (int e = threadIdx.x; e < m * ldc; e += NT) {
    const int k = e / ldc, c = e % ldc;
    C[e] = c < nsel ? V[(int64_t)sel[c] * m + k] : 0.0;
  }
}

// T = Rh Sigma^{-1} Rh^T (step 7): T[i][j] = sum_{k >= max(i, j)} Rh[i][k]
// Rh[j][k] / ev[sel[k]], Rh upper-triangular column-major, T column-major.
__global__ __launch_bounds__(NT) void k_rsr(const double *__restrict__ Rh,
                                            const double *__restrict__ ev,
                                            const int *__restrict__ sel, int m,
                                            double *__restrict__ T) {
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int i = e % m, j = e / m;
    double s = 0.0;
    for (int k = std::max(i, j); k < m; ++k)
      s += Rh[(int64_t)k * m + i] * Rh[(int64_t)k * m + j] / ev[sel[k]];
    T[e] = s;
  }
}

struct NysWork {
  LBuf<double> part, Gm, Rcm, Racc[2], Rinv, Csel, Aw, Vw, ev, ev2, T;
  LBuf<int> st, sel, sel2;
  int init(int64_t n, int L) {
    const int64_t nchunks = (n + GR_ROWS - 1) / GR_ROWS;
    const int nb = (int)std::min<int64_t>(GR_MAXB, nchunks);
    NFL_TRY(part.ensure((size_t)nb * L * L));
    NFL_TRY(Gm.ensure((size_t)L * L));
    NFL_TRY(Rcm.ensure((size_t)L * L));
    NFL_TRY(Racc[0].ensure((size_t)L * L));
    NFL_TRY(Racc[1].ensure((size_t)L * L));
    NFL_TRY(Rinv.ensure((size_t)L * NYS_LDC));
    NFL_TRY(Csel.ensure((size_t)L * NYS_LDC));
    NFL_TRY(Aw.ensure((size_t)L * L));
    NFL_TRY(Vw.ensure((size_t)L * L));
    NFL_TRY(ev.ensure(L));
    NFL_TRY(ev2.ensure(L));
    NFL_TRY(T.ensure((size_t)L * L));
    NFL_TRY(st.ensure(8));
    NFL_TRY(sel.ensure(L));
    NFL_TRY(sel2.ensure(L));
    return NFL_OK;
  }
};

int gram(nfl_plan *P, NysWork &W, const double *X, int a, const double *Y, int b, double *C) {
  const int64_t n = P->n;
  const int nb = (int)std::min<int64_t>(GR_MAXB, (n + GR_ROWS - 1) / GR_ROWS);
  hipLaunchKernelGGL(k_gram_partial, dim3(nb), dim3(NT), 0, P->stream, X, n, a, Y, n, b, n,
                     W.part.p);
  NFL_HIP(hipGetLastError());
  return colsum(P->stream, W.part.p, nb, a * b, C);
}

int rowmul(nfl_plan *P, const double *X, int a, const double *C, int ldc, int b, double *out) {
  return rowmul_dev(P->stream, X, P->n, a, C, ldc, b, P->n, out, P->n);
}

// Shifted CholeskyQR3 of the n x a block X (overwritten), with T as the second
// buffer.  *Q receives the orthonormal factor (it ends in T); when R is
// wanted, *R receives the product of the three triangular factors.  Pivot
// failures are reported in status[0..2] (read by the caller after a sync).
int cholqr3(nfl_plan *P, NysWork &W, double *X, double *T, int a, double **Q, double **R,
            int *status) {
  double *src = X, *dst = T;
  int cur = 0;
  for (int pass = 0; pass < 3; ++pass) {
    NFL_TRY(gram(P, W, src, a, src, a, W.Gm.p));
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(NT), 0, P->stream, W.Gm.p, a,
                       pass == 0 ? P->n : (int64_t)0, W.Rcm.p, W.Rinv.p, NYS_LDC, status + pass);
    NFL_TRY(rowmul(P, src, a, W.Rinv.p, NYS_LDC, a, dst));
    if (R) {
      if (pass == 0) {
        NFL_HIP(hipMemcpyAsync(W.Racc[0].p, W.Rcm.p, (size_t)a * a * sizeof(double),
                               hipMemcpyDeviceToDevice, P->stream));
      } else {
        hipLaunchKernelGGL(k_trmul, dim3(1), dim3(NT), 0, P->stream, W.Rcm.p, W.Racc[cur].p, a,
                           W.Racc[cur ^ 1].p);
        cur ^= 1;
      }
    }
    NFL_HIP(hipGetLastError());
    std::swap(src, dst);
  }
  *Q = src;
  if (R) *R = W.Racc[cur].p;
  return NFL_OK;
}

int apply_A_sorted(nfl_plan *P, const double *q, double *w) {
  VecArgs va;
  va.x64 = q;
  va.y64 = w;
  return fastsum(P, IN_SORTED_F64_DINV, OUT_SORTED_F64_A, va);
}

}  // namespace

int nystrom(nfl_plan *P, const double *G_user, int64_t ldg, int L, int M, int k,
            double *evals_host, double *evecs_dev, int *m_used) {
  const int64_t n = P->n;
  if (L > NYS_MAXL) {
    set_error("nystrom: L above 64 is not supported");
    return NFL_ERR_UNSUPPORTED;
  }
  hipStream_t s = P->stream;
  LBuf<double> B[3];
  for (auto &b : B) NFL_TRY(b.ensure((size_t)n * L));
  NysWork W;
  NFL_TRY(W.init(n, L));

  // step 3: Y = A_E G (B[1]), Q = orth(Y) (ends in B[0])
  for (int c = 0; c < L; ++c) NFL_TRY(gather64(P, G_user + (int64_t)c * ldg, B[0].p + (int64_t)c * n));
  for (int c = 0; c < L; ++c)
    NFL_TRY(apply_A_sorted(P, B[0].p + (int64_t)c * n, B[1].p + (int64_t)c * n));
  double *Q = nullptr;
  NFL_TRY(cholqr3(P, W, B[1].p, B[0].p, L, &Q, nullptr, W.st.p));
  // step 4: B1 = A_E Q (B[2]), B2 = Q^T B1
  for (int c = 0; c < L; ++c)
    NFL_TRY(apply_A_sorted(P, Q + (int64_t)c * n, B[2].p + (int64_t)c * n));
  NFL_TRY(gram(P, W, Q, L, B[2].p, L, W.Gm.p));
  // step 5: eigendecomposition of (B2 + B2^T)/2
  NFL_TRY(sym_eig(s, W.Gm.p, L, L, W.Aw.p, W.Vw.p, W.ev.p, W.st.p + 3));
  std::vector<double> theta(L);
  int hst[8] = {0};
  NFL_HIP(hipMemcpyAsync(theta.data(), W.ev.p, L * sizeof(double), hipMemcpyDeviceToHost, s));
  NFL_HIP(hipMemcpyAsync(hst, W.st.p, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
  NFL_HIP(hipStreamSynchronize(s));
  if (hst[0] || hst[1] || hst[2]) {
    set_error("nystrom: A_E G is numerically rank deficient (CholeskyQR pivot not positive)");
    return NFL_ERR_ARG;
  }
  if (hst[3]) {
    set_error("nystrom: Jacobi eigensolver did not converge on Q^T A_E Q");
    return NFL_ERR_HIP;
  }
  double amax = 0.0;
  for (double v : theta) amax = std::max(amax, std::fabs(v));
  std::vector<int> order(L);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return theta[a] > theta[b]; });
  std::vector<int> sel;
  for (int i = 0; i < M && i < L; ++i)
    if (theta[order[i]] > POS_REL * amax) sel.push_back(order[i]);
  const int Mu = (int)sel.size();
  if (Mu < k) {
    set_error("nystrom: fewer than k positive eigenvalues in Q^T A_E Q");
    return NFL_ERR_ARG;
  }
  NFL_HIP(hipMemcpyAsync(W.sel.p, sel.data(), Mu * sizeof(int), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_select_cols, dim3(1), dim3(NT), 0, s, W.Vw.p, L, W.sel.p, Mu, W.Csel.p,
                     NYS_LDC);
  // step 6: Z = B1 U_M (B[1]), Qh Rh = Z (Qh ends in B[0])
  NFL_TRY(rowmul(P, B[2].p, L, W.Csel.p, NYS_LDC, Mu, B[1].p));
  double *Qh = nullptr, *Rh = nullptr;
  NFL_TRY(cholqr3(P, W, B[1].p, B[0].p, Mu, &Qh, &Rh, W.st.p + 4));
  // step 7: eigendecomposition of Rh Sigma_M^{-1} Rh^T, V = Qh Uh
  hipLaunchKernelGGL(k_rsr, dim3(1), dim3(NT), 0, s, Rh, W.ev.p, W.sel.p, Mu, W.T.p);
  NFL_HIP(hipGetLastError());
  NFL_TRY(sym_eig(s, W.T.p, Mu, Mu, W.Aw.p, W.Vw.p, W.ev2.p, W.st.p + 7));
  std::vector<double> lam(Mu);
  NFL_HIP(hipMemcpyAsync(lam.data(), W.ev2.p, Mu * sizeof(double), hipMemcpyDeviceToHost, s));
  NFL_HIP(hipMemcpyAsync(hst + 4, W.st.p + 4, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
  NFL_HIP(hipStreamSynchronize(s));
  if (hst[4] || hst[5] || hst[6]) {
    set_error("nystrom: B1 U_M is numerically rank deficient (CholeskyQR pivot not positive)");
    return NFL_ERR_ARG;
  }
  if (hst[7]) {
    set_error("nystrom: Jacobi eigensolver did not converge on Rh Sigma^{-1} Rh^T");
    return NFL_ERR_HIP;
  }
  // step 8: the k largest
  std::vector<int> ord2(Mu);
  std::iota(ord2.begin(), ord2.end(), 0);
  std::stable_sort(ord2.begin(), ord2.end(), [&](int a, int b) { return lam[a] > lam[b]; });
  ord2.resize(k);
  for (int c = 0; c < k; ++c) evals_host[c] = lam[ord2[c]];
  if (m_used) *m_used = Mu;
  if (evecs_dev) {
    NFL_HIP(hipMemcpyAsync(W.sel2.p, ord2.data(), k * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_select_cols, dim3(1), dim3(NT), 0, s, W.Vw.p, Mu, W.sel2.p, k, W.Csel.p,
                       NYS_LDC);
    NFL_TRY(rowmul(P, Qh, Mu, W.Csel.p, NYS_LDC, k, B[2].p));
    for (int c = 0; c < k; ++c)
      NFL_TRY(scatter64(P, B[2].p + (int64_t)c * n, evecs_dev + (int64_t)c * n));
    NFL_HIP(hipStreamSynchronize(s));
  }
  return NFL_OK;
}

}  // namespace nfl
