// C-ABI of the NFFT graph-Laplacian library: argument checks, plan
// lifecycle, call order.  See include/nfl.h for the contract of every entry.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nfl_internal.h"

namespace nfl {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }



// y[i] *= s, i < n (W and degree outputs of non-Gaussian kernels: the NFFT
// works with K / K(0))
__global__ void k_scale_f32(float *__restrict__ y, int64_t n, float s) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] *= s;
}

static int scale_out(nfl_plan *P, float *y) {
  if (P->wscale == 1.0) return NFL_OK;
  const int blocks = (int)std::min<int64_t>(4096, (P->n + 255) / 256);
  hipLaunchKernelGGL(k_scale_f32, dim3(blocks), dim3(256), 0, P->stream, y, P->n, (float)P->wscale);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

__global__ void k_scale_f64(double *__restrict__ y, int64_t n, double s) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i < n) y[i] *= s;
}

static int scale_out64(nfl_plan *P, double *y) {
  if (P->wscale == 1.0) return NFL_OK;
  const int blocks = (int)((P->n + 255) / 256);
  hipLaunchKernelGGL(k_scale_f64, dim3(blocks), dim3(256), 0, P->stream, y, P->n, P->wscale);
  NFL_HIP(hipGetLastError());
  return NFL_OK;
}

static bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

static int check_vec_args(nfl_plan *P, const void *x, const void *y, int nvec, int64_t ld) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("apply before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("apply on a plan of target nodes (nfl_set_points_frame): it has no degrees"); return NFL_ERR_ORDER; }
  if (!x || !y) { set_error("null vector pointer"); return NFL_ERR_ARG; }
  if (nvec < 1) { set_error("nvec < 1"); return NFL_ERR_ARG; }
  if (ld < P->n) { set_error("ld < n"); return NFL_ERR_ARG; }
  return NFL_OK;
}

// (min, max) of the degrees: small host copy of the FP32 vector (setup only).
static int degree_stats(nfl_plan *P) {
  std::vector<float> h((size_t)P->n);
  NFL_HIP(hipMemcpyAsync(h.data(), P->deg.p, (size_t)P->n * sizeof(float), hipMemcpyDeviceToHost,
                         P->stream));
  NFL_HIP(hipStreamSynchronize(P->stream));
  double lo = INFINITY, hi = -INFINITY, sum = 0.0;
  for (float v : h) {
    lo = std::fmin(lo, (double)v);
    hi = std::fmax(hi, (double)v);
    sum += (double)v;
  }
  P->dmin = lo;
  P->dmax = hi;
  P->dmean = sum / (double)h.size();
  return NFL_OK;
}

}  // namespace nfl

using namespace nfl;

extern "C" {

int nfl_create(nfl_handle *h, int d, void *hip_stream) {
  if (!h) { set_error("null handle pointer"); return NFL_ERR_ARG; }
  *h = nullptr;
  if (d < 1 || d > 3) { set_error("d must be 1, 2 or 3"); return NFL_ERR_ARG; }
  nfl_plan *P = new (std::nothrow) nfl_plan();
  if (!P) { set_error("host allocation failed"); return NFL_ERR_OOM; }
  P->d = d;
  P->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    set_error("hipGetDevice failed");
    return NFL_ERR_HIP;
  }
  *h = P;
  return NFL_OK;
}

int nfl_destroy(nfl_handle P) {
  if (!P) return NFL_OK;
  (void)hipStreamSynchronize(P->stream);
  mlp_detach_plan(P);
  delete P;   // every device buffer of the plan is freed by its destructor
  return NFL_OK;
}

int nfl_set_option(nfl_handle P, int opt, double value) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (opt == NFL_OPT_EPS_I) {
    if (!(value >= 0 && value < 0.5)) { set_error("eps_I must be in [0, 1/2) (0 = p/N)"); return NFL_ERR_ARG; }
    ++P->gen;
    P->opt_eps_I = value;
    return NFL_OK;
  }
  if (opt == NFL_OPT_RESTARTS) {   // a solver setting: the operator is unchanged
    if (value < 0 || value > 1000 || value != std::floor(value)) { set_error("restarts must be an integer in [0, 1000]"); return NFL_ERR_ARG; }
    P->opt_restarts = (int)value;
    return NFL_OK;
  }
  ++P->gen;
  switch (opt) {
    case NFL_OPT_P:
      if (value < 0 || value > 16 || value != std::floor(value)) { set_error("p must be 0 (= m) or 1..16"); return NFL_ERR_ARG; }
      P->opt_p = (int)value;
      return NFL_OK;
    case NFL_OPT_TILE:
      if (!is_pow2((int)value) || value < 4 || value > 32) { set_error("tile must be a power of 2 in [4, 32]"); return NFL_ERR_ARG; }
      P->opt_tile = (int)value;
      return NFL_OK;
    case NFL_OPT_CHUNK:
      if (value < 64 || value > (1 << 24)) { set_error("chunk must be in [64, 2^24]"); return NFL_ERR_ARG; }
      P->opt_chunk = (int)value;
      return NFL_OK;
    case NFL_OPT_EPS_B_DEFAULT:
      P->opt_eps_default = value != 0;
      return NFL_OK;
    case NFL_OPT_PRECISION:
      if (value != 32 && value != 64) { set_error("precision must be 32 or 64"); return NFL_ERR_ARG; }
      P->opt_prec = (int)value;
      return NFL_OK;
    case NFL_OPT_DETERMINISTIC:
      if (value != 0 && value != 1) { set_error("deterministic must be 0 or 1"); return NFL_ERR_ARG; }
      P->opt_det = value != 0;
      P->grid_clean = false;   // the next spread clears the grid in the new format
      return NFL_OK;
    case NFL_OPT_KERNEL:
      if (value != 0 && value != 1 && value != 2) { set_error("kernel must be 0 (matrix cores), 1 (vector ALU) or 2 (matrix cores, per-cell runs)"); return NFL_ERR_ARG; }
      P->opt_kernel = (int)value;
      return NFL_OK;
    default:
      set_error("unknown option");
      return NFL_ERR_ARG;
  }
}

int nfl_set_points(nfl_handle P, int64_t n, const float *v_dev) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (n < 2) { set_error("need n >= 2 points"); return NFL_ERR_ARG; }
  if (n > (int64_t)1 << 30) { set_error("n above 2^30 is not supported"); return NFL_ERR_UNSUPPORTED; }
  if (!v_dev) { set_error("null point pointer"); return NFL_ERR_ARG; }
  ++P->gen;
  P->have_points = false;
  P->have_kernel = false;
  P->frame_only = false;
  P->n = n;
  NFL_TRY(P->pts_user.ensure((size_t)n * P->d));
  NFL_HIP(hipMemcpyAsync(P->pts_user.p, v_dev, (size_t)n * P->d * sizeof(float),
                         hipMemcpyDeviceToDevice, P->stream));
  NFL_TRY(bbox_and_radius(P));
  if (!std::isfinite(P->radius)) { set_error("non-finite coordinates"); return NFL_ERR_ARG; }
  P->have_points = true;
  return NFL_OK;
}

int nfl_set_points_frame(nfl_handle P, int64_t n, const float *v_dev, nfl_handle src) {
  if (!P || !src) { set_error("null handle"); return NFL_ERR_ARG; }
  if (P == src) { set_error("a plan cannot be its own frame"); return NFL_ERR_ARG; }
  if (!src->have_points || src->frame_only) { set_error("frame plan without its own points"); return NFL_ERR_ORDER; }
  if (P->d != src->d) { set_error("dimension differs from the frame plan"); return NFL_ERR_ARG; }
  if (n < 1) { set_error("need n >= 1 target points"); return NFL_ERR_ARG; }
  if (n > (int64_t)1 << 30) { set_error("n above 2^30 is not supported"); return NFL_ERR_UNSUPPORTED; }
  if (!v_dev) { set_error("null point pointer"); return NFL_ERR_ARG; }
  ++P->gen;
  P->have_points = false;
  P->have_kernel = false;
  P->frame_only = true;
  P->n = n;
  NFL_TRY(P->pts_user.ensure((size_t)n * P->d));
  NFL_HIP(hipMemcpyAsync(P->pts_user.p, v_dev, (size_t)n * P->d * sizeof(float),
                         hipMemcpyDeviceToDevice, P->stream));
  double r = 0.0;
  NFL_TRY(radius_about(P, src->centre, &r));
  if (!std::isfinite(r)) { set_error("non-finite coordinates"); return NFL_ERR_ARG; }
  if (r > src->radius * (1.0 + 1e-6)) {
    set_error("target points outside the ball of the source points (all differences must stay "
              "inside the torus of the fast summation)");
    return NFL_ERR_ARG;
  }
  for (int t = 0; t < 3; ++t) P->centre[t] = src->centre[t];
  P->radius = src->radius;
  P->have_points = true;
  return NFL_OK;
}

int nfl_evaluate(nfl_handle S, const float *x_dev, nfl_handle T, float *y_dev) {
  if (!S || !T) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!S->have_kernel || !T->have_kernel) { set_error("evaluate before a successful nfl_set_kernel on both plans"); return NFL_ERR_ORDER; }
  if (S->frame_only) { set_error("the source plan must hold its own points"); return NFL_ERR_ARG; }
  if (S->kind == NFL_KERNEL_LAPLACIAN_RBF) { set_error("evaluate: the Laplacian RBF kernel needs a near-field sum between the two node sets, not built"); return NFL_ERR_UNSUPPORTED; }
  if (S->prec == 64 || T->prec == 64) { set_error("evaluate: not built for the FP64 path"); return NFL_ERR_UNSUPPORTED; }
  if (T != S && !T->frame_only) { set_error("the target plan must be made with nfl_set_points_frame"); return NFL_ERR_ARG; }
  if (T != S && (T->centre[0] != S->centre[0] || T->centre[1] != S->centre[1] ||
                 T->centre[2] != S->centre[2] || T->radius != S->radius || T->d != S->d ||
                 T->kind != S->kind || T->sigma != S->sigma || T->N != S->N || T->m != S->m ||
                 T->p != S->p || T->eps_B != S->eps_B)) {
    set_error("target plan and source plan differ in frame or kernel parameters");
    return NFL_ERR_ARG;
  }
  if (!x_dev || !y_dev) { set_error("null vector pointer"); return NFL_ERR_ARG; }
  if (T->stream != S->stream) NFL_HIP(hipStreamSynchronize(T->stream));
  // Alg. nfft_fastsum with the adjoint NFFT at the sources and the NFFT at the
  // targets: spread (sources), filter, interpolation (targets)
  VecArgs a;
  a.x32 = x_dev;
  const bool clear = !S->grid_clean;
  S->grid_clean = false;
  NFL_TRY(spread(S, IN_USER_F32, a, S->grid.p, clear));
  NFL_TRY(convolve(S, S->grid.p, S->grid2.p, true));
  S->grid_clean = true;
  VecArgs b;
  b.y32 = y_dev;
  hipStream_t keep = T->stream;
  T->stream = S->stream;               // one stream orders the three steps
  const int rc = interp(T, S->grid2.p, IN_USER_F32, OUT_USER_RAW, b);
  T->stream = keep;
  if (rc < 0) return rc;
  if (S->wscale != 1.0) {
    const int blocks = (int)std::min<int64_t>(4096, (T->n + 255) / 256);
    hipLaunchKernelGGL(k_scale_f32, dim3(blocks), dim3(256), 0, S->stream, y_dev, T->n,
                       (float)S->wscale);
    NFL_HIP(hipGetLastError());
  }
  return NFL_OK;
}

int nfl_set_kernel(nfl_handle P, double sigma, int N, int m, double eps_B) {
  return nfl_set_kernel_ex(P, NFL_KERNEL_GAUSSIAN, sigma, N, m, eps_B);
}

int nfl_set_kernel_ex(nfl_handle P, int kind, double sigma, int N, int m, double eps_B) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_points) { set_error("set_kernel before set_points"); return NFL_ERR_ORDER; }
  if (kind < NFL_KERNEL_GAUSSIAN || kind > NFL_KERNEL_LAPLACIAN_RBF) { set_error("unknown kernel kind"); return NFL_ERR_ARG; }
  if (!(sigma > 0) || !std::isfinite(sigma)) { set_error("kernel parameter must be > 0"); return NFL_ERR_ARG; }
  if (N < 2 || (N & 1)) { set_error("N must be even and >= 2"); return NFL_ERR_ARG; }
  if (m < 1) { set_error("m must be >= 1"); return NFL_ERR_ARG; }
  const int p = P->opt_p > 0 ? P->opt_p : m;
  if (eps_B < 0 && P->opt_eps_default) eps_B = (double)p / N;
  if (!(eps_B >= 0.0 && eps_B < 0.5)) { set_error("eps_B must be in [0, 1/2)"); return NFL_ERR_ARG; }
  if (!is_pow2(N) || N < 8 || N > 256) { set_error("this build needs N a power of 2 in [8, 256]"); return NFL_ERR_UNSUPPORTED; }
  if (m < 2 || m > 8) { set_error("this build supports 2 <= m <= 8"); return NFL_ERR_UNSUPPORTED; }
  if (2 * m > N) { set_error("window wider than half the grid (need m <= N/2)"); return NFL_ERR_UNSUPPORTED; }
  ++P->gen;
  P->have_kernel = false;
  double eps_I = 0.0;
  if (kind == NFL_KERNEL_LAPLACIAN_RBF) {
    eps_I = P->opt_eps_I > 0 ? P->opt_eps_I : (double)p / N;
    if (!(eps_I + eps_B < 0.5)) { set_error("need eps_I + eps_B < 1/2"); return NFL_ERR_ARG; }
  }
  P->kind = kind;
  P->sigma = sigma;
  P->eps_I = eps_I;
  P->wscale = (kind == NFL_KERNEL_GAUSSIAN || kind == NFL_KERNEL_LAPLACIAN_RBF)
                  ? 1.0 : (kind == NFL_KERNEL_MULTIQUADRIC ? sigma : 1.0 / sigma);
  P->N = N;
  P->m = m;
  P->p = p;
  P->eps_B = eps_B;
  P->nos = 2 * N;
  P->rho = P->radius > 0 ? (0.25 - 0.5 * eps_B) / P->radius : 1.0;
  P->sigma_t = sigma * P->rho;
  P->win.m = m;
  P->win.b = (float)(M_PI * 1.5);
  P->win.mm = (float)(m * m);

  {
    std::vector<float> wc;
    NFL_TRY(window_coefficients(m, wc));
    NFL_TRY(P->wcoef.ensure(wc.size()));
    NFL_HIP(hipMemcpyAsync(P->wcoef.p, wc.data(), wc.size() * sizeof(float),
                           hipMemcpyHostToDevice, P->stream));
  }
  NFL_TRY(build_filter_host(P));
  if (kind == NFL_KERNEL_LAPLACIAN_RBF) {
    std::vector<double> c;
    NFL_TRY(inner_poly(P->sigma_t, P->eps_I, p, c));
    std::vector<float> cf(c.begin(), c.end());
    NFL_TRY(P->ti_coef.ensure(cf.size()));
    NFL_HIP(hipMemcpyAsync(P->ti_coef.p, cf.data(), cf.size() * sizeof(float),
                           hipMemcpyHostToDevice, P->stream));
  }
  NFL_TRY(P->filt.ensure(P->filt_host.size()));
  {
    std::vector<float> f32(P->filt_host.size());
    for (size_t i = 0; i < f32.size(); ++i) f32[i] = (float)P->filt_host[i];
    NFL_HIP(hipMemcpyAsync(P->filt.p, f32.data(), f32.size() * sizeof(float),
                           hipMemcpyHostToDevice, P->stream));
    std::vector<float2> tw((size_t)P->nos / 2);
    for (int k = 0; k < P->nos / 2; ++k) {
      const double a = -2.0 * M_PI * k / P->nos;
      tw[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    NFL_TRY(P->tw.ensure(tw.size()));
    NFL_HIP(hipMemcpyAsync(P->tw.p, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice,
                           P->stream));
    NFL_HIP(hipStreamSynchronize(P->stream));
  }
  int64_t gsz = 1;
  for (int t = 0; t < P->d; ++t) gsz *= P->nos;
  NFL_TRY(P->grid.ensure(2 * gsz));   // room for the int64 fixed-point grid
  NFL_TRY(P->grid2.ensure(gsz));
  P->grid_clean = false;
  NFL_TRY(P->fx_max.ensure(FX_WORDS * FX_STRIDE));
  NFL_HIP(hipMemsetAsync(P->fx_max.p, 0, FX_WORDS * FX_STRIDE * sizeof(unsigned), P->stream));
  {
    const double b = M_PI * 1.5, m = P->m;   // Kaiser-Bessel window at t = 0
    P->win_max = (std::sinh(b * m) / m) / (b * std::exp(b * m));
  }
  const int Hz = N / 2 + 1, F = N + 1;
  size_t s1 = Hz, s2 = 0;
  if (P->d == 2) s1 = (size_t)P->nos * Hz;
  if (P->d == 3) {
    s1 = (size_t)P->nos * P->nos * Hz;
    s2 = (size_t)P->nos * F * Hz;
  }
  NFL_TRY(P->spec1.ensure(s1));
  if (s2) NFL_TRY(P->spec2.ensure(s2));
  NFL_TRY(build_sorted_nodes(P));
  NFL_TRY(P->deg.ensure(P->n));
  NFL_TRY(P->dinv.ensure(P->n));
  NFL_TRY(P->xs32.ensure(P->n));
  P->prec = 32;
  if (P->opt_prec == 64) {
    NFL_TRY(setup64(P));
    P->prec = 64;
  }

  if (P->frame_only) {   // target nodes: no degree pass
    P->have_kernel = true;
    return NFL_OK;
  }
  // step 4 of Alg. nfft_normalized_matvec: D_E = diag(W~_E 1 - K(0) 1)
  VecArgs a;
  NFL_TRY(fastsum(P, IN_ONES, OUT_DEGREE, a));
  NFL_TRY(degree_stats(P));
  if (!(P->dmin > 0.0)) {
    set_error("approximate degree d_E <= 0 for some node (eps >= eta): raise N or m");
    return NFL_ERR_DEGREE;
  }
  P->have_kernel = true;
  return NFL_OK;
}

int nfl_degree(nfl_handle P, float *d_dev) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("degree before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("degree on a plan of target nodes (nfl_set_points_frame): it has no degrees"); return NFL_ERR_ORDER; }
  if (!d_dev) { set_error("null output"); return NFL_ERR_ARG; }
  NFL_TRY(scatter_f32(P, P->deg.p, d_dev));
  return scale_out(P, d_dev);
}

static int apply_common(nfl_handle P, const float *x, float *y, int nvec, int64_t ld, int in_mode,
                        int out_mode) {
  NFL_TRY(check_vec_args(P, x, y, nvec, ld));
  for (int k = 0; k < nvec; ++k) {
    VecArgs a;
    a.x32 = x + (int64_t)k * ld;
    a.y32 = y + (int64_t)k * ld;
    NFL_TRY(fastsum(P, in_mode, out_mode, a));
  }
  return NFL_OK;
}

int nfl_apply_W(nfl_handle P, const float *x, float *y, int nvec, int64_t ld) {
  NFL_TRY(apply_common(P, x, y, nvec, ld, IN_USER_F32, OUT_USER_W));
  for (int k = 0; k < nvec && P->wscale != 1.0; ++k) NFL_TRY(scale_out(P, y + (int64_t)k * ld));
  return NFL_OK;
}

int nfl_apply_Ls(nfl_handle P, const float *x, float *y, int nvec, int64_t ld) {
  return apply_common(P, x, y, nvec, ld, IN_USER_F32_DINV, OUT_USER_LS);
}

int nfl_apply_A(nfl_handle P, const float *x, float *y, int nvec, int64_t ld) {
  return apply_common(P, x, y, nvec, ld, IN_USER_F32_DINV, OUT_USER_A);
}

int nfl_apply_A64(nfl_handle P, const double *x, double *y) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("apply before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("apply_A64 on a plan of target nodes: it has no degrees"); return NFL_ERR_ORDER; }
  if (!x || !y || x == y) { set_error("null or aliased vector pointer"); return NFL_ERR_ARG; }
  return apply_A64_user(P, x, y);
}

int nfl_degree64(nfl_handle P, double *d) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("degree before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("degree on a plan of target nodes: it has no degrees"); return NFL_ERR_ORDER; }
  if (!d) { set_error("null output"); return NFL_ERR_ARG; }
  NFL_TRY(degree64_user(P, d));
  return scale_out64(P, d);
}

int nfl_lanczos_smallest(nfl_handle P, int k, int block, double tol, int maxit, double *evals_host,
                         double *evecs_dev, int *iters, double *max_resid) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("lanczos before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("lanczos on a plan of target nodes (nfl_set_points_frame): it has no degrees"); return NFL_ERR_ORDER; }
  if (!evals_host) { set_error("null eigenvalue output"); return NFL_ERR_ARG; }
  if (k < 1 || k >= P->n || maxit < k || !(tol > 0)) { set_error("need 1 <= k < n, maxit >= k, tol > 0"); return NFL_ERR_ARG; }
  if (block < 1 || block > 8) { set_error("block must be in 1..8"); return NFL_ERR_ARG; }
  return lanczos(P, k, block, tol, maxit, evals_host, evecs_dev, iters, max_resid);
}

int nfl_nystrom(nfl_handle P, const double *G_dev, int64_t ldg, int L, int M, int k,
                double *evals_host, double *evecs_dev, int *m_used) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("nystrom before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("nystrom on a plan of target nodes (nfl_set_points_frame): it has no degrees"); return NFL_ERR_ORDER; }
  if (!G_dev || !evals_host) { set_error("null G or eigenvalue output"); return NFL_ERR_ARG; }
  if (k < 1 || M < k || L < M || L > P->n) { set_error("need 1 <= k <= M <= L <= n"); return NFL_ERR_ARG; }
  if (ldg < P->n) { set_error("ldg < n"); return NFL_ERR_ARG; }
  return nystrom(P, G_dev, ldg, L, M, k, evals_host, evecs_dev, m_used);
}

int nfl_cg_solve(nfl_handle P, double tau, const double *f_dev, double *u_dev, int warm, double tol,
                 int maxit, int *iters, double *relres) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("cg before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("cg on a plan of target nodes (nfl_set_points_frame): it has no degrees"); return NFL_ERR_ORDER; }
  if (!f_dev || !u_dev) { set_error("null vector pointer"); return NFL_ERR_ARG; }
  if (!(tau >= 0) || !(tol > 0) || maxit < 0) { set_error("need tau >= 0, tol > 0, maxit >= 0"); return NFL_ERR_ARG; }
  if (warm < NFL_WARM_ZERO || warm > NFL_WARM_MLP) { set_error("bad warm-start mode"); return NFL_ERR_ARG; }
  return cg(P, tau, f_dev, u_dev, warm, tol, maxit, iters, relres);
}

int nfl_cg_solve_noalloc(nfl_handle P, double tau, const double *f_dev, double *u_dev, int warm,
                         double tol, int maxit, int *iters, double *relres) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("cg before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("cg on a plan of target nodes (nfl_set_points_frame): it has no degrees"); return NFL_ERR_ORDER; }
  if (!f_dev || !u_dev) { set_error("null vector pointer"); return NFL_ERR_ARG; }
  if (!(tau >= 0) || !(tol > 0) || maxit < 0) { set_error("need tau >= 0, tol > 0, maxit >= 0"); return NFL_ERR_ARG; }
  if (warm != NFL_WARM_ZERO && warm != NFL_WARM_USER) { set_error("nfl_cg_solve_noalloc: warm start NFL_WARM_ZERO or NFL_WARM_USER"); return NFL_ERR_ARG; }
  return cg_noalloc(P, tau, f_dev, u_dev, warm, tol, maxit, iters, relres);
}

int nfl_krr_solve(nfl_handle P, double beta, const double *f_dev, double *alpha_dev, int warm,
                  double tol, int maxit, int *iters, double *relres) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("krr before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (P->frame_only) { set_error("krr on a plan of target nodes (nfl_set_points_frame): it has no degrees"); return NFL_ERR_ORDER; }
  if (!f_dev || !alpha_dev) { set_error("null vector pointer"); return NFL_ERR_ARG; }
  if (!(beta >= 0) || !std::isfinite(beta) || !(tol > 0) || maxit < 0) { set_error("need beta >= 0, tol > 0, maxit >= 0"); return NFL_ERR_ARG; }
  if (warm != NFL_WARM_ZERO && warm != NFL_WARM_USER) { set_error("krr warm start: NFL_WARM_ZERO or NFL_WARM_USER"); return NFL_ERR_ARG; }
  return krr_solve(P, beta, f_dev, alpha_dev, warm, tol, maxit, iters, relres);
}

int nfl_get_info(nfl_handle P, double *rho, double *sigma_tilde, double *dmin, double *dmax,
                 double *eps_B, int *p) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("info before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (rho) *rho = P->rho;
  if (sigma_tilde) *sigma_tilde = P->sigma_t;
  if (dmin) *dmin = P->dmin * P->wscale;
  if (dmax) *dmax = P->dmax * P->wscale;
  if (eps_B) *eps_B = P->eps_B;
  if (p) *p = P->p;
  return NFL_OK;
}

int64_t nfl_grid_size(nfl_handle P) {
  if (!P || P->nos == 0) return 0;
  int64_t g = 1;
  for (int t = 0; t < P->d; ++t) g *= P->nos;
  return g;
}

int nfl_spread(nfl_handle P, const float *x_dev, float *grid_dev) {
  NFL_TRY(check_vec_args(P, x_dev, grid_dev, 1, P ? P->n : 0));
  VecArgs a;
  a.x32 = x_dev;
  return spread(P, IN_USER_F32, a, grid_dev);
}

int nfl_convolve(nfl_handle P, const float *gin, float *gout) {
  NFL_TRY(check_vec_args(P, gin, gout, 1, P ? P->n : 0));
  return convolve(P, gin, gout);
}

int nfl_interp(nfl_handle P, const float *grid_dev, float *f_dev) {
  NFL_TRY(check_vec_args(P, grid_dev, f_dev, 1, P ? P->n : 0));
  VecArgs a;
  a.y32 = f_dev;
  return interp(P, grid_dev, IN_USER_F32, OUT_USER_RAW, a);
}

int nfl_get_filter(nfl_handle P, double *filter_host, int64_t count) {
  if (!P) { set_error("null handle"); return NFL_ERR_ARG; }
  if (!P->have_kernel) { set_error("filter before a successful nfl_set_kernel"); return NFL_ERR_ORDER; }
  if (!filter_host || count < (int64_t)P->filt_host.size()) { set_error("filter buffer too small"); return NFL_ERR_ARG; }
  std::memcpy(filter_host, P->filt_host.data(), P->filt_host.size() * sizeof(double));
  return NFL_OK;
}

int nfl_compute_filter(int d, int N, int m, int p, double eps_B, double sigma_tilde,
                       double *filter_host, int64_t count) {
  return nfl_compute_filter_ex(NFL_KERNEL_GAUSSIAN, d, N, m, p, eps_B, sigma_tilde, 0.0,
                               filter_host, count);
}

int nfl_compute_filter_ex(int kind, int d, int N, int m, int p, double eps_B, double sigma_tilde,
                          double eps_I, double *filter_host, int64_t count) {
  if (!filter_host) { set_error("null output"); return NFL_ERR_ARG; }
  if (kind < NFL_KERNEL_GAUSSIAN || kind > NFL_KERNEL_LAPLACIAN_RBF) { set_error("unknown kernel kind"); return NFL_ERR_ARG; }
  if (kind == NFL_KERNEL_LAPLACIAN_RBF && !(eps_I > 0 && eps_I + eps_B < 0.5)) { set_error("need 0 < eps_I, eps_I + eps_B < 1/2"); return NFL_ERR_ARG; }
  if (d < 1 || d > 3 || N < 2 || (N & 1) || !is_pow2(N) || m < 1 || p < 1 ||
      !(eps_B >= 0 && eps_B < 0.5) || !(sigma_tilde > 0)) {
    set_error("bad filter arguments");
    return NFL_ERR_ARG;
  }
  std::vector<double> f;
  NFL_TRY(compute_filter(d, N, m, p, eps_B, sigma_tilde, f, kind, eps_I));
  if (count < (int64_t)f.size()) { set_error("filter buffer too small"); return NFL_ERR_ARG; }
  std::memcpy(filter_host, f.data(), f.size() * sizeof(double));
  return NFL_OK;
}

int nfl_profile_stages(nfl_handle P, const float *x_dev, float *y_dev, int nrep,
                       double *stage_ms) {
  NFL_TRY(check_vec_args(P, x_dev, y_dev, 1, P ? P->n : 0));
  if (nrep < 1 || !stage_ms) { set_error("need nrep >= 1 and an output array"); return NFL_ERR_ARG; }
  std::vector<hipEvent_t> ev((size_t)nrep * 5);
  for (auto &e : ev) NFL_HIP(hipEventCreate(&e));
  int rc = NFL_OK;
  for (int r = 0; r < nrep && rc == NFL_OK; ++r) {
    P->prof_ev = ev.data() + (size_t)r * 5;
    VecArgs a;
    a.x32 = x_dev;
    a.y32 = y_dev;
    rc = fastsum(P, IN_USER_F32_DINV, OUT_USER_LS, a);
  }
  P->prof_ev = nullptr;
  if (rc == NFL_OK && hipStreamSynchronize(P->stream) != hipSuccess) rc = NFL_ERR_HIP;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int r = 0; r < nrep && rc == NFL_OK; ++r) {
    hipEvent_t *e = ev.data() + (size_t)r * 5;
    for (int s = 0; s < 4; ++s) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e[s], e[s + 1]) != hipSuccess) { rc = NFL_ERR_HIP; break; }
      acc[s] += ms;
    }
    float tot = 0.f;
    if (hipEventElapsedTime(&tot, e[0], e[4]) != hipSuccess) rc = NFL_ERR_HIP;
    acc[4] += tot;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (rc != NFL_OK) { set_error("nfl_profile_stages: event timing failed"); return rc; }
  for (int s = 0; s < 5; ++s) stage_ms[s] = acc[s] / nrep;
  return NFL_OK;
}

int nfl_window_coefficients(int m, float *coef_host, int64_t count) {
  if (!coef_host || m < 1 || 2 * m > WIN_MAXW) { set_error("need 1 <= m <= 8 and an output"); return NFL_ERR_ARG; }
  std::vector<float> wc;
  NFL_TRY(window_coefficients(m, wc));
  const int64_t need = (int64_t)2 * m * WIN_NC;
  if (count < need) { set_error("coefficient buffer too small"); return NFL_ERR_ARG; }
  std::memcpy(coef_host, wc.data(), need * sizeof(float));
  return NFL_OK;
}

const char *nfl_strerror(int code) {
  switch (code) {
    case NFL_OK: return "ok";
    case NFL_NOT_CONVERGED: return "not converged (outputs hold the last iterate)";
    case NFL_ERR_ARG: return "invalid argument";
    case NFL_ERR_ORDER: return "call order (set_points / set_kernel first)";
    case NFL_ERR_DEGREE: return "approximate degree <= 0 (eps >= eta)";
    case NFL_ERR_HIP: return "HIP runtime error";
    case NFL_ERR_OOM: return "out of device memory";
    case NFL_ERR_UNSUPPORTED: return "unsupported by this build";
    default: return "unknown error code";
  }
}

const char *nfl_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

