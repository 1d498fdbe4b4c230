// Internal declarations of the NFFT graph-Laplacian library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nfl.h"

namespace nfl {

// Thread-local message of the last failure (nfl_last_error()).
void set_error(const std::string &msg);

#define NFL_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      nfl::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));           \
      return e_ == hipErrorOutOfMemory ? NFL_ERR_OOM : NFL_ERR_HIP;               \
    }                                                                              \
  } while (0)

#define NFL_TRY(expr)                                                              \
  do {                                                                             \
    int rc_ = (expr);                                                              \
    if (rc_ < 0) return rc_;                                                       \
  } while (0)

// A device buffer owned by its holder (a plan, a batch, a network, a
// function): freed by release() or at destruction (hipFree waits for the
// device work still using it).  Not copyable, so no second owner exists.
template <class T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() { release(); }
  int ensure(size_t count) {
    if (count <= n && p) return NFL_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    if (count == 0) return NFL_OK;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? NFL_ERR_OOM : NFL_ERR_HIP;
    }
    n = count;
    return NFL_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// A function-local device buffer (the same ownership as DBuf).
template <class T>
using LBuf = DBuf<T>;

// One unit of spread/interp work: a contiguous range of sorted nodes inside
// one grid tile.
struct Item {
  int tile;
  int start;
  int end;
  int pad;
};

// Window polynomials: WIN_NC coefficients for each of up to WIN_MAXW offsets.
constexpr int WIN_NC = 8;   // degree 7: the float32 rounding of the coefficients already bounds the fit (~3e-8 of psi(0))
constexpr int WIN_MAXW = 16;
int window_coefficients(int m, std::vector<float> &coef);

// Window constants in grid units: psi(t) for |t| <= m, t = k - u.
struct Window {
  int m;       // cut-off
  float b;     // Kaiser-Bessel shape parameter pi (2 - 1/sigma_os), sigma_os = 2
  float mm;    // m*m
};

}  // namespace nfl

struct nfl_plan {
  int d = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  uint64_t gen = 0;             // bumped by every call that changes the plan

  // points
  int64_t n = 0;
  nfl::DBuf<float> pts_user;    // n*d, caller order
  double centre[3] = {0, 0, 0};
  double radius = 0;
  bool have_points = false;
  bool frame_only = false;      // target nodes in another plan's frame (nfl_set_points_frame): no degrees

  // options
  int opt_p = 0;                // 0 -> p = m
  int opt_tile = 4;
  int opt_chunk = 512;
  bool opt_eps_default = false;

  // kernel / NFFT parameters; sigma is the kernel parameter (Gaussian width or
  // multiquadric c), sigma_t = rho * sigma its value in the scaled
  // coordinates; the NFFT works with the kernel divided by K(0), so W and the
  // degrees come out divided by wscale = K(0) (L_s and A do not change)
  int kind = NFL_KERNEL_GAUSSIAN;
  double wscale = 1.0;
  double eps_I = 0.0;           // inner regularisation radius (Laplacian RBF kernel), scaled coordinates
  double opt_eps_I = 0.0;       // 0: p/N
  nfl::DBuf<float> ti_coef;     // T_I(r) = sum_k c_k (r / eps_I)^(2k), k < p
  nfl::DBuf<int> tile_start;    // sorted-node offset of each grid tile, ntiles + 1 entries
  int64_t ntiles = 0;
  double sigma = 0, eps_B = 0, rho = 1, sigma_t = 0;
  int N = 0, m = 0, p = 0, nos = 0, tshift = 3;
  bool have_kernel = false;
  nfl::Window win{};

  // sorted nodes
  nfl::DBuf<float4> pts;        // (frac_x, frac_y, frac_z, packed cell) sorted
  nfl::DBuf<int> perm;          // sorted position -> caller index
  nfl::DBuf<nfl::Item> items;
  int nitems = 0;
  int max_item_len = 0;
  // the tile-stationary forms' work: the sorted nodes cut into ngroups groups
  // of near-equal cost, at most one per workgroup the GPU holds at once; group
  // g is the segments gitems[goff[g] .. goff[g + 1]), each the nodes of one
  // tile inside the group (contiguous in the sort)
  nfl::DBuf<nfl::Item> gitems;
  nfl::DBuf<int> goff;
  int ngroups = 0;

  // FFT / filter
  nfl::DBuf<float> wcoef;       // window polynomials, WIN_MAXW x WIN_NC
  int opt_kernel = 0;           // 0: MFMA (tile-stationary where possible), 1: VALU, 2: MFMA per-cell runs
  bool opt_det = true;          // deterministic spread: int64 fixed-point grid (NFL_OPT_DETERMINISTIC)
  int opt_prec = 32;            // NFFT precision: 32 (production) or 64 (NFL_OPT_PRECISION)
  int prec = 32;                // the precision the current kernel was set up with
  // all-FP64 path: real grid, complex grid, FP64 node fractions, degrees,
  // filter (exact window transform) and twiddles
  nfl::DBuf<double> grid64;
  nfl::DBuf<double2> spec64;
  nfl::DBuf<double4> frac64;
  nfl::DBuf<double> deg64, dinv64, filt64;
  nfl::DBuf<double2> tw64;
  nfl::DBuf<double> v64;        // 2 n FP64: sorted in/out of nfl_apply_A64
  // bits of max |input| of the current product (pre-pass; reset by c2r), as
  // the maximum of FX_WORDS words FX_STRIDE apart
  nfl::DBuf<unsigned> fx_max;
  float fx_mult = 0.f;          // grid values <= max |input| * fx_mult (set by the spread launch)
  double win_max = 0;           // largest window value (psi(0))
  int opt_restarts = 0;         // thick restarts of nfl_lanczos_smallest (0: none)
  nfl::DBuf<float> filt;        // half spectrum, FP32
  std::vector<double> filt_host;
  nfl::DBuf<float2> tw;         // e^{-2 pi i k / nos}, k < nos/2
  nfl::DBuf<float> grid;        // nos^d real: spread output, left zero by the r2c pass
  nfl::DBuf<float> grid2;       // nos^d real: c2r output, interpolation input
  bool grid_clean = false;      // `grid` is known to be zero
  nfl::DBuf<float2> spec1, spec2;
  nfl::DBuf<float> xs32;        // n: the product's input in sorted order (tile forms)
  // d = 3: the z-lines (x, y) of the grid that some node's window touches
  // (the padded tiles of the occupied tiles).  The spread writes and the
  // interpolation reads only these; the FFT passes process only them, the
  // x-slabs holding them and the spectrum entries above them; every other
  // entry of spec1 / spec2 stays zero (spec_clean) across products.
  nfl::DBuf<int> zs_lines;      // x * nos + y of the support lines, ascending
  nfl::DBuf<int> zs_x;          // the x holding a support line, ascending
  nfl::DBuf<uint8_t> zs_map;    // nos * nos line flags, then nos x flags
  int zs_nlines = 0, zs_nx = 0;
  bool spec_clean = false;      // spec1 / spec2 are zero off the support

  // degrees (sorted order)
  nfl::DBuf<float> deg;
  nfl::DBuf<float> dinv;        // d_E^{-1/2}
  double dmin = 0, dmax = 0, dmean = 1;

  // learned warm start attached with nfl_mlp_attach
  nfl_mlp *mlp = nullptr;
  int mlp_cls = 0;

  // stage profiling: when set, fastsum records events before the grid fill,
  // after it, after the spread kernel, after the convolution, after interp
  hipEvent_t *prof_ev = nullptr;

  // CG work space, allocated by the first solve and kept: r, p, q and the
  // sorted f, u (5 n FP64), reduction partials and scalars; the stop flag and
  // iteration count; pinned status words the solver's kernels write (host
  // checks one iteration behind the device) and two events for that check
  nfl::DBuf<double> cg_vec;
  nfl::DBuf<int> cg_st;
  int *cg_host = nullptr;
  hipEvent_t cg_ev[2] = {nullptr, nullptr};
  nfl::DBuf<float> krr_x32, krr_t32;   // FP32 copies of the KRR product's input and output
  // device stop flag of a running solve: passed to every kernel of a product,
  // which returns at once when it is set (null outside a solve)
  const int *stop = nullptr;

  ~nfl_plan() {
    if (cg_host) (void)hipHostFree(cg_host);
    for (hipEvent_t e : cg_ev)
      if (e) (void)hipEventDestroy(e);
  }

  // scratch
  nfl::DBuf<float> xs;          // sorted FP32 work vector
  nfl::DBuf<float> fs;          // sorted FP32 interp output
  nfl::DBuf<double> red;        // reduction partials
  nfl::DBuf<unsigned char> tmp; // sort temporaries
};

namespace nfl {

// ---- setup (setup.hip) -------------------------------------------------------
int bbox_and_radius(nfl_plan *P);                       // sets centre, radius
int radius_about(nfl_plan *P, const double *centre, double *radius);  // max ||v - centre||
int build_sorted_nodes(nfl_plan *P);                    // keys, sort, items
int build_filter_host(nfl_plan *P);                     // filt_host (FP64)
// the half-spectrum filter (FP64); exact_window: divide by the exact transform
// of the Kaiser-Bessel function (the FP64 path) instead of that of the
// polynomial window the FP32 kernels apply
int compute_filter(int d, int N, int m, int p, double eps_B, double sigma_t,
                   std::vector<double> &out, int kind, double eps_I, bool exact_window = false);
double kb_hat_exact(double xi, int m);                 // fp64.hip
int setup64(nfl_plan *P);   // all-FP64 path (fp64.hip): buffers, fractions, filter, twiddles
int exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t len, hipStream_t s,
                       DBuf<uint32_t> &scratch, size_t scratch_off);
int radix_sort_pairs(uint32_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s,
                     DBuf<unsigned char> &tmp);

// ---- NFFT (nfft.hip) -----------------------------------------------------------
// How the spread kernel gets its input value for sorted node i, and what the
// interp kernel does with f_i (the post-operations of Alg. nfft_normalized_matvec).
enum InMode {
  IN_USER_F32 = 0,      // x[perm[i]]
  IN_USER_F32_DINV = 1, // dinv[i] * x[perm[i]]
  IN_ONES = 2,          // 1
  IN_SORTED_F32 = 3,    // xs[i]
  IN_SORTED_F64_DINV = 4, // (float)(dinv[i] * x64[i])
};
enum OutMode {
  OUT_USER_RAW = 0,     // y[perm[i]] = f
  OUT_USER_W = 1,       // y[perm[i]] = f - x[perm[i]]                 (W x)
  OUT_USER_LS = 2,      // y[perm[i]] = x - dinv (f - dinv x)          (L_s x)
  OUT_USER_A = 3,       // y[perm[i]] = dinv (f - dinv x)              (A x)
  OUT_DEGREE = 4,       // deg[i] = f - 1, dinv[i] = 1/sqrt(deg)
  OUT_SORTED_F64_A = 5, // y64[i] = dinv (f - xt), xt = (float)(dinv x64)
  OUT_SORTED_F64_SSL = 6, // y64[i] = x64 + tau (x64 - dinv (f - xt))
};

// words of the deterministic spread's input bound (128 bytes apart)
constexpr int FX_WORDS = 8, FX_STRIDE = 32;

struct VecArgs {
  // the input's bound for the deterministic spread is already in the plan's
  // fx_max word (written by the kernel that produced the input)
  bool fx_ready = false;
  // the tile spread stores the caller-order input in sorted order here for
  // the tile interpolation's output step (null: it gathers x again)
  float *xs = nullptr;
  const float *x32 = nullptr;   // caller order
  float *y32 = nullptr;         // caller order
  const double *x64 = nullptr;  // sorted order
  double *y64 = nullptr;        // sorted order
  double tau = 0;
  // OUT_SORTED_F64_SSL: per-workgroup partials of x64 . y64, written by the
  // tile interpolation (product_dot_parts of them); null: not formed
  double *dot = nullptr;
};

int spread(nfl_plan *P, int in_mode, const VecArgs &a, float *grid, bool clear = true);
// workgroups of the tile-stationary forms that the GPU holds at once for the
// plan's window and tile (0 where those forms do not apply)
int tile_group_slots(const nfl_plan *P);
// most partials a product writes into VecArgs::dot
constexpr int DOT_PARTS_MAX = 4096;
// partials of x64 . y64 that the plan's SSL product writes into VecArgs::dot
// (one per workgroup of the tile interpolation), or 0 where its kernels do
// not form them
int product_dot_parts(const nfl_plan *P);
// zero_in: the r2c pass sets the input grid to 0 as it reads it
// support: the grids are the plan's own (spread and interpolation of its nodes):
// the d = 3 passes then take only the z-line support
int convolve(nfl_plan *P, const float *gin, float *gout, bool zero_in = false, bool support = false);
int interp(nfl_plan *P, const float *grid, int in_mode, int out_mode, const VecArgs &a);
// whole fast summation with the given input/output modes (grid = plan grid)
int fastsum(nfl_plan *P, int in_mode, int out_mode, const VecArgs &a);
// the same fast summation with FP64 spread, FFT and interpolation (fp64.hip)
int fastsum64(nfl_plan *P, int in_mode, int out_mode, const VecArgs &a);
int fill_f32(float *p, int64_t n, float v, hipStream_t s);
// Near-field correction of the Laplacian RBF kernel (nearfield.hip): adds the
// contribution of sum_{||v~_i - v~_j|| <= eps_I} x~_j (K - T_I)(v~_i - v~_j) to
// the output of the given mode, as the post-operation would have done.
int near_field(nfl_plan *P, int in_mode, int out_mode, const VecArgs &a);
// The regularised kernel K_R / K(0) in the scaled coordinates (setup.hip).
struct RegKernel {
  int kind;
  double sigma_t, eps_B, eps_I;
  int p;
  double r0, alpha, k_half = 0.0;
  std::vector<double> fa, fb, ia, ib;
  RegKernel(int kind, double sigma_t, double eps_B, double eps_I, int p);
  double K(double r) const;            // the kernel itself
  double operator()(double r) const;   // K_R
};
// b_l of eq. b_l::K_RF (normalised by N^d) for l in I_N^d, axis index l mod N.
void kernel_bhat(int d, int N, const RegKernel &KR, std::vector<double> &bhat);
// Monomial coefficients of the inner polynomial T_I in (r / eps_I)^2 (setup.hip).
int inner_poly(double sigma_t, double eps_I, int p, std::vector<double> &c);
int scatter_f32(nfl_plan *P, const float *src_sorted, float *dst_user);

// ---- Krylov (krylov.hip) -------------------------------------------------------
int lanczos(nfl_plan *P, int k, int block, double tol, int maxit, double *evals_host,
            double *evecs_dev, int *iters, double *max_resid);
int cg(nfl_plan *P, double tau, const double *f_dev, double *u_dev, int warm, double tol,
       int maxit, int *iters, double *relres);
// nfl_cg_solve_noalloc: the work space in the library's static device array
int cg_noalloc(nfl_plan *P, double tau, const double *f_dev, double *u_dev, int warm, double tol,
               int maxit, int *iters, double *relres);
int krr_solve(nfl_plan *P, double beta, const double *f_dev, double *alpha_dev, int warm,
              double tol, int maxit, int *iters, double *relres);
int apply_A64_user(nfl_plan *P, const double *x_user, double *y_user);
int degree64_user(nfl_plan *P, double *d_user);
int gather64(nfl_plan *P, const double *src_user, double *dst_sorted);
int scatter64(nfl_plan *P, const double *src_sorted, double *dst_user);
// out[:, j] = sum_k X[:, k] C[k * ldc + j] for j < b (X: n x a column-major,
// leading dimension ldx; C row-major, each row readable up to the next
// multiple of 16 or 32 beyond the columns used, zero-padded; out: n x b with
// leading dimension ldo, not overlapping X).  Asynchronous on s.
int rowmul_dev(hipStream_t s, const double *X, int64_t ldx, int a, const double *C, int ldc, int b,
               int64_t n, double *out, int64_t ldo);
// out[e] = sum_{w < nb} part[w * width + e] for e < width, in a fixed order.
int colsum(hipStream_t s, const double *part, int nb, int width, double *out);
// Eigendecomposition of the symmetric part of the leading m x m block of H
// (column-major, leading dimension ldH), m <= 1024, one workgroup of cyclic
// Jacobi: eval[m] unsorted, V[col * m + row]; A_work holds m * m doubles;
// status[0] = 1 if the sweeps did not converge.  Asynchronous on s.
int sym_eig(hipStream_t s, const double *H, int64_t ldH, int m, double *A_work, double *V,
            double *eval, int *status);

// ---- Nystrom-Gaussian-NFFT (nystrom.hip) ------------------------------------
int nystrom(nfl_plan *P, const double *G_user, int64_t ldg, int L, int M, int k,
            double *evals_host, double *evecs_dev, int *m_used);

// ---- learned warm start (mlp.hip) -------------------------------------------
int mlp_warm_start(nfl_plan *P, const double *f_sorted, double *u_sorted);
// Remove plan P from the attachment list of its warm-start network, if any.
void mlp_detach_plan(nfl_plan *P);
int mlp_forward_explicit(nfl_mlp *M, int64_t B, float *out);

}  // namespace nfl
