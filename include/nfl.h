/*
 * nfl.h -- NFFT fast summation for the graph Laplacian of a fully connected
 * Gaussian graph, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Alfke, Potts, Stoll, Volkmer, "NFFT meets Krylov methods: fast
 * matrix-vector products for the graph Laplacian of fully connected networks".
 * Section numbers, equation and algorithm labels below refer to that paper.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Return value: NFL_OK (0) on success; a negative NFL_ERR_* code on a hard
 *   error, in which case no output has been written; NFL_NOT_CONVERGED (> 0)
 *   when an iterative solver stopped at maxit (outputs hold the last iterate).
 *   nfl_strerror() names every code; nfl_last_error() gives the message of
 *   the last failure on the calling thread.
 * - Pointers named *_dev are device pointers (HBM of the device current when
 *   the handle was created); *_host are host pointers.  The caller owns every
 *   pointer it passes; the library never keeps one after the call returns
 *   (points are copied into handle-owned memory).
 * - Vectors at the boundary are in the caller's node order.  Internally the
 *   nodes are sorted by grid cell; that order never leaks out.
 * - All work is enqueued on the stream given to nfl_create() and is
 *   asynchronous, except where a call returns host scalars (noted below),
 *   which synchronises that stream.  A handle must not be used from two
 *   threads at once.
 * - The kernel is the Gaussian K(y) = exp(-||y||^2 / sigma^2), K(0) = 1
 *   (eq. W_gaussian).  W has zero diagonal (Section 2).
 * - Products are reproducible up to rounding order only: the spread (and,
 *   for the Laplacian RBF kernel, the near-field sum) add floating-point
 *   contributions with atomic operations whose order varies from run to run
 *   (differences at the FP32 rounding level of the sums).
 */
#ifndef NFL_H
#define NFL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NFL_OK              0
#define NFL_NOT_CONVERGED   1
#define NFL_ERR_ARG        -1   /* invalid argument (value or pointer) */
#define NFL_ERR_ORDER      -2   /* call order: e.g. apply before set_kernel */
#define NFL_ERR_DEGREE     -3   /* an approximate degree d_E,i <= 0 (Lemma of Section 3.1 needs eps < eta) */
#define NFL_ERR_HIP        -4   /* a HIP runtime call failed */
#define NFL_ERR_OOM        -5   /* device allocation failed */
#define NFL_ERR_UNSUPPORTED -6  /* valid for the method, not supported by this build (e.g. N not a power of 2) */

typedef struct nfl_plan *nfl_handle;
typedef struct nfl_mlp *nfl_mlp_handle;

/* Options for nfl_set_option (take effect at the next nfl_set_kernel). */
#define NFL_OPT_P          1   /* regularisation smoothness p of K_R (Fig. tab:fastsum_param); default p = m */
#define NFL_OPT_TILE       2   /* grid tile edge T for spread/interp (power of 2, 4..32); default 4 */
#define NFL_OPT_CHUNK      3   /* max nodes per work item of the per-cell, d <= 2, near-field and FP64
                                  kernels; default 512 (the tile-stationary d = 3 forms divide their
                                  work into one round of cost-balanced groups instead) */
#define NFL_OPT_EPS_B_DEFAULT 4 /* if value != 0, nfl_set_kernel with eps_B < 0 uses eps_B = p/N (the paper's default) */
#define NFL_OPT_KERNEL     5   /* d = 3 spread/interp: 0 = matrix-core (MFMA) kernels (default; tile-stationary
                                   where tile + 2m - 1 <= 16, else per-cell runs), 1 = vector-ALU kernels,
                                   2 = matrix-core kernels with per-cell runs only; takes effect immediately */
#define NFL_OPT_EPS_I      7   /* inner regularisation radius eps_I of the Laplacian RBF kernel in the
                                   scaled coordinates (0 = default p/N); eps_I + eps_B < 1/2; takes effect
                                   at the next nfl_set_kernel */
#define NFL_OPT_RESTARTS   6   /* thick restarts of nfl_lanczos_smallest (0 = none, default): with r > 0,
                                   maxit is the basis size and up to r restarts keep the leading Ritz
                                   vectors (see nfl_lanczos_smallest); takes effect immediately */
#define NFL_OPT_PRECISION  9   /* NFFT arithmetic, applied by the next nfl_set_kernel: 32 (default: FP32 spread,
                                 * FFT and interpolation on the matrix cores) or 64 (all FP64: the Kaiser-Bessel
                                 * window evaluated exactly, FP64 node fractions, degrees, FFT and filter; for
                                 * error studies, several times slower; d = 1..3, not with the Laplacian RBF
                                 * kernel, nfl_evaluate or the batched launch).  Inputs and outputs of the
                                 * apply calls stay float32; the Krylov solvers' FP64 vectors go through FP64
                                 * products. */
#define NFL_OPT_DETERMINISTIC 8 /* 1 (default): the spread into the plan's grid accumulates in int64 fixed
                                 * point (integer addition is associative), so every product is bitwise
                                 * reproducible run to run; 0: FP32 atomic additions, whose order (and so
                                 * the last bits of the result) varies between runs.  The batched launch
                                 * (nfl_batch_*) and the Laplacian RBF near field always use FP32 atomics. */

/* Create a plan for nodes in R^d, d in {1, 2, 3}.  `hip_stream` is a
 * hipStream_t (NULL = the default stream).  Allocates nothing on the device
 * yet. */
int nfl_create(nfl_handle *h, int d, void *hip_stream);

/* Release every device buffer of the plan.  Synchronises its stream. */
int nfl_destroy(nfl_handle h);

/* The vertex set {v_j} (Alg. nfft_fastsum input, Alg. nfft_normalized_matvec
 * input): n nodes, v_dev is n x d float32 row-major on the device, copied.
 * Computes the bounding-box midpoint c and R = max_j ||v_j - c|| on the
 * device (synchronises).  n >= 2.  Invalidates a previous set_kernel. */
int nfl_set_points(nfl_handle h, int64_t n, const float *v_dev);

/* Kernel and NFFT parameters (Fig. tab:fastsum_param): sigma > 0 in the
 * coordinates of the points; bandwidth N (even; this build needs a power of
 * 2, 8 <= N <= 256); window cut-off m (2 <= m <= 8); boundary region eps_B in
 * [0, 1/2) (or < 0 for the paper's default p/N when NFL_OPT_EPS_B_DEFAULT is
 * set).  The oversampled grid has 2N points per dimension.
 * Runs setup steps 1-4 of Alg. nfft_normalized_matvec: scales the nodes by
 * rho = (1/4 - eps_B/2)/R after shifting them to c (steps 1-2), computes the
 * Fourier coefficients b_l of the regularised kernel K_R by eq. b_l::K_RF
 * (step 3), sorts the nodes by grid cell, and computes the approximate
 * degrees D_E = diag(W~_E 1 - K(0) 1) (step 4).  Synchronises.  Returns
 * NFL_ERR_DEGREE if some d_E,i <= 0 (then apply calls fail with ORDER). */
int nfl_set_kernel(nfl_handle h, double sigma, int N, int m, double eps_B);

/* Radial kernels of eq. W_general for nfl_set_kernel_ex. */
#define NFL_KERNEL_GAUSSIAN               0  /* exp(-r^2 / param^2), K(0) = 1 */
#define NFL_KERNEL_MULTIQUADRIC           1  /* (r^2 + param^2)^{1/2}, K(0) = param */
#define NFL_KERNEL_INVERSE_MULTIQUADRIC   2  /* (r^2 + param^2)^{-1/2}, K(0) = 1/param */
#define NFL_KERNEL_LAPLACIAN_RBF          3  /* exp(-r / param) (eq. W_laplacian_rbf), K(0) = 1: not
                                                 smooth at 0, so K is regularised on r <= eps_I and a
                                                 near-field sum over pairs closer than eps_I restores it */

/* nfl_set_kernel for any kernel of eq. W_general above (Alg.
 * nfft_normalized_matvec, steps 1-4): W_ij = K(v_i - v_j) for i != j, W_ii = 0,
 * param > 0 in the coordinates of the points.  The parameter is a length: in
 * the scaled coordinates it becomes rho * param, and the multiquadric sums
 * come out times rho, the inverse multiquadric ones times 1/rho (homogeneity);
 * both are undone.  The NFFT works with the kernel divided by K(0), so that
 * L_s and A products run exactly as for the Gaussian; nfl_apply_W and
 * nfl_degree multiply their outputs by K(0), and nfl_get_info reports the
 * degree range in the original units.  The kernel-approximation error of
 * these slowly decaying kernels is much larger than the Gaussian's at the same
 * N (choose N = 64 or more and eps_B around 1/8); nfl_autotune and
 * nfl_direct_rows are for the Gaussian only.
 * NFL_KERNEL_LAPLACIAN_RBF: the regularised kernel K_R equals the even
 * polynomial T_I (degree 2p - 1, matching K and p - 1 radial derivatives at
 * r = +-eps_I) on r <= eps_I, the near-origin regularisation of the fast
 * summation for kernels that are not smooth at 0; every product then adds the
 * near-field sum over pairs with ||v~_i - v~_j|| <= eps_I of
 * x_j (K - T_I)(v~_i - v~_j) (diagonal included), computed directly from the
 * sorted nodes (cost grows with the number of such pairs: eps_I = p/N).
 * Batches and nfl_evaluate do not carry the near field and refuse this
 * kernel (NFL_ERR_UNSUPPORTED). */
int nfl_set_kernel_ex(nfl_handle h, int kind, double param, int N, int m, double eps_B);

int nfl_set_option(nfl_handle h, int opt, double value);

/* Target nodes for nfl_evaluate: n >= 1 points (n x d FP32 row-major on the
 * device, copied) placed in the frame of the plan `src` (its centre and
 * scaling, Alg. nfft_normalized_matvec steps 1-2), which must hold its own
 * points.  Every target must lie in the ball of the source points around
 * their centre (then all source-target differences stay inside the torus of
 * the fast summation); NFL_ERR_ARG otherwise.  Then call nfl_set_kernel(_ex)
 * on h with the source plan's kernel, N, m and eps_B (and the same
 * NFL_OPT_P): it sorts the targets and skips the degree pass.  Such a plan
 * only serves nfl_evaluate and the raw steps; operator and solver calls on it
 * return NFL_ERR_ORDER.  Synchronises. */
int nfl_set_points_frame(nfl_handle h, int64_t n, const float *v_dev, nfl_handle src);

/* y_j = sum_i x_i K(t_j - v_i): the fast summation of Alg. nfft_fastsum with
 * the adjoint NFFT at the source nodes v_i of plan src and the NFFT at the
 * target nodes t_j of plan tgt (made with nfl_set_points_frame(tgt, .., src),
 * same kernel parameters; tgt == src gives W~ x = W x + K(0) x).  This is the
 * kernel ridge regression prediction F(t) = sum_i alpha_i K(t - v_i)
 * (Section 6.3) for x = alpha.  x_dev: src->n FP32 in the sources' caller
 * order; y_dev: tgt->n FP32 in the targets' caller order.  Asynchronous on
 * src's stream (the target plan's stream is synchronised first). */
int nfl_evaluate(nfl_handle src, const float *x_dev, nfl_handle tgt, float *y_dev);

/* d_E (step 4 of Alg. nfft_normalized_matvec): n float32 in caller order. */
int nfl_degree(nfl_handle h, float *d_dev);

/* y = W_E x with W_E = W~_E - K(0) I (Section 3, Alg. nfft_fastsum followed by
 * removal of the diagonal).  x_dev, y_dev: nvec vectors of n float32, vector
 * k at offset k*ld (ld >= n); x and y must not overlap. */
int nfl_apply_W(nfl_handle h, const float *x_dev, float *y_dev, int nvec, int64_t ld);

/* y = L_s x = x - D_E^{-1/2} (W~_E (D_E^{-1/2} x) - K(0) D_E^{-1/2} x), the
 * symmetric normalised Laplacian (eq. nomlap) through step 5 of Alg.
 * nfft_normalized_matvec.  Same layout rules as nfl_apply_W. */
int nfl_apply_Ls(nfl_handle h, const float *x_dev, float *y_dev, int nvec, int64_t ld);

/* y = A_E x, A_E = D_E^{-1/2} W_E D_E^{-1/2} (step 5 of Alg.
 * nfft_normalized_matvec). */
int nfl_apply_A(nfl_handle h, const float *x_dev, float *y_dev, int nvec, int64_t ld);

/* FP64 vectors, caller order, one vector: y = A_E x = D_E^{-1/2} W_E D_E^{-1/2} x
 * (eq. nomlap; L_s x = x - A_E x, W x = D^{1/2} A_E D^{1/2} x).  With
 * NFL_OPT_PRECISION 64 the whole product is FP64 (the operator the Krylov
 * solvers use); otherwise the NFFT runs in FP32 between FP64 vectors.  x_dev
 * and y_dev must not overlap.  Device work memory: 2 n doubles (kept). */
int nfl_apply_A64(nfl_handle h, const double *x_dev, double *y_dev);
/* The degrees d_E (n doubles, caller order): FP64 on the FP64 path, else the
 * float32 degrees widened. */
int nfl_degree64(nfl_handle h, double *d_dev);

/* The k smallest eigenpairs of L_s (Section 4): Lanczos on A_E for its k
 * largest eigenvalues theta, lambda = 1 - theta (end of Section 2).  FP64
 * vectors, full reorthogonalisation (two classical Gram-Schmidt passes),
 * tridiagonal eigensolve on the device; stop when every wanted Ritz residual
 * |beta_{j+1} w_j| <= tol (Section 4) or after maxit steps.  block must be 1
 * (block > 1 runs a block Lanczos of that block size, 1..8).
 * evals_host: k doubles, ascending eigenvalues of L_s.  evecs_dev: n x k
 * FP64 column-major in caller order (NULL to skip).  iters, max_resid: host,
 * may be NULL.  Synchronises.  1 <= k < n, k <= maxit.
 * With NFL_OPT_RESTARTS r > 0 (any block size, 1 included) the basis holds at
 * most maxit columns (maxit >= k + 2 block); when it is full and the wanted
 * pairs have not converged, a thick restart (Wu and Simon 2000, block form)
 * keeps the l = min(J - b, max(k + b, J/2)) leading Ritz vectors and the next
 * block, with the projection diag(theta) plus the coupling R s_last, and the
 * iteration goes on; at most r restarts.  iters then counts A products. */
int nfl_lanczos_smallest(nfl_handle h, int k, int block, double tol, int maxit,
                         double *evals_host, double *evecs_dev, int *iters, double *max_resid);

/* The k largest eigenpairs of A_E = D_E^{-1/2} W_E D_E^{-1/2} by the
 * Nystrom-Gaussian-NFFT method (Alg. nystrom_hybrid, Section 5.2):
 * Y = A_E G, Q = orth(Y); B1 = A_E Q, B2 = Q^T B1; Sigma_M, U_M = the M
 * largest positive eigenpairs of B2; Qh Rh = B1 U_M;
 * Uh Lambda Uh^T = Rh Sigma_M^{-1} Rh^T; V = Qh Uh; the k largest of Lambda.
 * 2L NFFT products (FP32) and FP64 tall-skinny algebra; QR factorisations by
 * shifted CholeskyQR3.
 * G_dev: n x L FP64 column-major in caller order with leading dimension
 * ldg >= n, the Gaussian matrix (drawn by the caller; only its range
 * matters).  1 <= k <= M <= L <= n, L <= 64 in this build
 * (NFL_ERR_UNSUPPORTED above).  "Positive" in step 5 means above 1e-10 times
 * the largest absolute eigenvalue of B2; if fewer than M qualify, M shrinks to
 * their number (*m_used, host, may be NULL), and fewer than k is NFL_ERR_ARG,
 * as is a numerically rank-deficient A_E G or B1 U_M.
 * evals_host: k doubles, descending eigenvalues of the rank-M approximation
 * (1 - these approximate the smallest eigenvalues of L_s).  evecs_dev: n x k
 * FP64 column-major in caller order, orthonormal (NULL to skip).
 * Device work memory: 3 n L doubles.  Synchronises. */
int nfl_nystrom(nfl_handle h, const double *G_dev, int64_t ldg, int L, int M, int k,
                double *evals_host, double *evecs_dev, int *m_used);

/* Warm-start modes of nfl_cg_solve. */
#define NFL_WARM_ZERO 0
#define NFL_WARM_USER 1
#define NFL_WARM_MLP  2

/* CG for (I + tau L_s) u = f, the kernel-SSL system (eq. ssl::system), tau >= 0.
 * FP64 vectors and inner products, FP32 NFFT matvecs.  Stops when the
 * recurrence residual ||r|| / ||f|| <= tol or after maxit iterations; relres
 * (host, may be NULL) is the TRUE residual ||f - (I + tau L_s) u|| / ||f||
 * recomputed at the end with the same operator (one more product; with
 * relres NULL that product is skipped).  f_dev, u_dev: n doubles in
 * caller order.  warm: NFL_WARM_ZERO (u0 = 0), NFL_WARM_USER (u0 read from
 * u_dev), NFL_WARM_MLP (u0 from the plan's warm-start network, see
 * nfl_mlp_*).  The iteration runs on the device: the step lengths and the
 * stopping test are formed by the solver's kernels (fixed-order reductions,
 * so a solve is reproducible), and the host checks the status one iteration
 * behind without stalling the device.  NFL_NOT_CONVERGED also on a
 * breakdown (p.Mp <= 0).  Device work memory: 5 n doubles (plus the
 * reduction partials), allocated by the plan's first solve and kept with
 * the plan.  Synchronises. */
int nfl_cg_solve(nfl_handle h, double tau, const double *f_dev, double *u_dev, int warm,
                 double tol, int maxit, int *iters, double *relres);

/* nfl_cg_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, kernels and results, with the work space (5 n doubles, the
 * reduction partials, scalars and the stop flag) in the library's static
 * device array instead of plan-owned buffers; the call makes no hipMalloc,
 * hipFree or allocating library call.  Limits: n <= NFL_CG_NOALLOC_MAX_N
 * (else NFL_ERR_ARG, nothing written); warm is NFL_WARM_ZERO or
 * NFL_WARM_USER (the network's start allocates its feature buffers).  Each
 * GPU holds one such array (42 MB) until the process ends, shared by every
 * call on that GPU: calls that overlap on one GPU race (serialise them, e.g.
 * one stream).  The plan itself must have been built (points and kernel) by
 * the allocating calls beforehand.  Synchronises. */
#define NFL_CG_NOALLOC_MAX_N 1048576
int nfl_cg_solve_noalloc(nfl_handle h, double tau, const double *f_dev, double *u_dev, int warm,
                         double tol, int maxit, int *iters, double *relres);

/* Kernel ridge regression (Section 6.3): CG for (K + beta I) alpha = f with
 * the Gram matrix K_ij = K(v_i - v_j) of the plan's kernel, diagonal K(0)
 * included (K = W + K(0) I; Gaussian or inverse multiquadric: positive
 * definite; the multiquadric Gram matrix is not, and CG may fail on it).
 * beta >= 0.  The paper's preconditioner is unspecified; the diagonal one is
 * the scalar K(0) + beta here, so plain CG is run.  FP64 vectors in caller
 * order, FP32 NFFT products.  Stops when the recurrence residual
 * ||r|| / ||f|| <= tol or after maxit iterations; relres (host, may be NULL)
 * is the true residual recomputed with the same operator (skipped when NULL).  f_dev, alpha_dev:
 * n doubles; warm: NFL_WARM_ZERO (alpha0 = 0) or NFL_WARM_USER (alpha0 read
 * from alpha_dev).  The prediction at the training points is
 * K alpha = nfl_apply_W(alpha) + K(0) alpha.  Synchronises. */
int nfl_krr_solve(nfl_handle h, double beta, const double *f_dev, double *alpha_dev, int warm,
                  double tol, int maxit, int *iters, double *relres);

/* ---- learned warm start for nfl_cg_solve ------------------------------------
 * A pointwise network u0_i = net(features_i) predicts the solution of the
 * kernel-SSL system (eq. ssl::system) node by node; CG then runs to tolerance
 * from u0, so the network only changes the starting point.  Features of node
 * i: its position in the scaled torus coordinates (times 4), its right-hand
 * side f_i, d_E,i / mean(d_E), and a one-hot class index (one-vs-rest problems).
 * Architecture: 16 -> 64 -> 64 -> 64 -> 1 with tanh, BF16 matrix-core
 * operands, FP32 accumulation, FP32 master weights, Adam.  Parameter vector
 * (9473 floats): W1[64][16], b1[64], W2[64][64], b2[64], W3[64][64], b3[64],
 * W4[64], b4.  A network is independent of any plan; calls that take a plan
 * read its nodes and degrees.  All calls synchronise the network's stream. */
int nfl_mlp_create(nfl_mlp_handle *m, int n_classes, uint64_t seed, void *hip_stream);
int nfl_mlp_destroy(nfl_mlp_handle m);
/* One Adam step (learning rate lr) on nsample nodes of plan h drawn with seed:
 * inputs f_dev (right-hand side) and u_dev (target solution), n doubles each,
 * caller order; loss_host (may be NULL) receives the mean squared error
 * before the step. */
int nfl_mlp_train_step(nfl_mlp_handle m, nfl_handle h, const double *f_dev, const double *u_dev,
                       int cls, int64_t nsample, uint64_t seed, double lr, double *loss_host);
/* u_dev = net(features) for every node of h (caller order, doubles). */
int nfl_mlp_predict(nfl_mlp_handle m, nfl_handle h, const double *f_dev, int cls, double *u_dev);
/* Attach (m != NULL) or detach the network used by nfl_cg_solve(..., NFL_WARM_MLP),
 * with the class index of the right-hand sides that will be solved. */
int nfl_mlp_attach(nfl_handle h, nfl_mlp_handle m, int cls);
/* Save / load the parameters (flat little-endian file: 8-byte magic, 4 int32
 * header, 9473 float32).  Loading resets the optimiser state. */
int nfl_mlp_save(nfl_mlp_handle m, const char *path);
int nfl_mlp_load(nfl_mlp_handle m, const char *path);
int nfl_mlp_get_params(nfl_mlp_handle m, float *params_host, int64_t count);
int nfl_mlp_set_params(nfl_mlp_handle m, const float *params_host, int64_t count);
/* Explicit-feature entry points (for testing): feat_dev is B x 16 float32
 * row-major.  forward: out_dev = B network outputs.  gradient: the gradient
 * of the mean squared error (1/B) sum (out - target)^2 with respect to the
 * 9473 parameters (host) and the loss. */
int nfl_mlp_forward(nfl_mlp_handle m, const float *feat_dev, int64_t B, float *out_dev);
int nfl_mlp_gradient(nfl_mlp_handle m, const float *feat_dev, const float *target_dev, int64_t B,
                     float *grad_host, int64_t count, double *loss_host);

/* Plan information (host outputs, any may be NULL): rho, sigma_tilde = rho*sigma,
 * min and max of d_E, and eps_B / p actually used.  Synchronises. */
int nfl_get_info(nfl_handle h, double *rho, double *sigma_tilde, double *dmin, double *dmax,
                 double *eps_B, int *p);

/* A-posteriori error quantities of Section 3.1 (host outputs, any may be
 * NULL), for monitoring the accuracy of a plan:
 *   eta      = d_min / ||W||_inf, the quantity of the Lemma on normalisation
 *              (thm. normalization_propagation), from the plan's approximate
 *              degrees d_E (the kernels here are positive, so ||W||_inf is the
 *              largest degree);
 *   kerr_inf ~ ||K_ERR||_inf = max |K_R(y) - K_RF(y)| over ||y|| <= 1/2 - eps_B
 *              in the scaled coordinates (eq. KERR_estimate), the maximum taken
 *              over nsamples points y; K_RF(y) = sum_{l in I_N^d} b_l cos(2 pi l.y)
 *              with the plan's coefficients b_l (eq. b_l::K_RF), K_R the
 *              regularised kernel divided by K(0) (for the Laplacian RBF kernel
 *              K_R = T_I near 0, which the near field corrects exactly);
 *   eps_est  = n kerr_inf / ||W||_inf (eq. epsilon_KERR_estimate), the estimate
 *              of eps = ||E||_inf / ||W||_inf that ignores the NFFT's own error;
 *   lemma_bound = eps_est (1 + eta) / (eta (eta - eps_est)), the Lemma's bound
 *              on ||A - A_E||_inf with eps = eps_est (+infinity if eps_est >= eta).
 * The sample points are y_host (nsamples x d doubles, row-major, each inside
 * the ball, NFL_ERR_ARG otherwise) or, if y_host is NULL, nsamples points
 * uniform in the ball drawn from a splitmix64 stream seeded with seed.
 * 1 <= nsamples <= 2^20.  O(nsamples N^d) work on the GPU.  Synchronises. */
int nfl_error_estimate(nfl_handle h, int nsamples, uint64_t seed, const double *y_host,
                       double *eta, double *kerr_inf, double *eps_est, double *lemma_bound);

/* ---- the individual NFFT steps (for testing; same stream rules) ---------- */

/* Size of the oversampled grid: (2N)^d float32 cells, index ((x*2N)+y)*2N+z
 * (last dimension fastest).  Valid after nfl_set_kernel. */
int64_t nfl_grid_size(nfl_handle h);

/* Spread (adjoint NFFT gridding, step 1 of Alg. nfft_fastsum before its FFT):
 * g[k] = sum_i x_i psi~(k - u_i) with the periodised window psi~ on the grid,
 * u_i = 2N (v~_i + 1/2).  x_dev: n float32 (caller order); grid_dev: grid
 * size float32, overwritten. */
int nfl_spread(nfl_handle h, const float *x_dev, float *grid_dev);

/* FFT -> multiply by the kernel's Fourier coefficients divided by the
 * window's transform squared -> inverse FFT, on the real grid (the middle of
 * Alg. nfft_fastsum: end of step 1, step 2, start of step 3). */
int nfl_convolve(nfl_handle h, const float *grid_in_dev, float *grid_out_dev);

/* Interpolate (step 3 of Alg. nfft_fastsum after its inverse FFT):
 * f_i = sum_k g[k] psi~(k - u_i), the exact transpose of nfl_spread.  f_dev:
 * n float32 in caller order. */
int nfl_interp(nfl_handle h, const float *grid_dev, float *f_dev);

/* The filter the plan multiplies with, on the half spectrum
 * l_x, l_y in -N/2..N/2, l_z in 0..N/2 (d = 3; fewer axes for d < 3):
 * (N+1)^(d-1) (N/2+1) doubles, host.  Synchronises. */
int nfl_get_filter(nfl_handle h, double *filter_host, int64_t count);

/* Runs nrep products y = L_s x (as nfl_apply_Ls, one vector) with HIP
 * events recorded on the plan's stream between the stages, and returns the
 * average milliseconds per product of each stage in stage_ms[5]: grid
 * clear, spread, FFT + filter + inverse FFT, interpolation, whole product.
 * Synchronises. */
int nfl_profile_stages(nfl_handle h, const float *x_dev, float *y_dev, int nrep,
                       double *stage_ms);

/* The same filter computed from explicit parameters without a plan or a GPU
 * (host FP64; sigma_tilde is sigma in the scaled torus coordinates).  count
 * must be >= (N+1)^(d-1) (N/2+1).  N a power of 2. */
int nfl_compute_filter(int d, int N, int m, int p, double eps_B, double sigma_tilde,
                       double *filter_host, int64_t count);

/* nfl_compute_filter for a kernel kind (NFL_KERNEL_*): the filter of the
 * kernel divided by K(0), sigma_tilde = the scaled parameter, eps_I = the
 * inner regularisation radius (Laplacian RBF kernel only; 0 otherwise). */
int nfl_compute_filter_ex(int kind, int d, int N, int m, int p, double eps_B, double sigma_tilde,
                          double eps_I, double *filter_host, int64_t count);

/* The window the kernels apply (host, no GPU): for each of the 2m grid
 * offsets c of a node's window, NFL_WIN_NC float32 coefficients of the
 * polynomial in g = 2f - 1 (f = the node's fraction inside its cell) that
 * approximates the Kaiser-Bessel window psi(c - (m-1) - f),
 *   psi(t) = sinh(b sqrt(m^2 - t^2)) / (sqrt(m^2 - t^2) b e^{bm}), b = 3 pi / 2,
 * row-major [c][k], count >= 2m * NFL_WIN_NC.  The filter deconvolves with the
 * exact transform of this piecewise polynomial. */
#define NFL_WIN_NC 8
int nfl_window_coefficients(int m, float *coef_host, int64_t count);

/* ---- accuracy probe and parameter search ---------------------------------- */

/* Exact sums on sampled rows by a direct FP64 GPU kernel over all n points
 * (the definitions of Section 2, zero diagonal): for each r < nrows with
 * j = rows_host[r] (caller order, 0 <= j < n),
 *   wx_host[r]  = sum_{i != j} exp(-||v_j - v_i||^2 / sigma^2) x_i,
 *   deg_host[r] = sum_{i != j} exp(-||v_j - v_i||^2 / sigma^2).
 * wx_host or deg_host may be NULL (x_dev may be NULL when wx_host is).
 * Needs nfl_set_points only; 1 <= nrows <= 65535.  O(nrows * n) work.
 * Synchronises. */
int nfl_direct_rows(nfl_handle h, double sigma, const float *x_dev, const int64_t *rows_host,
                    int nrows, double *wx_host, double *deg_host);

/* Choose N, m, eps_B and the tile for this plan's points and sigma so that
 * max(rel_inf(d), rel_inf(W x)) on nrows seeded sampled rows (x uniform in
 * [-1, 1)) against nfl_direct_rows stays <= target, at the smallest product
 * time: smallest N (eps_B in {0, 1/16, 1/8}, widest window), then smallest m,
 * then the fastest tile in {4, 8, 16} (the paper's defaults of Section 3.2
 * are the starting point of this search, not its result).  The plan is left
 * set to the chosen configuration (as after nfl_set_kernel).  cache_path
 * (may be NULL): a text file of results keyed by (d, floor(log4 n),
 * floor(2 log2 sigma~), target); a cached configuration is verified on this
 * plan with the same probe and re-tuned if it misses.  Outputs (any may be
 * NULL): N, m, eps_B, tile, the probe error, ms per L_s product, cached =
 * 1 if the configuration came from the cache.  Returns NFL_NOT_CONVERGED
 * (plan set to the most accurate configuration tried) when no configuration
 * reaches the target.  Synchronises; runs many products. */
int nfl_autotune(nfl_handle h, double sigma, double target, int nrows, uint64_t seed,
                 const char *cache_path, int *N, int *m, double *eps_B, int *tile,
                 double *err, double *ms, int *cached);

/* ---- batches: many graphs, a block of vectors each, one graph launch ---- */

typedef struct nfl_batch_s *nfl_batch;

/* Group nplans plans into a batch that applies y = L_s x (Alg.
 * nfft_normalized_matvec, step 5) to nvec vectors of every plan at once.
 * Each plan must have d = 3, the matrix-core kernels (NFL_OPT_KERNEL 0) and a
 * successful nfl_set_kernel; plans may differ in n, sigma, N, m and tile.
 * The batch reads the plans' sorted nodes, degrees and filters (it does not
 * copy them), so every plan must outlive the batch and must not be changed
 * (set_points / set_kernel / set_option) while it exists: apply then fails
 * with NFL_ERR_ORDER.  The batch owns two grids and the spectra per (plan,
 * vector) pair (nfl_batch_info reports the bytes) and records the whole
 * product -- spread launches per window width and kernel form, five FFT
 * passes, interpolation launches -- as a HIP graph at creation.
 * hip_stream: the stream the graph is launched on (may be the null stream).
 * 1 <= nvec <= 64. */
int nfl_batch_create(nfl_batch *b, const nfl_handle *plans, int nplans, int nvec,
                     void *hip_stream);

/* Packed vector layout of a batch: offsets_host[g] = n_0 + ... + n_{g-1}
 * (count >= nplans + 1; offsets_host[nplans] = total n).  Plan g's block
 * occupies x[nvec * offsets[g] .. nvec * offsets[g+1]), vector j of it
 * starting at nvec * offsets[g] + j * n_g, each vector in plan g's caller
 * node order. */
int nfl_batch_offsets(nfl_batch b, int64_t *offsets_host, int64_t count);

/* y = L_s x for every (plan, vector) of the batch, packed as described at
 * nfl_batch_offsets (nvec * total n float32 each; x and y must not
 * overlap).  One graph launch, plus a one-thread kernel when x or y differs
 * from the previous call.  Asynchronous on the batch's stream; two applies
 * of one batch must not run concurrently (they share the grids). */
int nfl_batch_apply_Ls(nfl_batch b, const float *x_dev, float *y_dev);

/* Batch facts (any output may be NULL): total nodes, (plan, vector) jobs,
 * kernels in one product, device bytes of the grids and spectra. */
int nfl_batch_info(nfl_batch b, int64_t *total_n, int *njobs, int *nkernels,
                   int64_t *arena_bytes);

int nfl_batch_destroy(nfl_batch b);

const char *nfl_strerror(int code);
const char *nfl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NFL_H */
