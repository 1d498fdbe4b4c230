/*
 * Oracle (test infrastructure only): direct FP64 kernel sums.
 *
 * Only the tests, the smoke check and the bench's CPU-baseline leg may load
 * this library.  It shares no code with the HIP library.
 *
 * Weighted graph of Section 2: the weight between distinct nodes j != i is the
 * Gaussian exp(-||v_j - v_i||^2 / sigma^2) (the Gaussian weight equation,
 * eq. W_gaussian); a node has no loop, so W_jj = 0.  The degree d = W 1 and
 * every product with W are plain O(n^2) sums, in the order i = 0..n-1, with
 * no blocking or reassociation.  Duplicate points (j != i, same coordinates)
 * get weight exp(0) = 1: only the diagonal is zero.
 */
#include <math.h>
#include <stdint.h>

#define ORACLE_MAX_NVEC 64

/*
 * out[k*nrows + r] = sum_{i != rows[r]} W_{rows[r], i} * x[k*n + i]
 * v is n x d row-major (FP64), x is nvec vectors of length n (one per row).
 * Returns 0, or -1 for bad arguments.
 */
int oracle_w_rows(int64_t n, int d, const double *v, double sigma, int nvec,
                  const double *x, int64_t nrows, const int64_t *rows,
                  double *out)
{
    if (n < 1 || d < 1 || d > 8 || nvec < 1 || nvec > ORACLE_MAX_NVEC || sigma <= 0.0)
        return -1;
    const double inv_s2 = 1.0 / (sigma * sigma);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t j = rows[r];
        double acc[ORACLE_MAX_NVEC];
        for (int k = 0; k < nvec; ++k) acc[k] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (i == j) continue;
            double s = 0.0;
            for (int t = 0; t < d; ++t) {
                const double diff = v[j * d + t] - v[i * d + t];
                s += diff * diff;
            }
            const double w = exp(-s * inv_s2);
            for (int k = 0; k < nvec; ++k) acc[k] += w * x[(int64_t)k * n + i];
        }
        for (int k = 0; k < nvec; ++k) out[(int64_t)k * nrows + r] = acc[k];
    }
    return 0;
}

/* Degree rows: d_j = sum_{i != j} W_{j,i}  (the degree definition, Section 2). */
int oracle_degree_rows(int64_t n, int d, const double *v, double sigma,
                       int64_t nrows, const int64_t *rows, double *out)
{
    if (n < 1 || d < 1 || d > 8 || sigma <= 0.0) return -1;
    const double inv_s2 = 1.0 / (sigma * sigma);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t j = rows[r];
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (i == j) continue;
            double s = 0.0;
            for (int t = 0; t < d; ++t) {
                const double diff = v[j * d + t] - v[i * d + t];
                s += diff * diff;
            }
            acc += exp(-s * inv_s2);
        }
        out[r] = acc;
    }
    return 0;
}

/* Number of OpenMP threads the sums above use (reported with timings). */
int oracle_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
