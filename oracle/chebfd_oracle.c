/*
 * ORACLE -- test infrastructure only.
 *
 * Plain, unfused FP64 reference for the Chebyshev filter of ChebFD
 * (Kreutzer et al., "Chebyshev Filter Diagonalization on Modern Manycore
 * Processors and GPGPUs", Sect. 2, Alg. 1; subspace blocking Sect. 3.3,
 * Alg. 2).  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load this library.  It shares no code with the HIP library.
 *
 * Storage: the matrix is CRS (the paper's format, Sect. 3.1) with 64-bit row
 * pointers, 32-bit column indices and interleaved (re, im) doubles.  Block
 * vectors are column-major, one contiguous vector per column, leading
 * dimension n: the plain per-vector layout, not the paper's row-major one,
 * so that nothing here resembles the tuned path.
 *
 * Each routine does one operation of Alg. 1 over all rows with an OpenMP
 * parallel loop; there is no fusion.  Dot products sum each thread's
 * contiguous row range in row order and add the per-thread sums in thread
 * order, so results are reproducible for a fixed thread count.
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex zd;

/* Y(:,j) = (alpha*H + beta*I) X(:,j), j < m.  (Alg. 1: the spmmv() operation) */
void orc_spmmv(int64_t n, const int64_t *rowptr, const int32_t *col,
               const double *val, double alpha, double beta, int m,
               const zd *X, zd *Y)
{
    const zd *V = (const zd *)val;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < m; ++j) {
            zd acc = 0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                acc += V[k] * X[(int64_t)j * n + col[k]];
            Y[(int64_t)j * n + i] = alpha * acc + beta * X[(int64_t)j * n + i];
        }
    }
}

/* Y <- a*Y + b*X over an n x m block (Alg. 1: baxpy()/bscal()) */
void orc_axpby(int64_t n, int m, zd a, zd *Y, zd b, const zd *X)
{
    int64_t len = n * (int64_t)m;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < len; ++i)
        Y[i] = a * Y[i] + b * X[i];
}

/* out[j] = <A(:,j), B(:,j)> = sum_i conj(A_ij) B_ij  (Alg. 1: eta, mu dot products) */
void orc_dot(int64_t n, int m, const zd *A, const zd *B, zd *out)
{
    int nt = omp_get_max_threads();
    zd *part = (zd *)calloc((size_t)nt * (size_t)m, sizeof(zd));
#pragma omp parallel
    {
        int t = omp_get_thread_num();
        int T = omp_get_num_threads();
        int64_t lo = n * t / T, hi = n * (t + 1) / T;
        for (int j = 0; j < m; ++j) {
            zd s = 0;
            for (int64_t i = lo; i < hi; ++i)
                s += conj(A[(int64_t)j * n + i]) * B[(int64_t)j * n + i];
            part[(int64_t)t * m + j] = s;
        }
    }
    for (int j = 0; j < m; ++j) {
        zd s = 0;
        for (int t = 0; t < nt; ++t) s += part[(int64_t)t * m + j];
        out[j] = s;
    }
    free(part);
}

/*
 * Alg. 1 on one block of m vectors: X (n x m) is overwritten by the filtered
 * block  sum_{p=0}^{n_p} gamma_p T_p(alpha H + beta I) X.
 * U, W, T are n x m work blocks.  eta, nu receive, for p = 1..n_p,
 *   eta[p*m + j] = <T_p x_j, T_{p-1} x_j>,   nu[p*m + j] = <T_{p-1} x_j, T_{p-1} x_j>
 * (the moments of Alg. 1 for p >= 3, and the same two products for the start
 * vectors at p = 1, 2); row p = 0 is left untouched.
 */
void orc_filter_block(int64_t n, const int64_t *rowptr, const int32_t *col,
                      const double *val, double alpha, double beta, int n_p,
                      const double *gamma, int m, zd *X, zd *U, zd *W, zd *T,
                      zd *eta, zd *nu)
{
    if (n_p == 0) {                                       /* degree 0: X <- g0c0 X */
        orc_axpby(n, m, gamma[0], X, 0.0, X);
        return;
    }
    /* U <- (alpha H + beta I) X */
    orc_spmmv(n, rowptr, col, val, alpha, beta, m, X, U);
    orc_dot(n, m, U, X, eta + 1 * (int64_t)m);
    orc_dot(n, m, X, X, nu + 1 * (int64_t)m);
    if (n_p == 1) {                                       /* degree 1: X <- g0c0 X + g1c1 U */
        orc_axpby(n, m, gamma[0], X, gamma[1], U);
        return;
    }
    /* W <- 2 (alpha H + beta I) U - X */
    orc_spmmv(n, rowptr, col, val, alpha, beta, m, U, W);
    orc_axpby(n, m, 2.0, W, -1.0, X);
    orc_dot(n, m, W, U, eta + 2 * (int64_t)m);
    orc_dot(n, m, U, U, nu + 2 * (int64_t)m);
    /* X <- g0c0 X + g1c1 U + g2c2 W */
    orc_axpby(n, m, gamma[0], X, gamma[1], U);
    orc_axpby(n, m, 1.0, X, gamma[2], W);
    for (int p = 3; p <= n_p; ++p) {
        zd *tmp = U; U = W; W = tmp;                       /* swap(W, U) */
        orc_spmmv(n, rowptr, col, val, alpha, beta, m, U, T);
        orc_axpby(n, m, -1.0, W, 2.0, T);                 /* W <- 2 H~ U - W */
        orc_dot(n, m, W, U, eta + (int64_t)p * m);        /* eta_p <- <W, U> */
        orc_dot(n, m, U, U, nu + (int64_t)p * m);         /* mu_p  <- <U, U> */
        orc_axpby(n, m, 1.0, X, gamma[p], W);             /* X <- X + g_p c_p W */
    }
}

/* Alg. 2: the filter applied to n_s/n_b blocks of n_b vectors in turn.
 * X is n x n_s column-major; block b is columns [b n_b, (b+1) n_b).
 * eta, nu are (n_p+1) x n_s row-major (entry [p*n_s + column]). */
int orc_filter(int64_t n, const int64_t *rowptr, const int32_t *col,
               const double *val, double alpha, double beta, int n_p,
               const double *gamma, int n_s, int n_b, zd *X, zd *eta, zd *nu)
{
    if (n_b <= 0 || n_s % n_b != 0 || n_p < 0) return -1;
    size_t blk = (size_t)n * (size_t)n_b;
    zd *U = (zd *)malloc(blk * sizeof(zd));
    zd *W = (zd *)malloc(blk * sizeof(zd));
    zd *T = (zd *)malloc(blk * sizeof(zd));
    zd *eb = (zd *)calloc((size_t)(n_p + 1) * n_b, sizeof(zd));
    zd *nb = (zd *)calloc((size_t)(n_p + 1) * n_b, sizeof(zd));
    if (!U || !W || !T || !eb || !nb) { free(U); free(W); free(T); free(eb); free(nb); return -2; }
    for (int b = 0; b < n_s / n_b; ++b) {
        orc_filter_block(n, rowptr, col, val, alpha, beta, n_p, gamma, n_b,
                         X + (size_t)b * blk, U, W, T, eb, nb);
        for (int p = 1; p <= n_p; ++p)
            for (int j = 0; j < n_b; ++j) {
                eta[(int64_t)p * n_s + b * n_b + j] = eb[(int64_t)p * n_b + j];
                nu[(int64_t)p * n_s + b * n_b + j] = nb[(int64_t)p * n_b + j];
            }
    }
    free(U); free(W); free(T); free(eb); free(nb);
    return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

/* Thread count of the following calls (timing runs; results depend on it only
   through the order in which dot products add per-thread sums). */
void orc_set_num_threads(int t) { if (t >= 1) omp_set_num_threads(t); }
