/*
 * chebfd.h -- C ABI of libchebfd, a single-GPU (AMD MI355X, gfx950) library for
 * Chebyshev filter diagonalization (ChebFD) of large sparse Hermitian matrices.
 *
 * Method: Kreutzer, Hager, Ernst, Fehske, Bishop, Wellein, "Chebyshev Filter
 * Diagonalization on Modern Manycore Processors and GPGPUs" (arXiv:1803.02156).
 * ChebFD projects n_s search vectors onto the eigenvectors whose eigenvalues lie
 * in a search interval, using a polynomial window filter of degree n_p in the
 * scaled matrix alpha*H + beta*I (Sect. 2, Alg. 1), applied to blocks of n_b
 * vectors in turn (Sect. 3.3, Alg. 2).
 *
 * Conventions for every call:
 *  - Pointers named d_* are device (HIP) memory, h_* are host memory.  The
 *    library never allocates device memory: the caller passes buffers and the
 *    byte sizes it was told by the matching *_query call.  Host arrays are only
 *    read (or written, for outputs) during the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *    enqueued on it; a call returns before the work finishes unless stated.
 *  - Complex numbers are interleaved (re, im) pairs: c128 = 2 doubles,
 *    c64 = 2 floats.
 *  - Return value: 0 on success, > 0 a warning with valid outputs, < 0 an error
 *    (outputs untouched, nothing enqueued).  chebfd_last_error() gives a
 *    thread-local message for the last failing call.  No C++ exception crosses
 *    the interface.  All arguments are validated before the first launch.
 */
#ifndef CHEBFD_H
#define CHEBFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CHEBFD_OK               0
#define CHEBFD_NOT_CONVERGED    1   /* max_iter reached; outputs hold the last iterate */
#define CHEBFD_SUBSPACE_SMALL   2   /* more than 3/4 n_s Ritz values in the interval */
#define CHEBFD_EINVAL         (-1)  /* invalid argument (sizes, NULL, alignment, aliasing) */
#define CHEBFD_EHIP           (-2)  /* a HIP runtime call failed */
#define CHEBFD_EWORKSPACE     (-3)  /* caller buffer smaller than the queried size */
#define CHEBFD_EINTERVAL      (-4)  /* search interval not strictly inside the spectral bounds */
#define CHEBFD_ENUMERIC       (-5)  /* non-finite value or failed small eigensolve */

/* ---- precision of the block vectors and matrix values ------------------- */
#define CHEBFD_PREC_FP64   0   /* c128 vectors and matrix, FP64 arithmetic */
#define CHEBFD_PREC_MIXED  1   /* c64 vectors and matrix, FP32 sparse products, FP64 dot products */

/*
 * Device-resident sparse matrix in SELL-C-sigma format.  Rows are grouped in
 * chunks of C consecutive rows; within windows of sigma rows, rows are sorted by
 * decreasing length (stable, ties keep the original order), which is a
 * symmetric permutation P H P^T; each chunk is padded to its longest row and
 * stored column-major (slot k of the chunk's rows is contiguous).  Padding slots
 * hold value 0 and the row's own index.  Column indices are in permuted
 * numbering; all block vectors handled by the filter calls are in permuted row
 * order too (chebfd_pack/unpack convert).  This is a plain-old-data handle:
 * its pointers point into the d_buf given to chebfd_matrix_build, which the
 * caller owns and must keep alive.
 */
typedef struct chebfd_matrix {
    int64_t n;                  /* dimension */
    int64_t nnz;                /* stored entries of the input CRS matrix */
    int64_t n_chunks;           /* ceil(n / C) */
    int64_t slots;              /* stored slots including padding */
    int32_t C;                  /* chunk height */
    int32_t sigma;              /* sorting window (multiple of C, or 1) */
    int32_t prec;               /* CHEBFD_PREC_* of the stored values */
    int32_t max_width;          /* longest row */
    int32_t identity_perm;      /* 1 if the permutation is the identity */
    int32_t uniform_width;      /* slots per row of every chunk if all chunks are equally wide, else 0 */
    int32_t window_local[2];    /* stored entries per 1000 whose column lies in the row window of its
                                   tile (tiles of 32 and 64 rows, window 3 tiles either side); the
                                   filter gathers such entries from a copy of U staged in LDS */
    const int64_t *chunk_off;   /* [n_chunks + 1] first slot of each chunk */
    const int32_t *chunk_width; /* [n_chunks] slots per row in the chunk */
    const int32_t *col;         /* [slots] permuted column index */
    const void *val;            /* [slots] complex values (c128 or c64 per prec) */
    const int32_t *perm;        /* [n] perm[new] = old row */
    const int32_t *iperm;       /* [n] iperm[old] = new row */
} chebfd_matrix;

/* Version of the ABI (major*10000 + minor*100 + patch). */
int chebfd_version(void);

/* Message describing the last failing call on this thread ("" if none). */
const char *chebfd_last_error(void);

/* Device properties the launchers use: number of compute units and the name. */
int chebfd_device_info(int32_t *num_cus, char *name, int32_t name_len);

/*
 * Matrix ingest (the paper's CRS format, Sect. 3.1: 4-byte column indices,
 * complex double values) into SELL-C-sigma.
 * chebfd_matrix_query: bytes of device memory chebfd_matrix_build needs.
 * chebfd_matrix_build: builds the format on the host, copies it into d_buf on
 *   `stream` and synchronises that stream before returning (setup, once).
 *   h_rowptr[n+1] (int64, h_rowptr[0] = 0, non-decreasing), h_col[nnz] in [0, n),
 *   h_val[2*nnz] interleaved c128.  The matrix must be Hermitian (not checked).
 *   C in {1..1024}, sigma >= 1 and a multiple of C (or 1); prec per CHEBFD_PREC_*.
 *   d_buf must be 256-byte aligned.
 *   h_order (optional, NULL = natural order): a permutation of 0..n-1 giving the
 *   row order before the sigma sort (h_order[k] = original row placed k-th), a
 *   further symmetric permutation, e.g. one that keeps the rows a step gathers
 *   close together in memory.  Results do not depend on it beyond rounding
 *   order: vectors enter and leave through chebfd_pack/unpack in the original
 *   numbering, and device-drawn random vectors are keyed by original rows.
 */
int chebfd_matrix_query(int64_t n, const int64_t *h_rowptr, const int32_t *h_order, int32_t C,
                        int32_t sigma, int32_t prec, size_t *bytes);
int chebfd_matrix_build(int64_t n, const int64_t *h_rowptr, const int32_t *h_col,
                        const double *h_val, const int32_t *h_order, int32_t C, int32_t sigma,
                        int32_t prec, void *d_buf, size_t bytes, void *stream, chebfd_matrix *out);

/*
 * Gershgorin bounds of H (the interval that must be mapped onto [-1, 1] by the
 * scaling alpha*H + beta*I of Alg. 1): lam_lo = min_i (Re H_ii - r_i),
 * lam_hi = max_i (Re H_ii + r_i), r_i = sum_{j != i} |H_ij|.  Computed on the
 * device; d_work of chebfd_bounds_query bytes; synchronises `stream`.
 */
int chebfd_bounds_query(const chebfd_matrix *H, size_t *work_bytes);
int chebfd_bounds(const chebfd_matrix *H, void *d_work, size_t work_bytes, void *stream,
                  double *lam_lo, double *lam_hi);

/*
 * Filter coefficients (host): gamma_p = g_p c_p, p = 0..n_p, where c_p are the
 * Chebyshev coefficients of the indicator of the scaled interval
 * [a, b] = [alpha lam_L + beta, alpha lam_R + beta] (the window function of
 * Sect. 2) and g_p the Jackson damping factors for n_p + 1 terms (Alg. 1
 * weights each T_p x with the product g_p c_p).  Also returns alpha, beta from
 * the bounds [lam_lo, lam_hi].  CHEBFD_EINTERVAL unless -1 < a < b < 1.
 */
int chebfd_coefficients(double lam_lo, double lam_hi, double lam_L, double lam_R,
                        int32_t n_p, double *alpha, double *beta, double *h_gamma);

/*
 * Layout conversion between the user's column-major c128 block (n x m, ld = n,
 * original row order) and the filter's blocked layout (Fig. 3 of Sect. 3.3):
 * m/n_b blocks of n_b vectors, each block an n x n_b row-major array (the n_b
 * entries of a row contiguous), blocks stored one after another, rows in the
 * matrix's permuted order, elements c128 (prec FP64) or c64 (prec MIXED).
 * m % n_b == 0.  d_src and d_dst must not overlap.
 */
int chebfd_pack(const chebfd_matrix *H, int32_t m, int32_t n_b, int32_t prec,
                const void *d_colmajor, void *d_blocked, void *stream);
int chebfd_unpack(const chebfd_matrix *H, int32_t m, int32_t n_b, int32_t prec,
                  const void *d_blocked, void *d_colmajor, void *stream);

/*
 * Random-phase block in the blocked layout (the start block of chebfd_solve;
 * the paper leaves the start vectors open): entry (row r, column j) is
 * exp(2 pi i u) with u = top 53 bits of splitmix64(k_j xor r) * 2^-53,
 * k_j = splitmix64(splitmix64(seed) xor (col0 + j)) and r the row's index in
 * the caller's (original) order, so the block does not depend on H's row order
 * or on n_b.  m columns (m % n_b == 0), precision prec; d_blocked must be
 * 16-byte aligned and hold m n elements.  Enqueued on `stream`.
 */
int chebfd_random_phase(const chebfd_matrix *H, int32_t m, int32_t n_b, int32_t prec, uint64_t seed,
                        uint64_t col0, void *d_blocked, void *stream);

/*
 * The polynomial filter (Alg. 1 on each block, Alg. 2 over the blocks):
 * d_xy (blocked layout, n_s vectors, precision `prec`) holds X on entry and
 * Y = sum_{p=0}^{n_p} gamma_p T_p(alpha H + beta I) X on return (the paper
 * overwrites X by the filtered block).  Each step p >= 3 is one launch of the
 * fused kernel (chebfd_op: recurrence W <- 2(alpha H + beta I) U - W, the dot
 * products eta_p = <W, U>, mu_p = <U, U> and X <- X + gamma_p W in one pass).
 * d_u, d_w: n x n_b work blocks of the same precision.
 * d_eta: (n_p + 1) x n_s c128 and d_nu: (n_p + 1) x n_s FP64 (entry p*n_s + j,
 * column j in 0..n_s-1), receiving for p = 1..n_p
 *   eta[p] = <T_p x, T_{p-1} x>,  nu[p] = <T_{p-1} x, T_{p-1} x>
 * (with <a, b> = sum_i conj(a_i) b_i, FP64 accumulation, deterministic
 * summation order); row 0 is not written.  May be NULL together (moments not
 * needed is not faster: they are computed in the same pass).
 * d_work: chebfd_filter_query bytes (the partial sums of the dot products and
 * one progress word per workgroup of the window kernel, tagged per launch, so
 * nothing has to start at zero).  n_b in {1,2,4,8,16,32,64,128},
 * n_s % n_b == 0, n_p >= 0, gamma[n_p + 1] on the host.
 * Buffers must be 256-byte aligned and must not overlap.
 */
int chebfd_filter_query(const chebfd_matrix *H, int32_t n_b, size_t *work_bytes);

/*
 * The fused-step kernel that chebfd_filter, chebfd_op, chebfd_spmmv and the
 * moment calls launch for H and n_b (all compute the same step; they differ in
 * what they stage in LDS):
 *   CHEBFD_KERNEL_WINDOW   one workgroup per CU sweeps a contiguous row range and
 *                          gathers U from a window of U rows staged in LDS (FP64
 *                          n_b = 32, c64 n_b = 64, and c64 n_b = 32 from 32
 *                          tiles of 64 rows per CU on; C = 32; rows of at most 13 entries;
 *                          window_local[] >= 700 for the tile height); the
 *                          ranges of one XCD are held within a few tiles of
 *                          each other through progress words in the workspace
 *   CHEBFD_KERNEL_LDS      the tile's matrix slots staged in LDS, U gathered from
 *                          memory (rows of up to 16 entries, C <= 32)
 *   CHEBFD_KERNEL_ROW      one row per wavefront group (n_b >= 32, wider rows)
 *   CHEBFD_KERNEL_MULTIROW several rows per wavefront (n_b < 32, wider rows)
 */
#define CHEBFD_KERNEL_LDS      0
#define CHEBFD_KERNEL_ROW      1
#define CHEBFD_KERNEL_MULTIROW 2
#define CHEBFD_KERNEL_WINDOW   3
int chebfd_step_kernel(const chebfd_matrix *H, int32_t n_b, int32_t *kind);
int chebfd_filter(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma,
                  int32_t n_p, int32_t n_s, int32_t n_b, int32_t prec, void *d_xy, void *d_u,
                  void *d_w, double *d_eta, double *d_nu, void *d_work, size_t work_bytes,
                  void *stream);

/*
 * The same filter built from separate calls instead of the fused step (the
 * paper's comparison of chebfd_op with a minimum set of standard SpMMV and
 * BLAS1 calls, Sect. 3.2 and Fig. 2): per step p >= 3 one SpMMV launch
 * W <- 2(alpha H + beta I) U - W (the step kernel chebfd_step_kernel names,
 * without the dot products and the update), then the block dot products
 * eta_p = <W, U> and mu_p = <U, U> (one pass over their operands each, then a
 * small reduction launch) and the block axpby X <- X + gamma_p W; the start
 * steps use the same calls (W <- X copied before the second SpMMV, X <- g0 X
 * + g1 U + g2 W as a scal and two axpby).  Arguments, layouts, outputs,
 * workspace (chebfd_filter_query bytes) and errors as chebfd_filter; results
 * equal it up to rounding order.  Each extra call moves its operands through
 * HBM again: about 1.7x the bytes of the fused step at n_b = 32.
 */
int chebfd_filter_unfused(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma,
                          int32_t n_p, int32_t n_s, int32_t n_b, int32_t prec, void *d_xy, void *d_u,
                          void *d_w, double *d_eta, double *d_nu, void *d_work, size_t work_bytes,
                          void *stream);

/*
 * chebfd_filter without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the partial dot-product sums that the step kernels
 * hand from one launch to the next, and the window kernel's progress words,
 * live in a static device array of 4 MiB
 * (one copy per device, held until the process ends).  Every call on a device
 * shares that device's array: calls that overlap on one device (on different
 * streams, or from several threads) race; calls in sequence on a stream are
 * safe, since each launch overwrites the partials it later reads and nothing
 * has to start at zero.  Returns CHEBFD_EWORKSPACE, touching nothing, when
 * the launch geometry for H and n_b needs more than the array holds
 * (chebfd_filter_query bytes > 4 MiB: large n_b with many resident
 * workgroups).  Allocates nothing; other arguments, results and errors as
 * chebfd_filter (the same kernels in the same order: bitwise equal results).
 */
int chebfd_filter_noalloc(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma,
                          int32_t n_p, int32_t n_s, int32_t n_b, int32_t prec, void *d_xy, void *d_u,
                          void *d_w, double *d_eta, double *d_nu, void *stream);

/*
 * The filter on a search space held in host memory, for working sets larger
 * than the device memory (Sect. 3.5, Fig. 6: each block is loaded once and
 * then filtered for n_p steps, so the transfers are amortised over n_p).
 * h_xy: pinned host memory (hipHostMalloc or equivalent; pageable memory works
 * but its copies do not overlap) in the blocked layout of chebfd_pack, n_s
 * vectors of precision `prec`; X on entry, Y once `stream` has completed.
 * The blocks pass through two device staging blocks in d_work: block b + 1 is
 * copied in on `copy_stream` while block b is filtered on `stream` (with
 * chebfd_filter: same kernels, bitwise equal results), and block b is copied
 * back on `copy_stream` once its filter is done; `stream` finally waits for
 * the last copy.  d_u, d_w: n x n_b work blocks; d_eta, d_nu as chebfd_filter
 * (device memory, may be NULL together); d_work: chebfd_filter_streamed_query
 * bytes (two blocks of n x n_b, the moments of one block and the filter's
 * workspace), 256-byte aligned.  copy_stream must differ from stream and both
 * must belong to the current device.  Errors as chebfd_filter.
 */
int chebfd_filter_streamed_query(const chebfd_matrix *H, int32_t n_p, int32_t n_b, size_t *work_bytes);
int chebfd_filter_streamed(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma, int32_t n_p,
                           int32_t n_s, int32_t n_b, int32_t prec, void *h_xy, void *d_u, void *d_w, double *d_eta,
                           double *d_nu, void *d_work, size_t work_bytes, void *stream, void *copy_stream);

/*
 * One fused Chebyshev step on one block, as timed by the benchmarks (the
 * recurrence step of Alg. 1): W <- 2(alpha H + beta I) U - W in place, eta_p = <W, U>,
 * mu_p = <U, U>, Y <- Y + gamma W.  Same layouts and workspace as
 * chebfd_filter; the dot products stay in d_work (not reduced).
 */
int chebfd_op(const chebfd_matrix *H, double alpha, double beta, double gamma, int32_t n_b,
              int32_t prec, const void *d_u, void *d_w, void *d_y, void *d_work,
              size_t work_bytes, void *stream);

/*
 * Sparse matrix times one block (the first product of Alg. 1, spmmv()): Y = (alpha H + beta I) X
 * for an n x n_b block in the blocked layout and the matrix's precision.
 * d_work: chebfd_filter_query bytes.  X and Y must not overlap.
 */
int chebfd_spmmv(const chebfd_matrix *H, double alpha, double beta, int32_t n_b, int32_t prec,
                 const void *d_x, void *d_y, void *d_work, size_t work_bytes, void *stream);

/*
 * Kernel polynomial method moments (Sect. 2, the density-of-states and
 * eigenvalue-count estimate that Alg. 1's dot products feed): R random-phase
 * vectors x^(r) (|x_i| = 1, drawn on the device from `seed` with the same
 * counter-based generator as chebfd_solve's start block, columns 0..R-1) are
 * run through the Chebyshev recurrence of H~ = alpha H + beta I for n_steps
 * steps without forming a filtered block, and
 *   h_mu[m] = (1 / (n R)) sum_r Re <x^(r), T_m(H~) x^(r)>,  m = 0 .. 2 n_steps - 1
 * is returned on the host (h_mu: 2 n_steps doubles), the moments of order >=
 * n_steps + 1 from the product rule T_k T_k = (T_2k + T_0) / 2 and
 * T_{k+1} T_k = (T_2k+1 + T_1) / 2.  h_mu[0] is 1 up to rounding.
 * R: a power of two up to 32 or a multiple of 32 (blocks of min(R, 32)).
 * n_steps >= 1.  Precision: the matrix's (FP64 accumulation of the products).
 * d_work: chebfd_kpm_query bytes, 256-byte aligned.  Synchronises the stream.
 */
int chebfd_kpm_query(const chebfd_matrix *H, int32_t n_steps, int32_t R, size_t *work_bytes);
int chebfd_kpm_moments(const chebfd_matrix *H, double alpha, double beta, int32_t n_steps, int32_t R,
                       uint64_t seed, double *h_mu, void *d_work, size_t work_bytes, void *stream);

/*
 * Tall-skinny Gram product S = A^H B (FP64 complex, S column-major with leading
 * dimension ld >= m1) of two n x m1 and n x m2 block vectors in the blocked
 * layout (block width n_b, precision prec), with FP64 MFMA; the row range is
 * split over workgroups and the partial products are summed in a fixed order.
 * When d_a == d_b and m1 == m2 the product is Hermitian: only the 64 x 64 tiles
 * on and above the diagonal are formed and the rest of S is their mirror image
 * (exactly conj-symmetric).  d_work: chebfd_gram_query bytes.
 */
int chebfd_gram_query(int64_t n, int32_t m1, int32_t m2, size_t *work_bytes);
int chebfd_gram(int64_t n, int32_t n_b, int32_t m1, int32_t m2, int32_t prec, const void *d_a,
                const void *d_b, double *d_s, int32_t ld, void *d_work, size_t work_bytes,
                void *stream);

/*
 * Tall-skinny update Z = A M: A n x m1 (blocked, precision prec_a), M m1 x m2 FP64
 * complex column-major (ldm), Z n x m2 (blocked, precision prec_z), FP64 MFMA.
 * A and Z must not overlap.
 */
int chebfd_update(int64_t n, int32_t n_b, int32_t m1, int32_t m2, int32_t prec_a, const void *d_a,
                  const double *d_m, int32_t ldm, int32_t prec_z, void *d_z, void *stream);

/*
 * Tall-skinny QR (TSQR; Sect. 2 names it as the alternative to SVQB in the
 * orthogonalisation before the restart): d_y = Q R for an n x m block vector
 * d_y in the blocked layout (block width n_b, precision prec), 1 <= m <= n,
 * m <= 4096.  Q (n x m, same layout and precision) is written to d_q, which
 * must not overlap d_y; R (m x m, FP64 complex, column-major, ld_r >= m) to
 * d_r: upper triangular with a real non-negative diagonal (the unique such
 * factorisation when d_y has full column rank; for a dependent column k,
 * R_kk is at rounding level and column k of Q is an unspecified unit vector).
 * Columns are taken in panels of min(n_b, 32): each panel is projected
 * against the finished ones twice (block Gram-Schmidt with FP64 MFMA), then
 * factorised by a reduction tree of Householder QRs over 256-row blocks.  All
 * arithmetic is FP64.  d_work: chebfd_tsqr_query bytes, 256-byte aligned.
 * Asynchronous on `stream`.
 */
int chebfd_tsqr_query(int64_t n, int32_t m, int32_t n_b, size_t *work_bytes);
int chebfd_tsqr(int64_t n, int32_t m, int32_t n_b, int32_t prec, const void *d_y, void *d_q, double *d_r,
                int32_t ld_r, void *d_work, size_t work_bytes, void *stream);

/*
 * Eigendecomposition of a Hermitian m x m FP64 complex matrix (m <= 512) by
 * cyclic Jacobi rotations (one launch per round of disjoint rotations, one
 * workgroup per rotation pair): d_w receives the eigenvalues in
 * ascending order, d_v (ldv) the eigenvectors; d_a (lda) is overwritten.
 * Synchronises `stream`; CHEBFD_ENUMERIC if 40 sweeps do not reduce the
 * off-diagonal Frobenius norm below 4 m 2^-53 of the matrix's.
 */
int chebfd_heev_query(int32_t m, size_t *work_bytes);
int chebfd_heev(int32_t m, double *d_a, int32_t lda, double *d_v, int32_t ldv, double *d_w,
                void *d_work, size_t work_bytes, void *stream, int32_t *h_sweeps);

/*
 * The ChebFD iteration (Sect. 2): filter the search block, orthonormalise it
 * (rank revealing, tau = max(100 eps, (10 eps_store)^2)) by SVQB twice
 * (p->orth CHEBFD_ORTH_SVQB: Gram eigenvalues below tau times the largest are
 * dropped) or by TSQR (CHEBFD_ORTH_TSQR: chebfd_tsqr; a column k with
 * |R_kk|^2 <= tau ||y_k||^2 is dropped and the kept columns are factorised
 * again), Rayleigh-Ritz on the kept directions, residuals in FP64, restart
 * from the Ritz vectors plus fresh random-phase vectors in place of dropped
 * directions.
 * A Ritz pair inside the closed interval [lam_L, lam_R] is converged if its
 * residual ||H z - theta z|| (||z|| = 1) is <= tol, unresolved otherwise; the
 * iteration stops when the number of converged pairs repeats the previous
 * iteration's and the smallest unresolved residual did not halve since the
 * previous iteration, or no pair is unresolved (status CHEBFD_OK: an unresolved
 * pair whose residual no longer falls under the filter is a mixture of
 * eigenvectors at or beyond the interval's edges), after max_iter iterations
 * (CHEBFD_NOT_CONVERGED), or when, from the second iteration on, more than
 * 3/4 n_s Ritz pairs in the interval have residuals below (lam_R - lam_L) / 2
 * (CHEBFD_SUBSPACE_SMALL).
 *
 * Mixed precision (p->prec MIXED): the c64 basis bounds the residuals below by
 * about 2^-24 |lambda - theta|.  The iteration therefore runs in two stages:
 * c64 until the interval's pairs reach max(tol, 16 2^-24 max|lam_lo|,|lam_hi|)
 * or their residuals stop halving, then FP64 (filter with H64, blocks of
 * n_b / 2) on the Ritz vectors closest to the interval, the in-interval ones
 * first, at most n_s / 2 of them (kept in the c64 basis buffers), until the
 * convergence rule holds with tol.  Both stages count towards max_iter.
 *
 * H is the filter's matrix (precision p->prec); H64 an FP64 copy of the same
 * matrix (same n, C, sigma) for the Rayleigh-Ritz products and residuals (may
 * be H itself when p->prec is FP64).  d_x0: n x n_s c128 column-major start
 * block, or NULL for random phases exp(2 pi i u) with u from SplitMix64
 * (seed p->seed; the same vectors as topi.random_phase_block).  Refill vectors
 * of iteration k use the same generator with column offset k n_s.
 * Outputs: h_theta[n_s] and h_resid[n_s]: the converged pairs first (ascending),
 * then the other Ritz values (ascending); d_Z (n x n_s c128 column-major, may be
 * NULL): the Ritz vectors in the same order, each scaled so that its largest
 * entry is real positive; columns beyond the kept directions are zero.
 * With CHEBFD_VERBOSE=1 in the environment one progress line per iteration
 * goes to stderr.
 */
#define CHEBFD_ORTH_SVQB 0
#define CHEBFD_ORTH_TSQR 1

typedef struct chebfd_params {
    double lam_L, lam_R;   /* closed search interval, H's units */
    int32_t n_s, n_p, n_b; /* subspace size (multiple of n_b), filter degree, block width */
    int32_t prec;          /* CHEBFD_PREC_* of the filter */
    double tol;            /* residual tolerance */
    int32_t max_iter;
    int32_t orth;          /* CHEBFD_ORTH_SVQB (0) or CHEBFD_ORTH_TSQR (1) */
    uint64_t seed;
    double spec_lo, spec_hi; /* spectral bounds of H; NaN for Gershgorin bounds */
} chebfd_params;

typedef struct chebfd_stats {
    int32_t iterations, n_found, n_kept, status;
    double count_est;       /* eigenvalue count estimate from the first filter's moments */
    double t_total, t_filter, t_orth, t_rr, t_resid;  /* seconds (HIP events) */
    double filter_bytes;    /* algorithmic bytes of all filter applications */
} chebfd_stats;

int chebfd_solve_query(const chebfd_matrix *H, const chebfd_matrix *H64, const chebfd_params *p,
                       size_t *work_bytes);
int chebfd_solve(const chebfd_matrix *H, const chebfd_matrix *H64, const chebfd_params *p,
                 const void *d_x0, void *d_work, size_t work_bytes, void *stream, int32_t *n_found,
                 double *h_theta, void *d_Z, double *h_resid, chebfd_stats *st);

/*
 * Parameter choice (n_p, n_s) for chebfd_solve.  The paper fixes n_p and n_s
 * by hand (Sect. 2: n_s above the number of wanted eigenpairs; Sect. 2.1:
 * n_p around 10^3) and points to the KPM moments of the filter's dot products
 * as the cheap view of the spectrum (Sect. 2).  Two predictors use them:
 *  - a heuristic: n_s = max(n_b, round_up_{n_b}(2 n_hat)),
 *    n_p = clamp(round(kappa / delta), 50, 20000) with delta = (b~ - a~) / 2
 *    the half width of the scaled interval and n_hat the eigenvalue count
 *    estimate from the moments;
 *  - a small MLP (below) on the moment features, whose two outputs are
 *    scale-free ratios, standardised: log(n_p delta) (its own kappa) and
 *    log(n_s / max(2 n_hat, n_b)) (its factor on the heuristic's n_s).  Ratios
 *    transfer across matrix sizes: delta and n_hat already carry the size.
 */
#define CHEBFD_FEATURE_R        16   /* random-phase vectors of the feature moments */
#define CHEBFD_FEATURE_MOMENTS  256  /* moments mu~_0 .. mu~_255 (128 Chebyshev steps) */
#define CHEBFD_MLP_IN     258        /* 256 moments + [a~, b~] */
#define CHEBFD_MLP_HIDDEN 128
#define CHEBFD_MLP_OUT    2
#define CHEBFD_MLP_PARAMS 49922      /* 128*258 + 128 + 128*128 + 128 + 2*128 + 2 */
#define CHEBFD_NP_MIN     50
#define CHEBFD_NP_MAX     20000

typedef struct chebfd_predictor {
    double kappa;           /* heuristic: n_p = kappa / delta */
    double t_mean[2];       /* MLP output de-standardisation: log(n_p delta), log(n_s / max(2 n_hat, n_b)) */
    double t_std[2];
    double t_lo[2];         /* de-standardised outputs are clamped to [t_lo, t_hi] (the range of the */
    double t_hi[2];         /* training targets) where t_lo < t_hi; t_lo = t_hi = 0: no clamp */
} chebfd_predictor;

/*
 * Features of (H, [lam_L, lam_R]): Gershgorin scaling (alpha, beta), the
 * CHEBFD_FEATURE_MOMENTS averaged moments of chebfd_kpm_moments with
 * CHEBFD_FEATURE_R vectors from `seed`, then a~ = alpha lam_L + beta and
 * b~ = alpha lam_R + beta: h_features[258] (FP32, host), except that slot 0
 * (mu~_0, which is 1 by construction) holds log10(n) / 8: the moments are per
 * row and the network also needs the size.  *count_est: the
 * eigenvalue count estimate n sum_m g_m c_m mu~_m over the same moments (window
 * coefficients of [a~, b~] and Jackson damping for 256 terms).  Synchronises.
 * CHEBFD_EINTERVAL unless -1 < a~ < b~ < 1.
 */
int chebfd_features_query(const chebfd_matrix *H, size_t *work_bytes);
int chebfd_features(const chebfd_matrix *H, double lam_L, double lam_R, uint64_t seed, float *h_features,
                    double *count_est, double *alpha, double *beta, void *d_work, size_t work_bytes,
                    void *stream);

/*
 * (n_p, n_s) from the scaled interval [a, b], the count estimate and either the
 * MLP's two outputs (h_mlp_out, host: standardised log(n_p delta) and
 * log(n_s / max(2 n_hat, n_b)), so n_p = exp(t_std[0] y0 + t_mean[0]) / delta
 * and n_s = exp(t_std[1] y1 + t_mean[1]) max(2 n_hat, n_b), each exponent first
 * clamped to [t_lo, t_hi] when that range is set) or, with h_mlp_out NULL,
 * the heuristic.  Both are clamped: n_p to
 * [CHEBFD_NP_MIN, CHEBFD_NP_MAX]; n_s to a multiple of n_b that is at least
 * max(n_b, 1.2 n_hat) and at most 512.  Host only, no device work.
 */
int chebfd_choose_params(double a, double b, double count_est, int32_t n_b, const float *h_mlp_out,
                         const chebfd_predictor *pr, int32_t *n_p, int32_t *n_s);

/*
 * The predictor network (FP32, device): x (258) -> relu(W1 x + b1) (128)
 * -> relu(W2 h1 + b2) (128) -> y = W3 h2 + b3 (2).  d_params: the flat
 * CHEBFD_MLP_PARAMS vector W1, b1, W2, b2, W3, b3, weight matrices row-major
 * with the output index slowest (caller-owned).  Batches are row-major:
 * d_x batch x 258, d_y / d_t batch x 2.  d_work: chebfd_mlp_query bytes,
 * 256-byte aligned.  Results are bit-reproducible (fixed summation orders).
 *  forward: d_y = network(d_x).
 *  grad:    d_loss[0] = sum ||y - t||^2 / (2 batch), d_grad = d loss / d params.
 *  adam:    one Adam step (Kingma and Ba; bias-corrected, step counts from 1)
 *           on params with moment buffers d_m, d_v (zero before step 1).
 */
int chebfd_mlp_query(int32_t batch, int32_t *n_params, size_t *work_bytes);
int chebfd_mlp_forward(const float *d_params, int32_t batch, const float *d_x, float *d_y, void *d_work,
                       size_t work_bytes, void *stream);
int chebfd_mlp_grad(const float *d_params, int32_t batch, const float *d_x, const float *d_t, float *d_loss,
                    float *d_grad, void *d_work, size_t work_bytes, void *stream);
int chebfd_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step, float lr,
                    float beta1, float beta2, float eps, void *stream);

/*
 * HBM bandwidth probe (the STREAM analogue of Sect. 1.2, Table 2) over
 * `count` doubles (even): kind 0 = copy a = b (one 16-byte element per
 * thread), 1 = triad a = b + s c, 2 = copy a = b with non-temporal loads and
 * stores, four 16-byte elements per thread, 3 = read-only pass over b (one
 * sum per workgroup of 1024 doubles written to the front of a).
 */
int chebfd_probe_stream(int32_t kind, int64_t count, const double *d_b, const double *d_c,
                        double s, double *d_a, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CHEBFD_H */
