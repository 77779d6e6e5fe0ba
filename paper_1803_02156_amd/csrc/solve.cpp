// ChebFD outer loop on the device: filter (Alg. 1 / Alg. 2), SVQB
// orthonormalisation (twice, rank revealing), Rayleigh-Ritz on the kept
// directions, FP64 residuals, restart.  The paper describes the filter and names
// the orthogonalisation before the restart (Sect. 2); the restart and
// convergence rules used here are stated in include/chebfd.h.
//
// Host work per iteration: deciding how many SVQB directions to keep (needs the
// Gram eigenvalues), the convergence test (needs the Ritz values and
// residuals), and on the first iteration the eigenvalue-count estimate from the
// moments.  These are the only device -> host copies; everything else is
// enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace chebfd {
namespace {

size_t al(size_t v) { return round_up(v, 256); }

// Stopping tolerance of the Jacobi sweeps: off-diagonal Frobenius norm at most
// 4 m u ||A||_F (u = 2^-53).  Once the rotations are at rounding level each of
// the m(m-1) off-diagonal entries keeps a residue of order u ||A||, so a
// tolerance independent of m would never be met.
double jacobi_tol(int m) { return 4.0 * std::max(m, 1) * 0x1.0p-53; }

struct SolveLayout {
    size_t x, q, u, w, z64, t64, b64;
    size_t S, V, G, T, wv, d, theta, rr, phase, order;
    size_t eta, nu, fwork, gpart, rpart, jwork, tree;
    size_t fwork_bytes, gpart_bytes, rpart_bytes, jwork_bytes, total;
    int rgrid;
};

int solve_layout(const chebfd_matrix *H, const chebfd_matrix *H64, const chebfd_params *p,
                 SolveLayout *L) {
    const size_t n = H->n, ns = p->n_s, nb = p->n_b, sw = vec_elem_bytes(p->prec);
    size_t f1 = 0, f2 = 0;
    int rc = chebfd_filter_query(H, p->n_b, &f1);
    if (rc) return rc;
    if ((rc = chebfd_filter_query(H64, p->n_b, &f2))) return rc;
    L->fwork_bytes = std::max(f1, f2);
    if (p->prec != CHEBFD_PREC_FP64 && p->n_b > 1) {
        // the FP64 stage of a mixed run filters with n_b / 2
        size_t f3 = 0;
        if ((rc = chebfd_filter_query(H64, p->n_b / 2, &f3))) return rc;
        L->fwork_bytes = std::max(L->fwork_bytes, f3);
    }
    // the largest partial buffer of any Gram product the iteration forms (SVQB:
    // m x m with m <= n_s kept directions; Rayleigh-Ritz: m x n_b or n_b / 2)
    L->gpart_bytes = 0;
    const int tmax = (p->n_s + 63) / 64;
    for (int ta = 1; ta <= tmax; ++ta)
        for (int tb = 1; tb <= tmax; ++tb)
            L->gpart_bytes = std::max(L->gpart_bytes,
                                      gram_part_bytes(64 * ta, 64 * tb, gram_splits(H->n, 64 * ta, 64 * tb)));
    L->rgrid = resid_grid(H->n);
    L->rpart_bytes = (size_t)2 * nb * L->rgrid * 8;
    if ((rc = chebfd_heev_query(p->n_s, &L->jwork_bytes))) return rc;
    size_t at = 0;
    auto take = [&](size_t bytes) { size_t h = at; at += al(bytes); return h; };
    L->x = take(n * ns * sw);
    L->q = take(n * ns * sw);
    L->u = take(n * nb * sw);
    L->w = take(n * nb * sw);
    L->z64 = take(n * nb * 16);
    L->t64 = take(n * nb * 16);
    L->b64 = take(n * nb * 16);
    L->S = take(ns * ns * 16);
    L->V = take(ns * ns * 16);
    L->G = take(ns * ns * 16);
    L->T = take(ns * ns * 16);
    L->wv = take(ns * 8);
    L->d = take(ns * 8);
    L->theta = take(ns * 8);
    L->rr = take(2 * nb * 8);
    L->phase = take(2 * ns * 8);
    L->order = take(ns * 4);
    L->eta = take((size_t)(p->n_p + 1) * ns * 16);
    L->nu = take((size_t)(p->n_p + 1) * ns * 8);
    L->fwork = take(L->fwork_bytes);
    L->gpart = take(L->gpart_bytes);
    L->rpart = take(L->rpart_bytes);
    L->jwork = take(L->jwork_bytes);
    // TSQR: the panel and its projection use the FP64 blocks of the Rayleigh-Ritz step
    // (n x n_b each, free during the orthogonalisation); the reduction tree needs its own
    L->tree = take(p->orth == CHEBFD_ORTH_TSQR ? tsqr_tree_bytes(H->n, tsqr_panel_width(p->n_b)) : 0);
    L->total = at;
    return CHEBFD_OK;
}

int check_params(const chebfd_matrix *H, const chebfd_matrix *H64, const chebfd_params *p) {
    CHEBFD_REQUIRE(H && H64 && p, "NULL argument");
    CHEBFD_REQUIRE(H->n >= 1 && H->val && H64->val, "matrix handle not built");
    CHEBFD_REQUIRE(H64->prec == CHEBFD_PREC_FP64, "H64 must hold FP64 values");
    CHEBFD_REQUIRE(H->prec == p->prec, "p->prec %d differs from the matrix's %d", p->prec, H->prec);
    CHEBFD_REQUIRE(H64->n == H->n && H64->C == H->C && H64->sigma == H->sigma &&
                       H64->identity_perm == H->identity_perm,
                   "H and H64 must be built from the same matrix with the same C and sigma");
    CHEBFD_REQUIRE(p->n_b >= 1 && p->n_b <= 128 && (p->n_b & (p->n_b - 1)) == 0,
                   "n_b = %d must be a power of two in [1, 128]", p->n_b);
    CHEBFD_REQUIRE(p->n_s >= p->n_b && p->n_s % p->n_b == 0 && p->n_s <= 512,
                   "n_s = %d must be a multiple of n_b and at most 512", p->n_s);
    CHEBFD_REQUIRE(p->n_p >= 2, "n_p = %d < 2", p->n_p);
    CHEBFD_REQUIRE(p->max_iter >= 1, "max_iter < 1");
    CHEBFD_REQUIRE(std::isfinite(p->lam_L) && std::isfinite(p->lam_R) && p->lam_L < p->lam_R,
                   "search interval invalid");
    CHEBFD_REQUIRE(p->tol > 0.0, "tol must be positive");
    CHEBFD_REQUIRE(p->orth == CHEBFD_ORTH_SVQB || p->orth == CHEBFD_ORTH_TSQR, "orth = %d invalid", p->orth);
    return CHEBFD_OK;
}

double tau_for(int prec) {
    const double eps = 0x1.0p-53, es = prec == CHEBFD_PREC_FP64 ? 0x1.0p-53 : 0x1.0p-24;
    return std::max(100.0 * eps, (10.0 * es) * (10.0 * es));
}

struct Timer {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Timer() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

}  // namespace
}  // namespace chebfd

using namespace chebfd;

extern "C" {

int chebfd_gram_query(int64_t n, int32_t m1, int32_t m2, size_t *work_bytes) {
    clear_error();
    CHEBFD_REQUIRE(n >= 1 && m1 >= 1 && m2 >= 1 && work_bytes, "invalid Gram sizes");
    *work_bytes = gram_part_bytes(m1, m2, gram_splits(n, m1, m2));
    return CHEBFD_OK;
}

int chebfd_gram(int64_t n, int32_t n_b, int32_t m1, int32_t m2, int32_t prec, const void *d_a,
                const void *d_b, double *d_s, int32_t ld, void *d_work, size_t work_bytes,
                void *stream) {
    clear_error();
    CHEBFD_REQUIRE(n >= 1 && m1 >= 1 && m2 >= 1 && ld >= m1, "invalid Gram sizes");
    CHEBFD_REQUIRE(n_b >= 1 && n_b <= 128 && (n_b & (n_b - 1)) == 0, "n_b = %d invalid", n_b);
    CHEBFD_REQUIRE(prec == CHEBFD_PREC_FP64 || prec == CHEBFD_PREC_MIXED, "prec invalid");
    CHEBFD_REQUIRE(d_a && d_b && d_s && d_work, "NULL buffer");
    size_t need;
    int rc = chebfd_gram_query(n, m1, m2, &need);
    if (rc) return rc;
    if (work_bytes < need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "Gram workspace %zu < %zu", work_bytes, need);
    return launch_gram(d_a, prec, n_b, d_b, prec, n_b, n, m1, m2, static_cast<double *>(d_work),
                       gram_splits(n, m1, m2), d_s, ld, static_cast<hipStream_t>(stream));
}

int chebfd_update(int64_t n, int32_t n_b, int32_t m1, int32_t m2, int32_t prec_a, const void *d_a,
                  const double *d_m, int32_t ldm, int32_t prec_z, void *d_z, void *stream) {
    clear_error();
    CHEBFD_REQUIRE(n >= 1 && m1 >= 1 && m2 >= 1 && ldm >= m1, "invalid update sizes");
    CHEBFD_REQUIRE(n_b >= 1 && n_b <= 128 && (n_b & (n_b - 1)) == 0, "n_b = %d invalid", n_b);
    CHEBFD_REQUIRE(d_a && d_m && d_z, "NULL buffer");
    CHEBFD_REQUIRE(!overlap(d_a, vec_elem_bytes(prec_a) * (size_t)n * ((m1 + n_b - 1) / n_b * n_b), d_z,
                            vec_elem_bytes(prec_z) * (size_t)n * ((m2 + n_b - 1) / n_b * n_b)),
                   "A and Z overlap");
    return launch_update(d_a, prec_a, n_b, d_m, ldm, d_z, prec_z, n_b, n, m1, m2,
                         static_cast<hipStream_t>(stream));
}

int chebfd_tsqr_query(int64_t n, int32_t m, int32_t n_b, size_t *work_bytes) {
    clear_error();
    CHEBFD_REQUIRE(work_bytes, "NULL argument");
    CHEBFD_REQUIRE(n >= 1 && m >= 1 && m <= n && m <= 4096, "TSQR sizes n = %lld, m = %d invalid",
                   (long long)n, m);
    CHEBFD_REQUIRE(n_b >= 1 && n_b <= 128 && (n_b & (n_b - 1)) == 0, "n_b = %d invalid", n_b);
    const size_t pw = tsqr_panel_width(n_b);
    *work_bytes = al((size_t)n * pw * 16) + al(tsqr_tree_bytes(n, (int)pw)) + 2 * al((size_t)m * pw * 16) +
                  al(tsqr_gpart_bytes(n, m, n_b));
    return CHEBFD_OK;
}

int chebfd_tsqr(int64_t n, int32_t m, int32_t n_b, int32_t prec, const void *d_y, void *d_q, double *d_r,
                int32_t ld_r, void *d_work, size_t work_bytes, void *stream) {
    size_t need;
    int rc = chebfd_tsqr_query(n, m, n_b, &need);
    if (rc) return rc;
    CHEBFD_REQUIRE(prec == CHEBFD_PREC_FP64 || prec == CHEBFD_PREC_MIXED, "prec invalid");
    CHEBFD_REQUIRE(d_y && d_q && d_r && d_work, "NULL buffer");
    CHEBFD_REQUIRE(ld_r >= m, "ld_r = %d < m = %d", ld_r, m);
    const size_t es = vec_elem_bytes(prec);
    CHEBFD_REQUIRE(aligned(d_y, es) && aligned(d_q, es) && aligned(d_r, 16) && aligned(d_work, 256),
                   "misaligned buffer");
    const size_t vbytes = es * (size_t)n * ((m + n_b - 1) / n_b * n_b);
    CHEBFD_REQUIRE(!overlap(d_y, vbytes, d_q, vbytes), "Y and Q overlap");
    if (work_bytes < need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "TSQR workspace %zu < %zu", work_bytes, need);
    const size_t pw = tsqr_panel_width(n_b);
    char *base = static_cast<char *>(d_work);
    size_t at = 0;
    auto take = [&](size_t bytes) { double *h = reinterpret_cast<double *>(base + at); at += al(bytes); return h; };
    TsqrWork w;
    w.T = take((size_t)n * pw * 16);
    w.tree = take(tsqr_tree_bytes(n, (int)pw));
    w.C1 = take((size_t)m * pw * 16);
    w.C2 = take((size_t)m * pw * 16);
    w.ldc = m;
    w.gpart = take(tsqr_gpart_bytes(n, m, n_b));
    return tsqr_blocked(n, m, n_b, prec, d_y, prec, d_q, d_r, ld_r, w, static_cast<hipStream_t>(stream));
}

int chebfd_heev_query(int32_t m, size_t *work_bytes) {
    clear_error();
    CHEBFD_REQUIRE(m >= 1 && m <= 512 && work_bytes, "eigensolver size %d not in [1, 512]", m);
    *work_bytes = al(jacobi_scratch_bytes(m));
    return CHEBFD_OK;
}

int chebfd_heev(int32_t m, double *d_a, int32_t lda, double *d_v, int32_t ldv, double *d_w,
                void *d_work, size_t work_bytes, void *stream, int32_t *h_sweeps) {
    clear_error();
    size_t need;
    int rc = chebfd_heev_query(m, &need);
    if (rc) return rc;
    CHEBFD_REQUIRE(d_a && d_v && d_w && d_work && lda >= m && ldv >= m, "invalid eigensolver arguments");
    if (work_bytes < need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "eigensolver workspace %zu < %zu", work_bytes, need);
    CHEBFD_REQUIRE(aligned(d_work, 256), "d_work must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int sweeps = 0, converged = 0;
    if ((rc = launch_jacobi(m, d_a, lda, d_v, ldv, d_w, 40, jacobi_tol(m), d_work, &sweeps, &converged, s)))
        return rc;
    if (h_sweeps) *h_sweeps = sweeps;
    if (!converged) CHEBFD_FAIL(CHEBFD_ENUMERIC, "Jacobi eigensolver did not converge in %d sweeps", sweeps);
    return CHEBFD_OK;
}

int chebfd_solve_query(const chebfd_matrix *H, const chebfd_matrix *H64, const chebfd_params *p,
                       size_t *work_bytes) {
    clear_error();
    int rc = check_params(H, H64, p);
    if (rc) return rc;
    CHEBFD_REQUIRE(work_bytes != nullptr, "work_bytes is NULL");
    SolveLayout L;
    if ((rc = solve_layout(H, H64, p, &L))) return rc;
    *work_bytes = L.total;
    return CHEBFD_OK;
}

int chebfd_solve(const chebfd_matrix *H, const chebfd_matrix *H64, const chebfd_params *p,
                 const void *d_x0, void *d_work, size_t work_bytes, void *stream, int32_t *n_found,
                 double *h_theta, void *d_Z, double *h_resid, chebfd_stats *st) {
    clear_error();
    int rc = check_params(H, H64, p);
    if (rc) return rc;
    CHEBFD_REQUIRE(d_work && aligned(d_work, 256), "d_work must be non-NULL and 256-byte aligned");
    CHEBFD_REQUIRE(n_found && h_theta && h_resid, "output pointer is NULL");
    SolveLayout L;
    if ((rc = solve_layout(H, H64, p, &L))) return rc;
    if (work_bytes < L.total) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "solve workspace %zu < %zu", work_bytes, L.total);

    hipStream_t s = static_cast<hipStream_t>(stream);
    // CHEBFD_VERBOSE=1 in the environment: one progress line per iteration on stderr
    const char *venv = std::getenv("CHEBFD_VERBOSE");
    const bool verbose = venv && venv[0] == '1';
    char *base = static_cast<char *>(d_work);
    auto D = [&](size_t off) { return static_cast<void *>(base + off); };
    auto DD = [&](size_t off) { return reinterpret_cast<double *>(base + off); };
    const int64_t n = H->n;
    const int ns = p->n_s, nb = p->n_b, prec = p->prec;
    const size_t sw = vec_elem_bytes(prec);
    const int32_t *perm = H->identity_perm ? nullptr : H->perm;

    // spectral scaling and filter coefficients
    double lo = p->spec_lo, hi = p->spec_hi;
    if (!std::isfinite(lo) || !std::isfinite(hi)) {
        size_t bq;
        if ((rc = chebfd_bounds_query(H64, &bq))) return rc;
        if (bq > L.fwork_bytes) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "bounds workspace");
        if ((rc = chebfd_bounds(H64, D(L.fwork), L.fwork_bytes, stream, &lo, &hi))) return rc;
    }
    double alpha, beta;
    std::vector<double> gamma(p->n_p + 1), gamma2(2 * p->n_p);
    if ((rc = chebfd_coefficients(lo, hi, p->lam_L, p->lam_R, p->n_p, &alpha, &beta, gamma.data()))) return rc;
    if ((rc = chebfd_coefficients(lo, hi, p->lam_L, p->lam_R, 2 * p->n_p - 1, &alpha, &beta, gamma2.data())))
        return rc;

    // start block
    if (d_x0) {
        if ((rc = chebfd_pack(H, ns, nb, prec, d_x0, D(L.x), stream))) return rc;
    } else {
        if ((rc = launch_random_phase(D(L.x), prec, n, nb, 0, ns, p->seed, 0, perm, s))) return rc;
    }

    Timer ev[5];
    for (auto &t : ev)
        for (auto &e : t.e) CHEBFD_HIP(hipEventCreate(&e));
    double t_phase[4] = {0, 0, 0, 0};
    std::vector<double> hw(ns), hth(ns), hrr(2 * nb), hres(ns), hnrm(ns);
    std::vector<double> heta, hnu;
    double count_est = 0.0;
    int status = CHEBFD_NOT_CONVERGED, it = 0, k2 = 0;
    double fbytes = 0.0;

    // The working set of one stage of the iteration.  Stage 1 runs in the
    // caller's precision on all n_s vectors.  In mixed precision the c64
    // storage of the basis puts a floor of about 2^-24 |lambda - theta| under
    // the residuals; stage 2 then continues in FP64 (matrix H64) from the
    // Ritz vectors nearest the interval, at most n_s / 2 of them in blocks of
    // n_b / 2, held in the c64 basis buffers (same bytes).
    struct Stage {
        const chebfd_matrix *H;
        int prec, ns, nb;
        void *X, *Q, *U, *W;
        double tol;
    };
    Stage S1{H, prec, ns, nb, D(L.x), D(L.q), D(L.u), D(L.w), p->tol};
    const double hmax = std::max(std::fabs(lo), std::fabs(hi));
    if (prec != CHEBFD_PREC_FP64) S1.tol = std::max(p->tol, 16.0 * 0x1.0p-24 * hmax);

    // one SVQB step on the stage's basis: A (m columns) -> B (k kept columns)
    auto svqb = [&](const Stage &g, void *A, int m, void *B, int *k) -> int {
        int r;
        if ((r = launch_gram(A, g.prec, g.nb, A, g.prec, g.nb, n, m, m, DD(L.gpart), gram_splits(n, m, m), DD(L.S), ns,
                             s)))
            return r;
        if ((r = launch_svqb_scale(m, DD(L.S), ns, DD(L.d), s))) return r;
        if ((r = chebfd_heev(m, DD(L.S), ns, DD(L.V), ns, DD(L.wv), D(L.jwork), L.jwork_bytes, stream, nullptr)))
            return r;
        CHEBFD_HIP(hipMemcpyAsync(hw.data(), DD(L.wv), sizeof(double) * m, hipMemcpyDeviceToHost, s));
        CHEBFD_HIP(hipStreamSynchronize(s));
        const double wmax = hw[m - 1];
        if (!(wmax > 0.0) || !std::isfinite(wmax)) CHEBFD_FAIL(CHEBFD_ENUMERIC, "SVQB: non-positive Gram matrix");
        const double tau = tau_for(g.prec);
        int kk = 0;
        for (int i = 0; i < m; ++i) kk += hw[i] > tau * wmax ? 1 : 0;
        if ((r = launch_svqb_transform(m, kk, m - kk, DD(L.d), DD(L.V), ns, DD(L.wv), DD(L.T), ns, s))) return r;
        if ((r = launch_update(A, g.prec, g.nb, DD(L.T), ns, B, g.prec, g.nb, n, m, kk, s))) return r;
        *k = kk;
        return CHEBFD_OK;
    };

    // TSQR of the stage's basis X (all ns columns) into Q; columns whose part
    // outside the span of the earlier ones is at the resolved level
    // (|R_kk|^2 <= tau ||y_k||^2) are dropped and the kept ones factorised again.
    // On return X holds the k kept orthonormal directions (the buffers swap).
    std::vector<double> hinfo(2 * (size_t)ns), hsel;
    auto orth_tsqr = [&](Stage &g, int *k) -> int {
        int r;
        const TsqrWork w{DD(L.b64), DD(L.tree), DD(L.V), DD(L.G), ns, DD(L.gpart)};
        if ((r = tsqr_blocked(n, g.ns, g.nb, g.prec, g.X, g.prec, g.Q, DD(L.S), ns, w, s))) return r;
        if ((r = launch_tsqr_colinfo(g.ns, DD(L.S), ns, DD(L.T), s))) return r;
        CHEBFD_HIP(hipMemcpyAsync(hinfo.data(), DD(L.T), sizeof(double) * 2 * g.ns, hipMemcpyDeviceToHost, s));
        CHEBFD_HIP(hipStreamSynchronize(s));
        const double tau = tau_for(g.prec);
        std::vector<int> keep;
        for (int c = 0; c < g.ns; ++c) {
            if (!std::isfinite(hinfo[2 * c]) || !std::isfinite(hinfo[2 * c + 1]))
                CHEBFD_FAIL(CHEBFD_ENUMERIC, "TSQR: non-finite R");
            if (hinfo[2 * c] > tau * hinfo[2 * c + 1]) keep.push_back(c);
        }
        const int kk = static_cast<int>(keep.size());
        if (kk == 0) CHEBFD_FAIL(CHEBFD_ENUMERIC, "TSQR: no independent column");
        if (kk < g.ns) {
            // Y's kept columns into Q (a selection matrix through the update), then TSQR back into X
            hsel.assign((size_t)2 * ns * kk, 0.0);
            for (int c = 0; c < kk; ++c) hsel[2 * ((size_t)c * ns + keep[c])] = 1.0;
            CHEBFD_HIP(hipMemcpyAsync(DD(L.T), hsel.data(), sizeof(double) * hsel.size(), hipMemcpyHostToDevice, s));
            if ((r = launch_update(g.X, g.prec, g.nb, DD(L.T), ns, g.Q, g.prec, g.nb, n, g.ns, kk, s))) return r;
            if ((r = tsqr_blocked(n, kk, g.nb, g.prec, g.Q, g.prec, g.X, DD(L.S), ns, w, s))) return r;
        } else {
            std::swap(g.X, g.Q);
        }
        *k = kk;
        return CHEBFD_OK;
    };

    // Iterations of one stage until its convergence rule holds or max_iter is
    // reached.  prev: in-window converged count the first test compares with.
    // On return the stage's X holds the last kept basis, S its Ritz vectors
    // (coefficients), hth / hres the k2 Ritz values and residuals.
    auto run_stage = [&](Stage &g, int prev, bool stage1, bool *stagnated) -> int {
        const size_t swg = vec_elem_bytes(g.prec);
        double prev_max = INFINITY, prev_unres = INFINITY;
        int prev_inwin = -1;
        *stagnated = false;
        for (++it; it <= p->max_iter; ++it) {
            // --- filter (Alg. 2 over blocks, Alg. 1 per block) ---
            CHEBFD_HIP(hipEventRecord(ev[0].e[0], s));
            const bool moments = stage1 && it == 1;
            double *d_eta = moments ? DD(L.eta) : nullptr, *d_nu = moments ? DD(L.nu) : nullptr;
            int r;
            if ((r = chebfd_filter(g.H, alpha, beta, gamma.data(), p->n_p, g.ns, g.nb, g.prec, g.X, g.U, g.W, d_eta,
                                   d_nu, D(L.fwork), L.fwork_bytes, stream)))
                return r;
            CHEBFD_HIP(hipEventRecord(ev[0].e[1], s));
            fbytes += (double)(g.ns / g.nb) *
                      ((double)(p->n_p - 2) * (double)(g.H->nnz * (swg + 4) + 5 * n * g.nb * swg) +
                       2.0 * (double)(g.H->nnz * (swg + 4)) + 6.0 * n * g.nb * swg);
            if (moments) {
                // moments -> eigenvalue count estimate (trace of the damped window polynomial)
                heta.resize((size_t)2 * (p->n_p + 1) * ns);
                hnu.resize((size_t)(p->n_p + 1) * ns);
                CHEBFD_HIP(hipMemcpyAsync(heta.data(), DD(L.eta), sizeof(double) * heta.size(), hipMemcpyDeviceToHost, s));
                CHEBFD_HIP(hipMemcpyAsync(hnu.data(), DD(L.nu), sizeof(double) * hnu.size(), hipMemcpyDeviceToHost, s));
                CHEBFD_HIP(hipStreamSynchronize(s));
                std::vector<double> se(p->n_p + 1, 0.0), sn(p->n_p + 1, 0.0);
                for (int q = 1; q <= p->n_p; ++q)
                    for (int j = 0; j < ns; ++j) {
                        se[q] += heta[2 * ((size_t)q * ns + j)];
                        sn[q] += hnu[(size_t)q * ns + j];
                    }
                const double mu0 = sn[1], mu1 = se[1];
                double acc = gamma2[0] * mu0 + gamma2[1] * mu1;
                for (int k = 1; k < p->n_p; ++k)
                    acc += gamma2[2 * k] * (2.0 * sn[k + 1] - mu0) + gamma2[2 * k + 1] * (2.0 * se[k + 1] - mu1);
                count_est = acc / ns;   // n * sum g c mu~ with mu~ = mu / (n R)
            }

            // --- orthogonalisation: SVQB twice, or TSQR ---
            CHEBFD_HIP(hipEventRecord(ev[1].e[0], s));
            if (p->orth == CHEBFD_ORTH_TSQR) {
                if ((r = orth_tsqr(g, &k2))) return r;
            } else {
                int k1 = 0;
                if ((r = svqb(g, g.X, g.ns, g.Q, &k1))) return r;
                if ((r = svqb(g, g.Q, k1, g.X, &k2))) return r;
            }
            CHEBFD_HIP(hipEventRecord(ev[1].e[1], s));

            // --- Rayleigh-Ritz on the k2 kept directions (FP64 products) ---
            CHEBFD_HIP(hipEventRecord(ev[2].e[0], s));
            const int kb = (k2 + g.nb - 1) / g.nb;
            for (int b = 0; b < kb; ++b) {
                const void *Xb = static_cast<const char *>(g.X) + (size_t)b * n * g.nb * swg;
                const void *X64 = Xb;
                if (g.prec != CHEBFD_PREC_FP64) {
                    if ((r = launch_convert(Xb, g.prec, D(L.b64), CHEBFD_PREC_FP64, n * g.nb, s))) return r;
                    X64 = D(L.b64);
                }
                if ((r = chebfd_spmmv(H64, 1.0, 0.0, g.nb, CHEBFD_PREC_FP64, X64, D(L.t64), D(L.fwork), L.fwork_bytes,
                                      stream)))
                    return r;
                const int cols = std::min(g.nb, k2 - b * g.nb);
                if ((r = launch_gram(g.X, g.prec, g.nb, D(L.t64), CHEBFD_PREC_FP64, g.nb, n, k2, cols, DD(L.gpart),
                                     gram_splits(n, k2, cols), DD(L.G) + 2 * (size_t)b * g.nb * ns, ns, s)))
                    return r;
            }
            if ((r = launch_hermitise(k2, DD(L.G), ns, s))) return r;
            if ((r = chebfd_heev(k2, DD(L.G), ns, DD(L.S), ns, DD(L.theta), D(L.jwork), L.jwork_bytes, stream,
                                 nullptr)))
                return r;
            CHEBFD_HIP(hipEventRecord(ev[2].e[1], s));

            // --- residuals ||H z - theta z|| / ||z|| with z = X S in FP64 ---
            CHEBFD_HIP(hipEventRecord(ev[3].e[0], s));
            for (int b = 0; b < kb; ++b) {
                const int cols = std::min(g.nb, k2 - b * g.nb);
                if ((r = launch_update(g.X, g.prec, g.nb, DD(L.S) + 2 * (size_t)b * g.nb * ns, ns, D(L.z64),
                                       CHEBFD_PREC_FP64, g.nb, n, k2, cols, s)))
                    return r;
                if ((r = chebfd_spmmv(H64, 1.0, 0.0, g.nb, CHEBFD_PREC_FP64, D(L.z64), D(L.t64), D(L.fwork),
                                      L.fwork_bytes, stream)))
                    return r;
                if ((r = launch_resid(D(L.t64), D(L.z64), CHEBFD_PREC_FP64, n, g.nb, DD(L.theta) + (size_t)b * g.nb,
                                      DD(L.rpart), L.rgrid, DD(L.rr), s)))
                    return r;
                CHEBFD_HIP(hipMemcpyAsync(hrr.data(), DD(L.rr), sizeof(double) * 2 * g.nb, hipMemcpyDeviceToHost, s));
                CHEBFD_HIP(hipStreamSynchronize(s));
                for (int c = 0; c < cols; ++c) {
                    hres[b * g.nb + c] = std::sqrt(hrr[2 * c]);
                    hnrm[b * g.nb + c] = std::sqrt(hrr[2 * c + 1]);
                }
            }
            CHEBFD_HIP(hipMemcpyAsync(hth.data(), DD(L.theta), sizeof(double) * k2, hipMemcpyDeviceToHost, s));
            CHEBFD_HIP(hipEventRecord(ev[3].e[1], s));
            CHEBFD_HIP(hipStreamSynchronize(s));
            for (int q = 0; q < 4; ++q) {
                float ms = 0.0f;
                CHEBFD_HIP(hipEventElapsedTime(&ms, ev[q].e[0], ev[q].e[1]));
                t_phase[q] += ms * 1e-3;
            }
            for (int c = 0; c < k2; ++c) {
                hres[c] = hnrm[c] > 0.0 ? hres[c] / hnrm[c] : INFINITY;
                if (!std::isfinite(hth[c])) CHEBFD_FAIL(CHEBFD_ENUMERIC, "non-finite Ritz value");
            }

            // --- convergence test ---
            // in-interval pairs are converged (residual <= tol) or unresolved; the stage
            // stops once the converged count repeats and the smallest unresolved residual
            // has stopped falling (a pair whose residual no longer shrinks under the filter
            // is a stable mixture of eigenvectors at or beyond the interval's edges)
            int inwin = 0, conv = 0, settled = 0;
            double worst = 0.0, unres_min = INFINITY;
            for (int c = 0; c < k2; ++c) {
                if (hth[c] < p->lam_L || hth[c] > p->lam_R) continue;
                ++inwin;
                const bool cv = hres[c] <= g.tol;
                const bool spur = hres[c] > 0.5 * (p->lam_R - p->lam_L);
                conv += cv ? 1 : 0;
                settled += spur ? 0 : 1;
                if (!cv) unres_min = std::min(unres_min, hres[c]);
                if (!spur) worst = std::max(worst, hres[c]);
            }
            // too many eigenvalues for the subspace: judged from the second iteration on, on
            // the in-interval pairs whose residual already places them in the interval
            if (stage1 && it >= 2 && settled > 0.75 * g.ns) return CHEBFD_SUBSPACE_SMALL;
            const bool unres_settled = !(unres_min < INFINITY) || unres_min > 0.5 * prev_unres;
            if (verbose)
                std::fprintf(stderr,
                             "chebfd_solve: %s iteration %d: %d kept, %d in the interval, %d converged, "
                             "smallest unresolved residual %.3g; filter %.3f s, orthogonalisation %.3f s\n",
                             stage1 ? "stage 1" : "stage 2", it, k2, inwin, conv, unres_min, t_phase[0], t_phase[1]);
            if (conv == prev && unres_settled) return CHEBFD_OK;
            // stage 1 of a mixed run also ends when the residuals stop falling (storage floor)
            if (stage1 && g.prec != CHEBFD_PREC_FP64 && inwin > 0 && inwin == prev_inwin && conv == prev &&
                worst > 0.5 * prev_max) {
                *stagnated = true;
                return CHEBFD_OK;
            }
            prev = conv;
            prev_max = worst;
            prev_inwin = inwin;
            prev_unres = unres_min;
            if (it == p->max_iter) break;

            // --- restart: Ritz vectors, then fresh random phases for dropped directions ---
            if ((r = launch_update(g.X, g.prec, g.nb, DD(L.S), ns, g.Q, g.prec, g.nb, n, k2, k2, s))) return r;
            if ((r = launch_random_phase(g.Q, g.prec, n, g.nb, k2, g.ns, p->seed, (uint64_t)it * ns, perm, s)))
                return r;
            std::swap(g.X, g.Q);
        }
        return CHEBFD_NOT_CONVERGED;
    };

    bool stagnated = false;
    Stage *fin = &S1;
    status = run_stage(S1, -1, true, &stagnated);
    if (status < 0) return status;
    Stage S2{H64, CHEBFD_PREC_FP64, 0, std::max(1, nb / 2), S1.Q, S1.X, D(L.b64), D(L.t64), p->tol};
    if (prec != CHEBFD_PREC_FP64 && status == CHEBFD_OK && it < p->max_iter) {
        // --- stage 2 (mixed precision): FP64 iteration on the Ritz vectors nearest the interval ---
        // the non-spurious pairs in the interval first, then the other Ritz vectors by
        // distance of their values from the interval's centre
        const double half_w = 0.5 * (p->lam_R - p->lam_L), mid = 0.5 * (p->lam_L + p->lam_R);
        std::vector<int> pick, rest;
        for (int c = 0; c < k2; ++c) {
            if (hth[c] >= p->lam_L && hth[c] <= p->lam_R && hres[c] <= half_w)
                pick.push_back(c);
            else
                rest.push_back(c);
        }
        const int inwin = static_cast<int>(pick.size());
        const int ns2_max = ns / 2 / S2.nb * S2.nb;
        int ns2 = std::max(inwin + 2, (4 * inwin + 2) / 3 + 1);
        ns2 = std::min(ns2_max, (ns2 + S2.nb - 1) / S2.nb * S2.nb);
        ns2 = std::min(ns2, k2 / S2.nb * S2.nb);
        if (inwin > 0 && ns2 >= inwin) {
            std::stable_sort(rest.begin(), rest.end(),
                             [&](int a, int b) { return std::fabs(hth[a] - mid) < std::fabs(hth[b] - mid); });
            for (int c : rest)
                if ((int)pick.size() < ns2) pick.push_back(c);
            S2.ns = ns2;
            CHEBFD_HIP(hipMemcpyAsync(D(L.order), pick.data(), sizeof(int) * ns2, hipMemcpyHostToDevice, s));
            if ((rc = launch_permute_columns(k2, ns2, DD(L.S), ns, static_cast<const int *>(D(L.order)), DD(L.T), ns,
                                             s)))
                return rc;
            // FP64 Ritz vectors into the idle basis buffer (X of stage 2), block width n_b / 2
            if ((rc = launch_update(S1.X, prec, nb, DD(L.T), ns, S1.Q, CHEBFD_PREC_FP64, S2.nb, n, k2, ns2, s)))
                return rc;
            S2.X = S1.Q;
            S2.Q = S1.X;
            CHEBFD_HIP(hipStreamSynchronize(s));
            bool dummy;
            status = run_stage(S2, inwin, false, &dummy);
            if (status < 0) return status;
            fin = &S2;
        } else if (stagnated || S1.tol > p->tol) {
            status = CHEBFD_NOT_CONVERGED;
        }
    } else if (prec != CHEBFD_PREC_FP64 && status == CHEBFD_OK) {
        status = CHEBFD_NOT_CONVERGED;   // no iteration left for the FP64 stage
    }
    if (it > p->max_iter) it = p->max_iter;
    void *X = fin->X;
    const int fprec = fin->prec, fnb = fin->nb;

    // output order: converged pairs inside the interval first, then the rest
    std::vector<int> order;
    for (int c = 0; c < k2; ++c)
        if (hth[c] >= p->lam_L && hth[c] <= p->lam_R && hres[c] <= p->tol) order.push_back(c);
    const int nf = static_cast<int>(order.size());
    for (int c = 0; c < k2; ++c)
        if (!(hth[c] >= p->lam_L && hth[c] <= p->lam_R && hres[c] <= p->tol)) order.push_back(c);
    for (int c = 0; c < ns; ++c) {
        h_theta[c] = c < k2 ? hth[order[c]] : NAN;
        h_resid[c] = c < k2 ? hres[order[c]] : NAN;
    }
    *n_found = nf;
    if (d_Z) {
        CHEBFD_HIP(hipMemcpyAsync(D(L.order), order.data(), sizeof(int) * k2, hipMemcpyHostToDevice, s));
        if ((rc = launch_permute_columns(k2, k2, DD(L.S), ns, static_cast<const int *>(D(L.order)), DD(L.T), ns, s)))
            return rc;
        CHEBFD_HIP(hipMemsetAsync(d_Z, 0, sizeof(double) * 2 * (size_t)n * ns, s));
        const int kb = (k2 + fnb - 1) / fnb;
        for (int b = 0; b < kb; ++b) {
            const int cols = std::min(fnb, k2 - b * fnb);
            if ((rc = launch_update(X, fprec, fnb, DD(L.T) + 2 * (size_t)b * fnb * ns, ns, D(L.z64), CHEBFD_PREC_FP64,
                                    fnb, n, k2, cols, s)))
                return rc;
            if ((rc = launch_fix_phases(D(L.z64), CHEBFD_PREC_FP64, n, fnb, cols, DD(L.phase), s))) return rc;
            // columns b*fnb .. (b+1)*fnb-1 of the column-major output (fnb divides n_s)
            if ((rc = launch_pack(perm, n, fnb, fnb, CHEBFD_PREC_FP64, D(L.z64),
                                  static_cast<char *>(d_Z) + (size_t)b * fnb * n * 16, true, s)))
                return rc;
        }
        if (k2 % fnb) {
            // the last block's columns past k2 hold stale z64 data: zero them
            const size_t c0 = (size_t)k2, c1 = (size_t)(k2 / fnb + 1) * fnb;
            CHEBFD_HIP(hipMemsetAsync(static_cast<char *>(d_Z) + c0 * n * 16, 0, (c1 - c0) * n * 16, s));
        }
        CHEBFD_HIP(hipStreamSynchronize(s));
    }

    if (st) {
        st->iterations = it;
        st->n_found = nf;
        st->n_kept = k2;
        st->status = status;
        st->count_est = count_est;
        st->t_filter = t_phase[0];
        st->t_orth = t_phase[1];
        st->t_rr = t_phase[2];
        st->t_resid = t_phase[3];
        st->t_total = t_phase[0] + t_phase[1] + t_phase[2] + t_phase[3];
        st->filter_bytes = fbytes;
    }
    return status;
}

}  // extern "C"
