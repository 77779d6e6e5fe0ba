// Parameter choice for the ChebFD iteration: moment features of a matrix and
// search interval (KPM moments from the filter recurrence, Sect. 2), the
// eigenvalue-count estimate, and the mapping of a count estimate plus either
// the predictor network's outputs or the heuristic to (n_p, n_s).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

using namespace chebfd;

namespace {

constexpr int kSteps = CHEBFD_FEATURE_MOMENTS / 2;

}  // namespace

extern "C" {

int chebfd_features_query(const chebfd_matrix *H, size_t *work_bytes) {
    clear_error();
    CHEBFD_REQUIRE(work_bytes != nullptr, "work_bytes is NULL");
    size_t wb = 0, wk = 0;
    int rc;
    if ((rc = chebfd_bounds_query(H, &wb))) return rc;
    if ((rc = chebfd_kpm_query(H, kSteps, CHEBFD_FEATURE_R, &wk))) return rc;
    *work_bytes = std::max(wb, wk);
    return CHEBFD_OK;
}

int chebfd_features(const chebfd_matrix *H, double lam_L, double lam_R, uint64_t seed, float *h_features,
                    double *count_est, double *alpha, double *beta, void *d_work, size_t work_bytes,
                    void *stream) {
    clear_error();
    CHEBFD_REQUIRE(h_features && count_est && alpha && beta, "output pointer is NULL");
    CHEBFD_REQUIRE(std::isfinite(lam_L) && std::isfinite(lam_R) && lam_L < lam_R, "interval [%g, %g] invalid",
                   lam_L, lam_R);
    size_t need;
    int rc;
    if ((rc = chebfd_features_query(H, &need))) return rc;
    if (work_bytes < need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "features workspace %zu < %zu", work_bytes, need);
    double lo, hi;
    if ((rc = chebfd_bounds(H, d_work, work_bytes, stream, &lo, &hi))) return rc;
    // window coefficients of [a~, b~] and Jackson damping over all 256 moments
    std::vector<double> gc(CHEBFD_FEATURE_MOMENTS);
    double al, be;
    if ((rc = chebfd_coefficients(lo, hi, lam_L, lam_R, CHEBFD_FEATURE_MOMENTS - 1, &al, &be, gc.data())))
        return rc;
    std::vector<double> mu(CHEBFD_FEATURE_MOMENTS);
    if ((rc = chebfd_kpm_moments(H, al, be, kSteps, CHEBFD_FEATURE_R, seed, mu.data(), d_work, work_bytes,
                                 stream)))
        return rc;
    double acc = 0.0;
    for (int m = 0; m < CHEBFD_FEATURE_MOMENTS; ++m) {
        if (!std::isfinite(mu[m])) CHEBFD_FAIL(CHEBFD_ENUMERIC, "moment %d is not finite", m);
        acc += gc[m] * mu[m];
        h_features[m] = (float)mu[m];
    }
    // mu~_0 is 1 by construction; its slot carries the matrix size instead, which
    // sets the eigenvalue spacing the filter must resolve (the moments are per row)
    h_features[0] = (float)(std::log10((double)H->n) / 8.0);
    h_features[CHEBFD_FEATURE_MOMENTS] = (float)(al * lam_L + be);
    h_features[CHEBFD_FEATURE_MOMENTS + 1] = (float)(al * lam_R + be);
    *count_est = (double)H->n * acc;
    *alpha = al;
    *beta = be;
    return CHEBFD_OK;
}

int chebfd_choose_params(double a, double b, double count_est, int32_t n_b, const float *h_mlp_out,
                         const chebfd_predictor *pr, int32_t *n_p, int32_t *n_s) {
    clear_error();
    CHEBFD_REQUIRE(n_p && n_s, "output pointer is NULL");
    CHEBFD_REQUIRE(a > -1.0 && a < b && b < 1.0, "scaled interval [%g, %g] not inside (-1, 1)", a, b);
    CHEBFD_REQUIRE(std::isfinite(count_est), "count estimate not finite");
    CHEBFD_REQUIRE(n_b >= 1 && n_b <= 128 && (n_b & (n_b - 1)) == 0, "n_b = %d must be a power of two <= 128",
                   n_b);
    CHEBFD_REQUIRE(pr != nullptr, "predictor is NULL");
    const double nhat = std::max(count_est, 0.0);
    const double delta = (b - a) / 2.0;
    double np_real, ns_real;
    if (h_mlp_out) {
        // the network's outputs: standardised log(n_p delta) and log(n_s / max(2 n_hat, n_b))
        CHEBFD_REQUIRE(std::isfinite(h_mlp_out[0]) && std::isfinite(h_mlp_out[1]), "MLP output not finite");
        CHEBFD_REQUIRE(pr->t_std[0] > 0.0 && pr->t_std[1] > 0.0, "predictor scales must be positive");
        // a network asked far outside its training range extrapolates: its outputs
        // are held to the range of the training targets
        double y[2];
        for (int k = 0; k < 2; ++k) {
            y[k] = std::min(30.0, h_mlp_out[k] * pr->t_std[k] + pr->t_mean[k]);
            if (pr->t_lo[k] < pr->t_hi[k]) y[k] = std::min(pr->t_hi[k], std::max(pr->t_lo[k], y[k]));
        }
        np_real = std::exp(y[0]) / delta;
        ns_real = std::exp(y[1]) * std::max(2.0 * nhat, static_cast<double>(n_b));
        ns_real = std::max(ns_real, 1.2 * nhat);
    } else {
        CHEBFD_REQUIRE(pr->kappa > 0.0, "kappa must be positive");
        np_real = pr->kappa / delta;
        ns_real = 2.0 * nhat;
    }
    const double np_c = std::min<double>(CHEBFD_NP_MAX, std::max<double>(CHEBFD_NP_MIN, std::round(np_real)));
    double ns_c = std::ceil(ns_real / n_b) * n_b;
    ns_c = std::max<double>(ns_c, n_b);
    ns_c = std::min<double>(ns_c, std::max(n_b, 512 / n_b * n_b));
    *n_p = (int32_t)np_c;
    *n_s = (int32_t)ns_c;
    return CHEBFD_OK;
}

}  // extern "C"
