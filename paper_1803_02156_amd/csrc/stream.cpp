// The filter on a search space kept in host memory (working sets beyond HBM).
//
// The paper runs ChebFD on working sets larger than the fast memory of KNL
// and P100 and finds no significant slowdown once the filter degree is large
// enough, because each block of vectors is loaded once and then worked on for
// n_p steps (Sect. 3.5, Fig. 6).  Here the n_s / n_b blocks live in pinned
// host memory and pass through two device staging blocks: block b + 1 is
// copied in on the copy stream while block b is filtered on the compute
// stream, and block b is copied back once its filter is done.  The filter of
// one block is chebfd_filter itself; its moments go to a temporary in the
// workspace and are copied into their columns of eta and nu.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "kernels.h"

namespace chebfd {
namespace {

struct StreamLayout {
    size_t stage[2], eta, nu, fwork, fwork_bytes, total;
};

int stream_layout(const chebfd_matrix *H, int n_p, int n_b, int prec, StreamLayout *L) {
    size_t fb = 0;
    int rc = chebfd_filter_query(H, n_b, &fb);
    if (rc) return rc;
    const size_t blk = vec_elem_bytes(prec) * (size_t)H->n * n_b;
    size_t at = 0;
    auto take = [&](size_t b) { const size_t h = at; at = round_up(at + b, 256); return h; };
    L->stage[0] = take(blk);
    L->stage[1] = take(blk);
    L->eta = take(sizeof(double) * 2 * (size_t)(n_p + 1) * n_b);
    L->nu = take(sizeof(double) * (size_t)(n_p + 1) * n_b);
    L->fwork = take(fb);
    L->fwork_bytes = fb;
    L->total = at;
    return CHEBFD_OK;
}

struct Events {
    hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~Events() {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

}  // namespace
}  // namespace chebfd

using namespace chebfd;

extern "C" {

int chebfd_filter_streamed_query(const chebfd_matrix *H, int32_t n_p, int32_t n_b, size_t *work_bytes) {
    clear_error();
    CHEBFD_REQUIRE(H != nullptr && work_bytes != nullptr, "NULL argument");
    CHEBFD_REQUIRE(n_p >= 0, "n_p = %d < 0", n_p);
    CHEBFD_REQUIRE(H->prec == CHEBFD_PREC_FP64 || H->prec == CHEBFD_PREC_MIXED, "matrix handle invalid");
    StreamLayout L;
    int rc = stream_layout(H, n_p, n_b, H->prec, &L);
    if (rc) return rc;
    *work_bytes = L.total;
    return CHEBFD_OK;
}

int chebfd_filter_streamed(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma, int32_t n_p,
                           int32_t n_s, int32_t n_b, int32_t prec, void *h_xy, void *d_u, void *d_w, double *d_eta,
                           double *d_nu, void *d_work, size_t work_bytes, void *stream, void *copy_stream) {
    clear_error();
    CHEBFD_REQUIRE(H != nullptr && h_xy != nullptr && d_work != nullptr, "NULL argument");
    CHEBFD_REQUIRE(n_s >= 1 && n_b >= 1 && n_s % n_b == 0, "n_s = %d must be a positive multiple of n_b = %d", n_s,
                   n_b);
    CHEBFD_REQUIRE(n_p >= 0, "n_p = %d < 0", n_p);
    CHEBFD_REQUIRE((d_eta == nullptr) == (d_nu == nullptr), "d_eta and d_nu must both be set or both NULL");
    CHEBFD_REQUIRE(stream != copy_stream, "the copy stream must differ from the compute stream");
    CHEBFD_REQUIRE(aligned(d_work, 256), "d_work must be 256-byte aligned");
    StreamLayout L;
    int rc = stream_layout(H, n_p, n_b, prec, &L);
    if (rc) return rc;
    if (work_bytes < L.total) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "streamed filter workspace %zu < %zu", work_bytes, L.total);
    char *base = static_cast<char *>(d_work);
    void *stage[2] = {base + L.stage[0], base + L.stage[1]};
    double *teta = reinterpret_cast<double *>(base + L.eta);
    double *tnu = reinterpret_cast<double *>(base + L.nu);
    hipStream_t cs = static_cast<hipStream_t>(stream), xs = static_cast<hipStream_t>(copy_stream);
    const size_t blk = vec_elem_bytes(prec) * (size_t)H->n * n_b;
    const int nblk = n_s / n_b;
    char *host = static_cast<char *>(h_xy);

    // e[0], e[1]: block in slot k has arrived; e[2], e[3]: slot k's filter is done; e[4]: all copies done
    Events ev;
    for (hipEvent_t &x : ev.e) CHEBFD_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    // the copy stream starts after the work already queued on the compute stream
    CHEBFD_HIP(hipEventRecord(ev.e[4], cs));
    CHEBFD_HIP(hipStreamWaitEvent(xs, ev.e[4], 0));
    CHEBFD_HIP(hipMemcpyAsync(stage[0], host, blk, hipMemcpyHostToDevice, xs));
    CHEBFD_HIP(hipEventRecord(ev.e[0], xs));
    for (int b = 0; b < nblk; ++b) {
        const int k = b & 1;
        // prefetch the next block into the other slot (its previous block was copied
        // back earlier on the same stream)
        if (b + 1 < nblk) {
            CHEBFD_HIP(hipMemcpyAsync(stage[k ^ 1], host + (size_t)(b + 1) * blk, blk, hipMemcpyHostToDevice, xs));
            CHEBFD_HIP(hipEventRecord(ev.e[k ^ 1], xs));
        }
        CHEBFD_HIP(hipStreamWaitEvent(cs, ev.e[k], 0));
        if ((rc = chebfd_filter(H, alpha, beta, h_gamma, n_p, n_b, n_b, prec, stage[k], d_u, d_w,
                                d_eta ? teta : nullptr, d_eta ? tnu : nullptr, base + L.fwork, L.fwork_bytes,
                                stream)))
            return rc;
        if (d_eta && n_p >= 1) {
            // rows 1..n_p of the block's moments into columns b n_b .. b n_b + n_b - 1
            CHEBFD_HIP(hipMemcpy2DAsync(d_eta + 2 * ((size_t)n_s + (size_t)b * n_b), 16 * (size_t)n_s,
                                        teta + 2 * (size_t)n_b, 16 * (size_t)n_b, 16 * (size_t)n_b, n_p,
                                        hipMemcpyDeviceToDevice, cs));
            CHEBFD_HIP(hipMemcpy2DAsync(d_nu + (size_t)n_s + (size_t)b * n_b, 8 * (size_t)n_s, tnu + n_b,
                                        8 * (size_t)n_b, 8 * (size_t)n_b, n_p, hipMemcpyDeviceToDevice, cs));
        }
        CHEBFD_HIP(hipEventRecord(ev.e[2 + k], cs));
        CHEBFD_HIP(hipStreamWaitEvent(xs, ev.e[2 + k], 0));
        CHEBFD_HIP(hipMemcpyAsync(host + (size_t)b * blk, stage[k], blk, hipMemcpyDeviceToHost, xs));
    }
    // the caller synchronises the compute stream only
    CHEBFD_HIP(hipEventRecord(ev.e[4], xs));
    CHEBFD_HIP(hipStreamWaitEvent(cs, ev.e[4], 0));
    return CHEBFD_OK;
}

}  // extern "C"
