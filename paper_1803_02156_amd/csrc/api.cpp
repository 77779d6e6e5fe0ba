// C ABI of libchebfd: argument validation, SELL-C-sigma ingest on the host,
// the filter driver (Alg. 1 per block, Alg. 2 over blocks) and small helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace chebfd {

static thread_local std::string g_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
}

void clear_error() { g_error.clear(); }

int device_props(DeviceProps *out) {
    static std::mutex mu;
    static DeviceProps cache[64];
    static bool have[64] = {};
    int dev = 0;
    CHEBFD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) CHEBFD_FAIL(CHEBFD_EHIP, "device id %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!have[dev]) {
        hipDeviceProp_t p;
        CHEBFD_HIP(hipGetDeviceProperties(&p, dev));
        DeviceProps &d = cache[dev];
        d.id = dev;
        d.num_cus = p.multiProcessorCount;
        d.max_threads_per_cu = p.maxThreadsPerMultiProcessor;
        snprintf(d.name, sizeof(d.name), "%s", p.gcnArchName);
        have[dev] = true;
    }
    *out = cache[dev];
    return CHEBFD_OK;
}

// Static scratch of chebfd_filter_noalloc: the partial dot-product sums the step
// kernels pass from one launch to the next.  Each device holds its own copy
// until the process ends.  Host code never uses the array's name as a device
// address: scratch_ptr() looks the copy of the current device up once.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static int scratch_ptr(void **out) {
    static std::mutex mu;
    static void *ptr[64] = {};
    int dev = 0;
    CHEBFD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) CHEBFD_FAIL(CHEBFD_EHIP, "device id %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (ptr[dev] == nullptr) {
        void *p = nullptr;
        CHEBFD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr) CHEBFD_FAIL(CHEBFD_EHIP, "no device address for the static scratch buffer");
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return CHEBFD_OK;
}

// ---------------------------------------------------------------------------
// SELL-C-sigma layout on the host
// ---------------------------------------------------------------------------
struct SellPlan {
    int64_t n = 0, n_chunks = 0, slots = 0;
    int32_t max_width = 0;
    bool identity = true;
    std::vector<int32_t> perm;         // new -> old
    std::vector<int32_t> width;        // per chunk
    std::vector<int64_t> off;          // per chunk + 1
};

static int ilog2_exact(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return (1 << l) == v ? l : -1;
}

static int check_matrix_args(int64_t n, const int64_t *rowptr, int32_t C, int32_t sigma,
                             int32_t prec) {
    CHEBFD_REQUIRE(n >= 1 && n < (int64_t(1) << 31), "n = %lld out of range [1, 2^31)", (long long)n);
    CHEBFD_REQUIRE(rowptr != nullptr, "h_rowptr is NULL");
    CHEBFD_REQUIRE(C >= 1 && C <= 1024 && ilog2_exact(C) >= 0, "C = %d must be a power of two in [1, 1024]", C);
    CHEBFD_REQUIRE(sigma == 1 || (sigma >= C && sigma % C == 0), "sigma = %d must be 1 or a multiple of C", sigma);
    CHEBFD_REQUIRE(prec == CHEBFD_PREC_FP64 || prec == CHEBFD_PREC_MIXED, "prec = %d invalid", prec);
    CHEBFD_REQUIRE(rowptr[0] == 0, "h_rowptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        CHEBFD_REQUIRE(rowptr[i + 1] >= rowptr[i], "h_rowptr decreases at row %lld", (long long)i);
    return CHEBFD_OK;
}

static int check_order(int64_t n, const int32_t *order) {
    if (!order) return CHEBFD_OK;
    std::vector<char> seen(n, 0);
    for (int64_t k = 0; k < n; ++k) {
        CHEBFD_REQUIRE(order[k] >= 0 && order[k] < n && !seen[order[k]],
                       "h_order is not a permutation of 0..n-1 (entry %lld)", (long long)k);
        seen[order[k]] = 1;
    }
    return CHEBFD_OK;
}

// Row order of the SELL matrix: the caller's order (or the natural one), then
// a stable sort by row length inside each window of sigma rows.
static void make_plan(int64_t n, const int64_t *rowptr, const int32_t *order, int32_t C, int32_t sigma,
                      SellPlan &p) {
    p.n = n;
    p.perm.resize(n);
    if (order)
        std::copy(order, order + n, p.perm.begin());
    else
        std::iota(p.perm.begin(), p.perm.end(), 0);
    auto len = [&](int32_t r) { return rowptr[r + 1] - rowptr[r]; };
    if (sigma > 1) {
        for (int64_t w0 = 0; w0 < n; w0 += sigma) {
            const int64_t w1 = std::min<int64_t>(n, w0 + sigma);
            std::stable_sort(p.perm.begin() + w0, p.perm.begin() + w1,
                             [&](int32_t a, int32_t b) { return len(a) > len(b); });
        }
    }
    p.identity = true;
    for (int64_t i = 0; i < n; ++i)
        if (p.perm[i] != i) { p.identity = false; break; }
    p.n_chunks = (n + C - 1) / C;
    p.width.assign(p.n_chunks, 0);
    p.off.assign(p.n_chunks + 1, 0);
    p.max_width = 0;
    for (int64_t c = 0; c < p.n_chunks; ++c) {
        int64_t w = 0;
        for (int64_t i = c * C; i < std::min<int64_t>(n, (c + 1) * C); ++i)
            w = std::max<int64_t>(w, len(p.perm[i]));
        p.width[c] = static_cast<int32_t>(w);
        p.max_width = std::max<int32_t>(p.max_width, static_cast<int32_t>(w));
        p.off[c + 1] = p.off[c] + w * C;
    }
    p.slots = p.off[p.n_chunks];
}

// stored slots plus the zero padding the unrolled row kernel may read past the end
static int64_t padded_slots(const SellPlan &p, int C) { return p.slots + (int64_t)kRowMaxUnrolled * C; }

struct MatrixLayout {
    size_t o_off, o_width, o_col, o_val, o_perm, o_iperm, total;
};

static MatrixLayout matrix_layout(const SellPlan &p, int prec, int C) {
    MatrixLayout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t here = at;
        at = round_up(at + bytes, 256);
        return here;
    };
    L.o_off = take(sizeof(int64_t) * (p.n_chunks + 1));
    L.o_width = take(sizeof(int32_t) * p.n_chunks);
    L.o_col = take(sizeof(int32_t) * padded_slots(p, C));
    L.o_val = take(vec_elem_bytes(prec) * padded_slots(p, C));
    L.o_perm = take(sizeof(int32_t) * p.n);
    L.o_iperm = take(sizeof(int32_t) * p.n);
    L.total = at;
    return L;
}

}  // namespace chebfd

using namespace chebfd;

namespace chebfd {
int32_t next_step_epoch() {
    static std::atomic<uint32_t> counter{0};
    for (;;) {
        const uint32_t v = (counter.fetch_add(1, std::memory_order_relaxed) + 1) & 0x7fffffffu;
        if (v != 0) return static_cast<int32_t>(v);
    }
}
}  // namespace chebfd

extern "C" {

int chebfd_version(void) { return 100; }

const char *chebfd_last_error(void) { return g_error.c_str(); }

int chebfd_device_info(int32_t *num_cus, char *name, int32_t name_len) {
    DeviceProps d;
    int rc = device_props(&d);
    if (rc) return rc;
    if (num_cus) *num_cus = d.num_cus;
    if (name && name_len > 0) snprintf(name, name_len, "%s", d.name);
    return CHEBFD_OK;
}

int chebfd_matrix_query(int64_t n, const int64_t *h_rowptr, const int32_t *h_order, int32_t C,
                        int32_t sigma, int32_t prec, size_t *bytes) {
    clear_error();
    int rc = check_matrix_args(n, h_rowptr, C, sigma, prec);
    if (rc || (rc = check_order(n, h_order))) return rc;
    CHEBFD_REQUIRE(bytes != nullptr, "bytes is NULL");
    SellPlan p;
    make_plan(n, h_rowptr, h_order, C, sigma, p);
    *bytes = matrix_layout(p, prec, C).total;
    return CHEBFD_OK;
}

int chebfd_matrix_build(int64_t n, const int64_t *h_rowptr, const int32_t *h_col,
                        const double *h_val, const int32_t *h_order, int32_t C, int32_t sigma,
                        int32_t prec, void *d_buf, size_t bytes, void *stream, chebfd_matrix *out) {
    clear_error();
    int rc = check_matrix_args(n, h_rowptr, C, sigma, prec);
    if (rc || (rc = check_order(n, h_order))) return rc;
    const int64_t nnz = h_rowptr[n];
    CHEBFD_REQUIRE(nnz == 0 || (h_col && h_val), "h_col / h_val is NULL");
    CHEBFD_REQUIRE(d_buf != nullptr && aligned(d_buf, 256), "d_buf must be non-NULL and 256-byte aligned");
    CHEBFD_REQUIRE(out != nullptr, "out is NULL");
    for (int64_t k = 0; k < nnz; ++k)
        CHEBFD_REQUIRE(h_col[k] >= 0 && h_col[k] < n, "column index %d at entry %lld out of range",
                       h_col[k], (long long)k);
    SellPlan p;
    make_plan(n, h_rowptr, h_order, C, sigma, p);
    const MatrixLayout L = matrix_layout(p, prec, C);
    if (bytes < L.total)
        CHEBFD_FAIL(CHEBFD_EWORKSPACE, "matrix buffer has %zu bytes, needs %zu", bytes, L.total);

    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) iperm[p.perm[i]] = static_cast<int32_t>(i);
    const int64_t pslots = padded_slots(p, C);
    std::vector<int32_t> col(pslots, 0);
    std::vector<double> vd;
    std::vector<float> vf;
    if (prec == CHEBFD_PREC_FP64)
        vd.assign(2 * pslots, 0.0);
    else
        vf.assign(2 * pslots, 0.0f);
    for (int64_t c = 0; c < p.n_chunks; ++c) {
        const int w = p.width[c];
        for (int r = 0; r < C; ++r) {
            const int64_t i = c * C + r;
            const int64_t base = p.off[c] + r;
            if (i >= n) {
                for (int k = 0; k < w; ++k) col[base + (int64_t)k * C] = 0;
                continue;
            }
            const int32_t old = p.perm[i];
            const int64_t b = h_rowptr[old], len = h_rowptr[old + 1] - b;
            for (int k = 0; k < w; ++k) {
                const int64_t s = base + (int64_t)k * C;
                if (k < len) {
                    col[s] = iperm[h_col[b + k]];
                    if (prec == CHEBFD_PREC_FP64) {
                        vd[2 * s] = h_val[2 * (b + k)];
                        vd[2 * s + 1] = h_val[2 * (b + k) + 1];
                    } else {
                        vf[2 * s] = static_cast<float>(h_val[2 * (b + k)]);
                        vf[2 * s + 1] = static_cast<float>(h_val[2 * (b + k) + 1]);
                    }
                } else {
                    col[s] = static_cast<int32_t>(i);  // padding: own row, value 0
                }
            }
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(d_buf);
    CHEBFD_HIP(hipMemcpyAsync(base + L.o_off, p.off.data(), sizeof(int64_t) * (p.n_chunks + 1),
                              hipMemcpyHostToDevice, s));
    CHEBFD_HIP(hipMemcpyAsync(base + L.o_width, p.width.data(), sizeof(int32_t) * p.n_chunks,
                              hipMemcpyHostToDevice, s));
    CHEBFD_HIP(hipMemcpyAsync(base + L.o_col, col.data(), sizeof(int32_t) * col.size(),
                              hipMemcpyHostToDevice, s));
    if (prec == CHEBFD_PREC_FP64)
        CHEBFD_HIP(hipMemcpyAsync(base + L.o_val, vd.data(), sizeof(double) * vd.size(),
                                  hipMemcpyHostToDevice, s));
    else
        CHEBFD_HIP(hipMemcpyAsync(base + L.o_val, vf.data(), sizeof(float) * vf.size(),
                                  hipMemcpyHostToDevice, s));
    CHEBFD_HIP(hipMemcpyAsync(base + L.o_perm, p.perm.data(), sizeof(int32_t) * n,
                              hipMemcpyHostToDevice, s));
    CHEBFD_HIP(hipMemcpyAsync(base + L.o_iperm, iperm.data(), sizeof(int32_t) * n,
                              hipMemcpyHostToDevice, s));
    CHEBFD_HIP(hipStreamSynchronize(s));

    chebfd_matrix m;
    std::memset(&m, 0, sizeof(m));
    m.n = n;
    m.nnz = nnz;
    m.n_chunks = p.n_chunks;
    m.slots = p.slots;
    m.C = C;
    m.sigma = sigma;
    m.prec = prec;
    m.max_width = p.max_width;
    m.identity_perm = p.identity ? 1 : 0;
    m.uniform_width = p.max_width;
    for (int64_t c = 0; c < p.n_chunks; ++c)
        if (p.width[c] != p.max_width) { m.uniform_width = 0; break; }
    // locality of the gathers: entries whose column lies within the window
    // kernel's halo of their row's tile (tiles of 32 and 64 rows)
    for (int v = 0; v < 2; ++v) {
        const int64_t tr = 32 << v;
        const int64_t halo = win_halo(static_cast<int>(tr));
        int64_t local = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t t0 = i / tr * tr;
            const int32_t old = p.perm[i];
            for (int64_t k = h_rowptr[old]; k < h_rowptr[old + 1]; ++k) {
                const int64_t q = iperm[h_col[k]];
                local += (q >= t0 - halo * tr && q < t0 + (halo + 1) * tr) ? 1 : 0;
            }
        }
        m.window_local[v] = nnz > 0 ? static_cast<int32_t>(local * 1000 / nnz) : 1000;
    }
    m.chunk_off = reinterpret_cast<const int64_t *>(base + L.o_off);
    m.chunk_width = reinterpret_cast<const int32_t *>(base + L.o_width);
    m.col = reinterpret_cast<const int32_t *>(base + L.o_col);
    m.val = base + L.o_val;
    m.perm = reinterpret_cast<const int32_t *>(base + L.o_perm);
    m.iperm = reinterpret_cast<const int32_t *>(base + L.o_iperm);
    *out = m;
    return CHEBFD_OK;
}

static int check_handle(const chebfd_matrix *H) {
    CHEBFD_REQUIRE(H != nullptr, "matrix handle is NULL");
    CHEBFD_REQUIRE(H->n >= 1 && H->chunk_off && H->chunk_width && H->col && H->val && H->perm,
                   "matrix handle is not built");
    CHEBFD_REQUIRE(ilog2_exact(H->C) >= 0, "matrix handle has invalid C");
    return CHEBFD_OK;
}

static int bounds_grid(const DeviceProps &d, int64_t n) {
    int64_t G = (n + 255) / 256;
    G = std::min<int64_t>(G, (int64_t)d.num_cus * 4);
    return static_cast<int>(std::max<int64_t>(G, 1));
}

int chebfd_bounds_query(const chebfd_matrix *H, size_t *work_bytes) {
    clear_error();
    int rc = check_handle(H);
    if (rc) return rc;
    CHEBFD_REQUIRE(work_bytes != nullptr, "work_bytes is NULL");
    DeviceProps d;
    if ((rc = device_props(&d))) return rc;
    *work_bytes = round_up(sizeof(double) * (2 * bounds_grid(d, H->n) + 2), 256);
    return CHEBFD_OK;
}

int chebfd_bounds(const chebfd_matrix *H, void *d_work, size_t work_bytes, void *stream,
                  double *lam_lo, double *lam_hi) {
    clear_error();
    int rc = check_handle(H);
    if (rc) return rc;
    CHEBFD_REQUIRE(lam_lo && lam_hi, "lam_lo / lam_hi is NULL");
    CHEBFD_REQUIRE(d_work && aligned(d_work, 256), "d_work must be non-NULL and 256-byte aligned");
    DeviceProps d;
    if ((rc = device_props(&d))) return rc;
    const int G = bounds_grid(d, H->n);
    const size_t need = round_up(sizeof(double) * (2 * G + 2), 256);
    if (work_bytes < need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "bounds workspace %zu < %zu", work_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(d_work);
    double *res = part + 2 * G;
    if ((rc = launch_bounds(H->chunk_off, H->chunk_width, H->col, H->val, H->prec, H->n, H->C,
                            ilog2_exact(H->C), part, G, s)))
        return rc;
    if ((rc = launch_bounds_final(part, G, res, s))) return rc;
    double h[2];
    CHEBFD_HIP(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s));
    CHEBFD_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(h[0]) || !std::isfinite(h[1]))
        CHEBFD_FAIL(CHEBFD_ENUMERIC, "non-finite Gershgorin bounds");
    *lam_lo = h[0];
    *lam_hi = h[1];
    return CHEBFD_OK;
}

int chebfd_coefficients(double lam_lo, double lam_hi, double lam_L, double lam_R, int32_t n_p,
                        double *alpha, double *beta, double *h_gamma) {
    clear_error();
    CHEBFD_REQUIRE(alpha && beta && h_gamma, "output pointer is NULL");
    CHEBFD_REQUIRE(n_p >= 0, "n_p = %d < 0", n_p);
    CHEBFD_REQUIRE(std::isfinite(lam_lo) && std::isfinite(lam_hi) && lam_hi > lam_lo,
                   "spectral bounds [%g, %g] invalid", lam_lo, lam_hi);
    const double al = 2.0 / (lam_hi - lam_lo);
    const double be = -(lam_hi + lam_lo) / (lam_hi - lam_lo);
    const double a = al * lam_L + be, b = al * lam_R + be;
    if (!(a > -1.0 && a < b && b < 1.0))
        CHEBFD_FAIL(CHEBFD_EINTERVAL, "scaled interval [%g, %g] not strictly inside (-1, 1)", a, b);
    // window: Chebyshev series of the indicator of [a, b] in theta = arccos x
    const double ta = std::acos(a), tb = std::acos(b);
    // Jackson damping with M = n_p + 1 terms, q = pi / (M + 1)
    const double M = n_p + 1.0;
    const double q = M_PI / (M + 1.0);
    const double cotq = std::cos(q) / std::sin(q);
    for (int p = 0; p <= n_p; ++p) {
        const double c = p == 0 ? (ta - tb) / M_PI
                                : 2.0 * (std::sin(p * ta) - std::sin(p * tb)) / (p * M_PI);
        const double g = ((M - p + 1.0) * std::cos(p * q) + std::sin(p * q) * cotq) / (M + 1.0);
        h_gamma[p] = g * c;
    }
    *alpha = al;
    *beta = be;
    return CHEBFD_OK;
}

static int check_prec_nb(int32_t prec, int32_t n_b) {
    CHEBFD_REQUIRE(prec == CHEBFD_PREC_FP64 || prec == CHEBFD_PREC_MIXED, "prec = %d invalid", prec);
    CHEBFD_REQUIRE(n_b >= 1 && n_b <= 128 && ilog2_exact(n_b) >= 0,
                   "n_b = %d must be a power of two in [1, 128]", n_b);
    return CHEBFD_OK;
}

int chebfd_pack(const chebfd_matrix *H, int32_t m, int32_t n_b, int32_t prec,
                const void *d_colmajor, void *d_blocked, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(prec, n_b))) return rc;
    CHEBFD_REQUIRE(m >= 1 && m % n_b == 0, "m = %d must be a positive multiple of n_b = %d", m, n_b);
    CHEBFD_REQUIRE(d_colmajor && d_blocked, "NULL buffer");
    CHEBFD_REQUIRE(aligned(d_colmajor, 16) && aligned(d_blocked, 16), "buffers must be 16-byte aligned");
    CHEBFD_REQUIRE(!overlap(d_colmajor, 16 * H->n * m, d_blocked, vec_elem_bytes(prec) * H->n * m),
                   "source and destination overlap");
    return launch_pack(H->identity_perm ? nullptr : H->perm, H->n, m, n_b, prec, d_colmajor,
                       d_blocked, false, static_cast<hipStream_t>(stream));
}

int chebfd_unpack(const chebfd_matrix *H, int32_t m, int32_t n_b, int32_t prec,
                  const void *d_blocked, void *d_colmajor, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(prec, n_b))) return rc;
    CHEBFD_REQUIRE(m >= 1 && m % n_b == 0, "m = %d must be a positive multiple of n_b = %d", m, n_b);
    CHEBFD_REQUIRE(d_colmajor && d_blocked, "NULL buffer");
    CHEBFD_REQUIRE(aligned(d_colmajor, 16) && aligned(d_blocked, 16), "buffers must be 16-byte aligned");
    CHEBFD_REQUIRE(!overlap(d_colmajor, 16 * H->n * m, d_blocked, vec_elem_bytes(prec) * H->n * m),
                   "source and destination overlap");
    return launch_pack(H->identity_perm ? nullptr : H->perm, H->n, m, n_b, prec, d_blocked,
                       d_colmajor, true, static_cast<hipStream_t>(stream));
}

int chebfd_random_phase(const chebfd_matrix *H, int32_t m, int32_t n_b, int32_t prec, uint64_t seed,
                        uint64_t col0, void *d_blocked, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(prec, n_b))) return rc;
    CHEBFD_REQUIRE(m >= 1 && m % n_b == 0, "m = %d must be a positive multiple of n_b = %d", m, n_b);
    CHEBFD_REQUIRE(d_blocked && aligned(d_blocked, 16), "d_blocked must be non-NULL and 16-byte aligned");
    return launch_random_phase(d_blocked, prec, H->n, n_b, 0, m, seed, col0, H->identity_perm ? nullptr : H->perm,
                               static_cast<hipStream_t>(stream));
}

// workspace of the filter: two partial buffers [3*n_b][G] (double buffered),
// then one progress word per workgroup (the window kernel's lead control)
static size_t filter_part_bytes(int nb, int G) { return round_up(sizeof(double) * 3 * nb * (size_t)G, 256); }
static size_t filter_work_bytes(int nb, int G) {
    return 2 * filter_part_bytes(nb, G) + round_up(sizeof(int64_t) * (size_t)G, 256);
}
static int64_t *filter_prog(void *d_work, int nb, int G) {
    return reinterpret_cast<int64_t *>(static_cast<char *>(d_work) + 2 * filter_part_bytes(nb, G));
}

// Launch geometry of the step kernels.  The window kernel (U staged in LDS)
// serves the block widths it has instances for when the row order keeps most
// gathers within its window; otherwise the LDS-staged kernel (matrix slots in
// LDS) is used for chunks of C = 32 rows with rows of at most 16 entries (its
// instances' tile width); otherwise n_b >= 32 uses the row-per-wavefront
// kernel and smaller n_b the multi-row kernel.
struct StepGeometry {
    int kind;           // 0 = LDS-staged, 1 = row per wavefront, 2 = multi-row, 3 = window
    int64_t npass;      // passes (kinds 1, 2)
    int G;
    LdsGeometry lds;
    WinGeometry win;
};

static int filter_geometry(const chebfd_matrix *H, int prec, int nb, StepGeometry *g) {
    DeviceProps d;
    int rc = device_props(&d);
    if (rc) return rc;
    if (win_geometry(H, prec, nb, d.num_cus, &g->win)) {
        g->kind = 3;
        g->npass = g->win.ntiles;
        g->G = g->win.G;
    } else if (lds_geometry(H, prec, nb, d.num_cus, &g->lds)) {
        g->kind = 0;
        g->npass = g->lds.ntiles;
        g->G = g->lds.G;
    } else if (nb >= kRowKernelMinNb) {
        g->kind = 1;
        const int rows = row_kernel_rows_per_pass(nb);
        g->npass = (H->n + rows - 1) / rows;
        int64_t G = static_cast<int64_t>(d.num_cus) * row_occupancy(prec, nb);
        if (G > g->npass) G = g->npass;
        if (G >= 8) G -= G % 8;
        g->G = static_cast<int>(G < 1 ? 1 : G);
    } else {
        g->kind = 2;
        const int rows = 256 / nb;
        g->npass = (H->n + rows - 1) / rows;
        g->G = step_grid(prec, nb, g->npass, d.num_cus);
    }
    return CHEBFD_OK;
}

static int launch_any(const chebfd_matrix *H, int prec, int nb, int mode, StepArgs a,
                      const StepGeometry &g, hipStream_t s) {
    a.npass = g.npass;
    if (g.kind == 3) return launch_win_step(prec, nb, mode, a, g.win, s);
    if (g.kind == 0) return launch_lds_step(prec, nb, mode, a, g.lds, s);
    if (g.kind == 1) return launch_row_step(prec, nb, H->max_width, mode, a, g.G, s);
    return launch_step(prec, nb, mode, a, g.G, s);
}

int chebfd_filter_query(const chebfd_matrix *H, int32_t n_b, size_t *work_bytes) {
    clear_error();
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(H->prec, n_b))) return rc;
    CHEBFD_REQUIRE(work_bytes != nullptr, "work_bytes is NULL");
    StepGeometry g;
    if ((rc = filter_geometry(H, H->prec, n_b, &g))) return rc;
    *work_bytes = filter_work_bytes(n_b, g.G);
    return CHEBFD_OK;
}

int chebfd_step_kernel(const chebfd_matrix *H, int32_t n_b, int32_t *kind) {
    clear_error();
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(H->prec, n_b))) return rc;
    CHEBFD_REQUIRE(kind != nullptr, "kind is NULL");
    StepGeometry g;
    if ((rc = filter_geometry(H, H->prec, n_b, &g))) return rc;
    *kind = g.kind;
    return CHEBFD_OK;
}

static StepArgs base_args(const chebfd_matrix *H, double alpha, double beta) {
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = H->n;
    a.n_chunks = H->n_chunks;
    a.chunk_off = H->chunk_off;
    a.chunk_width = H->chunk_width;
    a.col = H->col;
    a.val = H->val;
    a.C = H->C;
    a.log2C = ilog2_exact(H->C);
    a.alpha = alpha;
    a.beta = beta;
    a.uniform_width = H->uniform_width;
    return a;
}

static int filter_run(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma, int n_p,
                      int n_s, int n_b, int prec, void *d_xy, void *d_u, void *d_w, double *d_eta,
                      double *d_nu, void *d_work, size_t need, const StepGeometry &geo, bool moments_only,
                      hipStream_t s);

// Argument checks shared by chebfd_filter and chebfd_filter_unfused; on
// success *geo holds the step kernels' launch geometry.
static int check_filter_args(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma, int32_t n_p,
                             int32_t n_s, int32_t n_b, int32_t prec, void *d_xy, void *d_u, void *d_w,
                             double *d_eta, double *d_nu, void *d_work, size_t work_bytes, StepGeometry *geo,
                             size_t *need_out) {
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(prec, n_b))) return rc;
    CHEBFD_REQUIRE(prec == H->prec, "prec %d differs from the matrix's %d", prec, H->prec);
    CHEBFD_REQUIRE(n_p >= 0 && h_gamma != nullptr, "n_p = %d / gamma invalid", n_p);
    CHEBFD_REQUIRE(n_s >= 1 && n_s % n_b == 0, "n_s = %d must be a positive multiple of n_b = %d", n_s, n_b);
    CHEBFD_REQUIRE(std::isfinite(alpha) && std::isfinite(beta), "alpha/beta not finite");
    for (int p = 0; p <= n_p; ++p)
        CHEBFD_REQUIRE(std::isfinite(h_gamma[p]), "gamma[%d] not finite", p);
    CHEBFD_REQUIRE((d_eta == nullptr) == (d_nu == nullptr), "d_eta and d_nu must both be set or both NULL");
    CHEBFD_REQUIRE(d_xy && d_u && d_w && d_work, "NULL device buffer");
    for (const void *ptr : {(const void *)d_xy, (const void *)d_u, (const void *)d_w,
                            (const void *)d_work, (const void *)d_eta, (const void *)d_nu})
        CHEBFD_REQUIRE(ptr == nullptr || aligned(ptr, 256), "device buffers must be 256-byte aligned");
    const size_t eb = vec_elem_bytes(prec);
    const size_t blk = eb * (size_t)H->n * n_b;
    const size_t xy_bytes = blk * (n_s / n_b);
    if ((rc = filter_geometry(H, prec, n_b, geo))) return rc;
    const size_t need = filter_work_bytes(n_b, geo->G);
    if (work_bytes < need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "filter workspace %zu < %zu", work_bytes, need);
    CHEBFD_REQUIRE(!overlap(d_xy, xy_bytes, d_u, blk) && !overlap(d_xy, xy_bytes, d_w, blk) &&
                       !overlap(d_u, blk, d_w, blk) && !overlap(d_work, need, d_xy, xy_bytes) &&
                       !overlap(d_work, need, d_u, blk) && !overlap(d_work, need, d_w, blk),
                   "filter buffers overlap");
    if (d_eta) {
        const size_t mb = sizeof(double) * (size_t)(n_p + 1) * n_s;
        CHEBFD_REQUIRE(!overlap(d_eta, 2 * mb, d_nu, mb), "d_eta and d_nu overlap");
    }
    *need_out = need;
    return CHEBFD_OK;
}

int chebfd_filter(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma,
                  int32_t n_p, int32_t n_s, int32_t n_b, int32_t prec, void *d_xy, void *d_u,
                  void *d_w, double *d_eta, double *d_nu, void *d_work, size_t work_bytes,
                  void *stream) {
    clear_error();
    StepGeometry geo;
    size_t need = 0;
    int rc = check_filter_args(H, alpha, beta, h_gamma, n_p, n_s, n_b, prec, d_xy, d_u, d_w, d_eta, d_nu, d_work,
                               work_bytes, &geo, &need);
    if (rc) return rc;
    return filter_run(H, alpha, beta, h_gamma, n_p, n_s, n_b, prec, d_xy, d_u, d_w, d_eta, d_nu, d_work, need,
                      geo, false, static_cast<hipStream_t>(stream));
}

static int filter_unfused_run(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma, int n_p,
                              int n_s, int n_b, int prec, void *d_xy, void *d_u, void *d_w, double *d_eta,
                              double *d_nu, void *d_work, const StepGeometry &geo, hipStream_t s);

int chebfd_filter_noalloc(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma,
                          int32_t n_p, int32_t n_s, int32_t n_b, int32_t prec, void *d_xy, void *d_u,
                          void *d_w, double *d_eta, double *d_nu, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(prec, n_b))) return rc;
    StepGeometry geo;
    if ((rc = filter_geometry(H, prec, n_b, &geo))) return rc;
    const size_t need = filter_work_bytes(n_b, geo.G);
    if (need > kNoAllocScratchBytes)
        CHEBFD_FAIL(CHEBFD_EWORKSPACE,
                    "n_b = %d needs %zu bytes of partial sums here; the static scratch holds %zu "
                    "(use chebfd_filter with a workspace)",
                    n_b, need, kNoAllocScratchBytes);
    void *work = nullptr;
    if ((rc = scratch_ptr(&work))) return rc;
    size_t need2 = 0;
    if ((rc = check_filter_args(H, alpha, beta, h_gamma, n_p, n_s, n_b, prec, d_xy, d_u, d_w, d_eta, d_nu, work,
                                kNoAllocScratchBytes, &geo, &need2)))
        return rc;
    return filter_run(H, alpha, beta, h_gamma, n_p, n_s, n_b, prec, d_xy, d_u, d_w, d_eta, d_nu, work, need2, geo,
                      false, static_cast<hipStream_t>(stream));
}

int chebfd_filter_unfused(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma,
                          int32_t n_p, int32_t n_s, int32_t n_b, int32_t prec, void *d_xy, void *d_u,
                          void *d_w, double *d_eta, double *d_nu, void *d_work, size_t work_bytes,
                          void *stream) {
    clear_error();
    StepGeometry geo;
    size_t need = 0;
    int rc = check_filter_args(H, alpha, beta, h_gamma, n_p, n_s, n_b, prec, d_xy, d_u, d_w, d_eta, d_nu, d_work,
                               work_bytes, &geo, &need);
    if (rc) return rc;
    return filter_unfused_run(H, alpha, beta, h_gamma, n_p, n_s, n_b, prec, d_xy, d_u, d_w, d_eta, d_nu, d_work,
                              geo, static_cast<hipStream_t>(stream));
}

// The unfused filter: Alg. 1 from separate calls, each one pass over its
// operands in HBM (the SpMMV with the recurrence's scaling and shift, two
// block dot products and the axpby of the filtered block), as in the paper's
// comparison of chebfd_op with standard SpMMV and BLAS1 calls (Sect. 3.2).
// Arguments validated by the caller; the partials of the dot products go to
// the first half of the filter workspace and are reduced once per step.
static int filter_unfused_run(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma, int n_p,
                              int n_s, int n_b, int prec, void *d_xy, void *d_u, void *d_w, double *d_eta,
                              double *d_nu, void *d_work, const StepGeometry &geo, hipStream_t s) {
    int rc;
    const int G = geo.G;
    const size_t blk = vec_elem_bytes(prec) * (size_t)H->n * n_b;
    double *part = static_cast<double *>(d_work);
    const int64_t count = H->n * (int64_t)n_b;
    // eta_p = <new, prior>, nu_p = <prior, prior> of block b into row p of the moments
    auto moments = [&](const void *nw, const void *prior, int p, int b) -> int {
        if (!d_eta) return CHEBFD_OK;
        int r;
        if ((r = launch_block_dot(prec, n_b, H->n, nw, prior, part, G, 0, true, s))) return r;
        if ((r = launch_block_dot(prec, n_b, H->n, prior, prior, part, G, 2, false, s))) return r;
        StepArgs a;
        std::memset(&a, 0, sizeof(a));
        a.part_in = part;
        a.red_eta = d_eta + 2 * ((int64_t)p * n_s + (int64_t)b * n_b);
        a.red_nu = d_nu + ((int64_t)p * n_s + (int64_t)b * n_b);
        a.G_prev = G;
        return launch_reduce(n_b, a, s);
    };
    for (int b = 0; b < n_s / n_b; ++b) {
        char *X = static_cast<char *>(d_xy) + blk * b;
        if (n_p == 0) {
            if ((rc = launch_block_axpby(prec, count, h_gamma[0], X, 0.0, nullptr, s))) return rc;
            continue;
        }
        // U <- (aH + bI) X                                          (Alg. 1, first product)
        StepArgs a = base_args(H, alpha, beta);
        a.P = X;
        a.N = d_u;
        if ((rc = launch_any(H, prec, n_b, kModeSpmv, a, geo, s))) return rc;
        if ((rc = moments(d_u, X, 1, b))) return rc;
        if (n_p == 1) {
            if ((rc = launch_block_axpby(prec, count, h_gamma[0], X, h_gamma[1], d_u, s))) return rc;
            continue;
        }
        // W <- X, W <- 2(aH + bI) U - W                             (Alg. 1, second product)
        if ((rc = launch_block_axpby(prec, count, 0.0, d_w, 1.0, X, s))) return rc;
        a = base_args(H, alpha, beta);
        a.P = d_u;
        a.O = d_w;
        if ((rc = launch_any(H, prec, n_b, kModeSpmvRec, a, geo, s))) return rc;
        if ((rc = moments(d_w, d_u, 2, b))) return rc;
        // X <- g0c0 X + g1c1 U + g2c2 W                              (Alg. 1, bscal + baxpy)
        if ((rc = launch_block_axpby(prec, count, h_gamma[0], X, h_gamma[1], d_u, s))) return rc;
        if ((rc = launch_block_axpby(prec, count, 1.0, X, h_gamma[2], d_w, s))) return rc;
        // p = 3..n_p: swap(W, U); W <- 2(aH + bI) U - W; eta, nu; X += g_p c_p W
        void *Ub = d_w, *Wb = d_u;
        for (int p = 3; p <= n_p; ++p) {
            a = base_args(H, alpha, beta);
            a.P = Ub;
            a.O = Wb;
            if ((rc = launch_any(H, prec, n_b, kModeSpmvRec, a, geo, s))) return rc;
            if ((rc = moments(Wb, Ub, p, b))) return rc;
            if ((rc = launch_block_axpby(prec, count, 1.0, X, h_gamma[p], Wb, s))) return rc;
            std::swap(Ub, Wb);
        }
    }
    return CHEBFD_OK;
}

// The filter driver shared by chebfd_filter and chebfd_kpm_moments (arguments
// validated by the caller).  moments_only: Alg. 1 without the filtered-block
// update (the KPM moments); X is then overwritten by Chebyshev vectors.
static int filter_run(const chebfd_matrix *H, double alpha, double beta, const double *h_gamma, int n_p,
                      int n_s, int n_b, int prec, void *d_xy, void *d_u, void *d_w, double *d_eta,
                      double *d_nu, void *d_work, size_t need, const StepGeometry &geo, bool moments_only,
                      hipStream_t s) {
    int rc;
    const int G = geo.G;
    const size_t blk = vec_elem_bytes(prec) * (size_t)H->n * n_b;
    double *part[2];
    part[0] = static_cast<double *>(d_work);
    part[1] = reinterpret_cast<double *>(static_cast<char *>(d_work) + filter_part_bytes(n_b, G));
    int64_t *prog = filter_prog(d_work, n_b, G);
    (void)need;
    const int nblocks = n_s / n_b;
    const int64_t count = H->n * (int64_t)n_b;

    // pending reduction: the partials of the last launch and where they go
    const double *pend_part = nullptr;
    double *pend_eta = nullptr, *pend_nu = nullptr;
    int flip = 0;
    auto next_args = [&](StepArgs a, int p, int b) {
        a.part_out = part[flip];
        a.part_in = pend_part;
        a.red_eta = pend_eta;
        a.red_nu = pend_nu;
        a.G_prev = G;
        a.prog = prog;
        a.epoch = next_step_epoch();
        pend_part = part[flip];
        if (d_eta) {
            pend_eta = d_eta + 2 * ((int64_t)p * n_s + (int64_t)b * n_b);
            pend_nu = d_nu + ((int64_t)p * n_s + (int64_t)b * n_b);
        } else {
            pend_eta = nullptr;
            pend_nu = nullptr;
        }
        if (!d_eta) a.part_in = nullptr;
        flip ^= 1;
        return a;
    };

    for (int b = 0; b < nblocks; ++b) {
        char *X = static_cast<char *>(d_xy) + blk * b;
        void *A = d_u, *B = d_w;
        if (n_p == 0) {
            if (!moments_only &&
                (rc = launch_axpby_blocked(prec, count, h_gamma[0], X, 0.0, nullptr, s)))
                return rc;
            continue;
        }
        StepArgs a = base_args(H, alpha, beta);
        // U <- (aH + bI) X                                         (Alg. 1, first product)
        a.P = X;
        a.N = A;
        if ((rc = launch_any(H, prec, n_b, kModeFirst, next_args(a, 1, b), geo, s))) return rc;
        if (moments_only) {
            // X <- 2(aH + bI) U - X = T_2 x, then alternate in place (no Y)
            void *cur = A, *prv = X;
            for (int p = 2; p <= n_p; ++p) {
                a = base_args(H, alpha, beta);
                a.P = cur;
                a.O = prv;
                if ((rc = launch_any(H, prec, n_b, kModeKpm, next_args(a, p, b), geo, s))) return rc;
                std::swap(cur, prv);
            }
            continue;
        }
        if (n_p == 1) {
            if ((rc = launch_axpby_blocked(prec, count, h_gamma[0], X, h_gamma[1], A, s))) return rc;
            continue;
        }
        // W <- 2(aH + bI) U - X;  X <- g0c0 X + g1c1 U + g2c2 W         (Alg. 1, start of Y)
        a = base_args(H, alpha, beta);
        a.P = A;
        a.O = X;
        a.N = B;
        a.Y = X;
        a.g0 = h_gamma[0];
        a.g1 = h_gamma[1];
        a.g2 = h_gamma[2];
        if ((rc = launch_any(H, prec, n_b, kModeSecond, next_args(a, 2, b), geo, s))) return rc;
        // p = 3..n_p: swap(W, U); chebfd_op(H, U, W, X)                  (Alg. 1, recurrence)
        void *Ub = B, *Wb = A;  // after the swap U holds T_2, W holds T_1
        for (int p = 3; p <= n_p; ++p) {
            a = base_args(H, alpha, beta);
            a.P = Ub;
            a.O = Wb;
            a.Y = X;
            a.g2 = h_gamma[p];
            if ((rc = launch_any(H, prec, n_b, kModeStep, next_args(a, p, b), geo, s))) return rc;
            std::swap(Ub, Wb);
        }
    }
    if (d_eta && pend_part) {
        StepArgs a;
        std::memset(&a, 0, sizeof(a));
        a.part_in = pend_part;
        a.red_eta = pend_eta;
        a.red_nu = pend_nu;
        a.G_prev = G;
        if ((rc = launch_reduce(n_b, a, s))) return rc;
    }
    return CHEBFD_OK;
}

// KPM workspace: X (R vectors, blocked by n_b = min(R, 32)), U, eta, nu and the
// filter partials, each 256-byte aligned.  Moments-only runs need no W block.
struct KpmLayout {
    size_t x, u, eta, nu, part, filter_bytes, total;
};

static int kpm_layout(const chebfd_matrix *H, int n_steps, int R, StepGeometry *geo, KpmLayout *L) {
    int rc;
    if ((rc = check_handle(H))) return rc;
    CHEBFD_REQUIRE(n_steps >= 1, "n_steps = %d < 1", n_steps);
    CHEBFD_REQUIRE(R >= 1 && ((R <= 32 && (R & (R - 1)) == 0) || R % 32 == 0),
                   "R = %d must be a power of two up to 32 or a multiple of 32", R);
    const int n_b = R < 32 ? R : 32;
    if ((rc = filter_geometry(H, H->prec, n_b, geo))) return rc;
    L->filter_bytes = filter_work_bytes(n_b, geo->G);
    const size_t sw = vec_elem_bytes(H->prec), n = H->n;
    size_t at = 0;
    auto take = [&](size_t b) { size_t h = at; at = round_up(at + b, 256); return h; };
    L->x = take(n * R * sw);
    L->u = take(n * n_b * sw);
    L->eta = take(sizeof(double) * 2 * (size_t)(n_steps + 1) * R);
    L->nu = take(sizeof(double) * (size_t)(n_steps + 1) * R);
    L->part = take(L->filter_bytes);
    L->total = at;
    return CHEBFD_OK;
}

int chebfd_kpm_query(const chebfd_matrix *H, int32_t n_steps, int32_t R, size_t *work_bytes) {
    clear_error();
    CHEBFD_REQUIRE(work_bytes != nullptr, "work_bytes is NULL");
    StepGeometry geo;
    KpmLayout L;
    int rc = kpm_layout(H, n_steps, R, &geo, &L);
    if (rc) return rc;
    *work_bytes = L.total;
    return CHEBFD_OK;
}

int chebfd_kpm_moments(const chebfd_matrix *H, double alpha, double beta, int32_t n_steps, int32_t R,
                       uint64_t seed, double *h_mu, void *d_work, size_t work_bytes, void *stream) {
    clear_error();
    StepGeometry geo;
    KpmLayout L;
    int rc = kpm_layout(H, n_steps, R, &geo, &L);
    if (rc) return rc;
    CHEBFD_REQUIRE(h_mu != nullptr, "h_mu is NULL");
    CHEBFD_REQUIRE(std::isfinite(alpha) && std::isfinite(beta), "alpha/beta not finite");
    CHEBFD_REQUIRE(d_work && aligned(d_work, 256), "d_work must be non-NULL and 256-byte aligned");
    if (work_bytes < L.total) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "KPM workspace %zu < %zu", work_bytes, L.total);
    const int n_b = R < 32 ? R : 32;
    const int prec = H->prec;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(d_work);
    double *eta = reinterpret_cast<double *>(w + L.eta), *nu = reinterpret_cast<double *>(w + L.nu);
    if ((rc = launch_random_phase(w + L.x, prec, H->n, n_b, 0, R, seed, 0,
                                  H->identity_perm ? nullptr : H->perm, s)))
        return rc;
    // W is never touched by a moments-only run; U stands in for it
    if ((rc = filter_run(H, alpha, beta, nullptr, n_steps, R, n_b, prec, w + L.x, w + L.u, w + L.u, eta, nu,
                         w + L.part, L.filter_bytes, geo, true, s)))
        return rc;
    std::vector<double> he(2 * (size_t)(n_steps + 1) * R), hn((size_t)(n_steps + 1) * R);
    CHEBFD_HIP(hipMemcpyAsync(he.data(), eta, sizeof(double) * he.size(), hipMemcpyDeviceToHost, s));
    CHEBFD_HIP(hipMemcpyAsync(hn.data(), nu, sizeof(double) * hn.size(), hipMemcpyDeviceToHost, s));
    CHEBFD_HIP(hipStreamSynchronize(s));
    // Column sums of eta_q = <T_q x, T_{q-1} x> and nu_q = <T_{q-1} x, T_{q-1} x>,
    // then the product rule: mu_0 = nu_1, mu_1 = eta_1, mu_2k = 2 nu_{k+1} - mu_0,
    // mu_{2k+1} = 2 eta_{k+1} - mu_1.  Real parts: H is Hermitian.
    std::vector<double> se(n_steps + 1, 0.0), sn(n_steps + 1, 0.0);
    for (int q = 1; q <= n_steps; ++q)
        for (int j = 0; j < R; ++j) {
            se[q] += he[2 * ((size_t)q * R + j)];
            sn[q] += hn[(size_t)q * R + j];
        }
    const double scale = 1.0 / ((double)H->n * R);
    const double mu0 = sn[1], mu1 = se[1];
    h_mu[0] = mu0 * scale;
    h_mu[1] = mu1 * scale;
    for (int k = 1; k < n_steps; ++k) {
        h_mu[2 * k] = (2.0 * sn[k + 1] - mu0) * scale;
        h_mu[2 * k + 1] = (2.0 * se[k + 1] - mu1) * scale;
    }
    return CHEBFD_OK;
}

int chebfd_op(const chebfd_matrix *H, double alpha, double beta, double gamma, int32_t n_b,
              int32_t prec, const void *d_u, void *d_w, void *d_y, void *d_work, size_t work_bytes,
              void *stream) {
    clear_error();
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(prec, n_b))) return rc;
    CHEBFD_REQUIRE(prec == H->prec, "prec %d differs from the matrix's %d", prec, H->prec);
    CHEBFD_REQUIRE(d_u && d_w && d_y && d_work, "NULL device buffer");
    const size_t blk = vec_elem_bytes(prec) * (size_t)H->n * n_b;
    StepGeometry geo;
    if ((rc = filter_geometry(H, prec, n_b, &geo))) return rc;
    const int G = geo.G;
    const size_t need = filter_work_bytes(n_b, G);
    if (work_bytes < need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "workspace %zu < %zu", work_bytes, need);
    CHEBFD_REQUIRE(!overlap(d_u, blk, d_w, blk) && !overlap(d_u, blk, d_y, blk) &&
                       !overlap(d_w, blk, d_y, blk) && !overlap(d_work, need, d_u, blk) &&
                       !overlap(d_work, need, d_w, blk) && !overlap(d_work, need, d_y, blk),
                   "buffers overlap");
    StepArgs a = base_args(H, alpha, beta);
    a.P = d_u;
    a.O = d_w;
    a.Y = d_y;
    a.g2 = gamma;
    a.part_out = static_cast<double *>(d_work);
    a.prog = filter_prog(d_work, n_b, G);
    a.epoch = next_step_epoch();
    return launch_any(H, prec, n_b, kModeStep, a, geo, static_cast<hipStream_t>(stream));
}

int chebfd_spmmv(const chebfd_matrix *H, double alpha, double beta, int32_t n_b, int32_t prec,
                 const void *d_x, void *d_y, void *d_work, size_t work_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_handle(H)) || (rc = check_prec_nb(prec, n_b))) return rc;
    CHEBFD_REQUIRE(prec == H->prec, "prec %d differs from the matrix's %d", prec, H->prec);
    CHEBFD_REQUIRE(d_x && d_y && d_work, "NULL device buffer");
    CHEBFD_REQUIRE(std::isfinite(alpha) && std::isfinite(beta), "alpha/beta not finite");
    const size_t blk = vec_elem_bytes(prec) * (size_t)H->n * n_b;
    StepGeometry geo;
    if ((rc = filter_geometry(H, prec, n_b, &geo))) return rc;
    const size_t need = filter_work_bytes(n_b, geo.G);
    if (work_bytes < need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "workspace %zu < %zu", work_bytes, need);
    CHEBFD_REQUIRE(!overlap(d_x, blk, d_y, blk) && !overlap(d_work, need, d_x, blk) &&
                       !overlap(d_work, need, d_y, blk),
                   "buffers overlap");
    StepArgs a = base_args(H, alpha, beta);
    a.P = d_x;
    a.N = d_y;
    a.part_out = static_cast<double *>(d_work);
    return launch_any(H, prec, n_b, kModeFirst, a, geo, static_cast<hipStream_t>(stream));
}

int chebfd_probe_stream(int32_t kind, int64_t count, const double *d_b, const double *d_c, double s,
                        double *d_a, void *stream) {
    clear_error();
    CHEBFD_REQUIRE(kind >= 0 && kind <= 3, "kind = %d invalid", kind);
    CHEBFD_REQUIRE(count >= 2 && count % 2 == 0, "count must be even and >= 2");
    CHEBFD_REQUIRE(d_a && d_b && (kind != 1 || d_c), "NULL buffer");
    CHEBFD_REQUIRE(aligned(d_a, 16) && aligned(d_b, 16) && (kind != 1 || aligned(d_c, 16)),
                   "buffers must be 16-byte aligned");
    DeviceProps d;
    int rc = device_props(&d);
    if (rc) return rc;
    return launch_stream_probe(kind, count, d_b, d_c, s, d_a, d.num_cus,
                               static_cast<hipStream_t>(stream));
}

}  // extern "C"
