// Fused block Chebyshev filter kernels for gfx950 (MI355X).
//
// One kernel template covers the start of the filter and its inner step
// (Alg. 1 of the ChebFD paper, Sect. 2): a SELL-C-sigma complex sparse
// matrix times a row-major block of NB vectors (SpMMV), the Chebyshev
// three-term recurrence, the filtered-block update and the two per-column dot
// products, all in one pass over the rows (the fusion of Sect. 3.1 that the
// paper calls chebfd_op).
//
// Thread mapping: a 256-thread workgroup covers ROWS = 256/NB rows per pass;
// lane t works on column j = t % NB of row t / NB.  For NB >= 32 every row
// spans half a wavefront or more, so the lanes of a row read one matrix entry
// (a broadcast) and NB consecutive vector entries (a coalesced 16*NB or 8*NB
// byte segment of the row-major block).  For small NB the lanes of a
// wavefront cover consecutive rows of a SELL chunk, whose column-major slots
// are then read coalesced.
//
// Grid: a persistent grid of G workgroups (the device's resident capacity).
// Workgroups are dispatched round-robin over the 8 XCDs, so workgroup w runs on
// XCD w % 8; each XCD is given one contiguous eighth of the row passes and its
// workgroups sweep it together, which keeps the neighbouring rows gathered
// from the block vector in that XCD's L2.
//
// Dot products are accumulated per lane in FP64, reduced in the workgroup in a
// fixed order and written as per-workgroup partials.  The next launch on the
// stream (the next step) reduces the previous step's partials in a fixed
// order in G-independent workgroups, so the reduction costs no extra launch
// and is bitwise reproducible (no floating-point atomics).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "kernels.h"

namespace chebfd {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };

constexpr int kThreads = 256;
constexpr int kXcds = 8;

// Reduce the previous step's partials: item q in [0, 3*NB) is the sum over
// g < G_prev of part_in[q*G_prev + g]; comp = q / NB selects Re eta, Im eta, nu.
template <int NB>
__device__ void reduce_previous(const StepArgs &a, double *sred) {
    const int tid = threadIdx.x;
    for (int q = blockIdx.x; q < 3 * NB; q += gridDim.x) {
        const double *src = a.part_in + (int64_t)q * a.G_prev;
        double s = 0.0;
        for (int g = tid; g < a.G_prev; g += kThreads) s += src[g];
        sred[tid] = s;
        __syncthreads();
        for (int h = kThreads / 2; h > 0; h >>= 1) {
            if (tid < h) sred[tid] += sred[tid + h];
            __syncthreads();
        }
        if (tid == 0) {
            const int comp = q / NB, jj = q % NB;
            if (comp < 2)
                a.red_eta[2 * jj + comp] = sred[0];
            else
                a.red_nu[jj] = sred[0];
        }
        __syncthreads();
    }
}

template <typename T, int NB, int MODE>
__global__ __launch_bounds__(kThreads) void cheb_step_kernel(StepArgs a) {
    using VT = typename V2<T>::type;
    constexpr int ROWS = kThreads / NB;
    __shared__ double sred[3 * kThreads];

    const int tid = threadIdx.x;
    const int j = tid % NB;
    const int rr = tid / NB;

    if (a.part_in != nullptr) reduce_previous<NB>(a, sred);

    const VT *__restrict__ P = static_cast<const VT *>(a.P);
    VT *O = static_cast<VT *>(a.O);  // Y may alias O (start of the filter)
    VT *__restrict__ N = static_cast<VT *>(a.N);
    VT *Y = static_cast<VT *>(a.Y);
    const VT *__restrict__ val = static_cast<const VT *>(a.val);
    const int32_t *__restrict__ col = a.col;

    const T alpha = static_cast<T>(a.alpha), beta = static_cast<T>(a.beta);
    const T g0 = static_cast<T>(a.g0), g1 = static_cast<T>(a.g1), g2 = static_cast<T>(a.g2);

    double e_re = 0.0, e_im = 0.0, nu = 0.0;

    // pass range of this workgroup: XCD-contiguous sweep
    const int G = gridDim.x, w = blockIdx.x;
    int64_t begin, end, stride;
    if (G % kXcds == 0 && a.npass >= G) {
        const int x = w % kXcds, k = w / kXcds;
        begin = a.npass * x / kXcds + k;
        end = a.npass * (x + 1) / kXcds;
        stride = G / kXcds;
    } else {
        begin = w;
        end = a.npass;
        stride = G;
    }

    for (int64_t pass = begin; pass < end; pass += stride) {
        const int64_t i = pass * ROWS + rr;
        if (i >= a.n) continue;
        const int64_t c = i >> a.log2C;
        const int r = static_cast<int>(i & (a.C - 1));
        const int64_t off = a.chunk_off[c] + r;
        const int wdt = a.chunk_width[c];

        T acc_re = 0, acc_im = 0;
        int k = 0;
        for (; k + 4 <= wdt; k += 4) {
            int cc[4];
            VT h[4], u[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) cc[q] = col[off + (int64_t)(k + q) * a.C];
#pragma unroll
            for (int q = 0; q < 4; ++q) h[q] = val[off + (int64_t)(k + q) * a.C];
#pragma unroll
            for (int q = 0; q < 4; ++q) u[q] = P[(int64_t)cc[q] * NB + j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc_re = fma(h[q].x, u[q].x, acc_re);
                acc_re = fma(-h[q].y, u[q].y, acc_re);
                acc_im = fma(h[q].x, u[q].y, acc_im);
                acc_im = fma(h[q].y, u[q].x, acc_im);
            }
        }
        for (; k < wdt; ++k) {
            const int cc = col[off + (int64_t)k * a.C];
            const VT h = val[off + (int64_t)k * a.C];
            const VT u = P[(int64_t)cc * NB + j];
            acc_re = fma(h.x, u.x, acc_re);
            acc_re = fma(-h.y, u.y, acc_re);
            acc_im = fma(h.x, u.y, acc_im);
            acc_im = fma(h.y, u.x, acc_im);
        }

        const int64_t e = i * NB + j;
        const VT up = P[e];
        // (alpha H + beta I) U at (i, j)
        const T hu_re = fma(alpha, acc_re, beta * up.x);
        const T hu_im = fma(alpha, acc_im, beta * up.y);

        VT nw;
        if constexpr (mode_first(MODE)) {
            nw.x = hu_re;
            nw.y = hu_im;
            N[e] = nw;
        } else {
            const VT o = O[e];
            nw.x = fma(T(2), hu_re, -o.x);
            nw.y = fma(T(2), hu_im, -o.y);
            if constexpr (MODE == kModeSecond) {
                N[e] = nw;
                VT y;
                y.x = fma(g0, o.x, fma(g1, up.x, g2 * nw.x));
                y.y = fma(g0, o.y, fma(g1, up.y, g2 * nw.y));
                Y[e] = y;  // Y aliases O: row i's old entry is read only here
            } else {
                O[e] = nw;
                if constexpr (MODE == kModeStep) {
                    VT y = Y[e];
                    y.x = fma(g2, nw.x, y.x);
                    y.y = fma(g2, nw.y, y.y);
                    Y[e] = y;
                }
            }
        }
        if constexpr (mode_dots(MODE)) {
            // eta += conj(new) * prior, nu += |prior|^2 (FP64)
            const double nr = nw.x, ni = nw.y, ur = up.x, ui = up.y;
            e_re = fma(nr, ur, fma(ni, ui, e_re));
            e_im = fma(nr, ui, fma(-ni, ur, e_im));
            nu = fma(ur, ur, fma(ui, ui, nu));
        }
    }
    if constexpr (!mode_dots(MODE)) return;

    // workgroup reduction over the ROWS lanes of each column, fixed order
    sred[tid] = e_re;
    sred[kThreads + tid] = e_im;
    sred[2 * kThreads + tid] = nu;
    __syncthreads();
    if (tid < NB) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int q = 0; q < ROWS; ++q) {
            s0 += sred[q * NB + tid];
            s1 += sred[kThreads + q * NB + tid];
            s2 += sred[2 * kThreads + q * NB + tid];
        }
        a.part_out[(int64_t)(0 * NB + tid) * G + w] = s0;
        a.part_out[(int64_t)(1 * NB + tid) * G + w] = s1;
        a.part_out[(int64_t)(2 * NB + tid) * G + w] = s2;
    }
}

// Reduce the last step's partials (no new step follows on the stream).
template <int NB>
__global__ __launch_bounds__(kThreads) void reduce_partials_kernel(StepArgs a) {
    __shared__ double sred[kThreads];
    reduce_previous<NB>(a, sred);
}

// ---------------------------------------------------------------------------
// host side: instantiation table and launch geometry
// ---------------------------------------------------------------------------
template <typename T, int NB, int MODE>
static int launch_one(const StepArgs &a0, int G, hipStream_t s) {
    StepArgs a = a0;
    hipLaunchKernelGGL((cheb_step_kernel<T, NB, MODE>), dim3(G), dim3(kThreads), 0, s, a);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

template <typename T, int NB>
static int launch_mode(int mode, const StepArgs &a, int G, hipStream_t s) {
    switch (mode) {
        case kModeFirst: return launch_one<T, NB, kModeFirst>(a, G, s);
        case kModeSecond: return launch_one<T, NB, kModeSecond>(a, G, s);
        case kModeStep: return launch_one<T, NB, kModeStep>(a, G, s);
        case kModeKpm: return launch_one<T, NB, kModeKpm>(a, G, s);
        case kModeSpmv: return launch_one<T, NB, kModeSpmv>(a, G, s);
        case kModeSpmvRec: return launch_one<T, NB, kModeSpmvRec>(a, G, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "bad step mode %d", mode);
}

template <typename T>
static int launch_nb(int nb, int mode, const StepArgs &a, int G, hipStream_t s) {
    switch (nb) {
        case 1: return launch_mode<T, 1>(mode, a, G, s);
        case 2: return launch_mode<T, 2>(mode, a, G, s);
        case 4: return launch_mode<T, 4>(mode, a, G, s);
        case 8: return launch_mode<T, 8>(mode, a, G, s);
        case 16: return launch_mode<T, 16>(mode, a, G, s);
        case 32: return launch_mode<T, 32>(mode, a, G, s);
        case 64: return launch_mode<T, 64>(mode, a, G, s);
        case 128: return launch_mode<T, 128>(mode, a, G, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "n_b = %d not supported (1, 2, 4, ..., 128)", nb);
}

int launch_step(int prec, int nb, int mode, const StepArgs &a, int G, hipStream_t s) {
    if (prec == CHEBFD_PREC_FP64) return launch_nb<double>(nb, mode, a, G, s);
    return launch_nb<float>(nb, mode, a, G, s);
}

template <int NB>
static int launch_reduce_nb(const StepArgs &a0, hipStream_t s) {
    StepArgs a = a0;
    const int G = 3 * NB;
    hipLaunchKernelGGL((reduce_partials_kernel<NB>), dim3(G), dim3(kThreads), 0, s, a);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int launch_reduce(int nb, const StepArgs &a, hipStream_t s) {
    switch (nb) {
        case 1: return launch_reduce_nb<1>(a, s);
        case 2: return launch_reduce_nb<2>(a, s);
        case 4: return launch_reduce_nb<4>(a, s);
        case 8: return launch_reduce_nb<8>(a, s);
        case 16: return launch_reduce_nb<16>(a, s);
        case 32: return launch_reduce_nb<32>(a, s);
        case 64: return launch_reduce_nb<64>(a, s);
        case 128: return launch_reduce_nb<128>(a, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "n_b = %d not supported", nb);
}

// Resident workgroups per CU for the step kernel (same for every mode and
// precision in practice; taken from the FP64 step kernel of this NB).
template <typename T, int NB>
static int occupancy_nb() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, cheb_step_kernel<T, NB, kModeStep>,
                                                     kThreads, 0) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    return blocks;
}

template <typename T>
static int occupancy_t(int nb) {
    switch (nb) {
        case 1: return occupancy_nb<T, 1>();
        case 2: return occupancy_nb<T, 2>();
        case 4: return occupancy_nb<T, 4>();
        case 8: return occupancy_nb<T, 8>();
        case 16: return occupancy_nb<T, 16>();
        case 32: return occupancy_nb<T, 32>();
        case 64: return occupancy_nb<T, 64>();
        case 128: return occupancy_nb<T, 128>();
    }
    return 1;
}

int step_grid(int prec, int nb, int64_t npass, int num_cus) {
    static int cache[2][8] = {};
    int lg = 0;
    while ((1 << lg) < nb) ++lg;
    int &occ = cache[prec == CHEBFD_PREC_FP64 ? 0 : 1][lg];
    if (occ == 0) occ = prec == CHEBFD_PREC_FP64 ? occupancy_t<double>(nb) : occupancy_t<float>(nb);
    int64_t G = static_cast<int64_t>(num_cus) * occ;
    if (G > npass) G = npass;
    if (G >= kXcds) G -= G % kXcds;
    if (G < 1) G = 1;
    return static_cast<int>(G);
}

}  // namespace chebfd
