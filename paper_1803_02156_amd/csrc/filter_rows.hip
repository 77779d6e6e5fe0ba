// Row-per-wavefront variant of the fused Chebyshev step for block widths
// n_b >= 32 (gfx950, wave64).
//
// Each wavefront owns one matrix row per pass, so the row's SELL-C-sigma slots
// (column index and value of each stored entry) are wave-uniform and are read
// with scalar loads into SGPRs: no vector-memory instructions are spent on the
// matrix, and all of a row's gathers can be issued back to back.
//
// A wavefront covers 32 columns of its row (n_b / 32 wavefronts per row).  Its
// 64 lanes are two halves of 32 columns and lane (j, h) handles component h
// (re or im) of column j in every access: the gathers, the stream loads and
// stores of U, W, Y.  Each such access of the wavefront is one contiguous
// segment of the row-major block (512 bytes in FP64).  The complex products are
// formed from one component per lane and completed by one exchange across the
// halves.
//
// The column indices of a wavefront's next row are loaded while the current
// row's gathers are in flight (a two-stage software pipeline); the values enter
// the FMAs directly as SGPR operands.  The dot products and the cross-launch
// reduction follow the same fixed-order scheme as the multi-row kernel.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "kernels.h"

namespace chebfd {

namespace {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kXcds = 8;

template <int NB>
__device__ void reduce_prev(const StepArgs &a, double *sred) {
    const int tid = threadIdx.x;
    for (int q = blockIdx.x; q < 3 * NB; q += gridDim.x) {
        const double *src = a.part_in + (int64_t)q * a.G_prev;
        double s = 0.0;
        for (int g = tid; g < a.G_prev; g += kThreads) s += src[g];
        sred[tid] = s;
        __syncthreads();
        for (int hh = kThreads / 2; hh > 0; hh >>= 1) {
            if (tid < hh) sred[tid] += sred[tid + hh];
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

}  // namespace

template <typename T, int NB, int MODE, int ME>
__global__ __launch_bounds__(kThreads) void cheb_row_kernel(StepArgs a) {
    using VT = typename V2<T>::type;
    using CT = const __attribute__((address_space(4))) T *;          // scalar (SMEM) loads
    using CI32 = const __attribute__((address_space(4))) int32_t *;
    using CI64 = const __attribute__((address_space(4))) int64_t *;
    constexpr int CB = NB / 32;            // 32-column blocks per row
    constexpr int RPP = kWaves / CB;       // rows per workgroup pass
    static_assert(NB == 32 || NB == 64 || NB == 128, "row kernel covers n_b in {32, 64, 128}");
    __shared__ double sred[3 * kThreads];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rin = wv / CB;                  // row of this wave within the pass
    const int cb = wv % CB;                   // column block of this wave
    const int h = lane >> 5;                  // component of this lane: 0 = re, 1 = im
    const int j = cb * 32 + (lane & 31);      // column

    if (a.part_in != nullptr) reduce_prev<NB>(a, sred);

    const T *__restrict__ Pc = static_cast<const T *>(a.P);
    const CT valT = (CT)(a.val);  // interleaved (re, im)
    const CI32 col = (CI32)(a.col);
    const CI64 chunk_off = (CI64)(a.chunk_off);
    const CI32 chunk_width = (CI32)(a.chunk_width);

    const T alpha = static_cast<T>(a.alpha), beta = static_cast<T>(a.beta);
    const T g0 = static_cast<T>(a.g0), g1 = static_cast<T>(a.g1), g2 = static_cast<T>(a.g2);

    double d_re = 0.0, d_im = 0.0, d_nu = 0.0;

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

    // slot offset and width of row i: arithmetic when every chunk is equally wide
    auto locate = [&](int64_t i, int64_t &off, int &wdt) {
        const int64_t c = i >> a.log2C;
        const int64_t r = i & (a.C - 1);
        if (a.uniform_width > 0) {
            wdt = a.uniform_width;
            off = c * (int64_t)wdt * a.C + r;
        } else {
            off = chunk_off[c] + r;
            wdt = chunk_width[c];
        }
    };

    // Software pipeline over this wavefront's rows: the column indices of the
    // next row are loaded (scalar) while the current row's gathers are in
    // flight, so a row costs one gather round trip.  Slots k >= wdt (readable:
    // the matrix buffer is padded) gather the row's own entry with coefficient 0.
    int64_t pass = begin;
    int64_t i_n = pass * RPP + rin, off_n = 0;
    int w_n = 0;
    bool have = pass < end && i_n < a.n;
    int32_t cn[ME];
    if (have) {
        locate(i_n, off_n, w_n);
#pragma unroll
        for (int k = 0; k < ME; ++k) cn[k] = col[off_n + (int64_t)k * a.C];
    }
    while (have) {
        const int64_t i = i_n, off = off_n;
        const int wdt = w_n;
        int32_t cs[ME];
#pragma unroll
        for (int k = 0; k < ME; ++k) cs[k] = cn[k];

        // gathers of component h of U[col, j] for the row's entries
        T u[ME];
        if (wdt <= ME) {
#pragma unroll
            for (int k = 0; k < ME; ++k) {
                const int64_t cc = k < wdt ? cs[k] : i;
                u[k] = Pc[(cc * NB + j) * 2 + h];
            }
        }
        // stream loads of row i, component h of column j
        const int64_t e2 = ((int64_t)i * NB + j) * 2 + h;
        const T up_c = Pc[e2];
        T o_c = 0, y_c = 0;
        if constexpr (!mode_first(MODE)) o_c = static_cast<const T *>(a.O)[e2];
        if constexpr (MODE == kModeStep) y_c = static_cast<const T *>(a.Y)[e2];

        // prefetch the next row's column indices
        pass += stride;
        i_n = pass * RPP + rin;
        have = pass < end && i_n < a.n;
        if (have) {
            locate(i_n, off_n, w_n);
#pragma unroll
            for (int k = 0; k < ME; ++k) cn[k] = col[off_n + (int64_t)k * a.C];
        }

        // With H = hr + i hi and u the component h of U: A = sum hr u, B = sum hi u.
        // Re (HU) = A(re lane) - B(im lane), Im (HU) = A(im lane) + B(re lane).
        T A = 0, B = 0;
        if (wdt <= ME) {
#pragma unroll
            for (int k = 0; k < ME; ++k) {
                const int64_t sl = off + (int64_t)k * a.C;
                const T hr = k < wdt ? valT[2 * sl] : T(0);
                const T hi = k < wdt ? valT[2 * sl + 1] : T(0);
                A = fma(hr, u[k], A);
                B = fma(hi, u[k], B);
            }
        } else {
            for (int k = 0; k < wdt; ++k) {
                const int64_t sl = off + (int64_t)k * a.C;
                const int64_t cc = col[sl];
                const T uu = Pc[(cc * NB + j) * 2 + h];
                A = fma(valT[2 * sl], uu, A);
                B = fma(valT[2 * sl + 1], uu, B);
            }
        }
        const T B_other = __shfl_xor(B, 32);
        const T acc_c = h ? A + B_other : A - B_other;
        const T hu = fma(alpha, acc_c, beta * up_c);
        T nw;
        if constexpr (mode_first(MODE)) {
            nw = hu;
            static_cast<T *>(a.N)[e2] = nw;
        } else {
            nw = fma(T(2), hu, -o_c);
            if constexpr (MODE == kModeSecond) {
                static_cast<T *>(a.N)[e2] = nw;
                static_cast<T *>(a.Y)[e2] = fma(g0, o_c, fma(g1, up_c, g2 * nw));
            } else {
                static_cast<T *>(a.O)[e2] = nw;
                if constexpr (MODE == kModeStep) static_cast<T *>(a.Y)[e2] = fma(g2, nw, y_c);
            }
        }
        // eta = sum conj(nw) up: Re from same-component products, Im from the
        // other component of nw (exchanged across halves); nu = sum |up|^2
        if constexpr (mode_dots(MODE)) {
            const double nwd = nw, upd = up_c;
            const double nwo = __shfl_xor(nwd, 32);
            d_re = fma(nwd, upd, d_re);
            d_im = fma(h ? nwo : -nwo, upd, d_im);
            d_nu = fma(upd, upd, d_nu);
        }
    }
    if constexpr (!mode_dots(MODE)) return;

    // workgroup reduction in a fixed order: the two halves, then the rows of
    // the pass that share this column block
    d_re += __shfl_xor(d_re, 32);
    d_im += __shfl_xor(d_im, 32);
    d_nu += __shfl_xor(d_nu, 32);
    __syncthreads();
    if (h == 0) {
        sred[0 * kThreads + wv * 64 + lane] = d_re;
        sred[1 * kThreads + wv * 64 + lane] = d_im;
        sred[2 * kThreads + wv * 64 + lane] = d_nu;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NB; t += kThreads) {
        const int tcb = t / 32, tl = t % 32;
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
            double sum = 0.0;
            for (int r = 0; r < RPP; ++r) sum += sred[comp * kThreads + (r * CB + tcb) * 64 + tl];
            a.part_out[(int64_t)(comp * NB + t) * G + w] = sum;
        }
    }
}

namespace {

template <typename T, int NB, int MODE, int ME>
int launch_row_one(const StepArgs &a0, int G, hipStream_t s) {
    StepArgs a = a0;
    hipLaunchKernelGGL((cheb_row_kernel<T, NB, MODE, ME>), dim3(G), dim3(kThreads), 0, s, a);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

template <typename T, int NB, int ME>
int launch_row_mode(int mode, const StepArgs &a, int G, hipStream_t s) {
    switch (mode) {
        case kModeFirst: return launch_row_one<T, NB, kModeFirst, ME>(a, G, s);
        case kModeSecond: return launch_row_one<T, NB, kModeSecond, ME>(a, G, s);
        case kModeStep: return launch_row_one<T, NB, kModeStep, ME>(a, G, s);
        case kModeKpm: return launch_row_one<T, NB, kModeKpm, ME>(a, G, s);
        case kModeSpmv: return launch_row_one<T, NB, kModeSpmv, ME>(a, G, s);
        case kModeSpmvRec: return launch_row_one<T, NB, kModeSpmvRec, ME>(a, G, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "bad step mode %d", mode);
}

template <typename T, int NB>
int launch_row_me(int max_width, int mode, const StepArgs &a, int G, hipStream_t s) {
    if (max_width <= 13) return launch_row_mode<T, NB, 13>(mode, a, G, s);
    return launch_row_mode<T, NB, kRowMaxUnrolled>(mode, a, G, s);
}

template <typename T>
int launch_row_nb(int nb, int max_width, int mode, const StepArgs &a, int G, hipStream_t s) {
    switch (nb) {
        case 32: return launch_row_me<T, 32>(max_width, mode, a, G, s);
        case 64: return launch_row_me<T, 64>(max_width, mode, a, G, s);
        case 128: return launch_row_me<T, 128>(max_width, mode, a, G, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "row kernel: n_b = %d not in {32, 64, 128}", nb);
}

template <typename T, int NB>
int occ_row() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, cheb_row_kernel<T, NB, kModeStep, kRowMaxUnrolled>, kThreads, 0) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    return blocks;
}

}  // namespace

int launch_row_step(int prec, int nb, int max_width, int mode, const StepArgs &a, int G,
                    hipStream_t s) {
    if (prec == CHEBFD_PREC_FP64) return launch_row_nb<double>(nb, max_width, mode, a, G, s);
    return launch_row_nb<float>(nb, max_width, mode, a, G, s);
}

int row_occupancy(int prec, int nb) {
    static int cache[2][3] = {};
    const int p = prec == CHEBFD_PREC_FP64 ? 0 : 1;
    const int q = nb == 32 ? 0 : nb == 64 ? 1 : 2;
    int &o = cache[p][q];
    if (o == 0) {
        if (p == 0)
            o = nb == 32 ? occ_row<double, 32>() : nb == 64 ? occ_row<double, 64>() : occ_row<double, 128>();
        else
            o = nb == 32 ? occ_row<float, 32>() : nb == 64 ? occ_row<float, 64>() : occ_row<float, 128>();
    }
    return o;
}

}  // namespace chebfd
