// BLAS1 building blocks of the unfused filter (gfx950): per-column dot
// products of two blocked n x NB blocks and a blocked axpby.
//
// The paper compares its fused chebfd_op with a version built from a minimum
// set of standard calls, the SpMMV and BLAS1 kernels run one after another
// (Sect. 3.2, the GHOST-nofuse variant of Fig. 2).  These are the BLAS1 calls
// of that version: each one streams its operands through HBM once.
//
// Dot products: lane t works on columns [CPL (t % LPR), CPL (t % LPR) + CPL)
// of row t / LPR of a pass (every access of a row segment contiguous, 16 bytes
// per lane), FP64 accumulation, fixed-order workgroup reduction, one partial
// per workgroup and column; launch_reduce turns the partials into the result.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "kernels.h"
#include "step_io.h"

namespace chebfd {
namespace {

using namespace step_io;

// The dot kernel runs on the step kernel's grid (its partials feed the same
// reduction), often one workgroup per CU: 1024 threads (four waves per SIMD),
// each with kDotUnroll row passes in flight, keep enough loads outstanding.
constexpr int kDotThreads = 1024;
constexpr int kDotUnroll = 4;
constexpr int kXcdN = 8;

template <typename T, int NB, bool IM>
__global__ __launch_bounds__(kDotThreads) void block_dot_kernel(int64_t n, const T *__restrict__ A,
                                                               const T *__restrict__ B, double *part,
                                                               int comp0) {
    constexpr int CPL = cols_per_lane<T, NB>();
    constexpr int LPR = NB / CPL;
    constexpr int ROWS = kDotThreads / LPR;
    __shared__ double sred[2 * CPL * kDotThreads];
    const int tid = threadIdx.x;
    const int jc = (tid % LPR) * CPL;
    const int rr = tid / LPR;
    const int G = gridDim.x, w = blockIdx.x;
    const int64_t npass = (n + ROWS - 1) / ROWS;
    // contiguous pass range per workgroup, one eighth of the rows per XCD
    int64_t begin, end;
    if (G % kXcdN == 0) {
        const int x = w % kXcdN, k = w / kXcdN, per = G / kXcdN;
        const int64_t xb = npass * x / kXcdN, xe = npass * (x + 1) / kXcdN;
        begin = xb + (xe - xb) * k / per;
        end = xb + (xe - xb) * (k + 1) / per;
    } else {
        begin = npass * w / G;
        end = npass * (w + 1) / G;
    }
    double s_re[CPL], s_im[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) s_re[c] = s_im[c] = 0.0;
    const bool same = A == B;
    for (int64_t pass = begin; pass < end; pass += kDotUnroll) {
        // the loads of kDotUnroll passes first, then the sums in pass order
        Pack<T, CPL> a[kDotUnroll], b[kDotUnroll];
#pragma unroll
        for (int u = 0; u < kDotUnroll; ++u) {
            const int64_t i = (pass + u) * ROWS + rr;
#pragma unroll
            for (int c = 0; c < CPL; ++c) a[u].re[c] = a[u].im[c] = b[u].re[c] = b[u].im[c] = T(0);
            if (pass + u < end && i < n) {
                const int64_t e = 2 * (i * NB + jc);
                a[u] = load_pack<T, CPL, true>(A + e);
                if (!same) b[u] = load_pack<T, CPL, true>(B + e);
            }
        }
#pragma unroll
        for (int u = 0; u < kDotUnroll; ++u) {
            const Pack<T, CPL> &bu = same ? a[u] : b[u];
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const double ar = a[u].re[c], ai = a[u].im[c], br = bu.re[c], bi = bu.im[c];
                // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
                s_re[c] = fma(ar, br, fma(ai, bi, s_re[c]));
                if constexpr (IM) s_im[c] = fma(ar, bi, fma(-ai, br, s_im[c]));
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        sred[(0 * CPL + c) * kDotThreads + tid] = s_re[c];
        sred[(1 * CPL + c) * kDotThreads + tid] = s_im[c];
    }
    __syncthreads();
    if (tid < NB) {
        const int lj = tid / CPL, c = tid % CPL;
        double r0 = 0.0, r1 = 0.0;
        for (int q = 0; q < ROWS; ++q) {
            r0 += sred[(0 * CPL + c) * kDotThreads + q * LPR + lj];
            if constexpr (IM) r1 += sred[(1 * CPL + c) * kDotThreads + q * LPR + lj];
        }
        part[(int64_t)(comp0 * NB + tid) * G + w] = r0;
        if constexpr (IM) part[(int64_t)((comp0 + 1) * NB + tid) * G + w] = r1;
    }
}

template <typename T, int NB>
int launch_dot_nb(int64_t n, const void *A, const void *B, double *part, int G, int comp0, bool im,
                  hipStream_t s) {
    const T *a = static_cast<const T *>(A), *b = static_cast<const T *>(B);
    if (im)
        hipLaunchKernelGGL((block_dot_kernel<T, NB, true>), dim3(G), dim3(kDotThreads), 0, s, n, a, b, part, comp0);
    else
        hipLaunchKernelGGL((block_dot_kernel<T, NB, false>), dim3(G), dim3(kDotThreads), 0, s, n, a, b, part,
                           comp0);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

template <typename T>
int launch_dot_t(int nb, int64_t n, const void *A, const void *B, double *part, int G, int comp0, bool im,
                 hipStream_t s) {
    switch (nb) {
        case 1: return launch_dot_nb<T, 1>(n, A, B, part, G, comp0, im, s);
        case 2: return launch_dot_nb<T, 2>(n, A, B, part, G, comp0, im, s);
        case 4: return launch_dot_nb<T, 4>(n, A, B, part, G, comp0, im, s);
        case 8: return launch_dot_nb<T, 8>(n, A, B, part, G, comp0, im, s);
        case 16: return launch_dot_nb<T, 16>(n, A, B, part, G, comp0, im, s);
        case 32: return launch_dot_nb<T, 32>(n, A, B, part, G, comp0, im, s);
        case 64: return launch_dot_nb<T, 64>(n, A, B, part, G, comp0, im, s);
        case 128: return launch_dot_nb<T, 128>(n, A, B, part, G, comp0, im, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "n_b = %d not supported", nb);
}

// y = a y + b x over `vecs` 16-byte vectors (W scalars of type T each) and, for
// an odd c64 count, one trailing complex number; y is not read when a == 0 and
// x not when b == 0.
template <typename T>
__global__ __launch_bounds__(256) void block_axpby_kernel(int64_t vecs, int tail, double a, T *y, double b,
                                                          const T *x) {
    typedef T v4 __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int W = 16 / sizeof(T);
    const T ta = static_cast<T>(a), tb = static_cast<T>(b);
    const bool ry = a != 0.0, rx = b != 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < vecs;
         t += (int64_t)gridDim.x * blockDim.x) {
        v4 yv = {}, xv = {};
        if (ry) yv = __builtin_nontemporal_load(reinterpret_cast<const v4 *>(y) + t);
        if (rx) xv = __builtin_nontemporal_load(reinterpret_cast<const v4 *>(x) + t);
        v4 r;
#pragma unroll
        for (int k = 0; k < W; ++k) r[k] = ry ? fma(ta, yv[k], tb * xv[k]) : tb * xv[k];
        __builtin_nontemporal_store(r, reinterpret_cast<v4 *>(y) + t);
    }
    if (tail && blockIdx.x == 0 && threadIdx.x < 2) {
        const int64_t k = vecs * W + threadIdx.x;
        const T yv = ry ? y[k] : T(0), xv = rx ? x[k] : T(0);
        y[k] = ry ? fma(ta, yv, tb * xv) : tb * xv;
    }
}

}  // namespace

int launch_block_dot(int prec, int nb, int64_t n, const void *A, const void *B, double *part, int G, int comp0,
                     bool want_im, hipStream_t s) {
    if (prec == CHEBFD_PREC_FP64) return launch_dot_t<double>(nb, n, A, B, part, G, comp0, want_im, s);
    return launch_dot_t<float>(nb, n, A, B, part, G, comp0, want_im, s);
}

int launch_block_axpby(int prec, int64_t count, double a, void *y, double b, const void *x, hipStream_t s) {
    const size_t eb = vec_elem_bytes(prec);
    const int64_t vecs = (int64_t)(count * eb / 16);
    const int tail = static_cast<int>((count * eb) % 16 != 0);
    // one 16-byte vector per thread over a flat grid (the launch shape of the
    // fastest stream probe; a persistent grid-stride loop streams about 13 %
    // slower here); the loop only matters past 2^31 workgroups
    int64_t G = (vecs + 255) / 256;
    if (G > 0x7fffffff) G = 0x7fffffff;
    if (G < 1) G = 1;
    if (prec == CHEBFD_PREC_FP64)
        hipLaunchKernelGGL((block_axpby_kernel<double>), dim3(G), dim3(256), 0, s, vecs, tail, a,
                           static_cast<double *>(y), b, static_cast<const double *>(x));
    else
        hipLaunchKernelGGL((block_axpby_kernel<float>), dim3(G), dim3(256), 0, s, vecs, tail, a,
                           static_cast<float *>(y), b, static_cast<const float *>(x));
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

}  // namespace chebfd
