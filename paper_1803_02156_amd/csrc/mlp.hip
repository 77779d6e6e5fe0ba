// Parameter predictor: a small FP32 multilayer perceptron from KPM moment
// features to (n_p, n_s), with forward pass, loss gradient and Adam update on
// the device.  The moments it reads are those of the filter's dot products
// (Sect. 2: KPM moments and the eigenvalue count come out of Alg. 1); the
// predictor replaces the hand-tuned choice of n_p and n_s (Sect. 2, Sect. 2.1).
//
// Network: x (258) -> relu(W1 x + b1) (128) -> relu(W2 h1 + b2) (128) -> W3 h2 + b3 (2).
// Parameters: one flat FP32 vector W1, b1, W2, b2, W3, b3 (weights row-major,
// output index slowest).  Batches are row-major (batch x features).
//
// The layers are small (2000 x 258 x 128 at most): a 64 x 64 LDS-tiled FP32
// VALU GEMM with fused bias / ReLU / ReLU-mask epilogues covers the forward
// and the backward products.  Every output is accumulated by one thread in a
// fixed order, and the reductions (loss, bias gradients) use fixed orders, so
// results are bit-reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"

namespace chebfd {
namespace {

constexpr int kIn = CHEBFD_MLP_IN, kHid = CHEBFD_MLP_HIDDEN, kOut = CHEBFD_MLP_OUT;
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kHid * kIn;
constexpr int64_t kOffW2 = kOffB1 + kHid;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kHid * kHid;
constexpr int64_t kOffW3 = kOffB2 + kHid;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kOut * kHid;
constexpr int64_t kParams = kOffB3 + kOut;
static_assert(kParams == CHEBFD_MLP_PARAMS, "parameter count");

constexpr int kTile = 64, kKT = 16, kThreads = 256;

// C[i][j] = epi( sum_k opA[i][k] opB[k][j] ),  opA[i][k] = TA ? A[k lda + i] : A[i lda + k],
// opB[k][j] = TB ? B[j ldb + k] : B[k ldb + j];  epi: + bias[j], relu, * (mask[i ldm + j] > 0).
template <bool TA, bool TB>
__global__ __launch_bounds__(kThreads) void gemm_kernel(int M, int N, int K, const float *__restrict__ A, int lda,
                                                        const float *__restrict__ B, int ldb, float *__restrict__ C,
                                                        int ldc, const float *__restrict__ bias, int relu,
                                                        const float *__restrict__ mask, int ldm) {
    __shared__ float sa[kKT][kTile + 1];
    __shared__ float sb[kKT][kTile + 1];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
    float acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0f;

    for (int k0 = 0; k0 < K; k0 += kKT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + kThreads * q;  // 0 .. 1023
            int row, kk;
            if (TA) {
                kk = e / kTile;
                row = e % kTile;
            } else {
                row = e / kKT;
                kk = e % kKT;
            }
            const int i = i0 + row, k = k0 + kk;
            float v = 0.0f;
            if (i < M && k < K) v = TA ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k];
            sa[kk][row] = v;
            int col;
            if (TB) {
                col = e / kKT;
                kk = e % kKT;
            } else {
                kk = e / kTile;
                col = e % kTile;
            }
            const int j = j0 + col, kb = k0 + kk;
            float w = 0.0f;
            if (j < N && kb < K) w = TB ? B[(int64_t)j * ldb + kb] : B[(int64_t)kb * ldb + j];
            sb[kk][col] = w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKT; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = sa[kk][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = sb[kk][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + ty + 16 * r;
        if (i >= M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + tx + 16 * c;
            if (j >= N) continue;
            float v = acc[r][c];
            if (bias) v += bias[j];
            if (relu) v = fmaxf(v, 0.0f);
            if (mask && !(mask[(int64_t)i * ldm + j] > 0.0f)) v = 0.0f;
            C[(int64_t)i * ldc + j] = v;
        }
    }
}

// dY = (Y - T) / B and loss = sum (Y - T)^2 / (2 B); one workgroup, fixed order.
__global__ __launch_bounds__(kThreads) void loss_kernel(int count, float inv_b, const float *__restrict__ Y,
                                                        const float *__restrict__ T, float *__restrict__ dY,
                                                        float *__restrict__ loss) {
    __shared__ float s[kThreads];
    float acc = 0.0f;
    for (int e = threadIdx.x; e < count; e += kThreads) {
        const float d = Y[e] - T[e];
        dY[e] = d * inv_b;
        acc = fmaf(d, d, acc);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w /= 2) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = 0.5f * s[0] * inv_b;
}

// g[j] = sum_i D[i][j] over the rows of a rows x N row-major matrix.
__global__ __launch_bounds__(kThreads) void colsum_kernel(int rows, int N, const float *__restrict__ D,
                                                          float *__restrict__ g) {
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= N) return;
    float acc = 0.0f;
    for (int i = 0; i < rows; ++i) acc += D[(int64_t)i * N + j];
    g[j] = acc;
}

// Adam with bias correction factors c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ __launch_bounds__(kThreads) void adam_kernel(int64_t count, float *__restrict__ p,
                                                        const float *__restrict__ g, float *__restrict__ m,
                                                        float *__restrict__ v, float lr, float b1, float b2,
                                                        float c1, float c2, float eps) {
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * kThreads) {
        const float ge = g[e];
        const float me = fmaf(b1, m[e], (1.0f - b1) * ge);
        const float ve = fmaf(b2, v[e], (1.0f - b2) * ge * ge);
        m[e] = me;
        v[e] = ve;
        p[e] -= lr * (me * c1) / (sqrtf(ve * c2) + eps);
    }
}

template <bool TA, bool TB>
int gemm(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
         const float *bias, bool relu, const float *mask, int ldm, hipStream_t s) {
    const dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile);
    hipLaunchKernelGGL((gemm_kernel<TA, TB>), grid, dim3(kThreads), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       relu ? 1 : 0, mask, ldm);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

// Workspace of a batch: H1, H2 (batch x 128), Y, dY (batch x 2), dZ2, dZ1 (batch x 128).
struct MlpWork {
    float *h1, *h2, *y, *dy, *dz2, *dz1;
};

size_t mlp_work_layout(int batch, char *base, MlpWork *w) {
    size_t at = 0;
    auto take = [&](size_t floats) {
        char *p = base ? base + at : nullptr;
        at = round_up(at + floats * sizeof(float), 256);
        return reinterpret_cast<float *>(p);
    };
    MlpWork t;
    t.h1 = take((size_t)batch * kHid);
    t.h2 = take((size_t)batch * kHid);
    t.y = take((size_t)batch * kOut);
    t.dy = take((size_t)batch * kOut);
    t.dz2 = take((size_t)batch * kHid);
    t.dz1 = take((size_t)batch * kHid);
    if (w) *w = t;
    return at;
}

int check_batch(int batch, const void *d_work, size_t work_bytes, size_t *need) {
    CHEBFD_REQUIRE(batch >= 1 && batch <= (1 << 20), "batch = %d out of range [1, 2^20]", batch);
    *need = mlp_work_layout(batch, nullptr, nullptr);
    CHEBFD_REQUIRE(d_work && aligned(d_work, 256), "d_work must be non-NULL and 256-byte aligned");
    if (work_bytes < *need) CHEBFD_FAIL(CHEBFD_EWORKSPACE, "MLP workspace %zu < %zu", work_bytes, *need);
    return CHEBFD_OK;
}

int forward(const float *P, int batch, const float *X, float *Y, const MlpWork &w, hipStream_t s) {
    int rc;
    if ((rc = gemm<false, true>(batch, kHid, kIn, X, kIn, P + kOffW1, kIn, w.h1, kHid, P + kOffB1, true, nullptr,
                                0, s)))
        return rc;
    if ((rc = gemm<false, true>(batch, kHid, kHid, w.h1, kHid, P + kOffW2, kHid, w.h2, kHid, P + kOffB2, true,
                                nullptr, 0, s)))
        return rc;
    return gemm<false, true>(batch, kOut, kHid, w.h2, kHid, P + kOffW3, kHid, Y, kOut, P + kOffB3, false, nullptr,
                             0, s);
}

int colsum(int rows, int N, const float *D, float *g, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, s, rows, N, D, g);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

}  // namespace
}  // namespace chebfd

using namespace chebfd;

extern "C" {

int chebfd_mlp_query(int32_t batch, int32_t *n_params, size_t *work_bytes) {
    clear_error();
    CHEBFD_REQUIRE(batch >= 1 && batch <= (1 << 20), "batch = %d out of range [1, 2^20]", batch);
    if (n_params) *n_params = (int32_t)kParams;
    if (work_bytes) *work_bytes = mlp_work_layout(batch, nullptr, nullptr);
    return CHEBFD_OK;
}

int chebfd_mlp_forward(const float *d_params, int32_t batch, const float *d_x, float *d_y, void *d_work,
                       size_t work_bytes, void *stream) {
    clear_error();
    size_t need;
    int rc;
    if ((rc = check_batch(batch, d_work, work_bytes, &need))) return rc;
    CHEBFD_REQUIRE(d_params && d_x && d_y, "NULL device buffer");
    CHEBFD_REQUIRE(!overlap(d_y, sizeof(float) * kOut * (size_t)batch, d_work, need), "d_y overlaps d_work");
    MlpWork w;
    mlp_work_layout(batch, static_cast<char *>(d_work), &w);
    return forward(d_params, batch, d_x, d_y, w, static_cast<hipStream_t>(stream));
}

int chebfd_mlp_grad(const float *d_params, int32_t batch, const float *d_x, const float *d_t, float *d_loss,
                    float *d_grad, void *d_work, size_t work_bytes, void *stream) {
    clear_error();
    size_t need;
    int rc;
    if ((rc = check_batch(batch, d_work, work_bytes, &need))) return rc;
    CHEBFD_REQUIRE(d_params && d_x && d_t && d_loss && d_grad, "NULL device buffer");
    CHEBFD_REQUIRE(!overlap(d_grad, sizeof(float) * kParams, d_params, sizeof(float) * kParams) &&
                       !overlap(d_grad, sizeof(float) * kParams, d_work, need),
                   "d_grad overlaps d_params or d_work");
    hipStream_t s = static_cast<hipStream_t>(stream);
    MlpWork w;
    mlp_work_layout(batch, static_cast<char *>(d_work), &w);
    const float *P = d_params;
    float *G = d_grad;
    if ((rc = forward(P, batch, d_x, w.y, w, s))) return rc;
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(kThreads), 0, s, batch * kOut, 1.0f / (float)batch, w.y, d_t,
                       w.dy, d_loss);
    CHEBFD_HIP(hipGetLastError());
    // output layer: gW3 = dY^T H2, gb3 = colsum dY, dZ2 = (dY W3) * [H2 > 0]
    if ((rc = gemm<true, false>(kOut, kHid, batch, w.dy, kOut, w.h2, kHid, G + kOffW3, kHid, nullptr, false,
                                nullptr, 0, s)))
        return rc;
    if ((rc = colsum(batch, kOut, w.dy, G + kOffB3, s))) return rc;
    if ((rc = gemm<false, false>(batch, kHid, kOut, w.dy, kOut, P + kOffW3, kHid, w.dz2, kHid, nullptr, false, w.h2,
                                 kHid, s)))
        return rc;
    // second layer: gW2 = dZ2^T H1, gb2, dZ1 = (dZ2 W2) * [H1 > 0]
    if ((rc = gemm<true, false>(kHid, kHid, batch, w.dz2, kHid, w.h1, kHid, G + kOffW2, kHid, nullptr, false,
                                nullptr, 0, s)))
        return rc;
    if ((rc = colsum(batch, kHid, w.dz2, G + kOffB2, s))) return rc;
    if ((rc = gemm<false, false>(batch, kHid, kHid, w.dz2, kHid, P + kOffW2, kHid, w.dz1, kHid, nullptr, false,
                                 w.h1, kHid, s)))
        return rc;
    // first layer: gW1 = dZ1^T X, gb1
    if ((rc = gemm<true, false>(kHid, kIn, batch, w.dz1, kHid, d_x, kIn, G + kOffW1, kIn, nullptr, false, nullptr,
                                0, s)))
        return rc;
    return colsum(batch, kHid, w.dz1, G + kOffB1, s);
}

int chebfd_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step, float lr,
                    float beta1, float beta2, float eps, void *stream) {
    clear_error();
    CHEBFD_REQUIRE(d_params && d_grad && d_m && d_v, "NULL device buffer");
    CHEBFD_REQUIRE(step >= 1, "step = %d must count from 1", step);
    CHEBFD_REQUIRE(lr > 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f,
                   "Adam hyper-parameters out of range");
    const double c1 = 1.0 / (1.0 - std::pow((double)beta1, step));
    const double c2 = 1.0 / (1.0 - std::pow((double)beta2, step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((kParams + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), kParams, d_params, d_grad, d_m, d_v, lr, beta1, beta2,
                       (float)c1, (float)c2, eps);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

}  // extern "C"
