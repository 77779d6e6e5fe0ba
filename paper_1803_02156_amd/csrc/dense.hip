// Dense kernels of the orthogonalisation and Rayleigh-Ritz steps (gfx950):
//  * tall-skinny Gram  S = A^H B  over the rows of two blocked block vectors
//    (FP64 MFMA, split over row ranges, deterministic fixed-order reduction);
//  * tall-skinny update  Z = A M  with a small FP64 complex matrix M (FP64 MFMA);
//  * a cyclic Jacobi eigensolver for small Hermitian matrices (one workgroup);
//  * column norms, scaled copies and the residual reduction.
//
// Block vectors use the filter's blocked layout: element (i, c) of an n x m
// block vector with block width nb is at ((c / nb) n + i) nb + c % nb, stored
// as c128 (prec FP64) or c64 (prec MIXED).  Small matrices are FP64 complex,
// column-major with leading dimension ld.
//
// MFMA: v_mfma_f64_16x16x4_f64 computes D(16x16) += A(16x4) B(4x16); lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[l / 16 + 4 r][l % 16] in its r-th accumulator (r = 0..3; measured on gfx950).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace chebfd {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kT = 256;

__device__ inline double2 load_c(const void *base, int prec, int64_t idx) {
    if (prec == CHEBFD_PREC_FP64) return static_cast<const double2 *>(base)[idx];
    const float2 f = static_cast<const float2 *>(base)[idx];
    double2 r;
    r.x = f.x;
    r.y = f.y;
    return r;
}

__device__ inline void store_c(void *base, int prec, int64_t idx, double2 v) {
    if (prec == CHEBFD_PREC_FP64) {
        static_cast<double2 *>(base)[idx] = v;
    } else {
        float2 f;
        f.x = static_cast<float>(v.x);
        f.y = static_cast<float>(v.y);
        static_cast<float2 *>(base)[idx] = f;
    }
}

// nb is a power of two (the launchers check): shifts instead of an integer division
__device__ inline int64_t blocked_index(int64_t n, int nb, int64_t i, int c) {
    const int lg = __ffs(nb) - 1;
    return ((int64_t)(c >> lg) * n + i) * nb + (c & (nb - 1));
}

// ---------------------------------------------------------------------------
// Gram: S(a, b) = sum_i conj(A(i, a)) B(i, b), 64 x 64 complex output tile per
// workgroup (4 waves, 32 x 32 each = 2 x 2 MFMA tiles x 4 real products), rows
// [r0, r1) of one split; partial tiles go to part[split][tile] and are summed
// in split order by gram_reduce_kernel.  For the Hermitian product A^H A only
// the tiles on and above the diagonal are formed (tile index t enumerates them
// column by column) and the reduction mirrors them.
// ---------------------------------------------------------------------------
constexpr int kGT = 64;   // output tile edge
constexpr int kGK = 16;   // rows per LDS stage

// (row tile, column tile) of output tile t: column-major over all tiles, or
// over the upper triangle (row tile <= column tile) when herm
__device__ inline void gram_tile(int t, int tiles_a, bool herm, int *ta, int *tb) {
    if (!herm) {
        *ta = t % tiles_a;
        *tb = t / tiles_a;
        return;
    }
    int c = 0;
    while ((c + 1) * (c + 2) / 2 <= t) ++c;
    *tb = c;
    *ta = t - c * (c + 1) / 2;
}

// Element types TA, TB of A and B (double: c128, float: c64) are template
// parameters: a storage precision chosen at run time made every element access
// a branch and kept the prefetch registers FP64 wide (two waves per SIMD
// instead of three; 287 -> 162 ms for a 33.5 M x 256 c64 product).  Stages stay
// in registers in the storage type until they go to LDS as FP64.
template <typename TA, typename TB, int BW>
__global__ __launch_bounds__(kT) void gram_kernel(const void *A, int nb_a, const void *B, int nb_b, int64_t n,
                                                   int m1, int m2, int tiles_a, int herm, int64_t rows_per_split,
                                                   double *part) {
    // output tile 64 (columns of A) x BW (columns of B); BW = 32 for products of at
    // most 32 columns of B (Rayleigh-Ritz and TSQR panels), so no wave multiplies zeros
    constexpr int KG = kGK;
    constexpr int NY = BW / 32;                // 16-column MFMA tiles per wave
    using RA = typename std::conditional<std::is_same<TA, double>::value, double2, float2>::type;
    using RB = typename std::conditional<std::is_same<TB, double>::value, double2, float2>::type;
    __shared__ double2 sa[KG][kGT];
    __shared__ double2 sb[KG][BW];
    const int tile = blockIdx.x;
    const int split = blockIdx.y;
    int ta, tb;
    gram_tile(tile, tiles_a, herm != 0, &ta, &tb);
    const int a0 = ta * kGT, b0 = tb * BW;
    const int64_t r0 = (int64_t)split * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < n ? r0 + rows_per_split : n;

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wa = (wv & 1) * 32, wb = (wv >> 1) * (BW / 2);  // wave's 32 x BW/2 sub-tile

    // two accumulators per 16 x 16 tile: real and imaginary part of the sum
    d4v acc[2][NY][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[x][y][q] = d4v{0.0, 0.0, 0.0, 0.0};

    // Stages of KG rows x 64 columns of A and KG rows x BW columns of B (zero
    // outside the matrices): the next stage's global loads are issued before the
    // current stage's products, so their latency hides behind the matrix-core work.
    constexpr int kPerA = KG * kGT / kT, kPerB = KG * BW / kT;   // elements per thread
    RA ra[kPerA];
    RB rb2[kPerB];
    auto fetch = [&](int64_t rbase) {
#pragma unroll
        for (int q = 0; q < kPerA; ++q) {
            const int t = threadIdx.x + q * kT;
            const int rr = t / kGT, cc = t % kGT;
            const int64_t i = rbase + rr;
            RA va{};
            if (i < r1 && a0 + cc < m1) va = static_cast<const RA *>(A)[blocked_index(n, nb_a, i, a0 + cc)];
            ra[q] = va;
        }
#pragma unroll
        for (int q = 0; q < kPerB; ++q) {
            const int t = threadIdx.x + q * kT;
            const int rr = t / BW, cc = t % BW;
            const int64_t i = rbase + rr;
            RB vb{};
            if (i < r1 && b0 + cc < m2) vb = static_cast<const RB *>(B)[blocked_index(n, nb_b, i, b0 + cc)];
            rb2[q] = vb;
        }
    };
    if (r0 < r1) fetch(r0);
    for (int64_t rb = r0; rb < r1; rb += KG) {
#pragma unroll
        for (int q = 0; q < kPerA; ++q) {
            const int t = threadIdx.x + q * kT;
            sa[t / kGT][t % kGT] = double2{(double)ra[q].x, (double)ra[q].y};
        }
#pragma unroll
        for (int q = 0; q < kPerB; ++q) {
            const int t = threadIdx.x + q * kT;
            sb[t / BW][t % BW] = double2{(double)rb2[q].x, (double)rb2[q].y};
        }
        __syncthreads();
        if (rb + KG < r1) fetch(rb + KG);
#pragma unroll
        for (int k0 = 0; k0 < KG; k0 += 4) {
            const int kk = k0 + lane / 16;
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const double2 av = sa[kk][wa + 16 * x + lane % 16];
#pragma unroll
                for (int y = 0; y < NY; ++y) {
                    const double2 bv = sb[kk][wb + 16 * y + lane % 16];
                    // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
                    acc[x][y][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, acc[x][y][0], 0, 0, 0);
                    acc[x][y][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.y, acc[x][y][0], 0, 0, 0);
                    acc[x][y][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, acc[x][y][1], 0, 0, 0);
                    acc[x][y][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.x, acc[x][y][1], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // write the partial tile into a 64 x 64 slot (column-major inside the slot;
    // a BW = 32 tile fills its first 32 columns, the reduction reads no others)
    double2 *out = reinterpret_cast<double2 *>(part) +
                   ((int64_t)split * gridDim.x + tile) * (kGT * kGT);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ra = wa + 16 * x + lane / 16 + 4 * r;  // row of S (column of A)
                const int cb = wb + 16 * y + lane % 16;            // column of S within the tile
                double2 v;
                v.x = acc[x][y][0][r];
                v.y = acc[x][y][1][r];
                out[(int64_t)cb * kGT + ra] = v;
            }
}

// S = sum over splits (in split order) of the partial tiles; S column-major, ld.
// herm: tiles above the diagonal also give their mirror image S(b, a) = conj S(a, b).
__global__ __launch_bounds__(kT) void gram_reduce_kernel(const double *part, int nsplit, int ntiles,
                                                         int tiles_a, int herm, int m1, int m2, double *S,
                                                         int ld) {
    const int64_t total = (int64_t)ntiles * kGT * kGT;
    const double2 *p = reinterpret_cast<const double2 *>(part);
    for (int64_t t = blockIdx.x * (int64_t)kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        const int tile = static_cast<int>(t / (kGT * kGT));
        const int e = static_cast<int>(t % (kGT * kGT));
        const int ra = e % kGT, cb = e / kGT;
        int ta, tb;
        gram_tile(tile, tiles_a, herm != 0, &ta, &tb);
        const int a = ta * kGT + ra, b = tb * kGT + cb;
        if (a >= m1 || b >= m2) continue;
        double sr = 0.0, si = 0.0;
        for (int s = 0; s < nsplit; ++s) {
            const double2 v = p[((int64_t)s * ntiles + tile) * (kGT * kGT) + e];
            sr += v.x;
            si += v.y;
        }
        reinterpret_cast<double2 *>(S)[(int64_t)b * ld + a] = double2{sr, si};
        if (herm && ta != tb) reinterpret_cast<double2 *>(S)[(int64_t)a * ld + b] = double2{sr, -si};
    }
}

// ---------------------------------------------------------------------------
// Update: Z(i, c) = sum_k A(i, k) M(k, c), M FP64 complex column-major (ld).
// 64 rows x 64 columns of Z per workgroup; k staged 16 at a time.
// ---------------------------------------------------------------------------
// Element types TA of A and TZ of Z (double: c128, float: c64) are template
// parameters, as for the Gram product.
// Z = A M, or Z = S - A M when TS (the storage type of S, blocked width nb_s) is
// not void; S may be Z itself (each entry is read by the thread that writes it).
template <typename TA, typename TZ, int BW, typename TS = void>
__global__ __launch_bounds__(kT) void update_kernel(const void *A, int nb_a, const double *M, int ldm, void *Z,
                                                    int nb_z, int64_t n, int m1, int m2, const void *S = nullptr,
                                                    int nb_s = 1) {
    // output tile 64 rows x BW columns of Z (BW = 32 when Z has at most 32 columns)
    constexpr int NY = BW / 32;                // 16-column MFMA tiles per wave
    using RA = typename std::conditional<std::is_same<TA, double>::value, double2, float2>::type;
    using RZ = typename std::conditional<std::is_same<TZ, double>::value, double2, float2>::type;
    __shared__ double2 sa[kGT][kGK + 1];
    __shared__ double2 sm[kGK][BW];
    const int64_t i0 = (int64_t)blockIdx.x * kGT;
    const int c0 = blockIdx.y * BW;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wi = (wv & 1) * 32, wc = (wv >> 1) * (BW / 2);
    const double2 *Mc = reinterpret_cast<const double2 *>(M);

    // two accumulators per 16 x 16 tile: real and imaginary part of the sum
    d4v acc[2][NY][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[x][y][q] = d4v{0.0, 0.0, 0.0, 0.0};

    // stages of kGK columns of A (64 rows) and kGK rows of M (BW columns): the next
    // stage's global loads are issued before the current stage's products
    constexpr int kPerA = kGT * kGK / kT, kPerM = BW * kGK / kT;   // elements per thread
    RA pa[kPerA];
    double2 pm[kPerM];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < kPerA; ++q) {
            const int t = threadIdx.x + q * kT;
            const int rr = t / kGK, kk = t % kGK;
            const int64_t i = i0 + rr;
            RA va{};
            if (i < n && k0 + kk < m1) va = static_cast<const RA *>(A)[blocked_index(n, nb_a, i, k0 + kk)];
            pa[q] = va;
        }
#pragma unroll
        for (int q = 0; q < kPerM; ++q) {
            const int t = threadIdx.x + q * kT;
            const int km = t / BW, cc = t % BW;
            double2 vm{0.0, 0.0};
            if (k0 + km < m1 && c0 + cc < m2) vm = Mc[(int64_t)(c0 + cc) * ldm + k0 + km];
            pm[q] = vm;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < m1; k0 += kGK) {
#pragma unroll
        for (int q = 0; q < kPerA; ++q) {
            const int t = threadIdx.x + q * kT;
            sa[t / kGK][t % kGK] = double2{(double)pa[q].x, (double)pa[q].y};
        }
#pragma unroll
        for (int q = 0; q < kPerM; ++q) {
            const int t = threadIdx.x + q * kT;
            sm[t / BW][t % BW] = pm[q];
        }
        __syncthreads();
        if (k0 + kGK < m1) fetch(k0 + kGK);
#pragma unroll
        for (int kb = 0; kb < kGK; kb += 4) {
            const int kk = kb + lane / 16;
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const double2 av = sa[wi + 16 * x + lane % 16][kk];
#pragma unroll
                for (int y = 0; y < NY; ++y) {
                    const double2 mv = sm[kk][wc + 16 * y + lane % 16];
                    // a m = (ar mr - ai mi) + i (ar mi + ai mr)
                    acc[x][y][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, mv.x, acc[x][y][0], 0, 0, 0);
                    acc[x][y][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, mv.y, acc[x][y][0], 0, 0, 0);
                    acc[x][y][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, mv.y, acc[x][y][1], 0, 0, 0);
                    acc[x][y][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, mv.x, acc[x][y][1], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + wi + 16 * x + lane / 16 + 4 * r;
                const int c = c0 + wc + 16 * y + lane % 16;
                if (i < n && c < m2) {
                    double vx = acc[x][y][0][r], vy = acc[x][y][1][r];
                    if constexpr (!std::is_void<TS>::value) {
                        using RS = typename std::conditional<std::is_same<TS, double>::value, double2, float2>::type;
                        const RS sv = static_cast<const RS *>(S)[blocked_index(n, nb_s, i, c)];
                        vx = static_cast<double>(sv.x) - vx;
                        vy = static_cast<double>(sv.y) - vy;
                    }
                    RZ v;
                    v.x = static_cast<TZ>(vx);
                    v.y = static_cast<TZ>(vy);
                    static_cast<RZ *>(Z)[blocked_index(n, nb_z, i, c)] = v;
                }
            }
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigensolver for a Hermitian m x m FP64 complex matrix.
// A sweep is me - 1 rounds (me = m rounded up to even) of the round-robin
// ordering; a round rotates me/2 disjoint (p, q) pairs.  For the pair block
// [[a, b], [conj(b), d]], b = |b| e^{i phi}, the rotation is
// J = diag(1, e^{-i phi}) [[c, s], [-s, c]] with t = s / c the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = (d - a) / (2 |b|); A <- J^H A J, V <- V J.
//
// One launch per round, one workgroup per pair: the workgroup first applies the
// previous round's row rotations (A <- J^H A, every pair) to its own two
// columns -- each column belongs to exactly one pair of every round, so every
// column receives them -- then forms its rotation from the updated columns and
// applies the column rotation to A and V.  The last round of a sweep is closed
// by a launch that applies its row rotations to all columns.  The rotated pair's
// off-diagonal entries are stored as exact zeros and its diagonal as real.
// ---------------------------------------------------------------------------
constexpr int kMaxM = 512;
constexpr int kJW = 256;       // threads per Jacobi workgroup
constexpr int kJNormG = 64;    // workgroups of the norm reduction

__device__ inline int rr_player(int m, int r, int k) {
    // round r, seat k of the circle method over players 0..m-1 (m even):
    // seat 0 holds player 0, the other seats rotate over 1..m-1
    return k == 0 ? 0 : ((k - 1 + r) % (m - 1)) + 1;
}

struct JacobiRound {
    int *p, *q;           // [2][kMaxM / 2] pair indices (p < q; q >= m: no rotation)
    double *c, *sr, *si;  // [2][kMaxM / 2] c and s e^{-i phi}
};

// rows p, q of column `col` <- J^H (rows p, q) for the rotation in slot `slot`, pair kk
__device__ inline void jacobi_row_rotate(double2 *Ac, int lda, const JacobiRound &jr, int slot, int kk, int col,
                                         int m) {
    const int h = slot * (kMaxM / 2) + kk;
    const int p = jr.p[h], q = jr.q[h];
    if (q >= m) return;
    const double c = jr.c[h], sr = jr.sr[h], si = -jr.si[h];  // s e^{+i phi}
    const double s = sqrt(sr * sr + si * si);
    const double er = s > 0.0 ? sr / s : 1.0, ei = s > 0.0 ? si / s : 0.0;
    const double2 x = Ac[(int64_t)col * lda + p], y = Ac[(int64_t)col * lda + q];
    double2 np, nq;
    np.x = c * x.x - (sr * y.x - si * y.y);
    np.y = c * x.y - (sr * y.y + si * y.x);
    nq.x = s * x.x + c * (er * y.x - ei * y.y);
    nq.y = s * x.y + c * (er * y.y + ei * y.x);
    if (col == q) np = double2{0.0, 0.0};
    if (col == p) {
        nq = double2{0.0, 0.0};
        np.y = 0.0;
    }
    if (col == q) nq.y = 0.0;
    Ac[(int64_t)col * lda + p] = np;
    Ac[(int64_t)col * lda + q] = nq;
}

__global__ __launch_bounds__(kJW) void jacobi_round_kernel(int m, int me, int r, int has_prev, double *A, int lda,
                                                           double *V, int ldv, JacobiRound jr) {
    __shared__ double s_par[3];
    double2 *Ac = reinterpret_cast<double2 *>(A);
    double2 *Vc = reinterpret_cast<double2 *>(V);
    const int half = me / 2, k = blockIdx.x, tid = threadIdx.x;
    int p = rr_player(me, r, k), q = rr_player(me, r, me - 1 - k);
    if (p > q) { const int tmp = p; p = q; q = tmp; }
    const int cur = r & 1, prv = cur ^ 1;
    // (a) the previous round's row rotations on columns p and q
    if (has_prev) {
        for (int t = tid; t < 2 * half; t += kJW) {
            const int col = t < half ? p : q;
            if (col < m) jacobi_row_rotate(Ac, lda, jr, prv, t % half, col, m);
        }
    }
    __syncthreads();
    // (b) this round's rotation from the updated columns
    if (tid == 0) {
        double c = 1.0, sr = 0.0, si = 0.0;
        if (q < m) {
            const double a = Ac[(int64_t)p * lda + p].x;
            const double d = Ac[(int64_t)q * lda + q].x;
            const double2 b = Ac[(int64_t)q * lda + p];  // A[p][q]
            const double ab = sqrt(b.x * b.x + b.y * b.y);
            if (ab > 0.0) {
                const double zeta = (d - a) / (2.0 * ab);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                c = 1.0 / sqrt(1.0 + t * t);
                const double sn = t * c;
                sr = sn * b.x / ab;   // s e^{-i phi} = s conj(b) / |b|
                si = -sn * b.y / ab;
            }
        }
        const int h = cur * (kMaxM / 2) + k;
        jr.p[h] = p;
        jr.q[h] = q;
        jr.c[h] = c;
        jr.sr[h] = sr;
        jr.si[h] = si;
        s_par[0] = c;
        s_par[1] = sr;
        s_par[2] = si;
    }
    __syncthreads();
    if (q >= m) return;
    // (c) columns: A(:,p) <- c A(:,p) - s e^{-i phi} A(:,q); A(:,q) <- s A(:,p) + c e^{-i phi} A(:,q); same for V
    const double c = s_par[0], sr = s_par[1], si = s_par[2];
    const double s = sqrt(sr * sr + si * si);
    const double er = s > 0.0 ? sr / s : 1.0, ei = s > 0.0 ? si / s : 0.0;
    for (int t = tid; t < 2 * m; t += kJW) {
        const int which = t / m, row = t % m;
        double2 *M = which ? Vc : Ac;
        const int ld = which ? ldv : lda;
        const double2 x = M[(int64_t)p * ld + row], y = M[(int64_t)q * ld + row];
        double2 np, nq;
        np.x = c * x.x - (sr * y.x - si * y.y);
        np.y = c * x.y - (sr * y.y + si * y.x);
        nq.x = s * x.x + c * (er * y.x - ei * y.y);
        nq.y = s * x.y + c * (er * y.y + ei * y.x);
        M[(int64_t)p * ld + row] = np;
        M[(int64_t)q * ld + row] = nq;
    }
}

// the row rotations of round slot `slot` on every column (closes a sweep)
__global__ __launch_bounds__(kJW) void jacobi_rows_kernel(int m, int me, int slot, double *A, int lda,
                                                          JacobiRound jr) {
    double2 *Ac = reinterpret_cast<double2 *>(A);
    const int half = me / 2;
    for (int col = blockIdx.x; col < m; col += gridDim.x)
        for (int t = threadIdx.x; t < half; t += kJW) jacobi_row_rotate(Ac, lda, jr, slot, t, col, m);
}

// partial sums of |A_ij|^2 (off-diagonal only if `off`), one per workgroup, fixed order
__global__ __launch_bounds__(kJW) void jacobi_norm_kernel(int m, const double *A, int lda, int off,
                                                          double *part) {
    __shared__ double sred[kJW];
    const double2 *Ac = reinterpret_cast<const double2 *>(A);
    double acc = 0.0;
    for (int t = blockIdx.x * kJW + threadIdx.x; t < m * m; t += gridDim.x * kJW) {
        const int r = t % m, c = t / m;
        if (off && r == c) continue;
        const double2 v = Ac[(int64_t)c * lda + r];
        acc += v.x * v.x + v.y * v.y;
    }
    sred[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kJW / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) sred[threadIdx.x] += sred[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sred[0];
}

__global__ __launch_bounds__(kJW) void jacobi_init_kernel(int m, double *V, int ldv) {
    double2 *Vc = reinterpret_cast<double2 *>(V);
    for (int t = blockIdx.x * kJW + threadIdx.x; t < m * m; t += gridDim.x * kJW) {
        const int r = t % m, c = t / m;
        Vc[(int64_t)c * ldv + r] = double2{r == c ? 1.0 : 0.0, 0.0};
    }
}

// eigenvalues ascending (ties by index) into w, eigenvectors permuted alike (one workgroup)
__global__ __launch_bounds__(kJW) void jacobi_sort_kernel(int m, double *A, int lda, double *V, int ldv,
                                                          double *w, double *scratch) {
    double2 *Ac = reinterpret_cast<double2 *>(A);
    double2 *Vc = reinterpret_cast<double2 *>(V);
    int *rank_of = reinterpret_cast<int *>(scratch + m);
    const int tid = threadIdx.x;
    for (int t = tid; t < m; t += kJW) scratch[t] = Ac[(int64_t)t * lda + t].x;
    __syncthreads();
    for (int t = tid; t < m; t += kJW) {
        const double d = scratch[t];
        int rank = 0;
        for (int u = 0; u < m; ++u) {
            const double e = scratch[u];
            rank += (e < d || (e == d && u < t)) ? 1 : 0;
        }
        w[rank] = d;
        rank_of[t] = rank;
    }
    __syncthreads();
    // permuted copy of V through A's storage (A is no longer needed)
    for (int t = tid; t < m * m; t += kJW) {
        const int r = t % m, c = t / m;
        Ac[(int64_t)rank_of[c] * lda + r] = Vc[(int64_t)c * ldv + r];
    }
    __syncthreads();
    for (int t = tid; t < m * m; t += kJW) {
        const int r = t % m, c = t / m;
        Vc[(int64_t)c * ldv + r] = Ac[(int64_t)c * lda + r];
    }
}

// ---------------------------------------------------------------------------
// small helpers of the SVQB / Rayleigh-Ritz / residual steps
// ---------------------------------------------------------------------------

// d_i = diag(S)_ii^{-1/2} (1 for non-positive entries); S <- D S D
__global__ __launch_bounds__(kT) void svqb_scale_kernel(int m, double *S, int ld, double *d) {
    double2 *Sc = reinterpret_cast<double2 *>(S);
    __shared__ double sd[kMaxM];
    for (int t = threadIdx.x; t < m; t += kT) {
        const double v = Sc[(int64_t)t * ld + t].x;
        sd[t] = v > 0.0 ? 1.0 / sqrt(v) : 1.0;
        d[t] = sd[t];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m * m; t += kT) {
        const int r = t % m, c = t / m;
        double2 v = Sc[(int64_t)c * ld + r];
        const double f = sd[r] * sd[c];
        v.x *= f;
        v.y *= f;
        Sc[(int64_t)c * ld + r] = v;
    }
}

// T(:, c) = D V(:, first + c) / sqrt(w[first + c]), c < k (the kept directions)
__global__ __launch_bounds__(kT) void svqb_transform_kernel(int m, int k, int first, const double *d,
                                                            const double *V, int ldv, const double *w,
                                                            double *T, int ldt) {
    const double2 *Vc = reinterpret_cast<const double2 *>(V);
    double2 *Tc = reinterpret_cast<double2 *>(T);
    for (int t = blockIdx.x * kT + threadIdx.x; t < m * k; t += gridDim.x * kT) {
        const int r = t % m, c = t / m;
        const double f = d[r] / sqrt(w[first + c]);
        double2 v = Vc[(int64_t)(first + c) * ldv + r];
        v.x *= f;
        v.y *= f;
        Tc[(int64_t)c * ldt + r] = v;
    }
}

// G <- (G + G^H) / 2
__global__ __launch_bounds__(kT) void hermitise_kernel(int m, double *G, int ld) {
    double2 *Gc = reinterpret_cast<double2 *>(G);
    for (int t = blockIdx.x * kT + threadIdx.x; t < m * m; t += gridDim.x * kT) {
        const int r = t % m, c = t / m;
        if (r > c) continue;
        const double2 a = Gc[(int64_t)c * ld + r], b = Gc[(int64_t)r * ld + c];
        const double2 u = double2{0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
        Gc[(int64_t)c * ld + r] = u;
        Gc[(int64_t)r * ld + c] = double2{u.x, -u.y};
    }
}

// Per column c of one n x nb block (blocked storage, precision prec): partial
// sums over the rows of this workgroup of |HZ - theta_c Z|^2 and |Z|^2, written
// to part[(2 c + q) * G + w]; reduced in order by colsum_reduce_kernel.
__global__ __launch_bounds__(kT) void resid_partial_kernel(const void *HZ, const void *Z, int prec,
                                                           int64_t n, int nb, const double *theta,
                                                           double *part) {
    __shared__ double s0[kT], s1[kT];
    const int cpt = nb < kT ? nb : kT;           // columns handled in parallel
    const int rows = kT / cpt;
    const int c = threadIdx.x % cpt, rr = threadIdx.x / cpt;
    for (int cb = 0; cb < nb; cb += cpt) {
        const int cc = cb + c;
        double a = 0.0, b = 0.0;
        const double th = theta ? theta[cc] : 0.0;
        for (int64_t i = (int64_t)blockIdx.x * rows + rr; i < n; i += (int64_t)gridDim.x * rows) {
            const int64_t e = i * nb + cc;
            const double2 h = load_c(HZ, prec, e), z = load_c(Z, prec, e);
            const double rx = h.x - th * z.x, ry = h.y - th * z.y;
            a += rx * rx + ry * ry;
            b += z.x * z.x + z.y * z.y;
        }
        s0[threadIdx.x] = a;
        s1[threadIdx.x] = b;
        __syncthreads();
        if (rr == 0) {
            double sa = 0.0, sb = 0.0;
            for (int q = 0; q < rows; ++q) {
                sa += s0[q * cpt + c];
                sb += s1[q * cpt + c];
            }
            part[(int64_t)(2 * cc) * gridDim.x + blockIdx.x] = sa;
            part[(int64_t)(2 * cc + 1) * gridDim.x + blockIdx.x] = sb;
        }
        __syncthreads();
    }
}

// out[q] = sum_g part[q * G + g], q < count (fixed order)
__global__ __launch_bounds__(kT) void colsum_reduce_kernel(const double *part, int G, int count,
                                                           double *out) {
    __shared__ double s[kT];
    for (int q = blockIdx.x; q < count; q += gridDim.x) {
        double a = 0.0;
        for (int g = threadIdx.x; g < G; g += kT) a += part[(int64_t)q * G + g];
        s[threadIdx.x] = a;
        __syncthreads();
        for (int h = kT / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = s[0];
        __syncthreads();
    }
}

// T(:, c) = S(:, order[c]) for c < m (FP64 complex, column-major)
__global__ __launch_bounds__(kT) void permute_columns_kernel(int rows, int m, const double *S, int lds,
                                                             const int *order, double *T, int ldt) {
    const double2 *Sc = reinterpret_cast<const double2 *>(S);
    double2 *Tc = reinterpret_cast<double2 *>(T);
    for (int t = blockIdx.x * kT + threadIdx.x; t < rows * m; t += gridDim.x * kT) {
        const int r = t % rows, c = t / rows;
        Tc[(int64_t)c * ldt + r] = Sc[(int64_t)order[c] * lds + r];
    }
}

// Precision conversion of a blocked block vector (count complex entries).
__global__ __launch_bounds__(kT) void convert_kernel(const void *src, int prec_src, void *dst,
                                                     int prec_dst, int64_t count) {
    for (int64_t t = blockIdx.x * (int64_t)kT + threadIdx.x; t < count; t += (int64_t)gridDim.x * kT)
        store_c(dst, prec_dst, t, load_c(src, prec_src, t));
}

// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Random-phase columns c in [c_begin, c_end) of a blocked block vector:
// entry (i, c) = exp(2 pi i u), u = top 53 bits of splitmix64(k ^ i) / 2^53,
// k = splitmix64(splitmix64(seed) ^ (col0 + c - c_begin)).
__global__ __launch_bounds__(kT) void random_phase_kernel(void *X, int prec, int64_t n, int nb,
                                                          int c_begin, int c_end, uint64_t seed,
                                                          uint64_t col0, const int32_t *perm) {
    const uint64_t base = splitmix64(seed);
    const int64_t cols = c_end - c_begin;
    for (int64_t t = blockIdx.x * (int64_t)kT + threadIdx.x; t < n * cols;
         t += (int64_t)gridDim.x * kT) {
        const int64_t cc = t / n, i = t % n;
        const uint64_t kj = splitmix64(base ^ (col0 + (uint64_t)cc));
        const uint64_t row = perm ? (uint64_t)perm[i] : (uint64_t)i;  // the row's original index
        const double u = (double)(splitmix64(kj ^ row) >> 11) * 0x1.0p-53;
        double sn, cs;
        sincospi(2.0 * u, &sn, &cs);
        store_c(X, prec, blocked_index(n, nb, i, c_begin + static_cast<int>(cc)), double2{cs, sn});
    }
}

// Per column: index of the largest-modulus entry (ties: smallest row) and the
// unit phase conj(z)/|z| that makes it real positive; then scale the column.
__global__ __launch_bounds__(kT) void phase_argmax_kernel(const void *Z, int prec, int64_t n, int nb,
                                                          int m, double *phase) {
    __shared__ double sv[kT];
    __shared__ int64_t si[kT];
    for (int c = blockIdx.x; c < m; c += gridDim.x) {
        double best = -1.0;
        int64_t bi = 0;
        for (int64_t i = threadIdx.x; i < n; i += kT) {
            const double2 z = load_c(Z, prec, blocked_index(n, nb, i, c));
            const double a = z.x * z.x + z.y * z.y;
            if (a > best) { best = a; bi = i; }
        }
        sv[threadIdx.x] = best;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int h = kT / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                const double o = sv[threadIdx.x + h];
                const int64_t oi = si[threadIdx.x + h];
                if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                    sv[threadIdx.x] = o;
                    si[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double2 z = load_c(Z, prec, blocked_index(n, nb, si[0], c));
            const double a = sqrt(z.x * z.x + z.y * z.y);
            phase[2 * c] = a > 0.0 ? z.x / a : 1.0;
            phase[2 * c + 1] = a > 0.0 ? -z.y / a : 0.0;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kT) void scale_columns_kernel(void *Z, int prec, int64_t n, int nb, int m,
                                                           const double *phase) {
    for (int64_t t = blockIdx.x * (int64_t)kT + threadIdx.x; t < n * m; t += (int64_t)gridDim.x * kT) {
        const int c = static_cast<int>(t / n);
        const int64_t i = t % n;
        const int64_t e = blocked_index(n, nb, i, c);
        const double2 z = load_c(Z, prec, e);
        const double pr = phase[2 * c], pi = phase[2 * c + 1];
        store_c(Z, prec, e, double2{z.x * pr - z.y * pi, z.x * pi + z.y * pr});
    }
}

}  // namespace

static bool pow2(int v) { return v >= 1 && (v & (v - 1)) == 0; }

int launch_gram(const void *A, int prec_a, int nb_a, const void *B, int prec_b, int nb_b, int64_t n,
                int m1, int m2, double *part, int nsplit, double *S, int ld, hipStream_t s) {
    if (!pow2(nb_a) || !pow2(nb_b)) CHEBFD_FAIL(CHEBFD_EINVAL, "block widths %d, %d must be powers of two", nb_a, nb_b);
    const int ta = (m1 + kGT - 1) / kGT, tb = (m2 + kGT - 1) / kGT;
    // A^H A: Hermitian, only the tiles on and above the diagonal
    const int herm = (A == B && prec_a == prec_b && nb_a == nb_b && m1 == m2) ? 1 : 0;
    const int ntiles = herm ? ta * (ta + 1) / 2 : ta * tb;
    const int64_t rps = ((n + nsplit - 1) / nsplit + 2 * kGK - 1) / (2 * kGK) * (2 * kGK);
    const dim3 grid(ntiles, nsplit);
    const bool a64 = prec_a == CHEBFD_PREC_FP64, b64 = prec_b == CHEBFD_PREC_FP64;
    // at most 32 columns of B: 64 x 32 output tiles (the slots and the reduction stay 64 x 64)
    const bool narrow = !herm && m2 <= 32;
#define CHEBFD_GRAM(TA_, TB_)                                                                              \
    do {                                                                                                   \
        if (narrow)                                                                                        \
            hipLaunchKernelGGL((gram_kernel<TA_, TB_, 32>), grid, dim3(kT), 0, s, A, nb_a, B, nb_b, n, m1, \
                               m2, ta, herm, rps, part);                                                   \
        else                                                                                               \
            hipLaunchKernelGGL((gram_kernel<TA_, TB_, 64>), grid, dim3(kT), 0, s, A, nb_a, B, nb_b, n, m1, \
                               m2, ta, herm, rps, part);                                                   \
    } while (0)
    if (a64 && b64)
        CHEBFD_GRAM(double, double);
    else if (a64)
        CHEBFD_GRAM(double, float);
    else if (b64)
        CHEBFD_GRAM(float, double);
    else
        CHEBFD_GRAM(float, float);
#undef CHEBFD_GRAM
    CHEBFD_HIP(hipGetLastError());
    const int64_t total = (int64_t)ntiles * kGT * kGT;
    int G = static_cast<int>((total + kT - 1) / kT);
    if (G > 4096) G = 4096;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(G), dim3(kT), 0, s, part, nsplit, ntiles, ta, herm, m1, m2,
                       S, ld);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

size_t gram_part_bytes(int m1, int m2, int nsplit) {
    const size_t ta = (m1 + kGT - 1) / kGT, tb = (m2 + kGT - 1) / kGT;
    return ta * tb * (size_t)nsplit * kGT * kGT * 16;
}

int launch_update(const void *A, int prec_a, int nb_a, const double *M, int ldm, void *Z, int prec_z,
                  int nb_z, int64_t n, int m1, int m2, hipStream_t s) {
    if (!pow2(nb_a) || !pow2(nb_z)) CHEBFD_FAIL(CHEBFD_EINVAL, "block widths %d, %d must be powers of two", nb_a, nb_z);
    // at most 32 columns of Z: 64 x 32 output tiles
    const int bw = m2 <= 32 ? 32 : kGT;
    const dim3 grid(static_cast<unsigned>((n + kGT - 1) / kGT), (m2 + bw - 1) / bw);
    const bool a64 = prec_a == CHEBFD_PREC_FP64, z64 = prec_z == CHEBFD_PREC_FP64;
#define CHEBFD_UPD(TA_, TZ_)                                                                                     \
    do {                                                                                                         \
        if (bw == 32)                                                                                            \
            hipLaunchKernelGGL((update_kernel<TA_, TZ_, 32>), grid, dim3(kT), 0, s, A, nb_a, M, ldm, Z, nb_z, n, \
                               m1, m2);                                                                          \
        else                                                                                                     \
            hipLaunchKernelGGL((update_kernel<TA_, TZ_, 64>), grid, dim3(kT), 0, s, A, nb_a, M, ldm, Z, nb_z, n, \
                               m1, m2);                                                                          \
    } while (0)
    if (a64 && z64)
        CHEBFD_UPD(double, double);
    else if (a64)
        CHEBFD_UPD(double, float);
    else if (z64)
        CHEBFD_UPD(float, double);
    else
        CHEBFD_UPD(float, float);
#undef CHEBFD_UPD
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int launch_update_sub(const void *A, int prec_a, int nb_a, const double *M, int ldm, const void *S, int prec_s,
                      int nb_s, double *Z, int nb_z, int64_t n, int m1, int m2, hipStream_t s) {
    if (!pow2(nb_a) || !pow2(nb_z) || !pow2(nb_s))
        CHEBFD_FAIL(CHEBFD_EINVAL, "block widths %d, %d, %d must be powers of two", nb_a, nb_s, nb_z);
    if (m2 > 32) CHEBFD_FAIL(CHEBFD_EINVAL, "Z = S - A M takes at most 32 columns (%d)", m2);
    const dim3 grid(static_cast<unsigned>((n + kGT - 1) / kGT), 1);
    const bool a64 = prec_a == CHEBFD_PREC_FP64, s64 = prec_s == CHEBFD_PREC_FP64;
#define CHEBFD_UPDS(TA_, TS_)                                                                                  \
    hipLaunchKernelGGL((update_kernel<TA_, double, 32, TS_>), grid, dim3(kT), 0, s, A, nb_a, M, ldm,          \
                       static_cast<void *>(Z), nb_z, n, m1, m2, S, nb_s)
    if (a64 && s64)
        CHEBFD_UPDS(double, double);
    else if (a64)
        CHEBFD_UPDS(double, float);
    else if (s64)
        CHEBFD_UPDS(float, double);
    else
        CHEBFD_UPDS(float, float);
#undef CHEBFD_UPDS
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

size_t jacobi_scratch_bytes(int m) {
    (void)m;
    // params [2][kMaxM/2] x (2 ints + 3 doubles), norm partials, sort scratch (2 kMaxM doubles)
    return round_up(2 * (kMaxM / 2) * (2 * sizeof(int) + 3 * sizeof(double)), 256) +
           round_up(kJNormG * sizeof(double), 256) + round_up(2 * kMaxM * sizeof(double), 256);
}

int launch_jacobi(int m, double *A, int lda, double *V, int ldv, double *w, int max_sweeps, double tol,
                  void *scratch, int *sweeps, int *converged, hipStream_t s) {
    if (m < 1 || m > kMaxM) CHEBFD_FAIL(CHEBFD_EINVAL, "eigensolver size %d not in [1, %d]", m, kMaxM);
    char *base = static_cast<char *>(scratch);
    const int H2 = 2 * (kMaxM / 2);
    JacobiRound jr;
    jr.p = reinterpret_cast<int *>(base);
    jr.q = jr.p + H2;
    jr.c = reinterpret_cast<double *>(base + round_up(2 * H2 * sizeof(int), 16));
    jr.sr = jr.c + H2;
    jr.si = jr.sr + H2;
    double *part = reinterpret_cast<double *>(base + round_up(2 * (kMaxM / 2) * (2 * sizeof(int) + 3 * sizeof(double)), 256));
    double *sortw = part + round_up(kJNormG * sizeof(double), 256) / sizeof(double);
    const int me = m + (m & 1), half = me / 2;
    const int G = std::min(kJNormG, std::max(1, (m * m + kJW - 1) / kJW));
    double hp[kJNormG];
    auto norm2 = [&](int off, double *out) -> int {
        hipLaunchKernelGGL(jacobi_norm_kernel, dim3(G), dim3(kJW), 0, s, m, A, lda, off, part);
        CHEBFD_HIP(hipGetLastError());
        CHEBFD_HIP(hipMemcpyAsync(hp, part, sizeof(double) * G, hipMemcpyDeviceToHost, s));
        CHEBFD_HIP(hipStreamSynchronize(s));
        double acc = 0.0;
        for (int g = 0; g < G; ++g) acc += hp[g];
        *out = acc;
        return CHEBFD_OK;
    };
    int rc;
    hipLaunchKernelGGL(jacobi_init_kernel, dim3(std::min(1024, (m * m + kJW - 1) / kJW)), dim3(kJW), 0, s, m, V,
                       ldv);
    CHEBFD_HIP(hipGetLastError());
    double fro2 = 0.0, off2 = 0.0;
    if ((rc = norm2(0, &fro2))) return rc;
    if ((rc = norm2(1, &off2))) return rc;
    *converged = off2 <= tol * tol * fro2 ? 1 : 0;
    int sweep = 0;
    for (; sweep < max_sweeps && !*converged; ++sweep) {
        for (int r = 0; r < me - 1; ++r) {
            hipLaunchKernelGGL(jacobi_round_kernel, dim3(half), dim3(kJW), 0, s, m, me, r, r > 0 ? 1 : 0, A, lda, V,
                               ldv, jr);
            CHEBFD_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(jacobi_rows_kernel, dim3(std::min(m, 256)), dim3(kJW), 0, s, m, me, (me - 2) & 1, A, lda,
                           jr);
        CHEBFD_HIP(hipGetLastError());
        if ((rc = norm2(1, &off2))) return rc;
        *converged = off2 <= tol * tol * fro2 ? 1 : 0;
    }
    *sweeps = sweep;
    hipLaunchKernelGGL(jacobi_sort_kernel, dim3(1), dim3(kJW), 0, s, m, A, lda, V, ldv, w, sortw);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

static int grid_cap(int64_t work, int cap = 8192) {
    int64_t g = (work + kT - 1) / kT;
    if (g > cap) g = cap;
    return static_cast<int>(g < 1 ? 1 : g);
}

int launch_svqb_scale(int m, double *S, int ld, double *d, hipStream_t s) {
    if (m > kMaxM) CHEBFD_FAIL(CHEBFD_EINVAL, "SVQB size %d > %d", m, kMaxM);
    hipLaunchKernelGGL(svqb_scale_kernel, dim3(1), dim3(kT), 0, s, m, S, ld, d);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int launch_svqb_transform(int m, int k, int first, const double *d, const double *V, int ldv,
                          const double *w, double *T, int ldt, hipStream_t s) {
    hipLaunchKernelGGL(svqb_transform_kernel, dim3(grid_cap((int64_t)m * k)), dim3(kT), 0, s, m, k,
                       first, d, V, ldv, w, T, ldt);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int launch_hermitise(int m, double *G, int ld, hipStream_t s) {
    hipLaunchKernelGGL(hermitise_kernel, dim3(grid_cap((int64_t)m * m)), dim3(kT), 0, s, m, G, ld);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int resid_grid(int64_t n) { return grid_cap(n, 1024); }

int launch_resid(const void *HZ, const void *Z, int prec, int64_t n, int nb, const double *theta,
                 double *part, int G, double *out, hipStream_t s) {
    hipLaunchKernelGGL(resid_partial_kernel, dim3(G), dim3(kT), 0, s, HZ, Z, prec, n, nb, theta, part);
    CHEBFD_HIP(hipGetLastError());
    hipLaunchKernelGGL(colsum_reduce_kernel, dim3(2 * nb), dim3(kT), 0, s, part, G, 2 * nb, out);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int launch_permute_columns(int rows, int m, const double *S, int lds, const int *order, double *T,
                           int ldt, hipStream_t s) {
    hipLaunchKernelGGL(permute_columns_kernel, dim3(grid_cap((int64_t)rows * m)), dim3(kT), 0, s, rows, m, S,
                       lds, order, T, ldt);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int launch_convert(const void *src, int prec_src, void *dst, int prec_dst, int64_t count,
                   hipStream_t s) {
    hipLaunchKernelGGL(convert_kernel, dim3(grid_cap(count, 65536)), dim3(kT), 0, s, src, prec_src, dst,
                       prec_dst, count);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int launch_random_phase(void *X, int prec, int64_t n, int nb, int c_begin, int c_end, uint64_t seed,
                        uint64_t col0, const int32_t *perm, hipStream_t s) {
    if (c_end <= c_begin) return CHEBFD_OK;
    if (!pow2(nb)) CHEBFD_FAIL(CHEBFD_EINVAL, "block width %d must be a power of two", nb);
    hipLaunchKernelGGL(random_phase_kernel, dim3(grid_cap(n * (c_end - c_begin), 65536)), dim3(kT), 0, s,
                       X, prec, n, nb, c_begin, c_end, seed, col0, perm);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

int launch_fix_phases(void *Z, int prec, int64_t n, int nb, int m, double *phase, hipStream_t s) {
    if (!pow2(nb)) CHEBFD_FAIL(CHEBFD_EINVAL, "block width %d must be a power of two", nb);
    hipLaunchKernelGGL(phase_argmax_kernel, dim3(m < 1024 ? m : 1024), dim3(kT), 0, s, Z, prec, n, nb, m,
                       phase);
    CHEBFD_HIP(hipGetLastError());
    hipLaunchKernelGGL(scale_columns_kernel, dim3(grid_cap(n * m, 65536)), dim3(kT), 0, s, Z, prec, n, nb,
                       m, phase);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

}  // namespace chebfd
