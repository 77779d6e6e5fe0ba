// Tall-skinny QR (TSQR) of a blocked block vector: the alternative to SVQB in
// the orthogonalisation before the restart (Sect. 2 names both; TSQR is the
// communication-avoiding QR of Demmel, Grigori, Hoemmen and Langou).
//
// Y (n x m, blocked layout of width nb, c128 or c64) = Q R with Q written to a
// second block vector and R (m x m, FP64 complex, column-major) upper
// triangular with a real non-negative diagonal, the unique such factorisation
// when Y has full column rank.  The columns are taken in panels of
// PW = min(nb, 32):
//   * panel p is projected against the finished panels twice (block classical
//     Gram-Schmidt with one reorthogonalisation) with the FP64 MFMA Gram and
//     update kernels; the projected panel T is FP64 whatever the storage;
//   * T is factorised by a reduction tree of Householder QRs.  A tree node
//     factorises kNode = 256 stacked rows in one workgroup: the half-wave that
//     owns column j holds rows l, l + 32, ..., l + 224 of it in lane l's
//     registers; per Householder step the owner of the pivot column puts its
//     reflector in LDS and the other columns form their products with it by a
//     32-lane sum (DPP within rows of 16 lanes, one permute across; one barrier
//     per step); the node's explicit Q is then formed in place from its
//     reflectors.  The leaves are the 256-row
//     ranges of T; a node of the next level stacks the R factors of 256 / PW
//     children.  The root's R is the panel's diagonal block of R after a phase
//     per column makes its diagonal real positive (the phase goes into Q);
//   * the explicit Q of the panel is the product down the tree: each node's Q
//     times the PW x PW block of its parent's product that belongs to it,
//     staged through LDS so that the product can overwrite the node's Q.
// Reflector of a column x (rows k..): u = x - beta e_k with
// beta = -(x_k / |x_k|) ||x||, H = I - u u^H / (||x|| (||x|| + |x_k|)), H x = beta e_k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace chebfd {

namespace {

constexpr int kNode = 256;      // rows per tree node
constexpr int kRpl = kNode / 32;  // rows per lane
constexpr int kEw = 256;        // threads of the elementwise kernels

constexpr int node_threads(int pw) { return ((pw + 1) / 2) * 64; }
constexpr int apply_cg(int pw) { return pw < 8 ? pw : 8; }  // output columns per thread
constexpr int apply_threads(int pw) { return kNode * (pw / apply_cg(pw)); }
constexpr size_t apply_lds_bytes(int pw) { return (size_t)(kNode * (pw + 1) + pw * pw) * 16; }

__device__ inline double2 ld_c(const void *base, int prec, int64_t idx) {
    if (prec == CHEBFD_PREC_FP64) return static_cast<const double2 *>(base)[idx];
    const float2 f = static_cast<const float2 *>(base)[idx];
    return double2{(double)f.x, (double)f.y};
}

__device__ inline void st_c(void *base, int prec, int64_t idx, double2 v) {
    if (prec == CHEBFD_PREC_FP64) {
        static_cast<double2 *>(base)[idx] = v;
    } else {
        static_cast<float2 *>(base)[idx] = float2{(float)v.x, (float)v.y};
    }
}

// lane permutation within rows of 16 lanes by DPP (no LDS round trip)
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// sum over the 32 lanes of a half-wave; every lane gets the same value (each
// stage adds a lane's value and its partner's, and a + b == b + a exactly).
// Partners: xor 1 and xor 2 within a quad, then lane i and 7 - i within eight
// lanes, then i and 15 - i within sixteen (DPP), then xor 16 (a permute).
__device__ inline double sum32(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    v += __shfl_xor(v, 16, 32);
    return v;
}

__device__ inline double2 cmul(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline double2 cjmul(double2 a, double2 b) {  // conj(a) b
    return double2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__device__ inline double2 unit_phase(double2 z) {
    const double a = hypot(z.x, z.y);
    return a > 0.0 ? double2{z.x / a, z.y / a} : double2{1.0, 0.0};
}

// Householder QR of the 256-row node blockIdx.x of `in` (rows >= `rows` read
// as zero; columns >= cols not touched).  Writes the node's explicit Q (rows <
// rows) to q (FP64, row i at q + i PW; q may equal in) and its R either to
// rnext (rows [PW node, PW node + PW), PW wide, zeros below the diagonal) or,
// at the root, phase-normalised to rroot (cols x cols, column-major, ldr).
template <int PW>
__global__ __launch_bounds__(node_threads(PW)) void tsqr_node_kernel(const void *in, int prec, int64_t ld,
                                                                     int64_t rows, int cols, double2 *q,
                                                                     double2 *rnext, int root, double2 *rroot,
                                                                     int ldr) {
    __shared__ double2 ub[2][kNode];
    __shared__ double cs[PW];
    __shared__ double2 rd[PW];
    const int lane = threadIdx.x & 63;
    const int l32 = lane & 31;
    const int j = 2 * (threadIdx.x >> 6) + (lane >> 5);
    const bool own = j < cols;
    const int64_t r0 = (int64_t)blockIdx.x * kNode;

    double2 a[kRpl];
#pragma unroll
    for (int s = 0; s < kRpl; ++s) {
        const int64_t g = r0 + l32 + 32 * s;
        a[s] = (own && g < rows) ? ld_c(in, prec, g * ld + j) : double2{0.0, 0.0};
    }

    // --- factorisation: reflector k annihilates column k below row k ---
    for (int k = 0; k < cols; ++k) {
        const int b = k & 1;
        if (j == k) {
            double s2 = 0.0;
            double2 al{0.0, 0.0};
#pragma unroll
            for (int s = 0; s < kRpl; ++s) {
                const int i = l32 + 32 * s;
                if (i > k) s2 += a[s].x * a[s].x + a[s].y * a[s].y;
                if (i == k) al = a[s];
            }
            s2 = sum32(s2);
            al.x = sum32(al.x);
            al.y = sum32(al.y);
            const double aa = hypot(al.x, al.y);
            const double xn = sqrt(aa * aa + s2);
            const double2 ph = unit_phase(al);
            const double c = xn > 0.0 ? 1.0 / (xn * (xn + aa)) : 0.0;
#pragma unroll
            for (int s = 0; s < kRpl; ++s) {
                const int i = l32 + 32 * s;
                double2 u{0.0, 0.0};
                if (i > k) u = a[s];
                if (i == k) u = double2{ph.x * (aa + xn), ph.y * (aa + xn)};
                ub[b][i] = u;
                if (i >= k) a[s] = u;   // rows < k keep R(i, k)
            }
            if (l32 == 0) {
                cs[k] = c;
                rd[k] = double2{-ph.x * xn, -ph.y * xn};
            }
        }
        __syncthreads();
        if (own && j > k) {
            const double c = cs[k];
            double2 u[kRpl];
            double wr = 0.0, wi = 0.0;
#pragma unroll
            for (int s = 0; s < kRpl; ++s) {
                u[s] = ub[b][l32 + 32 * s];
                const double2 t = cjmul(u[s], a[s]);
                wr += t.x;
                wi += t.y;
            }
            const double2 cw{c * sum32(wr), c * sum32(wi)};
#pragma unroll
            for (int s = 0; s < kRpl; ++s) {
                const double2 t = cmul(u[s], cw);
                a[s].x -= t.x;
                a[s].y -= t.y;
            }
        }
    }

    // --- R: column j, rows 0..PW-1 in lanes 0..PW-1 (register slot 0) ---
    if (own && l32 < PW) {
        const int i = l32;
        double2 v{0.0, 0.0};
        if (i < j) v = a[0];
        if (i == j) v = rd[j];
        if (root) {
            // conj(d_i) times row i; on the diagonal that is |beta_j|, real by construction
            if (i == j) v = double2{hypot(rd[j].x, rd[j].y), 0.0};
            else v = cjmul(unit_phase(rd[i]), v);
            if (i < cols) rroot[(int64_t)j * ldr + i] = v;
        } else {
            rnext[((int64_t)blockIdx.x * PW + i) * PW + j] = v;
        }
    }
    __syncthreads();   // the last reflector's buffer is reused below

    // --- explicit Q = H_0 ... H_{cols-1} [I; 0], formed in place from the last reflector back ---
    for (int k = cols - 1; k >= 0; --k) {
        const int b = k & 1;
        if (j == k) {
#pragma unroll
            for (int s = 0; s < kRpl; ++s) {
                const int i = l32 + 32 * s;
                ub[b][i] = i >= k ? a[s] : double2{0.0, 0.0};
            }
        }
        __syncthreads();
        const double c = cs[k];
        if (own && j > k) {
            double2 u[kRpl];
            double wr = 0.0, wi = 0.0;
#pragma unroll
            for (int s = 0; s < kRpl; ++s) {
                u[s] = ub[b][l32 + 32 * s];
                const double2 t = cjmul(u[s], a[s]);
                wr += t.x;
                wi += t.y;
            }
            const double2 cw{c * sum32(wr), c * sum32(wi)};
#pragma unroll
            for (int s = 0; s < kRpl; ++s) {
                const double2 t = cmul(u[s], cw);
                a[s].x -= t.x;
                a[s].y -= t.y;
            }
        } else if (j == k) {
            // H_k e_k = e_k - c u conj(u_k)
            const double2 ukk = ub[b][k];
            const double2 f{c * ukk.x, -c * ukk.y};
#pragma unroll
            for (int s = 0; s < kRpl; ++s) {
                const int i = l32 + 32 * s;
                double2 v{0.0, 0.0};
                if (i >= k) {
                    const double2 t = cmul(a[s], f);
                    v = double2{(i == k ? 1.0 : 0.0) - t.x, -t.y};
                }
                a[s] = v;
            }
        }
    }
    if (root && own) {
        const double2 d = unit_phase(rd[j]);
#pragma unroll
        for (int s = 0; s < kRpl; ++s) a[s] = cmul(a[s], d);
    }
#pragma unroll
    for (int s = 0; s < kRpl; ++s) {
        const int64_t g = r0 + l32 + 32 * s;
        if (own && g < rows) q[g * PW + j] = a[s];
    }
}

// out(rows of node blockIdx.x) = q(rows of the node) M_node, M_node = rows
// [PW node, PW node + PW) of m (PW wide), or the identity when m is null.
// The node's rows of q and M_node are staged in LDS first, so out may be q.
template <int PW>
__global__ __launch_bounds__(apply_threads(PW)) void tsqr_apply_kernel(const double2 *q, int64_t rows, int cols,
                                                                       const double2 *m, void *out, int prec,
                                                                       int64_t ld) {
    extern __shared__ double2 lds[];
    constexpr int CG = apply_cg(PW), NG = PW / CG, NT = apply_threads(PW), SQ = PW + 1;
    double2 *sq = lds;                 // [kNode][PW + 1]
    double2 *sm = lds + kNode * SQ;    // [PW][PW]
    const int64_t r0 = (int64_t)blockIdx.x * kNode;
    for (int t = threadIdx.x; t < kNode * PW; t += NT) {
        const int rr = t / PW, cc = t % PW;
        const int64_t g = r0 + rr;
        sq[rr * SQ + cc] = (g < rows && cc < cols) ? q[g * PW + cc] : double2{0.0, 0.0};
    }
    for (int t = threadIdx.x; t < PW * PW; t += NT) {
        const int kk = t / PW, cc = t % PW;
        double2 v{0.0, 0.0};
        if (kk < cols && cc < cols) {
            if (m)
                v = m[((int64_t)blockIdx.x * PW + kk) * PW + cc];
            else
                v = double2{kk == cc ? 1.0 : 0.0, 0.0};
        }
        sm[kk * PW + cc] = v;
    }
    __syncthreads();
    const int r = threadIdx.x / NG, c0 = (threadIdx.x % NG) * CG;
    double2 acc[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) acc[c] = double2{0.0, 0.0};
    for (int k = 0; k < cols; ++k) {
        const double2 x = sq[r * SQ + k];
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            const double2 y = sm[k * PW + c0 + c];
            acc[c].x += x.x * y.x - x.y * y.y;
            acc[c].y += x.x * y.y + x.y * y.x;
        }
    }
    const int64_t g = r0 + r;
    if (g < rows) {
#pragma unroll
        for (int c = 0; c < CG; ++c)
            if (c0 + c < cols) st_c(out, prec, g * ld + c0 + c, acc[c]);
    }
}

// Off-diagonal blocks of the panel's columns c0 .. c0 + cols - 1 of R:
// rows < c0 get C1 + C2 (the two projections; absent for the first panel),
// rows >= c0 + cols get zero.
__global__ __launch_bounds__(kEw) void tsqr_rblock_kernel(double2 *R, int ldr, int m, int c0, int cols,
                                                          const double2 *C1, const double2 *C2, int ldc) {
    const int total = m * cols;
    for (int t = blockIdx.x * kEw + threadIdx.x; t < total; t += gridDim.x * kEw) {
        const int c = t / m, i = t % m;
        if (i >= c0 && i < c0 + cols) continue;
        double2 v{0.0, 0.0};
        if (i < c0) {
            const double2 x = C1[(int64_t)c * ldc + i], y = C2[(int64_t)c * ldc + i];
            v = double2{x.x + y.x, x.y + y.y};
        }
        R[(int64_t)(c0 + c) * ldr + i] = v;
    }
}

// info[2k] = |R_kk|^2, info[2k + 1] = sum_{i <= k} |R_ik|^2 (the squared norm of column k of Y)
__global__ __launch_bounds__(kEw) void tsqr_colinfo_kernel(int m, const double2 *R, int ldr, double *info) {
    const int k = blockIdx.x * kEw + threadIdx.x;
    if (k >= m) return;
    double s = 0.0, d = 0.0;
    for (int i = 0; i <= k; ++i) {
        const double2 v = R[(int64_t)k * ldr + i];
        const double a2 = v.x * v.x + v.y * v.y;
        s += a2;
        if (i == k) d = a2;
    }
    info[2 * k] = d;
    info[2 * k + 1] = s;
}

int ew_grid(int64_t work) {
    int64_t g = (work + kEw - 1) / kEw;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, 8192)));
}

// row counts of the tree levels: level 0 has n rows, level l + 1 stacks PW rows per node of level l
std::vector<int64_t> tree_rows(int64_t n, int pw) {
    std::vector<int64_t> r{n};
    int64_t nodes = (n + kNode - 1) / kNode;
    while (nodes > 1) {
        r.push_back(nodes * pw);
        nodes = (nodes * pw + kNode - 1) / kNode;
    }
    return r;
}

// the LDS size above the default is a per-device attribute of the kernel: set
// it on every use (the current device may change between calls)
template <int PW>
bool set_apply_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(tsqr_apply_kernel<PW>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(apply_lds_bytes(PW))) == hipSuccess;
}

// QR of one panel: src (rows n, cols <= PW, element (i, c) at src[i ld + c])
// -> Q into dst (same addressing with ld_dst), R block into R (column-major, ldr)
template <int PW>
int tsqr_panel_t(int64_t n, int cols, const void *src, int prec_src, int64_t ld_src, double2 *T, double2 *tree,
                 void *dst, int prec_dst, int64_t ld_dst, double2 *R, int ldr, hipStream_t s) {
    if (!set_apply_attr<PW>()) CHEBFD_FAIL(CHEBFD_EHIP, "TSQR: cannot set the LDS size of the apply kernel");
    const std::vector<int64_t> rows = tree_rows(n, PW);
    const int L = static_cast<int>(rows.size()) - 1;
    std::vector<double2 *> arr{T};
    size_t off = 0;
    for (int l = 1; l <= L; ++l) {
        arr.push_back(reinterpret_cast<double2 *>(reinterpret_cast<char *>(tree) + off));
        off += round_up((size_t)rows[l] * PW * 16, 256);
    }
    for (int l = 0; l <= L; ++l) {
        const unsigned nodes = static_cast<unsigned>((rows[l] + kNode - 1) / kNode);
        const void *in = l == 0 ? src : arr[l];
        hipLaunchKernelGGL(tsqr_node_kernel<PW>, dim3(nodes), dim3(node_threads(PW)), 0, s, in,
                           l == 0 ? prec_src : (int)CHEBFD_PREC_FP64, l == 0 ? ld_src : (int64_t)PW, rows[l], cols,
                           arr[l], l < L ? arr[l + 1] : nullptr, l == L ? 1 : 0, R, ldr);
        CHEBFD_HIP(hipGetLastError());
    }
    for (int l = L > 0 ? L - 1 : 0; l >= 0; --l) {
        const unsigned nodes = static_cast<unsigned>((rows[l] + kNode - 1) / kNode);
        void *out = l == 0 ? dst : static_cast<void *>(arr[l]);
        hipLaunchKernelGGL(tsqr_apply_kernel<PW>, dim3(nodes), dim3(apply_threads(PW)), apply_lds_bytes(PW), s,
                           arr[l], rows[l], cols, L > 0 ? arr[l + 1] : nullptr, out,
                           l == 0 ? prec_dst : (int)CHEBFD_PREC_FP64, l == 0 ? ld_dst : (int64_t)PW);
        CHEBFD_HIP(hipGetLastError());
    }
    return CHEBFD_OK;
}

int tsqr_panel(int pw, int64_t n, int cols, const void *src, int prec_src, int64_t ld_src, double2 *T,
               double2 *tree, void *dst, int prec_dst, int64_t ld_dst, double2 *R, int ldr, hipStream_t s) {
    switch (pw) {
    case 1: return tsqr_panel_t<1>(n, cols, src, prec_src, ld_src, T, tree, dst, prec_dst, ld_dst, R, ldr, s);
    case 2: return tsqr_panel_t<2>(n, cols, src, prec_src, ld_src, T, tree, dst, prec_dst, ld_dst, R, ldr, s);
    case 4: return tsqr_panel_t<4>(n, cols, src, prec_src, ld_src, T, tree, dst, prec_dst, ld_dst, R, ldr, s);
    case 8: return tsqr_panel_t<8>(n, cols, src, prec_src, ld_src, T, tree, dst, prec_dst, ld_dst, R, ldr, s);
    case 16: return tsqr_panel_t<16>(n, cols, src, prec_src, ld_src, T, tree, dst, prec_dst, ld_dst, R, ldr, s);
    case 32: return tsqr_panel_t<32>(n, cols, src, prec_src, ld_src, T, tree, dst, prec_dst, ld_dst, R, ldr, s);
    default: CHEBFD_FAIL(CHEBFD_EINVAL, "TSQR panel width %d not in {1, 2, 4, 8, 16, 32}", pw);
    }
}

}  // namespace

int tsqr_panel_width(int nb) { return std::min(nb, 32); }

size_t tsqr_tree_bytes(int64_t n, int pw) {
    const std::vector<int64_t> rows = tree_rows(n, pw);
    size_t total = 0;
    for (size_t l = 1; l < rows.size(); ++l) total += round_up((size_t)rows[l] * pw * 16, 256);
    return total;
}

size_t tsqr_gpart_bytes(int64_t n, int m, int nb) {
    const int pw = tsqr_panel_width(nb);
    size_t b = 0;
    for (int c0 = pw; c0 < m; c0 += pw) {
        const int cols = std::min(pw, m - c0);
        b = std::max(b, gram_part_bytes(c0, cols, gram_splits(n, c0, cols)));
    }
    return b;
}

int tsqr_blocked(int64_t n, int m, int nb, int prec_y, const void *Y, int prec_q, void *Q, double *R, int ldr,
                 const TsqrWork &w, hipStream_t s) {
    const int pw = tsqr_panel_width(nb);
    const size_t ey = vec_elem_bytes(prec_y), eq = vec_elem_bytes(prec_q);
    double2 *T = reinterpret_cast<double2 *>(w.T);
    double2 *R2 = reinterpret_cast<double2 *>(R);
    int r;
    for (int c0 = 0; c0 < m; c0 += pw) {
        const int cols = std::min(pw, m - c0);
        const size_t eoff = ((size_t)(c0 / nb) * n) * nb + c0 % nb;   // element (0, c0) of the blocked layout
        const void *ysrc = static_cast<const char *>(Y) + eoff * ey;
        void *qdst = static_cast<char *>(Q) + eoff * eq;
        const void *src = ysrc;
        int prec_src = prec_y;
        int64_t ld_src = nb;
        if (c0 > 0) {
            // two rounds of projection against the finished panels, accumulated in FP64
            const int splits = gram_splits(n, c0, cols);
            if ((r = launch_gram(Q, prec_q, nb, ysrc, prec_y, nb, n, c0, cols, w.gpart, splits, w.C1, w.ldc, s)))
                return r;
            // T = Y - Q C1, then T = T - Q C2 (the subtraction in the update's epilogue)
            if ((r = launch_update_sub(Q, prec_q, nb, w.C1, w.ldc, ysrc, prec_y, nb, reinterpret_cast<double *>(T), pw,
                                       n, c0, cols, s)))
                return r;
            if ((r = launch_gram(Q, prec_q, nb, T, CHEBFD_PREC_FP64, pw, n, c0, cols, w.gpart, splits, w.C2, w.ldc,
                                 s)))
                return r;
            if ((r = launch_update_sub(Q, prec_q, nb, w.C2, w.ldc, T, CHEBFD_PREC_FP64, pw,
                                       reinterpret_cast<double *>(T), pw, n, c0, cols, s)))
                return r;
            src = T;
            prec_src = CHEBFD_PREC_FP64;
            ld_src = pw;
        }
        if ((r = tsqr_panel(pw, n, cols, src, prec_src, ld_src, T, reinterpret_cast<double2 *>(w.tree), qdst, prec_q,
                            nb, R2 + (size_t)c0 * ldr + c0, ldr, s)))
            return r;
        hipLaunchKernelGGL(tsqr_rblock_kernel, dim3(ew_grid((int64_t)m * cols)), dim3(kEw), 0, s, R2, ldr, m, c0,
                           cols, reinterpret_cast<const double2 *>(w.C1), reinterpret_cast<const double2 *>(w.C2),
                           w.ldc);
        CHEBFD_HIP(hipGetLastError());
    }
    return CHEBFD_OK;
}

int launch_tsqr_colinfo(int m, const double *R, int ldr, double *info, hipStream_t s) {
    hipLaunchKernelGGL(tsqr_colinfo_kernel, dim3((m + kEw - 1) / kEw), dim3(kEw), 0, s, m,
                       reinterpret_cast<const double2 *>(R), ldr, info);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

}  // namespace chebfd
