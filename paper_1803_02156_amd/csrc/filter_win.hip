// Fused Chebyshev step with the gathered block staged in LDS (gfx950).
//
// Same computation as the other step kernels (the recurrence step of Alg. 1 of
// the ChebFD paper, and its two start launches): per row i and block column j,
// W_ij <- 2 ((aH + bI) U)_ij - W_ij, the filtered-block update and the
// per-column dot products.
//
// The sparse product gathers whole row segments of U (NB complex numbers) at
// the matrix's column indices.  After a locality-preserving row order most of
// those columns lie close to the row, so one workgroup per CU sweeps a
// contiguous range of tiles and keeps a window of U in LDS: a ring of
// kWinBlocks blocks of TR rows (TR = rows of one tile, 16 KB per block).
// While tile t (rows [t TR, t TR + TR)) is processed the ring holds blocks
// t - h .. t + h (h = win_halo(TR): 3 tiles of 32 rows, 1 tile of 64) and
// receives block t + h + 1, which is loaded from HBM once (coalesced, one
// 16-byte access per thread) and read by the next 2 h + 1 tiles.  Gathers
// inside the window are LDS reads;
// columns outside it are gathered from global memory as before.  The vector
// memory pipeline then carries about one U access per row instead of one per
// stored entry, plus the streams of W and Y (non-temporal) and the matrix
// slots (staged in LDS per tile, double buffered).
//
// Lanes: TR = 1024 * CPL / NB rows per tile; lane t works on columns
// [CPL (t % LPR), CPL (t % LPR) + CPL) of row t / LPR of the tile.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "step_io.h"

namespace chebfd {
namespace {

using namespace step_io;

constexpr int kWinThreads = 1024;
constexpr int kXcdCount = 8;
constexpr int kWinLdsLimit = 160 * 1024;
// Lead control (see the kernel): every kWinCheckEvery tiles the first wave of a
// workgroup publishes its progress and reads that of the other workgroups of its
// XCD; more than kWinMaxLead tiles ahead of the slowest, it waits for it,
// polling at most kWinMaxPolls times.
constexpr int kWinCheckEvery = 32;
constexpr int kWinMaxLead = 4;
constexpr int kWinMaxPolls = 200;

template <typename T, int NB>
struct WinShape {
    static constexpr int CPL = cols_per_lane<T, NB>();
    static constexpr int LPR = NB / CPL;               // lanes per row
    static constexpr int TR = kWinThreads / LPR;       // rows per tile (one per lane group)
    static constexpr int RB = NB * 2 * sizeof(T);      // bytes of one row of U
    static constexpr int RING_ROWS = kWinBlocks * TR;  // power of two
    static constexpr int HALO = win_halo(TR);          // window: tiles t - HALO .. t + HALO
    static_assert(2 * HALO + 2 <= kWinBlocks, "the window and the incoming block fit the ring");
    static constexpr int CPT = TR / 32;                // SELL chunks (C = 32) per tile
};

template <typename T, int MAXW, int TR>
struct WinMatBuf {
    using VT = typename V2<T>::type;
    static constexpr int SLOTS = TR * MAXW;
    static constexpr int CPT = TR / 32;
    static constexpr int O_VALS = 0;
    static constexpr int O_COLS = O_VALS + SLOTS * static_cast<int>(sizeof(VT));
    static constexpr int O_COFF = O_COLS + 4 * SLOTS;
    static constexpr int O_CW = O_COFF + 4 * (CPT + 1);
    static constexpr int BYTES = (O_CW + 4 * CPT + 15) & ~15;
};

template <typename T, int NB, int MAXW>
constexpr int win_lds_bytes() {
    using S = WinShape<T, NB>;
    return S::RING_ROWS * S::RB + 2 * WinMatBuf<T, MAXW, S::TR>::BYTES;
}

template <typename T, int NB>
constexpr bool win_supported() {
    using S = WinShape<T, NB>;
    return S::TR >= 32 && S::TR % 32 == 0 && S::TR * kWinWidth <= kWinThreads &&
           win_lds_bytes<T, NB, kWinWidth>() <= kWinLdsLimit;
}

// partials of the previous launch (3 NB columns of G_prev values), fixed order
template <int NB>
__device__ void win_reduce_prev(const StepArgs &a, double *sred) {
    const int tid = threadIdx.x;
    for (int q = blockIdx.x; q < 3 * NB; q += gridDim.x) {
        const double *src = a.part_in + (int64_t)q * a.G_prev;
        double s = 0.0;
        for (int g = tid; g < a.G_prev; g += kWinThreads) s += src[g];
        sred[tid] = s;
        __syncthreads();
        for (int hh = kWinThreads / 2; hh > 0; hh >>= 1) {
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

// LDS layout (dynamic): ring[RING_ROWS][RB] | 2 x { vals[SLOTS], cols[SLOTS], coff[CPT + 1], cw[CPT] }.
// The ring area also serves the reductions before the first and after the last tile.
template <typename T, int NB, int MODE, int MAXW, bool UNI>
__global__ __launch_bounds__(kWinThreads) void cheb_win_kernel(StepArgs a, int64_t ntiles) {
    using S = WinShape<T, NB>;
    using MB = WinMatBuf<T, MAXW, S::TR>;
    using VT = typename V2<T>::type;
    using PK = Pack<T, S::CPL>;
    constexpr int CPL = S::CPL, LPR = S::LPR, TR = S::TR, RB = S::RB;
    constexpr int CPT = S::CPT;
    constexpr int HALO = S::HALO;
    constexpr int O_MAT = S::RING_ROWS * RB;
    static_assert(win_supported<T, NB>(), "tile shape does not fit the window kernel");
    static_assert(MB::SLOTS <= kWinThreads, "one matrix slot per thread and tile");

    extern __shared__ __align__(16) unsigned char smem[];
    double *sred = reinterpret_cast<double *>(smem);
#define CHEBFD_WV(b) reinterpret_cast<VT *>(smem + O_MAT + (b) * MB::BYTES + MB::O_VALS)
#define CHEBFD_WC(b) reinterpret_cast<int32_t *>(smem + O_MAT + (b) * MB::BYTES + MB::O_COLS)
#define CHEBFD_WCOFF(b) reinterpret_cast<int32_t *>(smem + O_MAT + (b) * MB::BYTES + MB::O_COFF)
#define CHEBFD_WCW(b) reinterpret_cast<int32_t *>(smem + O_MAT + (b) * MB::BYTES + MB::O_CW)
    // byte offset of row q of U inside the ring, plus this lane's columns
#define CHEBFD_RING(q) reinterpret_cast<const T *>(smem + ((q) & (S::RING_ROWS - 1)) * RB + lane_off)

    const int tid = threadIdx.x;
    const int jc = (tid % LPR) * CPL;          // first column of this lane
    const int rr = tid / LPR;                  // row within the tile
    const int lane_off = jc * 2 * static_cast<int>(sizeof(T));

    if (a.part_in != nullptr) win_reduce_prev<NB>(a, sred);

    const T *__restrict__ P = static_cast<const T *>(a.P);
    const VT *__restrict__ gval = static_cast<const VT *>(a.val);
    const int32_t *__restrict__ gcol = a.col;
    const T alpha = static_cast<T>(a.alpha), beta = static_cast<T>(a.beta);
    const T g0 = static_cast<T>(a.g0), g1 = static_cast<T>(a.g1), g2 = static_cast<T>(a.g2);
    // row and tile indices fit 32 bits (n < 2^31): scalar loop control stays in SGPRs
    const int n32 = static_cast<int>(a.n);
    const int nblk = (n32 + TR - 1) / TR;

    double e_re[CPL], e_im[CPL], nu[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) e_re[c] = e_im[c] = nu[c] = 0.0;

    // contiguous tile range of this workgroup; each XCD sweeps one eighth
    const int G = gridDim.x, w = blockIdx.x;
    int tb, te;
    if (G % kXcdCount == 0) {
        const int x = w % kXcdCount, k = w / kXcdCount, per = G / kXcdCount;
        const int64_t xb = ntiles * x / kXcdCount, xe = ntiles * (x + 1) / kXcdCount;
        tb = static_cast<int>(xb + (xe - xb) * k / per);
        te = static_cast<int>(xb + (xe - xb) * (k + 1) / per);
    } else {
        tb = static_cast<int>(ntiles * w / G);
        te = static_cast<int>(ntiles * (w + 1) / G);
    }

    // matrix slots of one tile: one slot per thread (prefetch register, then LDS)
    const int uw = UNI ? MAXW : 0;
    VT pv = VT{T(0), T(0)};
    int32_t pc = 0;
    int pf_ns = 0;
    int64_t pf_s0 = 0;
    auto fetch_mat = [&](int64_t tile) {
        const int64_t c0 = tile * CPT;
        int64_t c1 = c0 + CPT;
        if (c1 > a.n_chunks) c1 = a.n_chunks;
        if (uw > 0) {
            pf_s0 = c0 * 32 * uw;
            pf_ns = static_cast<int>((c1 - c0) * 32 * uw);
        } else {
            pf_s0 = a.chunk_off[c0];
            pf_ns = static_cast<int>(a.chunk_off[c1] - pf_s0);
        }
        // non-temporal: each slot is read once, and keeping the slots out of L2
        // leaves room for the U rows that neighbouring workgroups gather a few
        // tiles after they were loaded (the gathers that leave the window)
        if (tid < pf_ns) {
            pv = ld_nt(gval + pf_s0 + tid);
            pc = __builtin_nontemporal_load(gcol + pf_s0 + tid);
        }
    };
    auto deposit_mat = [&](int64_t tile, int b) {
        if (tid < pf_ns) {
            CHEBFD_WV(b)[tid] = pv;
            CHEBFD_WC(b)[tid] = pc;
        }
        if (uw > 0) return;
        if (tid < CPT) {
            const int64_t c = tile * CPT + tid;
            const bool in = c < a.n_chunks;
            CHEBFD_WCOFF(b)[tid] = in ? static_cast<int32_t>(a.chunk_off[c] - pf_s0) : 0;
            CHEBFD_WCW(b)[tid] = in ? a.chunk_width[c] : 0;
        }
    };
    // one block of U rows: row blk * TR + rr, this lane's columns
    auto ring_store = [&](int blk, const PK &v) {
        T *dst = reinterpret_cast<T *>(smem + ((blk * TR + rr) & (S::RING_ROWS - 1)) * RB + lane_off);
        if constexpr (CPL == 2) {
            *reinterpret_cast<float4 *>(dst) = float4{v.re[0], v.im[0], v.re[1], v.im[1]};
        } else {
            *reinterpret_cast<VT *>(dst) = VT{v.re[0], v.im[0]};
        }
    };
    auto row_ok = [&](int blk) { return blk >= 0 && blk < nblk && blk * TR + rr < n32; };


    // (the reduction above ends with a barrier: the ring area is free)
    if (tb < te) {
        // prologue: the window of the first tile and its matrix slots
        PK pro[2 * HALO + 1];
#pragma unroll
        for (int q = 0; q < 2 * HALO + 1; ++q) {
            const int blk = tb - HALO + q;
            if (row_ok(blk)) pro[q] = load_pack<T, CPL, false>(P + 2 * ((int64_t)(blk * TR + rr) * NB + jc));
        }
        fetch_mat(tb);
#pragma unroll
        for (int q = 0; q < 2 * HALO + 1; ++q) {
            const int blk = tb - HALO + q;
            if (row_ok(blk)) ring_store(blk, pro[q]);
        }
        deposit_mat(tb, 0);
    }
    __syncthreads();

    // One tile.  FULL: every row of the tile exists (all tiles but a ragged last
    // one), so every lane runs the same instruction stream; the partial tile guards
    // its rows.  (The compiler's wait counts are path-insensitive: a load whose use
    // sits under a lane-dependent branch stays "pending" at the loop's back edge,
    // and the next tile then drains the whole memory pipeline before its loads.)
    int buf = 0;
    // The previous tile's stored values, kept live (an empty asm statement uses
    // them) until this tile's loads are issued: otherwise the register allocator
    // reuses the store's data registers for this tile's gathers, and the compiler
    // then waits for the store to complete before issuing the next gathers.
    PK held_w, held_y;
#pragma unroll
    for (int c = 0; c < CPL; ++c) held_w.re[c] = held_w.im[c] = held_y.re[c] = held_y.im[c] = T(0);
    auto tile_body = [&](int tile, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        const bool more = tile + 1 < te;
        const int t0 = tile * TR;
        const int i = t0 + rr;
        const bool live = FULL || i < n32;
        const int wlo = t0 - HALO * TR;   // window [wlo, wlo + (2 HALO + 1) TR)
        const VT *sv = CHEBFD_WV(buf);
        const int32_t *sc = CHEBFD_WC(buf);

        // slots of the row (entries past its width gather the row itself with
        // coefficient 0; when every chunk holds MAXW slots per row the selects fold away)
        int cc[MAXW];
        int wdt = MAXW, base = 0;
        if (live) {
            const int cl = rr >> 5;
            base = (UNI ? cl * 32 * MAXW : CHEBFD_WCOFF(buf)[cl]) + (rr & 31);
            if constexpr (!UNI) wdt = CHEBFD_WCW(buf)[cl];
#pragma unroll
            for (int k = 0; k < MAXW; ++k) {
                const bool act = UNI || k < wdt;
                cc[k] = act ? sc[base + k * 32] : i;
            }
        }
        // gathers outside the window go to global memory (issued before the
        // prefetches, so waiting for them leaves the prefetches in flight)
        PK u[MAXW];
        bool inw[MAXW];
        if (live) {
#pragma unroll
            for (int k = 0; k < MAXW; ++k) {
                inw[k] = static_cast<unsigned>(cc[k] - wlo) < static_cast<unsigned>((2 * HALO + 1) * TR);
                if (!inw[k]) u[k] = load_pack<T, CPL, false>(P + 2 * ((int64_t)cc[k] * NB + jc));
            }
        }
        // prefetches: next tile's matrix slots, W and Y rows; the block entering the window
        PK rf;
        const int nb_in = tile + HALO + 1;
        const bool ring_in = more && row_ok(nb_in);
        if (ring_in) rf = load_pack<T, CPL, false>(P + 2 * ((int64_t)(nb_in * TR + rr) * NB + jc));
        if (more) fetch_mat(tile + 1);
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            asm volatile("" ::"v"(held_w.re[c]), "v"(held_w.im[c]), "v"(held_y.re[c]), "v"(held_y.im[c]));
        // row streams of W and Y
        const int64_t e = 2 * ((int64_t)i * NB + jc);
        PK o, yv;
#pragma unroll
        for (int c = 0; c < CPL; ++c) o.re[c] = o.im[c] = yv.re[c] = yv.im[c] = T(0);
        if (live) {
            if constexpr (!mode_first(MODE)) o = load_pack<T, CPL, true>(static_cast<const T *>(a.O) + e);
            if constexpr (MODE == kModeStep) yv = load_pack<T, CPL, true>(static_cast<const T *>(a.Y) + e);
        }

        if (live) {
            PK nw, yo;
            const PK up = load_pack<T, CPL, false>(CHEBFD_RING(i));
#pragma unroll
            for (int k = 0; k < MAXW; ++k)
                if (inw[k]) u[k] = load_pack<T, CPL, false>(CHEBFD_RING(cc[k]));

            T acc_re[CPL], acc_im[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc_re[c] = acc_im[c] = T(0);
#pragma unroll
            for (int k = 0; k < MAXW; ++k) {
                const bool act = UNI || k < wdt;
                VT h = sv[act ? base + k * 32 : 0];
                if (!act) h = VT{T(0), T(0)};
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    acc_re[c] = fma(h.x, u[k].re[c], acc_re[c]);
                    acc_re[c] = fma(-h.y, u[k].im[c], acc_re[c]);
                    acc_im[c] = fma(h.x, u[k].im[c], acc_im[c]);
                    acc_im[c] = fma(h.y, u[k].re[c], acc_im[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const T hu_re = fma(alpha, acc_re[c], beta * up.re[c]);
                const T hu_im = fma(alpha, acc_im[c], beta * up.im[c]);
                if constexpr (mode_first(MODE)) {
                    nw.re[c] = hu_re;
                    nw.im[c] = hu_im;
                } else {
                    nw.re[c] = fma(T(2), hu_re, -o.re[c]);
                    nw.im[c] = fma(T(2), hu_im, -o.im[c]);
                }
            }
            if constexpr (MODE == kModeSecond) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    yo.re[c] = fma(g0, o.re[c], fma(g1, up.re[c], g2 * nw.re[c]));
                    yo.im[c] = fma(g0, o.im[c], fma(g1, up.im[c], g2 * nw.im[c]));
                }
            } else if constexpr (MODE == kModeStep) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    yo.re[c] = fma(g2, nw.re[c], yv.re[c]);
                    yo.im[c] = fma(g2, nw.im[c], yv.im[c]);
                }
            }
            if constexpr (mode_first(MODE)) {
                store_pack_nt<T, CPL>(static_cast<T *>(a.N) + e, nw);
            } else if constexpr (MODE == kModeSecond) {
                store_pack_nt<T, CPL>(static_cast<T *>(a.N) + e, nw);
                store_pack_nt<T, CPL>(static_cast<T *>(a.Y) + e, yo);  // Y aliases O: row i's entry is read only here
            } else {
                store_pack_nt<T, CPL>(static_cast<T *>(a.O) + e, nw);
                if constexpr (MODE == kModeStep) store_pack_nt<T, CPL>(static_cast<T *>(a.Y) + e, yo);
            }
            held_w = nw;
            if constexpr (MODE == kModeSecond || MODE == kModeStep) held_y = yo;
            if constexpr (mode_dots(MODE)) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const double nr = nw.re[c], ni = nw.im[c], ur = up.re[c], ui = up.im[c];
                    e_re[c] = fma(nr, ur, fma(ni, ui, e_re[c]));
                    e_im[c] = fma(nr, ui, fma(-ni, ur, e_im[c]));
                    nu[c] = fma(ur, ur, fma(ui, ui, nu[c]));
                }
            }
        }
        // block tile + HALO + 1 replaces block tile - HALO - 1 (outside
        // this tile's window); the next tile's slots go to the idle buffer.  Their
        // loads were issued before the W and Y loads and the stores, so the wait
        // for them leaves those in flight; the stores also stay in flight across
        // the barrier (it orders LDS only; no other row reads this row's W or Y).
        if (ring_in) ring_store(nb_in, rf);
        if (more) deposit_mat(tile + 1, buf ^ 1);
        __syncthreads();
        buf ^= 1;
    };
    // Lead control between the sweep ranges of one XCD.  The row order deals
    // neighbouring pencils of the lattice to the ranges of one XCD at equal
    // offsets, so the gathers that leave the window read rows that another
    // range has just loaded into the shared L2 -- as long as the ranges advance
    // together; left alone they drift apart by far more than the few tiles the
    // L2 holds.  Every kWinCheckEvery tiles the first wave publishes
    // (launch tag, tiles done) in prog[x per + k] (workgroup w = x + 8 k on XCD
    // x) and, while the workgroup is more than kWinMaxLead tiles ahead of the
    // slowest range of its XCD that has started this launch, polls again (a
    // bounded wait: it only costs time).  Only the first wave touches the
    // counters (a wave-uniform branch); the others wait at the tile's barrier.
    const int per = G / kXcdCount;
    const bool lead = a.prog != nullptr && G % kXcdCount == 0 && per <= 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int64_t *const my_prog = lead ? a.prog + (w % kXcdCount) * per + w / kXcdCount : nullptr;
    const int64_t *const xcd_prog = lead ? a.prog + (w % kXcdCount) * per : nullptr;
    const int64_t tag = static_cast<int64_t>(a.epoch) << 32;
    auto check = [&](int done) {
        __hip_atomic_store(my_prog, tag | static_cast<uint32_t>(done), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int k = (tid & 63) % per;
        for (int poll = 0; poll < kWinMaxPolls; ++poll) {
            const int64_t v = __hip_atomic_load(xcd_prog + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // a range that has not started this launch (older tag) holds no one back
            int d = static_cast<int32_t>(v >> 32) == a.epoch ? static_cast<int>(v & 0xffffffff) : INT_MAX;
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) d = min(d, __shfl_xor(d, m));
            if (done - d <= kWinMaxLead) break;
            __builtin_amdgcn_s_sleep(16);
        }
    };

    // full tiles, then the ragged last tile of the matrix (if it is in this range)
    const int te_full = te < n32 / TR ? te : (n32 / TR > tb ? n32 / TR : tb);
    for (int tile = tb; tile < te_full; ++tile) {
        if (lead && wave == 0 && (tile - tb) % kWinCheckEvery == 0) check(tile - tb);
        tile_body(tile, std::true_type{});
    }
    for (int tile = te_full; tile < te; ++tile) tile_body(tile, std::false_type{});
    if (lead && wave == 0)
        __hip_atomic_store(my_prog, tag | static_cast<uint32_t>(te - tb), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    if constexpr (!mode_dots(MODE)) return;
    // workgroup reduction over the TR lanes of each column, fixed order;
    // sred[(component * CPL + c) * kWinThreads + lane] (over the ring: every
    // wave has passed the last barrier of the tile loop)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        sred[(0 * CPL + c) * kWinThreads + tid] = e_re[c];
        sred[(1 * CPL + c) * kWinThreads + tid] = e_im[c];
        sred[(2 * CPL + c) * kWinThreads + tid] = nu[c];
    }
    __syncthreads();
    if (tid < NB) {
        const int lj = tid / CPL, c = tid % CPL;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int q = 0; q < TR; ++q) {
            s0 += sred[(0 * CPL + c) * kWinThreads + q * LPR + lj];
            s1 += sred[(1 * CPL + c) * kWinThreads + q * LPR + lj];
            s2 += sred[(2 * CPL + c) * kWinThreads + q * LPR + lj];
        }
        a.part_out[(int64_t)(0 * NB + tid) * G + w] = s0;
        a.part_out[(int64_t)(1 * NB + tid) * G + w] = s1;
        a.part_out[(int64_t)(2 * NB + tid) * G + w] = s2;
    }
}
#undef CHEBFD_WV
#undef CHEBFD_WC
#undef CHEBFD_WCOFF
#undef CHEBFD_WCW
#undef CHEBFD_RING

namespace {

template <typename T, int NB, int MODE, int MAXW, bool UNI>
int launch_win_one(const StepArgs &a, const WinGeometry &g, hipStream_t s) {
    constexpr int lds = win_lds_bytes<T, NB, MAXW>();
    hipLaunchKernelGGL((cheb_win_kernel<T, NB, MODE, MAXW, UNI>), dim3(g.G), dim3(kWinThreads), lds, s, a,
                       g.ntiles);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

template <typename T, int NB, int MAXW, bool UNI>
int launch_win_mode(int mode, const StepArgs &a, const WinGeometry &g, hipStream_t s) {
    switch (mode) {
        case kModeFirst: return launch_win_one<T, NB, kModeFirst, MAXW, UNI>(a, g, s);
        case kModeSecond: return launch_win_one<T, NB, kModeSecond, MAXW, UNI>(a, g, s);
        case kModeStep: return launch_win_one<T, NB, kModeStep, MAXW, UNI>(a, g, s);
        case kModeKpm: return launch_win_one<T, NB, kModeKpm, MAXW, UNI>(a, g, s);
        case kModeSpmv: return launch_win_one<T, NB, kModeSpmv, MAXW, UNI>(a, g, s);
        case kModeSpmvRec: return launch_win_one<T, NB, kModeSpmvRec, MAXW, UNI>(a, g, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "bad step mode %d", mode);
}

template <typename T, int NB>
int launch_win_w(int mode, const StepArgs &a, const WinGeometry &g, hipStream_t s) {
    if (g.uniform) return launch_win_mode<T, NB, kWinWidth, true>(mode, a, g, s);
    return launch_win_mode<T, NB, kWinWidth, false>(mode, a, g, s);
}

template <typename T, int NB, int MAXW, bool UNI>
bool set_win_attr() {
    const int bytes = win_lds_bytes<T, NB, MAXW>();
    bool ok = true;
    ok &= hipFuncSetAttribute(reinterpret_cast<const void *>(cheb_win_kernel<T, NB, kModeFirst, MAXW, UNI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
    ok &= hipFuncSetAttribute(reinterpret_cast<const void *>(cheb_win_kernel<T, NB, kModeSecond, MAXW, UNI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
    ok &= hipFuncSetAttribute(reinterpret_cast<const void *>(cheb_win_kernel<T, NB, kModeStep, MAXW, UNI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
    ok &= hipFuncSetAttribute(reinterpret_cast<const void *>(cheb_win_kernel<T, NB, kModeKpm, MAXW, UNI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
    ok &= hipFuncSetAttribute(reinterpret_cast<const void *>(cheb_win_kernel<T, NB, kModeSpmv, MAXW, UNI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
    ok &= hipFuncSetAttribute(reinterpret_cast<const void *>(cheb_win_kernel<T, NB, kModeSpmvRec, MAXW, UNI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
    return ok;
}

}  // namespace

bool win_geometry(const chebfd_matrix *H, int prec, int nb, int num_cus, WinGeometry *g) {
    if (H->C != 32 || H->max_width > kWinWidth) return false;
    int tr;
    // instances where the window beats the LDS-staged kernel (measured): FP64
    // n_b = 32, c64 n_b = 64, and c64 n_b = 32 from 32 tiles of 64 rows per CU
    // (the 64x64x32 lattice: 141 against 151 us per step)
    if (prec == CHEBFD_PREC_FP64 && nb == 32)
        tr = WinShape<double, 32>::TR;
    else if (prec == CHEBFD_PREC_MIXED && nb == 64)
        tr = WinShape<float, 64>::TR;
    else if (prec == CHEBFD_PREC_MIXED && nb == 32 && H->n >= (int64_t)kWinC64Nb32Tiles * num_cus * 64)
        tr = WinShape<float, 32>::TR;
    else
        return false;
    const int local = H->window_local[tr == 32 ? 0 : 1];
    if (local < kWinMinLocal) return false;
    g->tr = tr;
    // every chunk exactly kWinWidth slots wide (lattice Hamiltonians of 4 orbitals): no width selects
    g->uniform = H->uniform_width == kWinWidth ? 1 : 0;
    g->ntiles = (H->n + tr - 1) / tr;
    // one workgroup per CU, at least two tiles each (the window needs a sweep to pay off)
    int64_t G = num_cus;
    while (G > kXcdCount && g->ntiles < 2 * G) G /= 2;
    if (g->ntiles < 2 * G) return false;
    static bool attr_ok =
        set_win_attr<double, 32, kWinWidth, true>() && set_win_attr<double, 32, kWinWidth, false>() &&
        set_win_attr<float, 64, kWinWidth, true>() && set_win_attr<float, 64, kWinWidth, false>() &&
        set_win_attr<float, 32, kWinWidth, true>() && set_win_attr<float, 32, kWinWidth, false>();
    if (!attr_ok) return false;
    g->G = static_cast<int>(G);
    return true;
}

int launch_win_step(int prec, int nb, int mode, const StepArgs &a, const WinGeometry &g, hipStream_t s) {
    if (prec == CHEBFD_PREC_FP64 && nb == 32) return launch_win_w<double, 32>(mode, a, g, s);
    if (prec == CHEBFD_PREC_MIXED && nb == 64) return launch_win_w<float, 64>(mode, a, g, s);
    if (prec == CHEBFD_PREC_MIXED && nb == 32) return launch_win_w<float, 32>(mode, a, g, s);
    CHEBFD_FAIL(CHEBFD_EINVAL, "window kernel has no instance for prec %d, n_b = %d", prec, nb);
}

}  // namespace chebfd
