// Fused Chebyshev step with the matrix staged in LDS (gfx950).
//
// Same computation as the step kernels of filter.hip (the recurrence step of
// Alg. 1 of the ChebFD paper, and its two start launches): per row i and block
// column j, W_ij <- 2 ((aH + bI) U)_ij - W_ij, the filtered-block update and
// the per-column dot products.
//
// Work unit: a tile of TR = max(C, 256 / NB) consecutive rows (whole SELL
// chunks).  A workgroup copies the tile's matrix slots (column index and value
// of every stored entry, contiguous in SELL order) from HBM into LDS with
// coalesced loads; the copy for the next tile is issued before the current
// tile is processed and lands in the second LDS buffer afterwards.  Rows read
// their slots from LDS as broadcasts, so the vector-memory pipeline only
// carries the block-vector traffic: the gathers of U (NB consecutive complex
// numbers per row segment, one per lane) and the row streams of U, W, Y.
// W and Y are streamed with non-temporal loads and stores so that the L2 keeps
// the lines of U, which other rows gather again.
//
// Lanes: 256 / NB rows per sub-pass, lane t works on column t % NB of row
// t / NB; all accesses of a row segment are contiguous.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "kernels.h"
#include "step_io.h"

namespace chebfd {
namespace {

using namespace step_io;

constexpr int kThreads = 256;
constexpr int kXcds = 8;

// Prefetch registers per thread: a tile holds max(32, rows per sub-pass) rows
// of at most 16 slots (wider rows or chunks above 32 rows use the other kernels).
constexpr int lds_prefetch_slots(int rows) {
    return ((rows > 32 ? rows : 32) * 16 + kThreads - 1) / kThreads;
}
constexpr int kMaxTileWidth = 16;

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

// LDS layout (dynamic): sred[3 * 256] doubles | 2 x { vals[S], cols[S] } | 2 x { coff[CPT + 1], cw[CPT] }
// where S = tile_slots (max slots of a tile) and CPT = chunks per tile.
template <typename T, int NB, int MODE, int MAXW>
__global__ __launch_bounds__(kThreads) void cheb_lds_kernel(StepArgs a, int tile_rows, int tile_slots,
                                                            int64_t ntiles) {
    using VT = typename V2<T>::type;
    constexpr int CPL = cols_per_lane<T, NB>();
    constexpr int LPR = NB / CPL;              // lanes per row
    constexpr int ROWS = kThreads / LPR;       // rows per sub-pass
    constexpr int PF = lds_prefetch_slots(ROWS);
    using PK = Pack<T, CPL>;
    extern __shared__ __align__(16) unsigned char smem[];
    double *sred = reinterpret_cast<double *>(smem);
    // byte offsets of the two tile buffers inside smem (pointers are formed
    // from smem at each use so the compiler keeps them in the LDS address space)
    const int cpt = tile_rows >> a.log2C;
    const int o_vals = static_cast<int>(sizeof(double)) * 3 * CPL * kThreads;
    const int o_cols = o_vals + static_cast<int>(sizeof(VT)) * tile_slots;
    const int o_coff = o_cols + 4 * tile_slots;
    const int o_cw = o_coff + 4 * (cpt + 1);
    const int buf_bytes = ((o_cw + 4 * cpt - o_vals) + 15) & ~15;
#define CHEBFD_SV(b) reinterpret_cast<VT *>(smem + o_vals + (b) * buf_bytes)
#define CHEBFD_SC(b) reinterpret_cast<int32_t *>(smem + o_cols + (b) * buf_bytes)
#define CHEBFD_SCOFF(b) reinterpret_cast<int32_t *>(smem + o_coff + (b) * buf_bytes)
#define CHEBFD_SCW(b) reinterpret_cast<int32_t *>(smem + o_cw + (b) * buf_bytes)

    const int tid = threadIdx.x;
    const int j = tid % LPR;
    const int jc = j * CPL;                    // first column of this lane
    const int rr = tid / LPR;

    if (a.part_in != nullptr) reduce_prev<NB>(a, sred);

    const T *__restrict__ P = static_cast<const T *>(a.P);   // interleaved re, im
    const VT *__restrict__ gval = static_cast<const VT *>(a.val);
    const int32_t *__restrict__ gcol = a.col;
    const T alpha = static_cast<T>(a.alpha), beta = static_cast<T>(a.beta);
    const T g0 = static_cast<T>(a.g0), g1 = static_cast<T>(a.g1), g2 = static_cast<T>(a.g2);

    double e_re[CPL], e_im[CPL], nu[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) e_re[c] = e_im[c] = nu[c] = 0.0;

    // tile range of this workgroup: each XCD sweeps one contiguous eighth
    const int G = gridDim.x, w = blockIdx.x;
    int64_t begin, end, stride;
    if (G % kXcds == 0 && ntiles >= G) {
        const int x = w % kXcds, k = w / kXcds;
        begin = ntiles * x / kXcds + k;
        end = ntiles * (x + 1) / kXcds;
        stride = G / kXcds;
    } else {
        begin = w;
        end = ntiles;
        stride = G;
    }

    // prefetch registers for one tile's slots (plain scalars: arrays of HIP
    // vector structs are not promoted to registers and would live in scratch)
    T pvr[PF], pvi[PF];
    int32_t pc[PF];
    int64_t pf_s0 = 0;
    int pf_ns = 0;
    // Equally wide chunks (every row padded to uw slots): chunk c starts at
    // slot c C uw, so no chunk metadata is read (a load of it would make the
    // wave wait for all its outstanding stores before the next tile).
    const int uw = a.uniform_width;
    auto fetch = [&](int64_t tile) {
        const int64_t c0 = (tile * tile_rows) >> a.log2C;
        int64_t c1 = c0 + cpt;
        if (c1 > a.n_chunks) c1 = a.n_chunks;
        if (uw > 0) {
            pf_s0 = c0 * a.C * uw;
            pf_ns = static_cast<int>((c1 - c0) * a.C * uw);
        } else {
            pf_s0 = a.chunk_off[c0];
            pf_ns = static_cast<int>(a.chunk_off[c1] - pf_s0);
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int s = tid + q * kThreads;
            if (s < pf_ns) {
                const VT v = gval[pf_s0 + s];
                pvr[q] = v.x;
                pvi[q] = v.y;
                pc[q] = gcol[pf_s0 + s];
            }
        }
    };
    auto deposit = [&](int64_t tile, int b) {
        const int64_t c0 = (tile * tile_rows) >> a.log2C;
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int s = tid + q * kThreads;
            if (s < pf_ns) {
                CHEBFD_SV(b)[s] = VT{pvr[q], pvi[q]};
                CHEBFD_SC(b)[s] = pc[q];
            }
        }
        if (uw > 0) return;
        for (int q = tid; q < cpt; q += kThreads) {
            const int64_t c = c0 + q;
            const bool in = c < a.n_chunks;
            CHEBFD_SCOFF(b)[q] = in ? static_cast<int32_t>(a.chunk_off[c] - pf_s0) : 0;
            CHEBFD_SCW(b)[q] = in ? a.chunk_width[c] : 0;
        }
    };

    int buf = 0;
    if (begin < end) {
        fetch(begin);
        deposit(begin, 0);
    }
    __syncthreads();

    for (int64_t tile = begin; tile < end; tile += stride) {
        const bool more = tile + stride < end;
        if (more) fetch(tile + stride);  // lands in registers while this tile runs

        const VT *sv = CHEBFD_SV(buf);
        const int32_t *sc = CHEBFD_SC(buf);
        const int32_t *scoffb = CHEBFD_SCOFF(buf);
        const int32_t *scwb = CHEBFD_SCW(buf);
        const int64_t t0 = tile * tile_rows;
        for (int sp = 0; sp < tile_rows; sp += ROWS) {
          const int r = sp + rr;             // row within the tile
          const int64_t i = t0 + r;
          if (i < a.n) {
            const int cl = r >> a.log2C;
            const int base = (uw > 0 ? cl * a.C * uw : scoffb[cl]) + (r & (a.C - 1));
            const int wdt = uw > 0 ? uw : scwb[cl];
            const int64_t e = 2 * (i * NB + jc);   // scalar offset of the lane's first column

            // row streams (U_i is also gathered by neighbours: cached; W, Y: streamed)
            const PK up = load_pack<T, CPL, false>(P + e);
            PK o, yv;
#pragma unroll
            for (int c = 0; c < CPL; ++c) o.re[c] = o.im[c] = yv.re[c] = yv.im[c] = T(0);
            if constexpr (!mode_first(MODE)) o = load_pack<T, CPL, true>(static_cast<const T *>(a.O) + e);
            if constexpr (MODE == kModeStep) yv = load_pack<T, CPL, true>(static_cast<const T *>(a.Y) + e);

            T acc_re[CPL], acc_im[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc_re[c] = acc_im[c] = T(0);
            if (wdt <= MAXW) {
                // Branch-free: slots past the row's width gather the row's own
                // entry and get coefficient 0; when every chunk holds exactly
                // MAXW slots per row (a kernel argument, uniform) the selects
                // fold away.
                const bool full = a.uniform_width == MAXW;
                int sidx[MAXW];
                int cc[MAXW];
#pragma unroll
                for (int k = 0; k < MAXW; ++k) {
                    const int sl = base + k * a.C;
                    sidx[k] = sl < tile_slots ? sl : tile_slots - 1;
                    const int c = sc[sidx[k]];
                    cc[k] = (full || k < wdt) ? c : static_cast<int>(i);
                }
                PK u[MAXW];
#pragma unroll
                for (int k = 0; k < MAXW; ++k) u[k] = load_pack<T, CPL, false>(P + 2 * ((int64_t)cc[k] * NB + jc));
#pragma unroll
                for (int k = 0; k < MAXW; ++k) {
                    VT h = sv[sidx[k]];
                    if (!(full || k < wdt)) h = VT{T(0), T(0)};
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        acc_re[c] = fma(h.x, u[k].re[c], acc_re[c]);
                        acc_re[c] = fma(-h.y, u[k].im[c], acc_re[c]);
                        acc_im[c] = fma(h.x, u[k].im[c], acc_im[c]);
                        acc_im[c] = fma(h.y, u[k].re[c], acc_im[c]);
                    }
                }
            } else {
                for (int k = 0; k < wdt; ++k) {
                    const int col = sc[base + k * a.C];
                    const VT h = sv[base + k * a.C];
                    const PK uu = load_pack<T, CPL, false>(P + 2 * ((int64_t)col * NB + jc));
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        acc_re[c] = fma(h.x, uu.re[c], acc_re[c]);
                        acc_re[c] = fma(-h.y, uu.im[c], acc_re[c]);
                        acc_im[c] = fma(h.x, uu.im[c], acc_im[c]);
                        acc_im[c] = fma(h.y, uu.re[c], acc_im[c]);
                    }
                }
            }

            PK nw;
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
            if constexpr (mode_first(MODE)) {
                store_pack_nt<T, CPL>(static_cast<T *>(a.N) + e, nw);
            } else if constexpr (MODE == kModeSecond) {
                store_pack_nt<T, CPL>(static_cast<T *>(a.N) + e, nw);
                PK y;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    y.re[c] = fma(g0, o.re[c], fma(g1, up.re[c], g2 * nw.re[c]));
                    y.im[c] = fma(g0, o.im[c], fma(g1, up.im[c], g2 * nw.im[c]));
                }
                store_pack_nt<T, CPL>(static_cast<T *>(a.Y) + e, y);  // Y aliases O: row i's entry is read only here
            } else {
                store_pack_nt<T, CPL>(static_cast<T *>(a.O) + e, nw);
                if constexpr (MODE == kModeStep) {
                    PK y;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        y.re[c] = fma(g2, nw.re[c], yv.re[c]);
                        y.im[c] = fma(g2, nw.im[c], yv.im[c]);
                    }
                    store_pack_nt<T, CPL>(static_cast<T *>(a.Y) + e, y);
                }
            }
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
          // The next tile's slots go to the idle buffer after the first
          // sub-pass: their loads have landed by then, and the wait for them
          // does not cover the stores of the later sub-passes.
          if (sp == 0 && more) deposit(tile + stride, buf ^ 1);
        }

        if (more) buf ^= 1;
        __syncthreads();
    }

    if constexpr (!mode_dots(MODE)) return;
    // workgroup reduction over the ROWS lanes of each column, fixed order;
    // sred[(component * CPL + c) * kThreads + lane]
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        sred[(0 * CPL + c) * kThreads + tid] = e_re[c];
        sred[(1 * CPL + c) * kThreads + tid] = e_im[c];
        sred[(2 * CPL + c) * kThreads + tid] = nu[c];
    }
    __syncthreads();
    if (tid < NB) {
        const int lj = tid / CPL, c = tid % CPL;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int q = 0; q < ROWS; ++q) {
            s0 += sred[(0 * CPL + c) * kThreads + q * LPR + lj];
            s1 += sred[(1 * CPL + c) * kThreads + q * LPR + lj];
            s2 += sred[(2 * CPL + c) * kThreads + q * LPR + lj];
        }
        a.part_out[(int64_t)(0 * NB + tid) * G + w] = s0;
        a.part_out[(int64_t)(1 * NB + tid) * G + w] = s1;
        a.part_out[(int64_t)(2 * NB + tid) * G + w] = s2;
    }
}
#undef CHEBFD_SV
#undef CHEBFD_SC
#undef CHEBFD_SCOFF
#undef CHEBFD_SCW

namespace {

template <typename T, int NB, int MODE, int MAXW>
int launch_lds_one(const StepArgs &a0, const LdsGeometry &g, hipStream_t s) {
    StepArgs a = a0;
    hipLaunchKernelGGL((cheb_lds_kernel<T, NB, MODE, MAXW>), dim3(g.G), dim3(kThreads), g.lds_bytes, s, a,
                       g.tile_rows, g.tile_slots, g.ntiles);
    CHEBFD_HIP(hipGetLastError());
    return CHEBFD_OK;
}

template <typename T, int NB, int MAXW>
int launch_lds_mode(int mode, const StepArgs &a, const LdsGeometry &g, hipStream_t s) {
    switch (mode) {
        case kModeFirst: return launch_lds_one<T, NB, kModeFirst, MAXW>(a, g, s);
        case kModeSecond: return launch_lds_one<T, NB, kModeSecond, MAXW>(a, g, s);
        case kModeStep: return launch_lds_one<T, NB, kModeStep, MAXW>(a, g, s);
        case kModeKpm: return launch_lds_one<T, NB, kModeKpm, MAXW>(a, g, s);
        case kModeSpmv: return launch_lds_one<T, NB, kModeSpmv, MAXW>(a, g, s);
        case kModeSpmvRec: return launch_lds_one<T, NB, kModeSpmvRec, MAXW>(a, g, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "bad step mode %d", mode);
}

template <typename T, int NB>
int launch_lds_w(int mode, const StepArgs &a, const LdsGeometry &g, hipStream_t s) {
    if (g.maxw == 13) return launch_lds_mode<T, NB, 13>(mode, a, g, s);
    return launch_lds_mode<T, NB, kMaxTileWidth>(mode, a, g, s);
}

template <typename T>
int launch_lds_nb(int nb, int mode, const StepArgs &a, const LdsGeometry &g, hipStream_t s) {
    switch (nb) {
        case 1: return launch_lds_w<T, 1>(mode, a, g, s);
        case 2: return launch_lds_w<T, 2>(mode, a, g, s);
        case 4: return launch_lds_w<T, 4>(mode, a, g, s);
        case 8: return launch_lds_w<T, 8>(mode, a, g, s);
        case 16: return launch_lds_w<T, 16>(mode, a, g, s);
        case 32: return launch_lds_w<T, 32>(mode, a, g, s);
        case 64: return launch_lds_w<T, 64>(mode, a, g, s);
        case 128: return launch_lds_w<T, 128>(mode, a, g, s);
    }
    CHEBFD_FAIL(CHEBFD_EINVAL, "n_b = %d not supported", nb);
}

template <typename T, int NB>
int occ_lds(int maxw, size_t lds) {
    int blocks = 0;
    const hipError_t e =
        maxw == 13 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, cheb_lds_kernel<T, NB, kModeStep, 13>,
                                                                  kThreads, lds)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                         &blocks, cheb_lds_kernel<T, NB, kModeStep, kMaxTileWidth>, kThreads, lds);
    return (e != hipSuccess || blocks < 1) ? 1 : blocks;
}

template <typename T>
int occ_lds_nb(int nb, int maxw, size_t lds) {
    switch (nb) {
        case 1: return occ_lds<T, 1>(maxw, lds);
        case 2: return occ_lds<T, 2>(maxw, lds);
        case 4: return occ_lds<T, 4>(maxw, lds);
        case 8: return occ_lds<T, 8>(maxw, lds);
        case 16: return occ_lds<T, 16>(maxw, lds);
        case 32: return occ_lds<T, 32>(maxw, lds);
        case 64: return occ_lds<T, 64>(maxw, lds);
        default: return occ_lds<T, 128>(maxw, lds);
    }
}

}  // namespace

bool lds_geometry(const chebfd_matrix *H, int prec, int nb, int num_cus, LdsGeometry *g) {
    if (H->max_width > kMaxTileWidth || H->C > 32) return false;
    const int cpl = (prec == CHEBFD_PREC_MIXED && nb >= 2) ? 2 : 1;   // cols_per_lane<T, NB>()
    const int rows = kThreads * cpl / nb;
    g->tile_rows = rows > H->C ? rows : H->C;
    g->maxw = H->max_width <= 13 ? 13 : kMaxTileWidth;
    const int64_t slots = (int64_t)H->max_width * g->tile_rows;
    if (slots > (int64_t)lds_prefetch_slots(rows) * kThreads) return false;
    g->tile_slots = static_cast<int>(slots < 1 ? 1 : slots);
    const int cpt = g->tile_rows / H->C;
    const size_t vb = prec == CHEBFD_PREC_FP64 ? 16 : 8;
    size_t per_buf = vb * g->tile_slots + 4 * g->tile_slots + 4 * (2 * cpt + 1);
    per_buf = (per_buf + 15) / 16 * 16;
    g->lds_bytes = sizeof(double) * 3 * cpl * kThreads + 2 * per_buf;
    g->ntiles = (H->n + g->tile_rows - 1) / g->tile_rows;
    const int occ = prec == CHEBFD_PREC_FP64 ? occ_lds_nb<double>(nb, g->maxw, g->lds_bytes)
                                             : occ_lds_nb<float>(nb, g->maxw, g->lds_bytes);
    int64_t G = (int64_t)num_cus * occ;
    if (G > g->ntiles) G = g->ntiles;
    if (G >= kXcds) G -= G % kXcds;
    g->G = static_cast<int>(G < 1 ? 1 : G);
    return true;
}

int launch_lds_step(int prec, int nb, int mode, const StepArgs &a, const LdsGeometry &g,
                    hipStream_t s) {
    if (prec == CHEBFD_PREC_FP64) return launch_lds_nb<double>(nb, mode, a, g, s);
    return launch_lds_nb<float>(nb, mode, a, g, s);
}

}  // namespace chebfd
