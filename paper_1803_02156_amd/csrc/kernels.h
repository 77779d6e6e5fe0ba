// Launchers of the libchebfd device kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chebfd {

// Variants of the fused step kernel.
//  kModeFirst : N = (aH+bI) P                                 (Alg. 1, first product)
//  kModeSecond: N = 2(aH+bI) P - O;  Y(=O) = g0 O + g1 P + g2 N   (Alg. 1, start of Y)
//  kModeStep  : O = 2(aH+bI) P - O (in place);  Y += g2 O       (Alg. 1, recurrence step)
//  kModeKpm   : O = 2(aH+bI) P - O (in place), no Y update      (moments only)
// These four also form the per-column products <new, P> and <P, P>.  The
// unfused filter (the SpMMV call of Alg. 1 on its own, followed by separate
// dot and axpy calls) uses two more, which form no dot products:
//  kModeSpmv   : N = (aH+bI) P
//  kModeSpmvRec: O = 2(aH+bI) P - O (in place)
enum { kModeFirst = 0, kModeSecond = 1, kModeStep = 2, kModeKpm = 3, kModeSpmv = 4, kModeSpmvRec = 5 };
constexpr bool mode_dots(int mode) { return mode <= kModeKpm; }
constexpr bool mode_first(int mode) { return mode == kModeFirst || mode == kModeSpmv; }

struct StepArgs {
    int64_t n;
    int64_t n_chunks;
    int64_t npass;              // ceil(n / (256 / NB)) row passes
    const int64_t *chunk_off;
    const int32_t *chunk_width;
    const int32_t *col;
    const void *val;
    int32_t C;
    int32_t log2C;
    const void *P;              // gathered block (T_{p-1} x)
    void *O;                    // previous block (T_{p-2} x); in place for Step/Kpm
    void *N;                    // new block for First/Second
    void *Y;                    // filtered block
    double alpha, beta;
    double g0, g1, g2;
    double *part_out;           // [3*NB][G] partial dot products of this launch
    const double *part_in;      // [3*NB][G_prev] partials of the previous launch, or null
    double *red_eta;            // destination of the reduced eta (re, im pairs) [NB]
    double *red_nu;             // destination of the reduced nu [NB]
    int32_t G_prev;
    int32_t uniform_width;      // every chunk has this many slots per row (0: read chunk_width)
    int64_t *prog;              // [G] progress words of the window kernel's lead control, or null
    int32_t epoch;              // this launch's tag in prog (nonzero, distinct from recent launches)
};
// A fresh launch tag for StepArgs::epoch (host, thread-safe).
int32_t next_step_epoch();

int launch_step(int prec, int nb, int mode, const StepArgs &a, int G, hipStream_t s);

// LDS-staged step kernel (filter_lds.hip): tiles of whole SELL chunks
struct LdsGeometry {
    int tile_rows;      // rows per tile: max(C, 256 / n_b)
    int tile_slots;     // LDS slots per tile buffer: max_width * tile_rows
    int maxw;           // compile-time row width of the kernel instance (13 or 16)
    int G;              // persistent grid
    int64_t ntiles;
    size_t lds_bytes;
};
bool lds_geometry(const chebfd_matrix *H, int prec, int nb, int num_cus, LdsGeometry *g);
int launch_lds_step(int prec, int nb, int mode, const StepArgs &a, const LdsGeometry &g,
                    hipStream_t s);
// Window step kernel (filter_win.hip): one 1024-thread workgroup per CU sweeps
// a contiguous range of tiles and gathers from a ring of U rows staged in LDS
// (kWinBlocks blocks of one tile each; tile t reads blocks t - h .. t + h,
// h = win_halo(tile rows)).  Used for FP64 n_b = 32, c64 n_b = 64 and c64
// n_b = 32, rows of at most kWinWidth entries, when at least kWinMinLocal of
// 1000 stored entries fall inside the window.
constexpr int kWinBlocks = 8;
// Window half-width in tiles: 3 tiles of 32 rows, 1 tile of 64 rows.  The
// z-neighbours of 4 x 4 pencils (4 orbitals) lie 64 rows away; with 32-row
// tiles a window of 2 tiles measured 7 % slower than 3, with 64-row tiles 1
// tile beats 3 (fewer prologue blocks: 64x64x32 c64 n_b = 32 step 151.6 ->
// 141.1 us).
constexpr int win_halo(int tr) { return tr >= 64 ? 1 : 3; }
constexpr int kWinWidth = 13;       // rows of at most this many stored entries
constexpr int kWinMinLocal = 700;
constexpr int kWinC64Nb32Tiles = 32;   // c64 n_b = 32 takes the window kernel from this many 64-row tiles per CU
struct WinGeometry {
    int tr;             // rows per tile
    int uniform;        // 1: every chunk holds exactly kWinWidth slots per row
    int G;              // workgroups (one per CU)
    int64_t ntiles;
};
bool win_geometry(const chebfd_matrix *H, int prec, int nb, int num_cus, WinGeometry *g);
int launch_win_step(int prec, int nb, int mode, const StepArgs &a, const WinGeometry &g, hipStream_t s);
// row-per-wavefront kernel for n_b in {32, 64, 128}: a pass covers 128 / n_b rows
// Rows up to kRowMaxUnrolled stored entries use the unrolled path, whose loads
// may read up to kRowMaxUnrolled * C slots past the last chunk: the matrix
// buffer carries that many zero slots as padding.
constexpr int kRowMaxUnrolled = 16;
int launch_row_step(int prec, int nb, int max_width, int mode, const StepArgs &a, int G,
                    hipStream_t s);
int row_occupancy(int prec, int nb);
constexpr int kRowKernelMinNb = 32;
inline int row_kernel_rows_per_pass(int nb) { return 128 / nb; }
int launch_reduce(int nb, const StepArgs &a, hipStream_t s);
// BLAS1 calls of the unfused filter (blas1.hip), on blocked n x nb blocks:
// per-workgroup partials of <A, B>_j = sum_i conj(A_ij) B_ij into
// part[(comp0 + c) NB + j][G] (c = 0 real part, 1 imaginary part; real part
// only when want_im is false), and Y = a Y + b X over count complex entries.
int launch_block_dot(int prec, int nb, int64_t n, const void *A, const void *B, double *part, int G, int comp0,
                     bool want_im, hipStream_t s);
int launch_block_axpby(int prec, int64_t count, double a, void *y, double b, const void *x, hipStream_t s);
int step_grid(int prec, int nb, int64_t npass, int num_cus);

// dense kernels (dense.hip)
int launch_gram(const void *A, int prec_a, int nb_a, const void *B, int prec_b, int nb_b, int64_t n,
                int m1, int m2, double *part, int nsplit, double *S, int ld, hipStream_t s);
size_t gram_part_bytes(int m1, int m2, int nsplit);
// Row splits of a Gram product S = A^H B (m1 x m2): enough workgroups for a few
// full waves of the device (about 4096 64 x 64 tile-splits; the Hermitian
// product forms about half of them) but at least 256 rows per split.
inline int gram_splits(int64_t n, int m1, int m2) {
    const int64_t tiles = (int64_t)((m1 + 63) / 64) * ((m2 + 63) / 64);
    const int64_t want = (4096 + tiles - 1) / tiles;
    const int64_t cap = n / 256 > 1 ? n / 256 : 1;
    return static_cast<int>(want < 1024 ? (want < cap ? want : cap) : (1024 < cap ? 1024 : cap));
}
int launch_update(const void *A, int prec_a, int nb_a, const double *M, int ldm, void *Z, int prec_z,
                  int nb_z, int64_t n, int m1, int m2, hipStream_t s);
// Z = S - A M (Z FP64, at most 32 columns, blocked width nb_z; S of precision
// prec_s, blocked width nb_s, may alias Z)
int launch_update_sub(const void *A, int prec_a, int nb_a, const double *M, int ldm, const void *S, int prec_s,
                      int nb_s, double *Z, int nb_z, int64_t n, int m1, int m2, hipStream_t s);
// Jacobi eigensolver (host-driven sweeps, one launch per round); synchronises `s`
// once per sweep to read the off-diagonal norm
size_t jacobi_scratch_bytes(int m);
int launch_jacobi(int m, double *A, int lda, double *V, int ldv, double *w, int max_sweeps, double tol,
                  void *scratch, int *sweeps, int *converged, hipStream_t s);

int launch_svqb_scale(int m, double *S, int ld, double *d, hipStream_t s);
int launch_svqb_transform(int m, int k, int first, const double *d, const double *V, int ldv,
                          const double *w, double *T, int ldt, hipStream_t s);
int launch_hermitise(int m, double *G, int ld, hipStream_t s);
int resid_grid(int64_t n);
int launch_resid(const void *HZ, const void *Z, int prec, int64_t n, int nb, const double *theta,
                 double *part, int G, double *out, hipStream_t s);
int launch_convert(const void *src, int prec_src, void *dst, int prec_dst, int64_t count,
                   hipStream_t s);
int launch_random_phase(void *X, int prec, int64_t n, int nb, int c_begin, int c_end, uint64_t seed,
                        uint64_t col0, const int32_t *perm, hipStream_t s);
int launch_permute_columns(int rows, int m, const double *S, int lds, const int *order, double *T,
                           int ldt, hipStream_t s);
int launch_fix_phases(void *Z, int prec, int64_t n, int nb, int m, double *phase, hipStream_t s);

// TSQR (tsqr.hip): Y (n x m, blocked width nb, prec_y) = Q R, Q into a second
// block vector (prec_q, same nb), R (m x m, FP64 complex, column-major, ldr)
// upper triangular with a real non-negative diagonal.  Panels of
// tsqr_panel_width(nb) columns; work buffers: T (n x panel width FP64
// complex), tree (tsqr_tree_bytes), C1 and C2 (m x panel width, leading
// dimension ldc >= m) and gpart (tsqr_gpart_bytes).
struct TsqrWork {
    double *T, *tree, *C1, *C2;
    int ldc;
    double *gpart;
};
int tsqr_panel_width(int nb);
size_t tsqr_tree_bytes(int64_t n, int pw);
size_t tsqr_gpart_bytes(int64_t n, int m, int nb);
int tsqr_blocked(int64_t n, int m, int nb, int prec_y, const void *Y, int prec_q, void *Q, double *R, int ldr,
                 const TsqrWork &w, hipStream_t s);
// info[2k] = |R_kk|^2, info[2k + 1] = squared norm of column k of R
int launch_tsqr_colinfo(int m, const double *R, int ldr, double *info, hipStream_t s);

// layout / misc kernels (layout.hip)
int launch_pack(const int32_t *perm, int64_t n, int m, int nb, int prec, const void *src,
                void *dst, bool unpack, hipStream_t s);
int launch_axpby_blocked(int prec, int64_t count, double a, void *y, double b, const void *x,
                         hipStream_t s);
int launch_bounds(const int64_t *chunk_off, const int32_t *chunk_width, const int32_t *col,
                  const void *val, int prec, int64_t n, int C, int log2C, double *part, int G,
                  hipStream_t s);
int launch_bounds_final(const double *part, int G, double *out2, hipStream_t s);
int launch_stream_probe(int kind, int64_t count, const double *b, const double *c, double sc,
                        double *a, int num_cus, hipStream_t s);

}  // namespace chebfd
