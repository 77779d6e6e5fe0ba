// Launchers of the libchebfd device kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chebfd {

// Variants of the fused step kernel.
//  kModeFirst : N = (aH+bI) P                                 (Alg. 1 line 4)
//  kModeSecond: N = 2(aH+bI) P - O;  Y(=O) = g0 O + g1 P + g2 N   (lines 5-6)
//  kModeStep  : O = 2(aH+bI) P - O (in place);  Y += g2 O       (lines 9-12)
//  kModeKpm   : O = 2(aH+bI) P - O (in place), no Y update      (moments only)
// Every mode also forms the per-column products <new, P> and <P, P>.
enum { kModeFirst = 0, kModeSecond = 1, kModeStep = 2, kModeKpm = 3 };

struct StepArgs {
    int64_t n;
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
    int32_t pad;
};

int launch_step(int prec, int nb, int mode, const StepArgs &a, int G, hipStream_t s);
int launch_reduce(int nb, const StepArgs &a, hipStream_t s);
int step_grid(int prec, int nb, int64_t npass, int num_cus);

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
