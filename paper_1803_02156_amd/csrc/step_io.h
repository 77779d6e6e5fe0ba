// Register packs of block-vector entries and their loads and stores, shared by
// the fused step kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace chebfd {
namespace step_io {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));

__device__ inline double2 ld_nt(const double2 *p) {
    const dv2 v = __builtin_nontemporal_load(reinterpret_cast<const dv2 *>(p));
    return double2{v.x, v.y};
}
__device__ inline float2 ld_nt(const float2 *p) {
    const fv2 v = __builtin_nontemporal_load(reinterpret_cast<const fv2 *>(p));
    return float2{v.x, v.y};
}
__device__ inline void st_nt(double2 *p, double2 r) {
    dv2 v;
    v.x = r.x;
    v.y = r.y;
    __builtin_nontemporal_store(v, reinterpret_cast<dv2 *>(p));
}
__device__ inline void st_nt(float2 *p, float2 r) {
    fv2 v;
    v.x = r.x;
    v.y = r.y;
    __builtin_nontemporal_store(v, reinterpret_cast<fv2 *>(p));
}

// Columns per lane: c64 blocks give each lane two adjacent columns (one
// 16-byte access per row segment instead of two 8-byte ones: the gathers are
// bound by the number of vector memory instructions as much as by bytes).
template <typename T, int NB>
constexpr int cols_per_lane() { return (sizeof(T) == 4 && NB >= 2) ? 2 : 1; }

// CPL complex numbers of one lane: re[c], im[c] of columns jc + c
template <typename T, int CPL> struct Pack {
    T re[CPL], im[CPL];
};

typedef float fv4 __attribute__((ext_vector_type(4)));

template <typename T, int CPL, bool NT>
__device__ inline Pack<T, CPL> load_pack(const T *p) {  // p: interleaved re, im of CPL columns
    Pack<T, CPL> r;
    if constexpr (CPL == 2) {
        const fv4 v = NT ? __builtin_nontemporal_load(reinterpret_cast<const fv4 *>(p))
                         : *reinterpret_cast<const fv4 *>(p);
        r.re[0] = v.x;
        r.im[0] = v.y;
        r.re[1] = v.z;
        r.im[1] = v.w;
    } else {
        using VT = typename V2<T>::type;
        const VT v = NT ? ld_nt(reinterpret_cast<const VT *>(p)) : *reinterpret_cast<const VT *>(p);
        r.re[0] = v.x;
        r.im[0] = v.y;
    }
    return r;
}

template <typename T, int CPL>
__device__ inline void store_pack_nt(T *p, const Pack<T, CPL> &r) {
    if constexpr (CPL == 2) {
        fv4 v;
        v.x = r.re[0];
        v.y = r.im[0];
        v.z = r.re[1];
        v.w = r.im[1];
        __builtin_nontemporal_store(v, reinterpret_cast<fv4 *>(p));
    } else {
        using VT = typename V2<T>::type;
        st_nt(reinterpret_cast<VT *>(p), VT{r.re[0], r.im[0]});
    }
}

}  // namespace step_io
}  // namespace chebfd
