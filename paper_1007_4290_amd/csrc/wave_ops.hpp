// Wavefront (64-lane) reductions built on DPP lane moves.
//
// A DPP move is a modifier on an ordinary VALU instruction, so a reduction
// step costs a few cycles instead of the ~100-cycle round trip of the LDS
// crossbar (ds_bpermute / ds_swizzle) that __shfl uses.  The idiom: row_shr
// by 1, 2, 4, 8 builds inclusive prefix sums inside each row of 16 lanes;
// row_bcast:15 and row_bcast:31 carry the row totals upward, leaving the
// wave total in lane 63, which v_readlane broadcasts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "cplx.hpp"

namespace wops {

enum : int {
    QP_XOR1 = 0xB1,            // quad_perm [1, 0, 3, 2]
    QP_XOR2 = 0x4E,            // quad_perm [2, 3, 0, 1]
    ROW_MIRROR = 0x140,        // lane i of a row of 16 reads lane 15 - i
    ROW_HALF_MIRROR = 0x141,   // lane i of a half row reads lane 7 - i
    ROW_SHR1 = 0x111,
    ROW_SHR2 = 0x112,
    ROW_SHR4 = 0x114,
    ROW_SHR8 = 0x118,
    ROW_BCAST15 = 0x142,
    ROW_BCAST31 = 0x143,
};

// DPP move of a 32-bit value; lanes whose source is outside the pattern
// (or masked rows) receive `fill`.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ int dpp_i32(int v, int fill) {
    return __builtin_amdgcn_update_dpp(fill, v, CTRL, ROWMASK, 0xf, false);
}

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ float dpp(float v, float fill) {
    return __int_as_float(dpp_i32<CTRL, ROWMASK>(__float_as_int(v), __float_as_int(fill)));
}

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp(double v, double fill) {
    const int64_t b = __double_as_longlong(v);
    const int64_t f = __double_as_longlong(fill);
    const int lo = dpp_i32<CTRL, ROWMASK>((int)(b & 0xffffffffll), (int)(f & 0xffffffffll));
    const int hi = dpp_i32<CTRL, ROWMASK>((int)(b >> 32), (int)(f >> 32));
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

template <typename T>
__device__ __forceinline__ T readlane63(T v);
template <>
__device__ __forceinline__ float readlane63<float>(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
template <>
__device__ __forceinline__ double readlane63<double>(double v) {
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int readlane63_i(int v) { return __builtin_amdgcn_readlane(v, 63); }

// Sum over all 64 lanes, returned to every lane.  Every lane must call it.
template <typename T>
__device__ __forceinline__ T sum(T v) {
    v += dpp<ROW_SHR1>(v, T(0));
    v += dpp<ROW_SHR2>(v, T(0));
    v += dpp<ROW_SHR4>(v, T(0));
    v += dpp<ROW_SHR8>(v, T(0));
    v += dpp<ROW_BCAST15, 0xa>(v, T(0));
    v += dpp<ROW_BCAST31, 0xc>(v, T(0));
    return readlane63(v);
}

template <typename T>
__device__ __forceinline__ cpx<T> sum(cpx<T> v) {
    return mk<T>(sum(v.re), sum(v.im));
}

// Sums over aligned segments of SEG lanes (SEG = 2, 4, 8 or 16); the segment
// total lands in the LAST lane of each segment (other lanes hold partial
// prefixes).  Every lane must call it.
template <int SEG, typename T>
__device__ __forceinline__ T seg_sum_last(T v) {
    static_assert(SEG == 2 || SEG == 4 || SEG == 8 || SEG == 16, "segment of 2..16 lanes");
    v += dpp<ROW_SHR1>(v, T(0));
    if constexpr (SEG >= 4) v += dpp<ROW_SHR2>(v, T(0));
    if constexpr (SEG >= 8) v += dpp<ROW_SHR4>(v, T(0));
    if constexpr (SEG >= 16) v += dpp<ROW_SHR8>(v, T(0));
    return v;
}

// Sum over aligned groups of G consecutive lanes (G = 1, 2, 4, ..., 64; the
// same on every lane), returned to every lane of the group.  The butterfly is
// symmetric, so all lanes of a group hold bitwise the same total.  Every lane
// must call it.
template <typename T>
__device__ __forceinline__ T gsum(T v, int G) {
    // the DPP steps always run and are selected away above the group size
    // (no branches); the cross-row steps use the LDS crossbar and are rare
    T t = dpp<QP_XOR1>(v, T(0));
    v += G >= 2 ? t : T(0);
    t = dpp<QP_XOR2>(v, T(0));
    v += G >= 4 ? t : T(0);
    t = dpp<ROW_HALF_MIRROR>(v, T(0));
    v += G >= 8 ? t : T(0);
    t = dpp<ROW_MIRROR>(v, T(0));
    v += G >= 16 ? t : T(0);
    if (G >= 32) {
        v += __shfl_xor(v, 16, 64);
        if (G >= 64) v += __shfl_xor(v, 32, 64);
    }
    return v;
}

template <typename T>
__device__ __forceinline__ cpx<T> gsum(cpx<T> v, int G) {
    return mk<T>(gsum(v.re, G), gsum(v.im, G));
}

// As gsum with a compile-time group size: no selects or branches.
template <int G, typename T>
__device__ __forceinline__ T gsum_ct(T v) {
    if constexpr (G >= 2) v += dpp<QP_XOR1>(v, T(0));
    if constexpr (G >= 4) v += dpp<QP_XOR2>(v, T(0));
    if constexpr (G >= 8) v += dpp<ROW_HALF_MIRROR>(v, T(0));
    if constexpr (G >= 16) v += dpp<ROW_MIRROR>(v, T(0));
    if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
    if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

template <int G, typename T>
__device__ __forceinline__ cpx<T> gsum_ct(cpx<T> v) {
    return mk<T>(gsum_ct<G>(v.re), gsum_ct<G>(v.im));
}

__device__ __forceinline__ int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Maximum of v over all lanes with the lowest index among ties; both
// returned to every lane.
template <typename T>
__device__ __forceinline__ void argmax(T& v, int& idx) {
    const T lo = -__builtin_huge_val();
#define WOPS_STEP(CTRL, RM)                                                                  \
    {                                                                                        \
        const T ov = dpp<CTRL, RM>(v, lo);                                                   \
        const int oi = dpp_i32<CTRL, RM>(idx, 0x7fffffff);                                   \
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }                           \
    }
    WOPS_STEP(ROW_SHR1, 0xf)
    WOPS_STEP(ROW_SHR2, 0xf)
    WOPS_STEP(ROW_SHR4, 0xf)
    WOPS_STEP(ROW_SHR8, 0xf)
    WOPS_STEP(ROW_BCAST15, 0xa)
    WOPS_STEP(ROW_BCAST31, 0xc)
#undef WOPS_STEP
    v = readlane63(v);
    idx = readlane63_i(idx);
}

// argmax as above when every lane of each aligned group of G lanes (G = 8, 16
// or 32) holds the same candidate: only the steps that combine groups run.
template <int G, typename T>
__device__ __forceinline__ void argmax_groups(T& v, int& idx) {
    const T lo = -__builtin_huge_val();
#define WOPS_STEP(CTRL, RM)                                                                  \
    {                                                                                        \
        const T ov = dpp<CTRL, RM>(v, lo);                                                   \
        const int oi = dpp_i32<CTRL, RM>(idx, 0x7fffffff);                                   \
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }                           \
    }
    if constexpr (G <= 8) WOPS_STEP(ROW_MIRROR, 0xf)
    if constexpr (G <= 16) WOPS_STEP(ROW_BCAST15, 0xa)
    WOPS_STEP(ROW_BCAST31, 0xc)
#undef WOPS_STEP
    v = readlane63(v);
    idx = readlane63_i(idx);
}

// Unsigned maximum over all 64 lanes, returned to every lane.
__device__ __forceinline__ unsigned umax(unsigned v) {
    int x = (int)v;
#define WOPS_UMAX(CTRL, RM) x = (int)max((unsigned)x, (unsigned)dpp_i32<CTRL, RM>(x, 0));
    WOPS_UMAX(ROW_SHR1, 0xf)
    WOPS_UMAX(ROW_SHR2, 0xf)
    WOPS_UMAX(ROW_SHR4, 0xf)
    WOPS_UMAX(ROW_SHR8, 0xf)
    WOPS_UMAX(ROW_BCAST15, 0xa)
    WOPS_UMAX(ROW_BCAST31, 0xc)
#undef WOPS_UMAX
    return (unsigned)readlane63_i(x);
}

// Pivot search on non-negative keys: the lane of largest key (ties: lowest
// idx, 0 <= idx < 64) among the lanes with eligible set.  The key and index
// are packed into one word (top bit: eligible; then the float key without its
// lowest mantissa bits; then 63 - idx), so the search is a single unsigned
// maximum.  Keys closer than about 2^-17 relative count as ties.  Returns the
// winning idx, or -1 when no lane is eligible.
__device__ __forceinline__ int argmax_nonneg(float key, int idx, bool eligible) {
    const unsigned kb = (__float_as_uint(key > 0.0f ? key : 0.0f) >> 1) & ~63u;
    const unsigned u = eligible ? (0x80000000u | kb | (unsigned)(63 - idx)) : 0u;
    const unsigned m = umax(u);
    return (m & 0x80000000u) ? 63 - (int)(m & 63u) : -1;
}

}  // namespace wops
