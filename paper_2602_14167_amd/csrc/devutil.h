// Device-side helpers shared by the tiled kernels: address-space views,
// uniform job lookup and a wave-wide float64 sum.
//
// Plan descriptors (jobs, passes, phases, ops, op matrices) are the same for
// every lane of a wave.  Reading them through generic pointers makes the
// compiler treat the loaded values as per-lane (a generic pointer may point
// into per-lane scratch), so every branch on an op field becomes an
// exec-masked branch and every gate's register block is copied at the join.
// Reading them through constant-address-space pointers yields scalar loads,
// uniform values in scalar registers and scalar branches.
#pragma once

#include "kernels.h"

namespace tcng {

// (the host pass of a HIP compile only sees the kernels' signatures; plain
// pointers keep it from checking device-only address-space conversions)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T>
using cptr = const T*;
template <typename T>
using gptr = T*;
#endif

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)(p);
}
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
    return (gptr<T>)(p);
}
template <typename T>
__device__ __forceinline__ gptr<const T> as_global(const T* p) {
    return (gptr<const T>)(p);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// block -> (job, block index inside the job); a single job travels by value
__device__ __forceinline__ Job load_job(const JobList& jl, const Job& single, int64_t blk, int64_t& local) {
    if (!jl.jobs) {
        local = blk;
        return single;
    }
    cptr<int64_t> prefix = as_const(jl.prefix);
    int lo = 0, hi = jl.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    local = blk - prefix[lo];
    return as_const(jl.jobs)[lo];
}

// v + (v of the DPP source lane); lanes of rows outside ROWMASK add zero
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_add(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROWMASK, 0xF, false);
    return v + __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// sum over the 64 lanes of a wave, returned uniformly (fixed order, so the
// result does not depend on scheduling): pairs and quads by quad
// permutations, 8 and 16 lanes by half-row and row mirrors, then rows 0+1 and
// 2+3 by the row-15 broadcast and all four rows by the lane-31 broadcast,
// which leaves the total in lane 63.
__device__ __forceinline__ double wave_sum(double v) {
    v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141, 0xF>(v);   // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);   // row_mirror
    v = dpp_add<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b), 63);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), 63);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// the same for float: v + (v of the DPP source lane)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_add(float v) {
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}

// float sum over the 64 lanes of a wave in the same fixed order, returned uniformly
__device__ __forceinline__ float wave_sum(float v) {
    v = dpp_add<0xB1, 0xF>(v);
    v = dpp_add<0x4E, 0xF>(v);
    v = dpp_add<0x141, 0xF>(v);
    v = dpp_add<0x140, 0xF>(v);
    v = dpp_add<0x142, 0xA>(v);
    v = dpp_add<0x143, 0xC>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

}  // namespace tcng
