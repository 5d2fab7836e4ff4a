// svf_device.h -- device-side helpers shared by the gfx950 kernel files
// (svf_kernels.hip: scale map and pre-integration; svf_fd.hip: finite difference).
#pragma once

#include <hip/hip_runtime.h>

#include "svf_internal.h"

namespace svf {
namespace {

constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kRsqrt2 = 0.70710678118654752440;
constexpr int kBufWord3 = 0x00020000;   // buffer resource word 3 for gfx9-family raw loads

// ---------------------------------------------------------------------------
// A descriptor read from a device table (batched launches) as wave-uniform values.
// The table is ordinary read-write memory, so the compiler reads it with vector
// loads and would treat everything derived from it (buffer resources above all)
// as varying per lane: each buffer access would then be wrapped in a loop over the
// distinct lane values.  One readfirstlane per dword restores the scalar form that
// a descriptor passed as a kernel argument has.
// ---------------------------------------------------------------------------
template <class S>
__device__ __forceinline__ S uniform_copy(const S *p)
{
    static_assert(sizeof(S) % 4 == 0, "whole dwords");
    uint32_t w[sizeof(S) / 4];
    __builtin_memcpy(w, p, sizeof(S));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(S) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    S v;
    __builtin_memcpy(&v, w, sizeof(S));
    return v;
}

// A load (store) through a pointer read from a device table, as a global one: the
// compiler cannot tell what such a pointer addresses and would issue a flat load,
// which also counts against the LDS wait counter (so every LDS barrier would wait
// for it).  Pointers that arrive as kernel arguments are known global already.
// four floats as a native vector: loads and stores of it are single accesses (the
// HIP float4 class would go through its member operators and a generic pointer)
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T load_global(const T *p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(1))) T *)p;
#else
    return *p;
#endif
}

template <class T>
__device__ __forceinline__ void store_global(T *p, const T &v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    *(__attribute__((address_space(1))) T *)p = v;
#else
    *p = v;
#endif
}

// ---------------------------------------------------------------------------
// LDS-only work-group barrier: orders LDS accesses without waiting for global
// loads in flight, so the row sweep keeps its input prefetches across barriers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Tile geometry shared by the pre-integration and the finite difference.
// Tile t covers rows [ti T, ...) x cols [tj T, ...).  A pixel n with pass
// half-widths (R1, R2) reads lattice columns [n1 - R1 - 2, n1 + R1 + 1] and rows
// [n2 - R2 - 3, n2 + R2]: the taps n + tau - x_i span [-R - 1/2, R - 1/2] x
// [-R - 3/2, R - 3/2] and the ZP stencil adds one sample on each side of the
// nearest lattice point.  One sample of margin is added on every side.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Window window_of(const Job &J, int tile)
{
    const int ti = tile / J.ntc, tj = tile - ti * J.ntc;
    const int64_t r0 = (int64_t)ti * J.T, c0 = (int64_t)tj * J.T;
    const int64_t r1 = min(r0 + (int64_t)J.T, J.H), c1 = min(c0 + (int64_t)J.T, J.W);
    const float rx = J.tstat[tile].rx * J.inv_sqrt_m;
    const float ry = J.tstat[tile].ry * J.inv_sqrt_m;
    const int hx = min(J.cap, (int)ceilf(rx * 1.000001f));
    const int hy = min(J.cap, (int)ceilf(ry * 1.000001f));
    Window w;
    w.c0 = c0 - hx - 3;
    w.w = (int)(c1 - c0) + 2 * hx + 5;
    // even origin and width (at most T + 2 cap + 6): rows of the window start
    // 16-byte aligned, and pairs of input columns from even columns are 8-byte aligned
    if (w.c0 & 1) {
        w.c0 -= 1;
        w.w += 1;
    }
    w.w += w.w & 1;
    w.r0 = r0 - hy - 4;
    w.h = (int)(r1 - r0) + 2 * hy + 5;
    return w;
}

// XCD-aware block order: consecutive hardware work-group ids go round-robin over
// the 8 XCDs; remap so that each XCD receives one contiguous range of logical
// blocks (the blocks of a tile share its window in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int pid, int nblocks)
{
    const int per = nblocks >> 3;   // nblocks is a multiple of 8
    return (pid & 7) * per + (pid >> 3);
}

__device__ __forceinline__ int find_job(const Job *jobs, int n, int idx, int which)
{
    // largest j with base_j <= idx (bases ascending)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int b = which == 0 ? jobs[mid].tile_base : which == 1 ? jobs[mid].blk_base : jobs[mid].smap_base;
        if (b <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace
}  // namespace svf
