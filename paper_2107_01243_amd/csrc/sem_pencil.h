// sem_pencil.h -- LDS helpers shared by the element kernels (pencil layout: the
// lanes of one element own lines of points and exchange them through an LDS copy
// of the element).
#pragma once
#include <hip/hip_runtime.h>

namespace sem {

// Synchronise the lanes that share one element's LDS buffers.  When whole elements
// fit inside one wave64 (lx*lx divides 64, e.g. lx = 8: one element per wave) no
// other wave touches those buffers, and LDS operations of one wave complete in
// order, so a wave-level barrier (a compiler fence, no s_barrier) suffices.
template <int LX>
__device__ __forceinline__ void esync()
{
    if constexpr (64 % (LX * LX) == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// The same for a workgroup of NT lanes that holds a single element: a wave-level
// barrier when the workgroup is one wave, else a workgroup barrier.
template <int NT>
__device__ __forceinline__ void bsync()
{
    if constexpr (NT <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// LDS index of point (i, j, k) inside one element buffer of LX^3 points (row
// stride LX + 1, so the three pencil access patterns are free of bank conflicts).
template <int LX>
__device__ __forceinline__ int lidx(int i, int j, int k) { return i + (LX + 1) * (j + LX * k); }

}  // namespace sem
