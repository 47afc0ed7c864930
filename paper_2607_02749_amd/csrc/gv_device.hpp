// gv_device.hpp -- device-side helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gv {

typedef uint64_t u64;

template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    cx<R> o;
    o.re = a.re * b.re - a.im * b.im;
    o.im = a.re * b.im + a.im * b.re;
    return o;
}

// State-vector loads and stores of the sweeps: every amplitude is read and
// written once per pass, so they carry the non-temporal (streaming) hint.
template <typename R>
__device__ __forceinline__ cx<R> ld_amp(const cx<R> *p)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load((const v2 *)p);
    return cx<R>{v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void st_amp(cx<R> *p, cx<R> a)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, (v2 *)p);
}

// k with a zero bit inserted at position q
__device__ __forceinline__ u64 insert_zero(u64 k, int q)
{
    const u64 lo = k & ((1ull << q) - 1);
    return ((k >> q) << (q + 1)) | lo;
}

// Sum of v over the block, in a fixed order (wave64 shuffles, then the waves
// in index order).  Valid in thread 0.  `sh` holds >= blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    // blocks of fewer than 64 threads fill part of a wave: skip the shifts
    // that would read the missing lanes
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        if (o < (int)blockDim.x) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += sh[i];
    }
    return s;
}

}  // namespace gv
