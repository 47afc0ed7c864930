// gv_stream.hip -- streaming kernels that measure what HBM delivers to
// plain, perfectly coalesced access patterns on this device: the practical
// ceiling the state-vector passes are compared against.
//
// Access patterns (one element = one vector of `width` bytes per lane):
//   READ   sum every element of src0 (written out only when it matches an
//          impossible value, so the loads are not dropped)
//   WRITE  store a constant to every element of dst
//   COPY   dst = src0
//   RMW    dst = src0 + dst   (read two streams, write one of them back:
//          the access pattern of a reverse pass that reads phi and lambda
//          and writes lambda)
//   TRIAD  dst = src0 + src1  (read two streams, write a third)
// Elements are taken in chunks of blockDim.x * U; lane t of a chunk touches
// elements t, t + blockDim.x, ..., so every instruction covers one
// contiguous run of 64 * width bytes.  A grid of 0 launches one block per
// chunk; a positive grid strides over the chunks.
// With tile_shift = s > 0 the element index e is placed at a permuted
// address, the layout a state-vector tile pass reads: its bits 0..3 stay,
// bits 4..11 move to bits s..s+7 and the others fill the rest in order, so
// every 16 consecutive lanes still read one contiguous run but the runs of
// one chunk lie 2^s elements apart.
#include "gv_device.hpp"
#include "gv_internal.hpp"

namespace gv {

namespace {

constexpr int kStreamBlock = 256;

// clang vector types: the non-temporal builtins take them directly
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int W>
struct Vec;
template <>
struct Vec<4> {
    typedef float T;
};
template <>
struct Vec<8> {
    typedef f32x2 T;
};
template <>
struct Vec<16> {
    typedef f32x4 T;
};

template <typename T, bool NT>
__device__ __forceinline__ T ld(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename T, bool NT>
__device__ __forceinline__ void st(T *p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__device__ __forceinline__ float first(float v) { return v; }
__device__ __forceinline__ float first(f32x2 v) { return v.x + v.y; }
__device__ __forceinline__ float first(f32x4 v) { return (v.x + v.y) + (v.z + v.w); }

__device__ __forceinline__ u64 place(u64 e, int s)
{
    if (s <= 0) return e;
    const u64 lo = e & 15, mid = (e >> 4) & 255, hi = e >> 12;
    const u64 hlo = hi & ((1ull << (s - 4)) - 1), hhi = hi >> (s - 4);
    return lo | (hlo << 4) | (mid << s) | (hhi << (s + 8));
}

template <int KIND, int W, int U, bool NT>
__global__ __launch_bounds__(kStreamBlock) void k_stream(void *dst_, const void *s0_,
                                                        const void *s1_, u64 nvec, int shift)
{
    typedef typename Vec<W>::T T;
    T *dst = (T *)dst_;
    const T *s0 = (const T *)s0_, *s1 = (const T *)s1_;
    const u64 per = (u64)kStreamBlock * U;
    const u64 nchunk = nvec / per;
    float acc = 0.f;
    for (u64 c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const u64 b = c * per + threadIdx.x;
        u64 o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) o[u] = place(b + (u64)u * kStreamBlock, shift);
        T a[U], e[U];
        if constexpr (KIND != STREAM_WRITE) {
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = ld<T, NT>(s0 + o[u]);
        }
        if constexpr (KIND == STREAM_RMW) {
#pragma unroll
            for (int u = 0; u < U; ++u) e[u] = ld<T, NT>(dst + o[u]);
        } else if constexpr (KIND == STREAM_TRIAD) {
#pragma unroll
            for (int u = 0; u < U; ++u) e[u] = ld<T, NT>(s1 + o[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            T *d = dst + o[u];
            if constexpr (KIND == STREAM_READ) acc += first(a[u]);
            else if constexpr (KIND == STREAM_WRITE) st<T, NT>(d, (T)((float)u));
            else if constexpr (KIND == STREAM_COPY) st<T, NT>(d, a[u]);
            else st<T, NT>(d, a[u] + e[u]);
        }
    }
    if constexpr (KIND == STREAM_READ)
        if (acc == 1.2345e-30f) dst[threadIdx.x] = (T)acc;
}

template <int KIND, int W, int U, bool NT>
hipError_t launch(void *dst, const void *s0, const void *s1, size_t bytes, int grid, int shift,
                  hipStream_t s)
{
    const u64 nvec = bytes / W;
    const u64 nchunk = nvec / ((u64)kStreamBlock * U);
    const u64 g = grid > 0 ? (u64)grid : nchunk;
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL((k_stream<KIND, W, U, NT>), dim3((unsigned)g), dim3(kStreamBlock), 0, s,
                       dst, s0, s1, nvec, shift);
    return hipGetLastError();
}

template <int KIND, int W, int U>
hipError_t by_nt(int nt, void *dst, const void *s0, const void *s1, size_t bytes, int grid,
                 int shift, hipStream_t s)
{
    return nt ? launch<KIND, W, U, true>(dst, s0, s1, bytes, grid, shift, s)
              : launch<KIND, W, U, false>(dst, s0, s1, bytes, grid, shift, s);
}

template <int KIND, int W>
hipError_t by_unroll(int unroll, int nt, void *dst, const void *s0, const void *s1, size_t bytes,
                     int grid, int shift, hipStream_t s)
{
    switch (unroll) {
    case 1: return by_nt<KIND, W, 1>(nt, dst, s0, s1, bytes, grid, shift, s);
    case 2: return by_nt<KIND, W, 2>(nt, dst, s0, s1, bytes, grid, shift, s);
    case 4: return by_nt<KIND, W, 4>(nt, dst, s0, s1, bytes, grid, shift, s);
    case 8: return by_nt<KIND, W, 8>(nt, dst, s0, s1, bytes, grid, shift, s);
    default: return by_nt<KIND, W, 16>(nt, dst, s0, s1, bytes, grid, shift, s);
    }
}

template <int KIND>
hipError_t by_width(int width, int unroll, int nt, void *dst, const void *s0, const void *s1,
                    size_t bytes, int grid, int shift, hipStream_t s)
{
    switch (width) {
    case 4: return by_unroll<KIND, 4>(unroll, nt, dst, s0, s1, bytes, grid, shift, s);
    case 8: return by_unroll<KIND, 8>(unroll, nt, dst, s0, s1, bytes, grid, shift, s);
    default: return by_unroll<KIND, 16>(unroll, nt, dst, s0, s1, bytes, grid, shift, s);
    }
}

}  // namespace

hipError_t stream_probe(int kind, int width, int unroll, int nt, void *dst, const void *s0,
                        const void *s1, size_t bytes, int grid, int shift, hipStream_t s)
{
    switch (kind) {
    case STREAM_READ: return by_width<STREAM_READ>(width, unroll, nt, dst, s0, s1, bytes, grid, shift, s);
    case STREAM_WRITE: return by_width<STREAM_WRITE>(width, unroll, nt, dst, s0, s1, bytes, grid, shift, s);
    case STREAM_COPY: return by_width<STREAM_COPY>(width, unroll, nt, dst, s0, s1, bytes, grid, shift, s);
    case STREAM_RMW: return by_width<STREAM_RMW>(width, unroll, nt, dst, s0, s1, bytes, grid, shift, s);
    default: return by_width<STREAM_TRIAD>(width, unroll, nt, dst, s0, s1, bytes, grid, shift, s);
    }
}

}  // namespace gv
