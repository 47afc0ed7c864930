// gv_ham.hip -- Hamiltonian side of the hot path (Eq. 6, Eq. 4):
//   * the FP64 diagonal of the Z-only part, built once per Hamiltonian by an
//     in-place fast Walsh-Hadamard transform of the coefficient histogram:
//     D_i = sum_z h[z] (-1)^{popcount(i & z)}, h[z] = sum of c_k with z_k = z;
//   * the energy reduction E = sum_i D_i |psi_i|^2 (FP64) with lam = D psi;
//   * the off-diagonal terms one by one: lam += c P psi, E += <psi|c P psi>;
//   * fixed-order reductions of per-block partials.
#include "gv_device.hpp"
#include "gv_internal.hpp"

namespace gv {

namespace {

constexpr int kBlock = 256;

__global__ void k_fill_zero(double *d, u64 count)
{
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < count;
         i += (u64)gridDim.x * blockDim.x)
        d[i] = 0.0;
}

// h[z_k] = c_k; the z_k are distinct (merged on the host), so no two threads
// write the same entry.
__global__ void k_scatter(double *h, const uint64_t *z, const double *c, int64_t m)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x)
        h[z[k]] = c[k];
}

__device__ __forceinline__ u64 deposit(u64 v, u64 mask)
{
    u64 out = 0;
    while (mask) {
        const u64 low = mask & (~mask + 1);
        if (v & 1) out |= low;
        v >>= 1;
        mask &= mask - 1;
    }
    return out;
}

struct WhtPass {
    int K;
    int8_t pos[kMaxTileBits];
    uint32_t active;
    u64 outside;   // mask of the bits not in the tile
    u64 ntiles;
};

// One tile pass of the transform: 2^K entries whose index bits pos[0..K) vary
// go through LDS; butterflies (a, b) -> (a + b, a - b) on the active bits.
__global__ __launch_bounds__(kBlock) void k_wht_pass(double *d, WhtPass w)
{
    __shared__ double t[1 << kMaxTileBits];
    const int tile_n = 1 << w.K;
    for (u64 tile = blockIdx.x; tile < w.ntiles; tile += gridDim.x) {
        const u64 base = deposit(tile, w.outside);
        __syncthreads();
        for (int u = threadIdx.x; u < tile_n; u += blockDim.x) {
            u64 off = 0;
            for (int j = 0; j < w.K; ++j) off |= (u64)((u >> j) & 1) << w.pos[j];
            t[u] = d[base | off];
        }
        __syncthreads();
        for (int j = 0; j < w.K; ++j) {
            if (!((w.active >> j) & 1)) continue;
            for (int k = threadIdx.x; k < tile_n / 2; k += blockDim.x) {
                const int lo = k & ((1 << j) - 1);
                const int i0 = ((k >> j) << (j + 1)) | lo, i1 = i0 | (1 << j);
                const double a = t[i0], b = t[i1];
                t[i0] = a + b;
                t[i1] = a - b;
            }
            __syncthreads();
        }
        for (int u = threadIdx.x; u < tile_n; u += blockDim.x) {
            u64 off = 0;
            for (int j = 0; j < w.K; ++j) off |= (u64)((u >> j) & 1) << w.pos[j];
            d[base | off] = t[u];
        }
    }
}

// The same pass for 12-bit tiles whose tile bits 4..7 and 8..11 sit at
// consecutive index positions: 256 threads hold 16 values each, and the
// butterflies of a tile bit run in registers while it is one of the
// thread's four register bits.  The register bits go 8..11 (load), 0..3,
// 4..7 (store), switched through LDS (padded one slot per 16 against bank
// conflicts).
__device__ __forceinline__ int wht_slot(int t, int r, int l)
{
    const int u = (t & ((1 << l) - 1)) | (r << l) | ((t >> l) << (l + 4));
    return u + (u >> 4);
}

__device__ __forceinline__ void wht_bfly(double (&v)[16], uint32_t m)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!((m >> k) & 1)) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r & (1 << k)) continue;
            const double a = v[r], b = v[r | (1 << k)];
            v[r] = a + b;
            v[r | (1 << k)] = a - b;
        }
    }
}

template <int LF, int LT>
__device__ __forceinline__ void wht_exchange(double (&v)[16], double *lds, int t)
{
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[wht_slot(t, r, LF)] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = lds[wht_slot(t, r, LT)];
}

__global__ __launch_bounds__(256) void k_wht_reg(double *d, WhtPass w)
{
    __shared__ double lds[4096 + 256];
    const int t = threadIdx.x;
    u64 toff0 = 0, toff2 = 0;
    for (int j = 0, tb = 0; j < 12; ++j)
        if (j < 8) toff0 |= (u64)((t >> tb++) & 1) << w.pos[j];
    for (int j = 0, tb = 0; j < 12; ++j)
        if (j < 4 || j >= 8) toff2 |= (u64)((t >> tb++) & 1) << w.pos[j];
    const int sh0 = w.pos[8], sh2 = w.pos[4];
    for (u64 tile = blockIdx.x; tile < w.ntiles; tile += gridDim.x) {
        const u64 base = deposit(tile, w.outside);
        double v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = d[base | toff0 | ((u64)r << sh0)];
        wht_bfly(v, w.active >> 8);
        wht_exchange<8, 0>(v, lds, t);
        wht_bfly(v, w.active & 0xf);
        wht_exchange<0, 4>(v, lds, t);
        wht_bfly(v, (w.active >> 4) & 0xf);
#pragma unroll
        for (int r = 0; r < 16; ++r) d[base | toff2 | ((u64)r << sh2)] = v[r];
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_energy_diag(const cx<R> *psi, const double *diag,
                                                         cx<R> *lam, u64 dim, double *epart,
                                                         int grid)
{
    __shared__ double sh[kBlock / 64];
    double acc = 0.0;
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x) {
        const cx<R> v = psi[i];
        const double dd = diag[i];
        acc += dd * ((double)v.re * v.re + (double)v.im * v.im);
        if (lam) {
            cx<R> o;
            o.re = (R)dd * v.re;
            o.im = (R)dd * v.im;
            lam[i] = o;
        }
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        epart[blockIdx.x] = tot;
        epart[grid + blockIdx.x] = 0.0;
    }
}

// lam_i += c i^{|x&z|} (-1)^{popcount((i^x)&z)} psi_{i^x} for one term;
// energy partials (re, im) of conj(psi_i) times that value are added.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_offdiag_term(const cx<R> *psi, cx<R> *lam, u64 dim,
                                                          u64 x, u64 z, double c, double *epart,
                                                          int grid)
{
    __shared__ double sh[kBlock / 64];
    const int ph = __popcll(x & z) & 3;
    double accr = 0.0, acci = 0.0;
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x) {
        const u64 j = i ^ x;
        const cx<R> pj = psi[j];
        const double sg = (__popcll(j & z) & 1) ? -c : c;
        double vr, vi;  // sg * i^ph * psi_j
        switch (ph) {
        case 0: vr = sg * pj.re; vi = sg * pj.im; break;
        case 1: vr = -sg * pj.im; vi = sg * pj.re; break;
        case 2: vr = -sg * pj.re; vi = -sg * pj.im; break;
        default: vr = sg * pj.im; vi = -sg * pj.re; break;
        }
        const cx<R> pi = psi[i];
        accr += (double)pi.re * vr + (double)pi.im * vi;
        acci += (double)pi.re * vi - (double)pi.im * vr;
        if (lam) {
            cx<R> o = lam[i];
            o.re += (R)vr;
            o.im += (R)vi;
            lam[i] = o;
        }
    }
    const double tr = block_sum(accr, sh);
    const double ti = block_sum(acci, sh);
    if (threadIdx.x == 0) {
        epart[blockIdx.x] += tr;
        epart[grid + blockIdx.x] += ti;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_rows(const double *part, int64_t rows, int cols,
                                                         const uint8_t *mask, double *out)
{
    __shared__ double sh[kBlock / 64];
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        double acc = 0.0;
        for (int c = threadIdx.x; c < cols; c += blockDim.x) acc += part[r * cols + c];
        const double tot = block_sum(acc, sh);
        if (threadIdx.x == 0) out[r] = (mask && !mask[r]) ? 0.0 : tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_energy(const double *epart, int grid,
                                                           double *energy)
{
    __shared__ double sh[kBlock / 64];
    double a = 0.0, b = 0.0;
    for (int c = threadIdx.x; c < grid; c += blockDim.x) {
        a += epart[c];
        b += epart[grid + c];
    }
    const double ta = block_sum(a, sh);
    const double tb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        energy[0] = ta;
        energy[1] = tb;
    }
}

inline int grid_for(u64 work, int cap)
{
    u64 b = (work + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (int)(b < (u64)cap ? b : cap);
}

}  // namespace

hipError_t fill_zero_f64(double *d, u64 count, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(count, 4096)), dim3(kBlock), 0, s, d, count);
    return hipGetLastError();
}

hipError_t scatter_coeffs(double *h, const uint64_t *z, const double *c, int64_t m, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for((u64)m, 1024)), dim3(kBlock), 0, s, h, z, c, m);
    return hipGetLastError();
}

hipError_t fwht_inplace(double *d, int n, hipStream_t s)
{
    const int K = n < kMaxTileBits ? n : kMaxTileBits;
    TilePlan plan;
    if (!make_tile_plan(n, K, K < 4 ? K : 4, &plan)) return hipErrorInvalidValue;
    for (int p = 0; p < plan.npass; ++p) {
        WhtPass w;
        w.K = K;
        u64 inside = 0;
        for (int j = 0; j < K; ++j) {
            w.pos[j] = plan.pass[p].pos[j];
            inside |= 1ull << w.pos[j];
        }
        w.active = plan.pass[p].active;
        w.outside = ((n >= 64) ? ~0ull : ((1ull << n) - 1)) & ~inside;
        w.ntiles = 1ull << (n - K);
        bool reg = K == 12;
        for (int k = 1; k < 4; ++k)
            reg = reg && w.pos[4 + k] == w.pos[4] + k && w.pos[8 + k] == w.pos[8] + k;
        if (reg) {
            const int grid = (int)(w.ntiles < 2048 ? w.ntiles : 2048);
            hipLaunchKernelGGL(k_wht_reg, dim3(grid), dim3(256), 0, s, d, w);
        } else {
            const int grid = (int)(w.ntiles < 8192 ? w.ntiles : 8192);
            hipLaunchKernelGGL(k_wht_pass, dim3(grid), dim3(kBlock), 0, s, d, w);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t energy_diag(int prec, const void *psi, const double *diag, void *lam, int n,
                       double *epart, int grid, hipStream_t s)
{
    const u64 dim = 1ull << n;
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_energy_diag<float>, dim3(grid), dim3(kBlock), 0, s,
                           (const cx<float> *)psi, diag, (cx<float> *)lam, dim, epart, grid);
    else
        hipLaunchKernelGGL(k_energy_diag<double>, dim3(grid), dim3(kBlock), 0, s,
                           (const cx<double> *)psi, diag, (cx<double> *)lam, dim, epart, grid);
    return hipGetLastError();
}

hipError_t energy_offdiag_terms(int prec, const void *psi, void *lam, int n, int64_t m,
                                const uint64_t *ox, const uint64_t *oz, const double *oc,
                                double *epart, int grid, hipStream_t s)
{
    const u64 dim = 1ull << n;
    for (int64_t k = 0; k < m; ++k) {
        if (prec == GV_C64)
            hipLaunchKernelGGL(k_offdiag_term<float>, dim3(grid), dim3(kBlock), 0, s,
                               (const cx<float> *)psi, (cx<float> *)lam, dim, ox[k], oz[k], oc[k],
                               epart, grid);
        else
            hipLaunchKernelGGL(k_offdiag_term<double>, dim3(grid), dim3(kBlock), 0, s,
                               (const cx<double> *)psi, (cx<double> *)lam, dim, ox[k], oz[k],
                               oc[k], epart, grid);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t reduce_rows(const double *part, int64_t rows, int cols, const uint8_t *mask,
                       double *out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    const int grid = (int)(rows < 4096 ? rows : 4096);
    hipLaunchKernelGGL(k_reduce_rows, dim3(grid), dim3(kBlock), 0, s, part, rows, cols, mask, out);
    return hipGetLastError();
}

hipError_t reduce_energy(const double *epart, int grid, double *energy, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(kBlock), 0, s, epart, grid, energy);
    return hipGetLastError();
}

hipError_t copy_vector(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

}  // namespace gv
