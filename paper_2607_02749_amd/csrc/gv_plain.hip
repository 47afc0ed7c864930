// gv_plain.hip -- the plain engine: one kernel per gate (Eq. 7 gates, CZ /
// CNOT entanglers) and one kernel per reverse-sweep step.  It is the direct
// GPU form of the method and the baseline the fused engine is measured
// against.  Every reduction is FP64 with a fixed order.
#include "gv_device.hpp"
#include "gv_internal.hpp"

namespace gv {

namespace {

inline int grid_for(u64 work)
{
    u64 b = (work + kPlainBlock - 1) / kPlainBlock;
    return (int)(b < (u64)kPlainGrid ? (b ? b : 1) : kPlainGrid);
}

template <typename R>
__global__ void k_zero_state(cx<R> *psi, u64 dim)
{
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x) {
        cx<R> v;
        v.re = i == 0 ? R(1) : R(0);
        v.im = R(0);
        psi[i] = v;
    }
}

// RY(t) on qubit q: (a, b) -> (c a - s b, s a + c b), c = cos t/2, s = sin t/2
template <typename R>
__global__ void k_ry(cx<R> *psi, int n, int q, const double *theta, int64_t p, int inv)
{
    double t = theta[p];
    if (inv) t = -t;
    double sd, cd;
    sincos(0.5 * t, &sd, &cd);
    const R c = (R)cd, s = (R)sd;
    const u64 half = 1ull << (n - 1), bit = 1ull << q;
    for (u64 k = blockIdx.x * (u64)blockDim.x + threadIdx.x; k < half;
         k += (u64)gridDim.x * blockDim.x) {
        const u64 i = insert_zero(k, q), j = i | bit;
        const cx<R> a = psi[i], b = psi[j];
        cx<R> a2, b2;
        a2.re = c * a.re - s * b.re;
        a2.im = c * a.im - s * b.im;
        b2.re = s * a.re + c * b.re;
        b2.im = s * a.im + c * b.im;
        psi[i] = a2;
        psi[j] = b2;
    }
}

// RZ(t) on qubit q: bit 0 times exp(-i t/2), bit 1 times exp(+i t/2)
template <typename R>
__global__ void k_rz(cx<R> *psi, int n, int q, const double *theta, int64_t p, int inv)
{
    double t = theta[p];
    if (inv) t = -t;
    double sd, cd;
    sincos(0.5 * t, &sd, &cd);
    cx<R> e0, e1;
    e0.re = (R)cd;
    e0.im = (R)-sd;
    e1.re = (R)cd;
    e1.im = (R)sd;
    const u64 dim = 1ull << n, bit = 1ull << q;
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x)
        psi[i] = cmul(psi[i], (i & bit) ? e1 : e0);
}

template <typename R>
__global__ void k_cz(cx<R> *psi, int n, int a, int b)
{
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const u64 quarter = 1ull << (n - 2), set = (1ull << a) | (1ull << b);
    for (u64 k = blockIdx.x * (u64)blockDim.x + threadIdx.x; k < quarter;
         k += (u64)gridDim.x * blockDim.x) {
        const u64 i = insert_zero(insert_zero(k, lo), hi) | set;
        cx<R> v = psi[i];
        v.re = -v.re;
        v.im = -v.im;
        psi[i] = v;
    }
}

// CNOT(ctl -> tgt): swap the pairs with control bit 1
template <typename R>
__global__ void k_cnot(cx<R> *psi, int n, int ctl, int tgt)
{
    const int lo = ctl < tgt ? ctl : tgt, hi = ctl < tgt ? tgt : ctl;
    const u64 quarter = 1ull << (n - 2);
    const u64 cb = 1ull << ctl, tb = 1ull << tgt;
    for (u64 k = blockIdx.x * (u64)blockDim.x + threadIdx.x; k < quarter;
         k += (u64)gridDim.x * blockDim.x) {
        const u64 i = insert_zero(insert_zero(k, lo), hi) | cb, j = i | tb;
        const cx<R> t = psi[i];
        psi[i] = psi[j];
        psi[j] = t;
    }
}

// Reverse-sweep step of RY on qubit q: partial of Im<lam|Y_q|phi>, then
// RY(-t) on both vectors.  part_row[blockIdx.x] receives the block sum.
template <typename R>
__global__ void k_adj_ry(cx<R> *phi, cx<R> *lam, int n, int q, const double *theta, int64_t p,
                         double *part_row)
{
    __shared__ double sh[kPlainBlock / 64];
    double sd, cd;
    sincos(-0.5 * theta[p], &sd, &cd);
    const R c = (R)cd, s = (R)sd;
    const u64 half = 1ull << (n - 1), bit = 1ull << q;
    double acc = 0.0;
    for (u64 k = blockIdx.x * (u64)blockDim.x + threadIdx.x; k < half;
         k += (u64)gridDim.x * blockDim.x) {
        const u64 i = insert_zero(k, q), j = i | bit;
        const cx<R> f0 = phi[i], f1 = phi[j], l0 = lam[i], l1 = lam[j];
        // Im<lam|Y|phi> over the pair = Re(conj(l1) f0) - Re(conj(l0) f1)
        acc += ((double)l1.re * f0.re + (double)l1.im * f0.im) -
               ((double)l0.re * f1.re + (double)l0.im * f1.im);
        cx<R> a, b;
        a.re = c * f0.re - s * f1.re;
        a.im = c * f0.im - s * f1.im;
        b.re = s * f0.re + c * f1.re;
        b.im = s * f0.im + c * f1.im;
        phi[i] = a;
        phi[j] = b;
        a.re = c * l0.re - s * l1.re;
        a.im = c * l0.im - s * l1.im;
        b.re = s * l0.re + c * l1.re;
        b.im = s * l0.im + c * l1.im;
        lam[i] = a;
        lam[j] = b;
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) part_row[blockIdx.x] = tot;
}

// Reverse-sweep step of RZ on qubit q: partial of Im<lam|Z_q|phi>, then
// RZ(-t) on both vectors.
template <typename R>
__global__ void k_adj_rz(cx<R> *phi, cx<R> *lam, int n, int q, const double *theta, int64_t p,
                         double *part_row)
{
    __shared__ double sh[kPlainBlock / 64];
    double sd, cd;
    sincos(0.5 * theta[p], &sd, &cd);
    // inverse: bit 0 times exp(+i t/2), bit 1 times exp(-i t/2)
    cx<R> e0, e1;
    e0.re = (R)cd;
    e0.im = (R)sd;
    e1.re = (R)cd;
    e1.im = (R)-sd;
    const u64 dim = 1ull << n, bit = 1ull << q;
    double acc = 0.0;
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x) {
        const cx<R> f = phi[i], l = lam[i];
        const double t = (double)l.re * f.im - (double)l.im * f.re;  // Im(conj(l) f)
        acc += (i & bit) ? -t : t;
        phi[i] = cmul(f, (i & bit) ? e1 : e0);
        lam[i] = cmul(l, (i & bit) ? e1 : e0);
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) part_row[blockIdx.x] = tot;
}

}  // namespace

template <typename R>
static inline cx<R> *C(void *p) { return (cx<R> *)p; }

hipError_t plain_set_zero_state(int prec, void *psi, int n, hipStream_t s)
{
    const u64 dim = 1ull << n;
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_zero_state<float>, dim3(grid_for(dim)), dim3(kPlainBlock), 0, s,
                           C<float>(psi), dim);
    else
        hipLaunchKernelGGL(k_zero_state<double>, dim3(grid_for(dim)), dim3(kPlainBlock), 0, s,
                           C<double>(psi), dim);
    return hipGetLastError();
}

hipError_t plain_ry(int prec, void *psi, int n, int q, const double *theta, int64_t p, int inv,
                    hipStream_t s)
{
    const int g = grid_for(1ull << (n - 1));
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_ry<float>, dim3(g), dim3(kPlainBlock), 0, s, C<float>(psi), n, q,
                           theta, p, inv);
    else
        hipLaunchKernelGGL(k_ry<double>, dim3(g), dim3(kPlainBlock), 0, s, C<double>(psi), n, q,
                           theta, p, inv);
    return hipGetLastError();
}

hipError_t plain_rz(int prec, void *psi, int n, int q, const double *theta, int64_t p, int inv,
                    hipStream_t s)
{
    const int g = grid_for(1ull << n);
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_rz<float>, dim3(g), dim3(kPlainBlock), 0, s, C<float>(psi), n, q,
                           theta, p, inv);
    else
        hipLaunchKernelGGL(k_rz<double>, dim3(g), dim3(kPlainBlock), 0, s, C<double>(psi), n, q,
                           theta, p, inv);
    return hipGetLastError();
}

hipError_t plain_cz(int prec, void *psi, int n, int a, int b, hipStream_t s)
{
    const int g = grid_for(1ull << (n - 2));
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_cz<float>, dim3(g), dim3(kPlainBlock), 0, s, C<float>(psi), n, a, b);
    else
        hipLaunchKernelGGL(k_cz<double>, dim3(g), dim3(kPlainBlock), 0, s, C<double>(psi), n, a,
                           b);
    return hipGetLastError();
}

hipError_t plain_cnot(int prec, void *psi, int n, int ctl, int tgt, hipStream_t s)
{
    const int g = grid_for(1ull << (n - 2));
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_cnot<float>, dim3(g), dim3(kPlainBlock), 0, s, C<float>(psi), n,
                           ctl, tgt);
    else
        hipLaunchKernelGGL(k_cnot<double>, dim3(g), dim3(kPlainBlock), 0, s, C<double>(psi), n,
                           ctl, tgt);
    return hipGetLastError();
}

hipError_t plain_adj_ry(int prec, void *phi, void *lam, int n, int q, const double *theta,
                        int64_t p, double *part_row, hipStream_t s)
{
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_adj_ry<float>, dim3(kPlainGrid), dim3(kPlainBlock), 0, s,
                           C<float>(phi), C<float>(lam), n, q, theta, p, part_row);
    else
        hipLaunchKernelGGL(k_adj_ry<double>, dim3(kPlainGrid), dim3(kPlainBlock), 0, s,
                           C<double>(phi), C<double>(lam), n, q, theta, p, part_row);
    return hipGetLastError();
}

hipError_t plain_adj_rz(int prec, void *phi, void *lam, int n, int q, const double *theta,
                        int64_t p, double *part_row, hipStream_t s)
{
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_adj_rz<float>, dim3(kPlainGrid), dim3(kPlainBlock), 0, s,
                           C<float>(phi), C<float>(lam), n, q, theta, p, part_row);
    else
        hipLaunchKernelGGL(k_adj_rz<double>, dim3(kPlainGrid), dim3(kPlainBlock), 0, s,
                           C<double>(phi), C<double>(lam), n, q, theta, p, part_row);
    return hipGetLastError();
}

}  // namespace gv
