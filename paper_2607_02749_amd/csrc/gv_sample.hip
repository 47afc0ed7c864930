// gv_sample.hip -- measurement side of the method (Sec. IV-F, Sec. V-A):
// bitstrings drawn from the Born distribution |psi_i|^2 by inverse-CDF
// sampling, the most probable bitstring (the decoded result), and the
// finite-shot energy estimate: the Z-only terms from shots of psi itself,
// every qubit-wise-commuting group from shots of psi rotated into the
// group's eigenbasis (H on its X qubits, H S^dagger on its Y qubits).
//
// Sampling: the 2^n probabilities are summed in FP64 over chunks of
// kChunk amplitudes (a fixed order per chunk), the chunk sums are scanned in
// FP64 by one block, and one wave per shot finds the chunk whose cumulative
// sum first exceeds u * total, then the amplitude inside it (lane segments
// scanned in lane order, then the segment walked in index order).
#include "gv_device.hpp"
#include "gv_internal.hpp"

namespace gv {

namespace {

constexpr int kChunk = 4096;
constexpr int kSampleBlock = 256;   // four shots per block, one per wave

template <typename R>
__device__ __forceinline__ double prob(const cx<R> &v)
{
    const double a = (double)v.re, b = (double)v.im;
    return a * a + b * b;
}

// S[c] = sum of |psi_i|^2 over chunk c (elements c * ch .. c * ch + ch - 1)
template <typename R>
__global__ __launch_bounds__(256) void k_chunk_sums(const cx<R> *psi, u64 ch, double *S)
{
    __shared__ double sh[4];
    const cx<R> *p = psi + (u64)blockIdx.x * ch;
    double acc = 0.0;
    for (u64 i = threadIdx.x; i < ch; i += blockDim.x) acc += prob(p[i]);
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) S[blockIdx.x] = tot;
}

// in-place inclusive scan of S[0..m) by one block: thread segments summed in
// index order, the segment totals scanned by thread 0, then each segment
// rewritten with its running sum
__global__ __launch_bounds__(1024) void k_scan_chunks(double *S, u64 m)
{
    __shared__ double seg[1024];
    const u64 per = (m + blockDim.x - 1) / blockDim.x;
    const u64 lo = threadIdx.x * per, hi = lo + per < m ? lo + per : m;
    double s = 0.0;
    for (u64 i = lo; i < hi; ++i) s += S[i];
    seg[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (unsigned t = 0; t < blockDim.x; ++t) {
            const double v = seg[t];
            seg[t] = run;
            run += v;
        }
    }
    __syncthreads();
    double run = seg[threadIdx.x];
    for (u64 i = lo; i < hi; ++i) {
        run += S[i];
        S[i] = run;
    }
}

// one wave per shot: out[j] = the index i with cdf(i - 1) <= u_j * total <
// cdf(i) (the last index with non-zero probability when rounding leaves the
// target at or above the total)
template <typename R>
__global__ __launch_bounds__(kSampleBlock) void k_sample(const cx<R> *psi, const double *cdf,
                                                          u64 nchunk, u64 ch, const double *u,
                                                          int64_t shots, uint64_t *out)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (kSampleBlock / 64) + (threadIdx.x >> 6);
    if (j >= shots) return;   // whole waves leave together
    const double total = cdf[nchunk - 1];
    const double target = u[j] * total;
    // first chunk whose inclusive sum exceeds the target
    u64 lo = 0, hi = nchunk - 1;
    while (lo < hi) {
        const u64 mid = (lo + hi) >> 1;
        if (cdf[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    const u64 c = lo;
    double rem = target - (c > 0 ? cdf[c - 1] : 0.0);
    const cx<R> *p = psi + c * ch;
    const u64 seg = (ch + 63) / 64;
    const u64 s0 = (u64)lane * seg, s1 = s0 + seg < ch ? s0 + seg : ch;
    double mine = 0.0;
    for (u64 i = s0; i < s1; ++i) mine += prob(p[i]);
    // inclusive scan over the lanes, in lane order
    double incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const double excl = incl - mine;
    const unsigned long long hit = __ballot(incl > rem && mine > 0.0);
    int owner;
    if (hit) {
        owner = __ffsll((long long)hit) - 1;
    } else {   // rounding: the last lane with any probability
        const unsigned long long nz = __ballot(mine > 0.0);
        owner = nz ? 63 - __clzll((long long)nz) : 63;
    }
    if (lane == owner) {
        double run = excl;
        u64 pick = s1 > s0 ? s1 - 1 : ch - 1;
        u64 last_nz = pick;
        bool found = false;
        for (u64 i = s0; i < s1; ++i) {
            const double pi = prob(p[i]);
            if (pi > 0.0) last_nz = i;
            run += pi;
            if (!found && run > rem && pi > 0.0) {
                pick = i;
                found = true;
            }
        }
        if (!found) pick = last_nz;
        out[j] = c * ch + pick;
    }
}

// per block: (max |psi_i|^2, smallest index reaching it) over a grid-stride
// range; then one block reduces the block results in block order
template <typename R>
__global__ __launch_bounds__(256) void k_argmax_blocks(const cx<R> *psi, u64 dim, double *bp,
                                                       uint64_t *bi)
{
    __shared__ double sp[256];
    __shared__ uint64_t si[256];
    double best = -1.0;
    uint64_t bidx = ~0ull;
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x) {
        const double p = prob(psi[i]);
        if (p > best) {   // increasing i: ties keep the smaller index
            best = p;
            bidx = i;
        }
    }
    sp[threadIdx.x] = best;
    si[threadIdx.x] = bidx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double q = sp[threadIdx.x + o];
            const uint64_t qi = si[threadIdx.x + o];
            if (q > sp[threadIdx.x] || (q == sp[threadIdx.x] && qi < si[threadIdx.x])) {
                sp[threadIdx.x] = q;
                si[threadIdx.x] = qi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bp[blockIdx.x] = sp[0];
        bi[blockIdx.x] = si[0];
    }
}

__global__ void k_argmax_final(const double *bp, const uint64_t *bi, int nb, uint64_t *idx,
                               double *p)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double best = -1.0;
    uint64_t bidx = ~0ull;
    for (int b = 0; b < nb; ++b)
        if (bp[b] > best || (bp[b] == best && bi[b] < bidx)) {
            best = bp[b];
            bidx = bi[b];
        }
    *idx = bidx;
    if (p) *p = best;
}

// dst = the single-qubit rotation of the group basis on qubit q applied to
// src (dst may equal src): letter 1 = X (H), 2 = Y (H S^dagger)
template <typename R>
__global__ void k_basis_qubit(const cx<R> *src, cx<R> *dst, u64 dim, int q, int letter)
{
    const R h = (R)0.70710678118654752440;
    const u64 half = dim >> 1, bit = 1ull << q;
    for (u64 k = blockIdx.x * (u64)blockDim.x + threadIdx.x; k < half;
         k += (u64)gridDim.x * blockDim.x) {
        const u64 i = insert_zero(k, q), i1 = i | bit;
        const cx<R> a = src[i];
        cx<R> b = src[i1];
        if (letter == 2) {   // S^dagger on the |1> component: times -i
            const R re = b.im, im = -b.re;
            b.re = re;
            b.im = im;
        }
        cx<R> o0, o1;
        o0.re = h * (a.re + b.re);
        o0.im = h * (a.im + b.im);
        o1.re = h * (a.re - b.re);
        o1.im = h * (a.im - b.im);
        dst[i] = o0;
        dst[i1] = o1;
    }
}

// shot estimate of a set of terms from the sampled indices: for term k,
// c_k times the mean over shots of (-1)^{popcount(b & mask_k)}; one block
// per term, block sums in a fixed order, then out += sum over terms (one
// thread, term order)
__global__ __launch_bounds__(256) void k_parity_means(const uint64_t *b, int64_t shots,
                                                     const uint64_t *mask, const double *c,
                                                     int64_t m, double *term_out)
{
    __shared__ double sh[4];
    for (int64_t k = blockIdx.x; k < m; k += gridDim.x) {
        const uint64_t mk = mask[k];
        double acc = 0.0;
        for (int64_t s = threadIdx.x; s < shots; s += blockDim.x)
            acc += (__popcll(b[s] & mk) & 1) ? -1.0 : 1.0;
        const double tot = block_sum(acc, sh);
        if (threadIdx.x == 0) term_out[k] = c[k] * tot / (double)shots;
        __syncthreads();
    }
}

// mean over shots of the FP64 diagonal at the sampled indices
__global__ __launch_bounds__(256) void k_diag_mean(const uint64_t *b, int64_t shots,
                                                   const double *diag, double *out)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int64_t s = threadIdx.x; s < shots; s += blockDim.x) acc += diag[b[s]];
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = tot / (double)shots;
}

__global__ void k_sum_terms(const double *term, int64_t m, const double *diag_part, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = diag_part ? *diag_part : 0.0;
    for (int64_t k = 0; k < m; ++k) s += term[k];
    out[0] = s;
    out[1] = 0.0;
}

inline unsigned grid_of(u64 work, unsigned block)
{
    const u64 g = (work + block - 1) / block;
    return (unsigned)(g < 8192 ? (g ? g : 1) : 8192);
}

}  // namespace

size_t sample_work_bytes(int n)
{
    const u64 dim = 1ull << n, ch = dim < (u64)kChunk ? dim : (u64)kChunk;
    return align_up((size_t)(dim / ch) * sizeof(double)) + align_up(8192 * 16);
}

hipError_t sample_born(int prec, const void *psi, int n, const double *u, int64_t shots,
                       void *work, uint64_t *out, hipStream_t s)
{
    const u64 dim = 1ull << n, ch = dim < (u64)kChunk ? dim : (u64)kChunk, nchunk = dim / ch;
    double *S = (double *)work;
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_chunk_sums<float>, dim3((unsigned)nchunk), dim3(256), 0, s,
                           (const cx<float> *)psi, ch, S);
    else
        hipLaunchKernelGGL(k_chunk_sums<double>, dim3((unsigned)nchunk), dim3(256), 0, s,
                           (const cx<double> *)psi, ch, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, s, S, nchunk);
    if ((e = hipGetLastError()) != hipSuccess || shots == 0) return e;
    const unsigned g = (unsigned)((shots + kSampleBlock / 64 - 1) / (kSampleBlock / 64));
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_sample<float>, dim3(g), dim3(kSampleBlock), 0, s,
                           (const cx<float> *)psi, S, nchunk, ch, u, shots, out);
    else
        hipLaunchKernelGGL(k_sample<double>, dim3(g), dim3(kSampleBlock), 0, s,
                           (const cx<double> *)psi, S, nchunk, ch, u, shots, out);
    return hipGetLastError();
}

hipError_t argmax_prob(int prec, const void *psi, int n, void *work, uint64_t *idx, double *p,
                       hipStream_t s)
{
    const u64 dim = 1ull << n;
    const int nb = (int)grid_of(dim, 256) < 1024 ? (int)grid_of(dim, 256) : 1024;
    double *bp = (double *)work;
    uint64_t *bi = (uint64_t *)((char *)work + align_up(1024 * sizeof(double)));
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_argmax_blocks<float>, dim3(nb), dim3(256), 0, s,
                           (const cx<float> *)psi, dim, bp, bi);
    else
        hipLaunchKernelGGL(k_argmax_blocks<double>, dim3(nb), dim3(256), 0, s,
                           (const cx<double> *)psi, dim, bp, bi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(1), 0, s, bp, bi, nb, idx, p);
    return hipGetLastError();
}

hipError_t basis_rotate(int prec, const void *src, void *dst, int n, u64 xmask, u64 ymask,
                        hipStream_t s)
{
    const u64 dim = 1ull << n;
    const void *from = src;
    bool any = false;
    for (int q = 0; q < n; ++q) {
        const int letter = ((ymask >> q) & 1) ? 2 : (((xmask >> q) & 1) ? 1 : 0);
        if (!letter) continue;
        if (prec == GV_C64)
            hipLaunchKernelGGL(k_basis_qubit<float>, dim3(grid_of(dim / 2, 256)), dim3(256), 0, s,
                               (const cx<float> *)from, (cx<float> *)dst, dim, q, letter);
        else
            hipLaunchKernelGGL(k_basis_qubit<double>, dim3(grid_of(dim / 2, 256)), dim3(256), 0,
                               s, (const cx<double> *)from, (cx<double> *)dst, dim, q, letter);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        from = dst;
        any = true;
    }
    if (!any) return copy_vector(dst, src, dim * (prec == GV_C64 ? 8 : 16), s);
    return hipSuccess;
}

hipError_t parity_means(const uint64_t *b, int64_t shots, const uint64_t *mask, const double *c,
                        int64_t m, double *term_out, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_parity_means, dim3((unsigned)(m < 4096 ? m : 4096)), dim3(256), 0, s, b,
                       shots, mask, c, m, term_out);
    return hipGetLastError();
}

hipError_t diag_mean(const uint64_t *b, int64_t shots, const double *diag, double *out,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_diag_mean, dim3(1), dim3(256), 0, s, b, shots, diag, out);
    return hipGetLastError();
}

hipError_t sum_terms(const double *term, int64_t m, const double *diag_part, double *out,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_terms, dim3(1), dim3(1), 0, s, term, m, diag_part, out);
    return hipGetLastError();
}

}  // namespace gv
