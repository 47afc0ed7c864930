// gv_fused.hip -- the fused engine for the ansatz of Sec. IV-B (Eq. 7, Eq. 8)
// and its reverse sweep.
//
// A layer of the ansatz is R_l = (x)_q RY(theta_{l,q}) followed by the
// diagonal D_l = (prod_q RZ(phi_{l,q})) * (CZ ladder).  R_l factorises over
// qubits, so it is applied in a few HBM sweeps ("passes"): a pass loads a
// tile of 2^K amplitudes whose index bits pos[0..K) vary (the low C bits are
// always in the tile so that every access is a run of >= 2^C contiguous
// amplitudes), applies the RY of every tile qubit that is new in this pass,
// and writes the tile back in place.  Inside a tile, each thread holds 2^LOGR
// amplitudes in registers; the tile bits a thread's registers span change
// between "assignments" by an exchange through LDS, so every tile bit is a
// register bit in one assignment and its 2x2 rotation runs in registers.
// D_l is applied in the last pass of the layer from three per-layer tables
// indexed by chunks of the amplitude index (FP64-built, rounded once).
// The first layer acts on |0...0>, so its state is a product state times
// D_0 and is written directly from tables.
//
// Reverse sweep (gradient): with phi = psi and lam = H psi, each layer is
// undone with the same tiles.  For a tile qubit q of layer l, at the start of
// its pass Im<lam|Z_q|phi> is the gradient of RZ(phi_{l,q}) (it commutes with
// every diagonal factor and with the RY of other qubits), and just before its
// RY is undone Im<lam|Y_q|phi> is the gradient of RY(theta_{l,q}).  Products
// are taken in the amplitude precision over at most 2^LOGR terms per thread;
// everything above that is FP64 with a fixed reduction order.
#include <string.h>

#include "gv_device.hpp"
#include "gv_internal.hpp"

namespace gv {

namespace {

struct FusedArgs {
    int n;
    int layer;              // rotation layer whose gates this pass applies
    int nparam_layer;       // 2n
    int8_t pos[kMaxTileBits];
    uint32_t active;
    int apply_diag;
    int nruns;              // tile id -> outside bits, as runs of contiguous bits
    int8_t run_src[kMaxTileBits + 1], run_w[kMaxTileBits + 1], run_dst[kMaxTileBits + 1];
    u64 ntiles;
    const double *ry;       // [P][2] cos, sin of half angles
    const void *dtab;       // this layer's tables T0 | T1 | T2
    int b1, b2;
    int s1off, s2off;       // entry offsets of T1, T2
    u64 m0, m1;             // chunk masks (after shifting)
    int nx;                 // cross-chunk CZ pairs
    int8_t xa[3], xb[3];
    double *part;           // reverse sweep: P x grid partials
    int grid;
};

template <int K, int LOGR>
struct Tile {
    static constexpr int NR = 1 << LOGR;
    static constexpr int NT = 1 << (K - LOGR);
    static constexpr int NA = 1 + (K - LOGR + LOGR - 1) / LOGR;
    static constexpr int LDS = (1 << K) + ((1 << K) >> 4);
    static constexpr int lo(int a)
    {
        return a == 0 ? K - LOGR : ((a - 1) * LOGR < K - LOGR ? (a - 1) * LOGR : K - LOGR);
    }
    static constexpr uint32_t bits(int a) { return ((1u << LOGR) - 1u) << lo(a); }
    static constexpr uint32_t newbits(int a)
    {
        uint32_t prev = 0;
        for (int b = 0; b < a; ++b) prev |= bits(b);
        return bits(a) & ~prev;
    }
    // tile-local index of register r of thread t in an assignment with
    // register bits [lo, lo + LOGR)
    __device__ static __forceinline__ int u_of(int t, int r, int l)
    {
        return (t & ((1 << l) - 1)) | (r << l) | ((t >> l) << (l + LOGR));
    }
    __device__ static __forceinline__ int pad(int u) { return u + (u >> 4); }
};

__device__ __forceinline__ u64 tile_base(u64 tile, const FusedArgs &a)
{
    u64 b = 0;
    for (int i = 0; i < a.nruns; ++i)
        b |= ((tile >> a.run_src[i]) & ((1ull << a.run_w[i]) - 1)) << a.run_dst[i];
    return b;
}

// physical offset of the thread bits of assignment lo (tile bits outside
// [lo, lo + LOGR) take thread-id bits in ascending order)
template <int K, int LOGR>
__device__ __forceinline__ u64 thread_off(int t, int l, const FusedArgs &a)
{
    u64 off = 0;
    int tb = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= l && j < l + LOGR) continue;
        off |= (u64)((t >> tb) & 1) << a.pos[j];
        ++tb;
    }
    return off;
}

template <int LOGR>
__device__ __forceinline__ u64 reg_off(int r, const u64 (&rb)[LOGR])
{
    u64 o = 0;
#pragma unroll
    for (int k = 0; k < LOGR; ++k)
        if ((r >> k) & 1) o |= rb[k];
    return o;
}

template <typename R>
__device__ __forceinline__ cx<R> diag_entry(u64 i, const FusedArgs &a)
{
    const cx<R> *T = (const cx<R> *)a.dtab;
    cx<R> d = cmul(cmul(T[i & a.m0], T[a.s1off + ((i >> a.b1) & a.m1)]), T[a.s2off + (i >> a.b2)]);
    int par = 0;
    for (int k = 0; k < a.nx; ++k) par ^= (int)((i >> a.xa[k]) & (i >> a.xb[k]) & 1);
    if (par) {
        d.re = -d.re;
        d.im = -d.im;
    }
    return d;
}

// RY on the pair (x, y): (c x - s y, s x + c y)
template <typename R>
__device__ __forceinline__ void rot_pair(cx<R> &x, cx<R> &y, R c, R s)
{
    const cx<R> a = x, b = y;
    x.re = c * a.re - s * b.re;
    x.im = c * a.im - s * b.im;
    y.re = s * a.re + c * b.re;
    y.im = s * a.im + c * b.im;
}

// forward rotations of the tile bits that are new in assignment AI
template <typename R, int K, int LOGR, int AI>
__device__ __forceinline__ void fwd_assign(cx<R> (&v)[1 << LOGR], const FusedArgs &a)
{
    using T = Tile<K, LOGR>;
    constexpr int LO = T::lo(AI);
    constexpr uint32_t NEW = T::newbits(AI);
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        const int j = LO + k;
        if (!((NEW >> j) & 1) || !((a.active >> j) & 1)) continue;
        const double *e = a.ry + 2 * ((int64_t)a.layer * a.nparam_layer + a.pos[j]);
        const R c = (R)e[0], s = (R)e[1];
#pragma unroll
        for (int r = 0; r < T::NR; ++r)
            if (!(r & (1 << k))) rot_pair(v[r], v[r | (1 << k)], c, s);
    }
}

// reverse step of the tile bits new in assignment AI: gradient partial of
// RY (Im<lam|Y_q|phi> = Re(conj(l1) f0) - Re(conj(l0) f1) over pairs), then
// RY(-theta) on both vectors
template <typename R, int K, int LOGR, int AI>
__device__ __forceinline__ void bwd_assign(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR],
                                           double (&accY)[K], const FusedArgs &a)
{
    using T = Tile<K, LOGR>;
    constexpr int LO = T::lo(AI);
    constexpr uint32_t NEW = T::newbits(AI);
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        const int j = LO + k;
        if (!((NEW >> j) & 1) || !((a.active >> j) & 1)) continue;
        const double *e = a.ry + 2 * ((int64_t)a.layer * a.nparam_layer + a.pos[j]);
        const R c = (R)e[0], s = -(R)e[1];
        R g = 0;
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            if (r & (1 << k)) continue;
            const int r1 = r | (1 << k);
            g += (l[r1].re * f[r].re + l[r1].im * f[r].im) - (l[r].re * f[r1].re + l[r].im * f[r1].im);
            rot_pair(f[r], f[r1], c, s);
            rot_pair(l[r], l[r1], c, s);
        }
        accY[j] += (double)g;
    }
}

template <typename R, int K, int LOGR>
__device__ __forceinline__ void exchange(cx<R> (&v)[1 << LOGR], cx<R> *lds, int t, int lfrom, int lto)
{
    using T = Tile<K, LOGR>;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < T::NR; ++r) lds[T::pad(T::u_of(t, r, lfrom))] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < T::NR; ++r) v[r] = lds[T::pad(T::u_of(t, r, lto))];
}

template <typename R, int K, int LOGR, int AI>
struct FwdChain {
    __device__ static __forceinline__ void run(cx<R> (&v)[1 << LOGR], cx<R> *lds, int t,
                                               const FusedArgs &a)
    {
        using T = Tile<K, LOGR>;
        exchange<R, K, LOGR>(v, lds, t, T::lo(AI - 1), T::lo(AI));
        fwd_assign<R, K, LOGR, AI>(v, a);
        if constexpr (AI + 1 < T::NA) FwdChain<R, K, LOGR, AI + 1>::run(v, lds, t, a);
    }
};

template <typename R, int K, int LOGR, int AI>
struct BwdChain {
    __device__ static __forceinline__ void run(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR],
                                               double (&accY)[K], cx<R> *lds, int t,
                                               const FusedArgs &a)
    {
        using T = Tile<K, LOGR>;
        exchange<R, K, LOGR>(f, lds, t, T::lo(AI - 1), T::lo(AI));
        exchange<R, K, LOGR>(l, lds, t, T::lo(AI - 1), T::lo(AI));
        bwd_assign<R, K, LOGR, AI>(f, l, accY, a);
        if constexpr (AI + 1 < T::NA) BwdChain<R, K, LOGR, AI + 1>::run(f, l, accY, lds, t, a);
    }
};

template <typename R, int K, int LOGR>
__global__ __launch_bounds__(1 << (K - LOGR)) void k_fwd_pass(cx<R> *psi, FusedArgs a)
{
    using T = Tile<K, LOGR>;
    __shared__ cx<R> lds[T::LDS];
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    u64 rb_ld[LOGR], rb_st[LOGR];
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        rb_ld[k] = 1ull << a.pos[LD + k];
        rb_st[k] = 1ull << a.pos[ST + k];
    }
    for (u64 tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const u64 base = tile_base(tile, a);
        cx<R> v[T::NR];
#pragma unroll
        for (int r = 0; r < T::NR; ++r) v[r] = psi[base | toff_ld | reg_off<LOGR>(r, rb_ld)];
        fwd_assign<R, K, LOGR, 0>(v, a);
        if constexpr (T::NA > 1) FwdChain<R, K, LOGR, 1>::run(v, lds, t, a);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            const u64 i = base | toff_st | reg_off<LOGR>(r, rb_st);
            if (a.apply_diag) v[r] = cmul(v[r], diag_entry<R>(i, a));
            psi[i] = v[r];
        }
    }
}

template <typename R, int K, int LOGR>
__global__ __launch_bounds__(1 << (K - LOGR)) void k_bwd_pass(const cx<R> *phi_in, cx<R> *phi,
                                                              cx<R> *lam, FusedArgs a)
{
    using T = Tile<K, LOGR>;
    __shared__ cx<R> lds[T::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    u64 rb_ld[LOGR], rb_st[LOGR];
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        rb_ld[k] = 1ull << a.pos[LD + k];
        rb_st[k] = 1ull << a.pos[ST + k];
    }
    double accY[K], accZ[K];
#pragma unroll
    for (int j = 0; j < K; ++j) accY[j] = accZ[j] = 0.0;

    for (u64 tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const u64 base = tile_base(tile, a);
        cx<R> f[T::NR], l[T::NR];
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            const u64 i = base | toff_ld | reg_off<LOGR>(r, rb_ld);
            f[r] = phi_in[i];
            l[r] = lam[i];
            if (a.apply_diag) {
                cx<R> d = diag_entry<R>(i, a);
                d.im = -d.im;
                f[r] = cmul(f[r], d);
                l[r] = cmul(l[r], d);
            }
        }
        // RZ gradients of the active tile qubits: sum_i z_q(i) Im(conj(lam_i) phi_i)
        {
            R tt[T::NR];
            R tsum = 0;
#pragma unroll
            for (int r = 0; r < T::NR; ++r) {
                tt[r] = l[r].re * f[r].im - l[r].im * f[r].re;
                tsum += tt[r];
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (!((a.active >> j) & 1)) continue;
                if (j >= LD) {  // register bit of the load assignment
                    const int k = j - LD;
                    R s = 0;
#pragma unroll
                    for (int r = 0; r < T::NR; ++r) s += ((r >> k) & 1) ? -tt[r] : tt[r];
                    accZ[j] += (double)s;
                } else {        // thread bit j of the load assignment
                    accZ[j] += ((t >> j) & 1) ? -(double)tsum : (double)tsum;
                }
            }
        }
        bwd_assign<R, K, LOGR, 0>(f, l, accY, a);
        if constexpr (T::NA > 1) BwdChain<R, K, LOGR, 1>::run(f, l, accY, lds, t, a);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            const u64 i = base | toff_st | reg_off<LOGR>(r, rb_st);
            phi[i] = f[r];
            lam[i] = l[r];
        }
    }
    // FP64 block sums of the gradient partials, one column per block
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!((a.active >> j) & 1)) continue;
        const int64_t row = (int64_t)a.layer * a.nparam_layer + a.pos[j];
        const double y = block_sum(accY[j], sh);
        if (t == 0) a.part[row * a.grid + blockIdx.x] = y;
        const double z = block_sum(accZ[j], sh);
        if (t == 0) a.part[(row + a.n) * a.grid + blockIdx.x] = z;
    }
}

// ------------------------------------------------------------ table kernels

// ry[p] = (cos(theta_p / 2), sin(theta_p / 2))
__global__ void k_ry_table(const double *theta, int64_t np, double *ry)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        double s, c;
        sincos(0.5 * theta[p], &s, &c);
        ry[2 * p] = c;
        ry[2 * p + 1] = s;
    }
}

struct TabArgs {
    int n;
    int rot_layers;
    int cz_layers;          // layers (entangled ones carry CZ when cz != 0)
    int cz;                 // 1 linear CZ, 2 circular CZ, 0 none
    int b[4];               // chunk bounds b0=0, b1, b2, b3=n
    int off[4];             // entry offsets of the chunks within a layer's table set
    size_t stride;          // bytes per layer
};

// in-chunk phase of RZ and CZ for entry v of chunk c in layer l:
// prod_{q in chunk} exp(-+ i phi_q / 2) * (-1)^{CZ pairs inside the chunk}
__device__ __forceinline__ void chunk_phase(const double *theta, const TabArgs &ta, int l, int c,
                                            u64 v, double &ang, int &par)
{
    const int lo = ta.b[c], hi = ta.b[c + 1];
    ang = 0.0;
    par = 0;
    for (int q = lo; q < hi; ++q) {
        const int bit = (int)((v >> (q - lo)) & 1);
        const double ph = theta[(int64_t)l * 2 * ta.n + ta.n + q];
        ang += bit ? 0.5 * ph : -0.5 * ph;
    }
    if (ta.cz && l < ta.cz_layers) {
        for (int q = lo; q + 1 < hi; ++q)
            par ^= (int)((v >> (q - lo)) & (v >> (q + 1 - lo)) & 1);
        if (ta.cz == 2 && ta.n > 2 && lo == 0 && hi == ta.n)
            par ^= (int)((v >> (ta.n - 1)) & v & 1);
    }
}

template <typename R>
__global__ void k_diag_tables(const double *theta, TabArgs ta, char *dtab)
{
    const int per = ta.off[3];
    const int64_t total = (int64_t)per * ta.rot_layers;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(e / per), w = (int)(e % per);
        const int c = w < ta.off[1] ? 0 : (w < ta.off[2] ? 1 : 2);
        const u64 v = (u64)(w - ta.off[c]);
        double ang;
        int par;
        chunk_phase(theta, ta, l, c, v, ang, par);
        double s, co;
        sincos(ang, &s, &co);
        if (par) {
            s = -s;
            co = -co;
        }
        cx<R> out;
        out.re = (R)co;
        out.im = (R)s;
        ((cx<R> *)(dtab + (size_t)l * ta.stride))[w] = out;
    }
}

// first-layer product-state tables: prod_{q in chunk} (bit ? sin : cos)(theta_q/2)
// times the chunk's diagonal phase of layer 0
template <typename R>
__global__ void k_init_tables(const double *theta, TabArgs ta, cx<R> *gtab)
{
    const int per = ta.off[3];
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < per; w += gridDim.x * blockDim.x) {
        const int c = w < ta.off[1] ? 0 : (w < ta.off[2] ? 1 : 2);
        const u64 v = (u64)(w - ta.off[c]);
        double ang;
        int par;
        chunk_phase(theta, ta, 0, c, v, ang, par);
        double mag = par ? -1.0 : 1.0;
        for (int q = ta.b[c]; q < ta.b[c + 1]; ++q) {
            double s, co;
            sincos(0.5 * theta[q], &s, &co);
            mag *= ((v >> (q - ta.b[c])) & 1) ? s : co;
        }
        double s, co;
        sincos(ang, &s, &co);
        cx<R> out;
        out.re = (R)(mag * co);
        out.im = (R)(mag * s);
        gtab[w] = out;
    }
}

template <typename R>
__global__ void k_init_state(cx<R> *psi, FusedArgs a, u64 dim)
{
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x)
        psi[i] = diag_entry<R>(i, a);
}

// CNOT ladder as an index permutation.  Forward ladder F = f o g with
// f = prefix XOR of the index bits (CNOT(q -> q+1) for q = 0, 1, ...) and
// g = CNOT(n-1 -> 0) for the circular form (identity otherwise).
// forward:  dst[j] = src[g(f^-1(j))];  inverse: dst[i] = src[f(g(i))].
template <typename R>
__global__ void k_cnot_gather(const cx<R> *src, cx<R> *dst, int n, int circular, int inverse)
{
    const u64 dim = 1ull << n, mask = dim - 1;
    for (u64 o = blockIdx.x * (u64)blockDim.x + threadIdx.x; o < dim;
         o += (u64)gridDim.x * blockDim.x) {
        u64 i;
        if (!inverse) {
            i = o ^ ((o << 1) & mask);
            if (circular) i ^= (i >> (n - 1)) & 1;
        } else {
            u64 v = o;
            if (circular) v ^= (v >> (n - 1)) & 1;
            for (int sh = 1; sh < 64; sh <<= 1) v ^= v << sh;
            i = v & mask;
        }
        dst[o] = src[i];
    }
}

// ------------------------------------------------------------ host helpers

void fill_runs(FusedArgs &a, const PassPlan &pp, int K, int n)
{
    bool in[64] = {false};
    for (int j = 0; j < K; ++j) in[pp.pos[j]] = true;
    a.nruns = 0;
    int src = 0;
    for (int q = 0; q < n;) {
        if (in[q]) {
            ++q;
            continue;
        }
        int w = 0;
        while (q + w < n && !in[q + w]) ++w;
        a.run_src[a.nruns] = (int8_t)src;
        a.run_w[a.nruns] = (int8_t)w;
        a.run_dst[a.nruns] = (int8_t)q;
        ++a.nruns;
        src += w;
        q += w;
    }
}

void fill_diag(FusedArgs &a, const gv_ansatz &an, const Chunks &ch, const void *tab, int layer)
{
    a.dtab = tab;
    a.b1 = ch.b1;
    a.b2 = ch.b2;
    a.s1off = ch.size0;
    a.s2off = ch.size0 + ch.size1;
    a.m0 = (u64)ch.size0 - 1;
    a.m1 = (u64)ch.size1 - 1;
    a.nx = 0;
    const int n = an.n;
    const bool cz = (an.ent == GV_ENT_CZ_LINEAR || an.ent == GV_ENT_CZ_CIRCULAR) && layer < an.layers;
    if (!cz) return;
    if (ch.b1 < n) {
        a.xa[a.nx] = (int8_t)(ch.b1 - 1);
        a.xb[a.nx++] = (int8_t)ch.b1;
    }
    if (ch.b2 < n) {
        a.xa[a.nx] = (int8_t)(ch.b2 - 1);
        a.xb[a.nx++] = (int8_t)ch.b2;
    }
    // circular pair (n-1, 0) lies in one chunk only when there is one chunk
    if (an.ent == GV_ENT_CZ_CIRCULAR && n > 2 && ch.b1 < n) {
        a.xa[a.nx] = (int8_t)(n - 1);
        a.xb[a.nx++] = 0;
    }
}

TabArgs make_tab_args(const gv_ansatz &an, const Chunks &ch, size_t stride)
{
    TabArgs ta;
    ta.n = an.n;
    ta.rot_layers = rot_layers(an);
    ta.cz_layers = an.layers;
    ta.cz = an.ent == GV_ENT_CZ_LINEAR ? 1 : (an.ent == GV_ENT_CZ_CIRCULAR ? 2 : 0);
    ta.b[0] = 0;
    ta.b[1] = ch.b1;
    ta.b[2] = ch.b2;
    ta.b[3] = an.n;
    ta.off[0] = 0;
    ta.off[1] = ch.size0;
    ta.off[2] = ch.size0 + ch.size1;
    ta.off[3] = ch.size0 + ch.size1 + ch.size2;
    ta.stride = stride;
    return ta;
}

template <typename R, int K, int LOGR>
hipError_t launch_fwd(void *psi, const FusedArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_fwd_pass<R, K, LOGR>), dim3(grid), dim3(1 << (K - LOGR)), 0, s,
                       (cx<R> *)psi, a);
    return hipGetLastError();
}

template <typename R, int K, int LOGR>
hipError_t launch_bwd(const void *phi_in, void *phi, void *lam, const FusedArgs &a, int grid,
                      hipStream_t s)
{
    hipLaunchKernelGGL((k_bwd_pass<R, K, LOGR>), dim3(grid), dim3(1 << (K - LOGR)), 0, s,
                       (const cx<R> *)phi_in, (cx<R> *)phi, (cx<R> *)lam, a);
    return hipGetLastError();
}

FusedArgs base_args(const gv_ansatz &an, const TilePlan &plan, int pass, int layer,
                    int apply_diag, const Chunks &ch, const FusedTables &t, int prec)
{
    FusedArgs a;
    memset(&a, 0, sizeof(a));
    a.n = an.n;
    a.layer = layer;
    a.nparam_layer = 2 * an.n;
    for (int j = 0; j < plan.K; ++j) a.pos[j] = plan.pass[pass].pos[j];
    a.active = plan.pass[pass].active;
    a.apply_diag = apply_diag;
    fill_runs(a, plan.pass[pass], plan.K, an.n);
    a.ntiles = 1ull << (an.n - plan.K);
    a.ry = t.ry;
    fill_diag(a, an, ch, (const char *)t.dtab + (size_t)layer * t.dtab_stride, layer);
    (void)prec;
    return a;
}

}  // namespace

int fused_grid(int prec, const TilePlan &plan, int n)
{
    // persistent blocks: enough to fill 256 CUs several times over
    const u64 ntiles = 1ull << (n - plan.K);
    const u64 want = prec == GV_C64 ? 1024 : 512;
    return (int)(ntiles < want ? ntiles : want);
}

hipError_t fused_build_tables(int prec, const gv_ansatz &an, const Chunks &ch,
                              const double *theta, const FusedTables &t, hipStream_t s)
{
    const int64_t np = nparams(an);
    hipLaunchKernelGGL(k_ry_table, dim3((int)((np + 255) / 256)), dim3(256), 0, s, theta, np,
                       (double *)t.ry);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TabArgs ta = make_tab_args(an, ch, t.dtab_stride);
    const int64_t total = (int64_t)ta.off[3] * ta.rot_layers;
    const int g = (int)((total + 255) / 256 < 2048 ? (total + 255) / 256 : 2048);
    if (prec == GV_C64) {
        hipLaunchKernelGGL(k_diag_tables<float>, dim3(g), dim3(256), 0, s, theta, ta,
                           (char *)t.dtab);
        hipLaunchKernelGGL(k_init_tables<float>, dim3((ta.off[3] + 255) / 256), dim3(256), 0, s,
                           theta, ta, (cx<float> *)t.gtab);
    } else {
        hipLaunchKernelGGL(k_diag_tables<double>, dim3(g), dim3(256), 0, s, theta, ta,
                           (char *)t.dtab);
        hipLaunchKernelGGL(k_init_tables<double>, dim3((ta.off[3] + 255) / 256), dim3(256), 0, s,
                           theta, ta, (cx<double> *)t.gtab);
    }
    return hipGetLastError();
}

hipError_t fused_init_state(int prec, void *psi, const gv_ansatz &an, const Chunks &ch,
                            const FusedTables &t, hipStream_t s)
{
    FusedArgs a;
    memset(&a, 0, sizeof(a));
    a.n = an.n;
    fill_diag(a, an, ch, t.gtab, 0);
    const u64 dim = 1ull << an.n;
    const u64 b = (dim + 255) / 256;
    const int g = (int)(b < 8192 ? b : 8192);
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_init_state<float>, dim3(g), dim3(256), 0, s, (cx<float> *)psi, a, dim);
    else
        hipLaunchKernelGGL(k_init_state<double>, dim3(g), dim3(256), 0, s, (cx<double> *)psi, a,
                           dim);
    return hipGetLastError();
}

hipError_t fused_forward_pass(int prec, void *psi, const gv_ansatz &an, const TilePlan &plan,
                              int pass, int layer, int apply_diag, const Chunks &ch,
                              const FusedTables &t, hipStream_t s)
{
    FusedArgs a = base_args(an, plan, pass, layer, apply_diag, ch, t, prec);
    const int grid = fused_grid(prec, plan, an.n);
    switch (plan.K) {
    case 12: return prec == GV_C64 ? launch_fwd<float, 12, 4>(psi, a, grid, s)
                                   : launch_fwd<double, 12, 4>(psi, a, grid, s);
    case 10: return prec == GV_C64 ? launch_fwd<float, 10, 4>(psi, a, grid, s)
                                   : launch_fwd<double, 10, 4>(psi, a, grid, s);
    case 8: return prec == GV_C64 ? launch_fwd<float, 8, 3>(psi, a, grid, s)
                                  : launch_fwd<double, 8, 3>(psi, a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t fused_backward_pass(int prec, const void *phi_in, void *phi, void *lam,
                               const gv_ansatz &an, const TilePlan &plan, int pass, int layer,
                               int apply_diag, const Chunks &ch, const FusedTables &t,
                               double *part, int grid, hipStream_t s)
{
    FusedArgs a = base_args(an, plan, pass, layer, apply_diag, ch, t, prec);
    a.part = part;
    a.grid = grid;
    switch (plan.K) {
    case 12: return prec == GV_C64 ? launch_bwd<float, 12, 4>(phi_in, phi, lam, a, grid, s)
                                   : launch_bwd<double, 12, 4>(phi_in, phi, lam, a, grid, s);
    case 10: return prec == GV_C64 ? launch_bwd<float, 10, 4>(phi_in, phi, lam, a, grid, s)
                                   : launch_bwd<double, 10, 4>(phi_in, phi, lam, a, grid, s);
    case 8: return prec == GV_C64 ? launch_bwd<float, 8, 3>(phi_in, phi, lam, a, grid, s)
                                  : launch_bwd<double, 8, 3>(phi_in, phi, lam, a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t cnot_ladder_gather(int prec, const void *src, void *dst, int n, int circular,
                              int inverse, hipStream_t s)
{
    const u64 dim = 1ull << n;
    const u64 b = (dim + 255) / 256;
    const int g = (int)(b < 8192 ? b : 8192);
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_cnot_gather<float>, dim3(g), dim3(256), 0, s, (const cx<float> *)src,
                           (cx<float> *)dst, n, circular, inverse);
    else
        hipLaunchKernelGGL(k_cnot_gather<double>, dim3(g), dim3(256), 0, s,
                           (const cx<double> *)src, (cx<double> *)dst, n, circular, inverse);
    return hipGetLastError();
}

}  // namespace gv
