// gv_fused.hip -- the fused engine for the ansatz of Sec. IV-B (Eq. 7, Eq. 8)
// and its reverse sweep.
//
// Layer l of the ansatz is R_l = (x)_q RY(theta_{l,q}) followed by the
// diagonal D_l = (prod_q RZ(phi_{l,q})) * (CZ ladder) (for the CNOT ladder,
// D_l holds only the RZ phases and the ladder is an index permutation).
// R_l factorises over qubits, so it is applied in a few HBM sweeps
// ("passes"): a pass loads a tile of 2^K amplitudes whose index bits
// pos[0..K) vary (the low C bits are always in the tile, so every access is a
// run of >= 2^C contiguous amplitudes), applies the RY of every tile qubit
// that is new in this pass, and writes the tile back in place.  Inside a tile
// each thread holds 2^LOGR amplitudes in registers; the tile bits a thread's
// registers span change between "assignments" by an exchange through LDS, so
// every tile bit is a register bit in one assignment and its 2x2 rotation
// runs in registers.
//
// What sits in HBM between layers is the state just before a diagonal,
// psi~_l = R_l D_{l-1} ... ; the diagonal D_{l-1} is applied on the fly when
// the first pass of layer l loads its tiles (from three per-layer tables
// indexed by chunks of the amplitude index, FP64-built and rounded once).
// The first layer's state R_0|0...0> is a product state and is generated
// from tables instead of being read.
//
// Reverse sweep (gradient): with phi = psi~_l and lam its adjoint partner,
// for a tile qubit q of layer l, Im<lam|Z_q|phi> at the start of its pass is
// the gradient of RZ(phi_{l,q}) (it commutes with every diagonal factor and
// with the RY of other qubits), and Im<lam|Y_q|phi> just before its RY is
// undone is the gradient of RY(theta_{l,q}).  The last pass of layer l
// undoes D_{l-1} as it stores.  For a Z-only Hamiltonian the last forward
// pass, the energy E = sum_i D_i |psi_i|^2, lam = D psi and the first
// reverse pass run as one "turnaround" kernel.
//
// Products are taken in the amplitude precision over at most 2^LOGR terms
// per thread; everything above that is FP64 with a fixed reduction order.
#include <string.h>

#include "gv_device.hpp"
#include "gv_internal.hpp"

namespace gv {

namespace {

// Diagonal tables of one layer over four chunks of the amplitude index,
// chunk c covering bits [b_c, b_{c+1}) with b_0 = 0, b_1 = K - LOGR, b_2 = K
// (so in the contiguous pass 0, chunk 0 is the thread bits and chunk 1 the
// register bits of the load assignment) and b_4 = n.  Entry v of chunk c is
// the product of the RZ phases of the chunk's qubits and the sign of the CZ
// pairs inside the chunk; CZ pairs that straddle chunks are listed apart.
struct DiagTab {
    const void *tab;
    int b1, b2, b3;
    int off1, off2, off3;
    u64 m0, m1, m2;
    int npair;
    int8_t pa[4], pb[4];
};

enum { IN_LOAD = 0, IN_LOAD_DIAG = 1, IN_GENERATE = 2 };

struct FusedArgs {
    int n;
    int layer;               // rotation layer whose RY gates this pass applies
    int nparam_layer;        // 2n
    int8_t pos[kMaxTileBits];
    uint32_t active;
    int in_mode;             // forward / turnaround: IN_* (diag and generate only in pass 0)
    int diag_phi, diag_lam;  // reverse, pass 0: times conj(dt) on load
    int phi_gen;             // reverse, pass 0: phi from gt instead of a load
    int store_phi, store_lam;
    int nruns;               // tile id -> outside bits, as runs of contiguous bits
    int8_t run_src[kMaxTileBits + 1], run_w[kMaxTileBits + 1], run_dst[kMaxTileBits + 1];
    u64 ntiles;
    const double *ry;        // [P][2] cos, sin of half angles
    DiagTab dt;              // layer diagonal (or the first layer's generator in forward)
    DiagTab gt;              // reverse: generator of R_0|0...0>
    const double *hdiag;     // turnaround: diagonal of the Hamiltonian
    double *part;            // P x grid gradient partials
    double *epart;           // turnaround: 2 x grid energy partials
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
    // tile-local index of register r of thread t in the assignment whose
    // register bits are [l, l + LOGR)
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

// physical offset of the thread bits of the assignment with register bits
// [l, l + LOGR) (the other tile bits take thread-id bits in ascending order)
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

// physical offset of register r: with CONTIG the register bits of the
// assignment sit at consecutive positions (the planner guarantees it for
// K >= 10), so the offset is r shifted by the first position
template <int LOGR, bool CONTIG>
struct RegMap {
    u64 rb[CONTIG ? 1 : LOGR];
    int sh;
    __device__ __forceinline__ void init(const int8_t *p)
    {
        sh = p[0];
        if constexpr (!CONTIG)
#pragma unroll
            for (int k = 0; k < LOGR; ++k) rb[k] = 1ull << p[k];
    }
    __device__ __forceinline__ u64 off(int r) const
    {
        if constexpr (CONTIG) {
            return (u64)r << sh;
        } else {
            u64 o = 0;
#pragma unroll
            for (int k = 0; k < LOGR; ++k)
                if ((r >> k) & 1) o |= rb[k];
            return o;
        }
    }
};

template <typename R>
__device__ __forceinline__ cx<R> cneg(cx<R> v)
{
    v.re = -v.re;
    v.im = -v.im;
    return v;
}

template <typename R>
__device__ __forceinline__ cx<R> diag_entry(u64 i, const DiagTab &d)
{
    const cx<R> *T = (const cx<R> *)d.tab;
    cx<R> v = cmul(cmul(T[i & d.m0], T[d.off1 + ((i >> d.b1) & d.m1)]),
                   cmul(T[d.off2 + ((i >> d.b2) & d.m2)], T[d.off3 + (i >> d.b3)]));
    int par = 0;
    for (int k = 0; k < d.npair; ++k) par ^= (int)((i >> d.pa[k]) & (i >> d.pb[k]) & 1);
    return par ? cneg(v) : v;
}

// The diagonal over the tiles of pass 0 (tile bits = index bits 0..K-1) in
// the load assignment: thread t's bits are chunk 0, register r's bits chunk
// 1, the tile id's bits chunks 2 and 3.  D = T0[t] T1[r] T2 T3 times the
// signs of the straddling CZ pairs, collected per (thread, tile) as a mask
// over the registers.
template <typename R, int K, int LOGR>
struct P0Diag {
    static constexpr int NR = 1 << LOGR;
    cx<R> t0;        // T0[t], per thread
    cx<R> w;         // T0[t] T2 T3, per thread and tile
    uint32_t neg;    // bit r: register r's entry is negated
    __device__ __forceinline__ void init(const DiagTab &d, int t)
    {
        t0 = ((const cx<R> *)d.tab)[t];
    }
    __device__ static __forceinline__ uint32_t reg_pattern(int k)
    {
        uint32_t m = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if ((r >> k) & 1) m |= 1u << r;
        return m;
    }
    __device__ static __forceinline__ uint32_t src_mask(int q, int t, u64 base)
    {
        constexpr uint32_t ALL = (NR >= 32) ? 0xffffffffu : ((1u << NR) - 1u);
        if (q < K - LOGR) return ((t >> q) & 1) ? ALL : 0u;
        if (q < K) {
            uint32_t m = 0;
#pragma unroll
            for (int k = 0; k < LOGR; ++k)
                if (q - (K - LOGR) == k) m = reg_pattern(k);
            return m;
        }
        return ((base >> q) & 1) ? ALL : 0u;
    }
    __device__ __forceinline__ void tile(const DiagTab &d, u64 base, int t)
    {
        const cx<R> *T = (const cx<R> *)d.tab;
        w = cmul(t0, cmul(T[d.off2 + ((base >> d.b2) & d.m2)], T[d.off3 + (base >> d.b3)]));
        neg = 0;
        for (int k = 0; k < d.npair; ++k) neg ^= src_mask(d.pa[k], t, base) & src_mask(d.pb[k], t, base);
    }
    __device__ __forceinline__ cx<R> at(const DiagTab &d, int r) const
    {
        const cx<R> v = cmul(w, ((const cx<R> *)d.tab)[d.off1 + r]);
        return ((neg >> r) & 1) ? cneg(v) : v;
    }
};

template <typename R>
__device__ __forceinline__ cx<R> cmul_conj(cx<R> a, cx<R> d)  // a * conj(d)
{
    cx<R> o;
    o.re = a.re * d.re + a.im * d.im;
    o.im = a.im * d.re - a.re * d.im;
    return o;
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
// RY (Im<lam|Y_q|phi> = Re(conj(l1) f0) - Re(conj(l0) f1) over the pairs),
// then RY(-theta) on both vectors
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

// reverse assignments AI = 1 .. NA-1, each after an exchange from AI-1
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

// reverse assignments in the order AI, AI-1, ..., 0 (each after an exchange
// from AI+1), used by the turnaround whose data ends the forward part in the
// last assignment
template <typename R, int K, int LOGR, int AI>
struct BwdChainRev {
    __device__ static __forceinline__ void run(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR],
                                               double (&accY)[K], cx<R> *lds, int t,
                                               const FusedArgs &a)
    {
        using T = Tile<K, LOGR>;
        exchange<R, K, LOGR>(f, lds, t, T::lo(AI + 1), T::lo(AI));
        exchange<R, K, LOGR>(l, lds, t, T::lo(AI + 1), T::lo(AI));
        bwd_assign<R, K, LOGR, AI>(f, l, accY, a);
        if constexpr (AI > 0) BwdChainRev<R, K, LOGR, AI - 1>::run(f, l, accY, lds, t, a);
    }
};

// Load a pass's tile in the load assignment.  In pass 0 the loaded values
// may be multiplied by the layer diagonal (IN_LOAD_DIAG) or replaced by the
// generated first-layer state (IN_GENERATE).
template <typename R, int K, int LOGR, bool CONTIG>
__device__ __forceinline__ void load_tile(cx<R> (&v)[1 << LOGR], const cx<R> *src, u64 base,
                                          u64 toff, const RegMap<LOGR, CONTIG> &m, int mode,
                                          P0Diag<R, K, LOGR> &pd, const DiagTab &d, int t)
{
    constexpr int NR = 1 << LOGR;
    if (mode != IN_LOAD) pd.tile(d, base, t);
    if (mode == IN_GENERATE) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = pd.at(d, r);
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = src[base | toff | m.off(r)];
        if (mode == IN_LOAD_DIAG) {
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r] = cmul(v[r], pd.at(d, r));
        }
    }
}

template <typename R, int K, int LOGR, bool CONTIG>
__global__ __launch_bounds__(1 << (K - LOGR)) void k_fwd_pass(void *psi_, FusedArgs a)
{
    using T = Tile<K, LOGR>;
    cx<R> *psi = (cx<R> *)psi_;
    __shared__ cx<R> lds[T::LDS];
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    RegMap<LOGR, CONTIG> mld, mst;
    mld.init(a.pos + LD);
    mst.init(a.pos + ST);
    P0Diag<R, K, LOGR> pd;
    if (a.in_mode != IN_LOAD) pd.init(a.dt, t);
    for (u64 tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const u64 base = tile_base(tile, a);
        cx<R> v[T::NR];
        load_tile<R, K, LOGR, CONTIG>(v, psi, base, toff_ld, mld, a.in_mode, pd, a.dt, t);
        fwd_assign<R, K, LOGR, 0>(v, a);
        if constexpr (T::NA > 1) FwdChain<R, K, LOGR, 1>::run(v, lds, t, a);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) psi[base | toff_st | mst.off(r)] = v[r];
    }
}

template <typename R, int K>
__device__ __forceinline__ void write_partials(const double (&accY)[K], const double (&accZ)[K],
                                               bool zeroZ, double *sh, const FusedArgs &a)
{
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!((a.active >> j) & 1)) continue;
        const int64_t row = (int64_t)a.layer * a.nparam_layer + a.pos[j];
        const double y = block_sum(accY[j], sh);
        if (threadIdx.x == 0) a.part[row * a.grid + blockIdx.x] = y;
        const double z = zeroZ ? 0.0 : block_sum(accZ[j], sh);
        if (threadIdx.x == 0) a.part[(row + a.n) * a.grid + blockIdx.x] = z;
    }
}

template <typename R, int K, int LOGR, bool CONTIG>
__global__ __launch_bounds__(1 << (K - LOGR)) void k_bwd_pass(const void *phi_in_, void *phi_,
                                                              void *lam_, FusedArgs a)
{
    using T = Tile<K, LOGR>;
    const cx<R> *phi_in = (const cx<R> *)phi_in_;
    cx<R> *phi = (cx<R> *)phi_, *lam = (cx<R> *)lam_;
    __shared__ cx<R> lds[T::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    RegMap<LOGR, CONTIG> mld, mst;
    mld.init(a.pos + LD);
    mst.init(a.pos + ST);
    P0Diag<R, K, LOGR> pd, pg;
    const bool any_diag = a.diag_phi || a.diag_lam;
    if (any_diag) pd.init(a.dt, t);
    if (a.phi_gen) pg.init(a.gt, t);
    double accY[K], accZ[K];
#pragma unroll
    for (int j = 0; j < K; ++j) accY[j] = accZ[j] = 0.0;

    for (u64 tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const u64 base = tile_base(tile, a);
        cx<R> f[T::NR], l[T::NR];
        if (a.phi_gen) {
            pg.tile(a.gt, base, t);
#pragma unroll
            for (int r = 0; r < T::NR; ++r) f[r] = pg.at(a.gt, r);
        } else {
#pragma unroll
            for (int r = 0; r < T::NR; ++r) f[r] = phi_in[base | toff_ld | mld.off(r)];
        }
#pragma unroll
        for (int r = 0; r < T::NR; ++r) l[r] = lam[base | toff_ld | mld.off(r)];
        if (any_diag) {
            pd.tile(a.dt, base, t);
#pragma unroll
            for (int r = 0; r < T::NR; ++r) {
                const cx<R> d = pd.at(a.dt, r);
                if (a.diag_phi) f[r] = cmul_conj(f[r], d);
                if (a.diag_lam) l[r] = cmul_conj(l[r], d);
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
            const u64 i = base | toff_st | mst.off(r);
            if (a.store_phi) phi[i] = f[r];
            if (a.store_lam) lam[i] = l[r];
        }
    }
    write_partials<R, K>(accY, accZ, false, sh, a);
}

// Last forward pass of the last layer + energy + first reverse pass, for a
// Z-only Hamiltonian with diagonal D: in each tile psi gets the pass's RY
// gates, E += sum D_i |psi_i|^2, lam = D psi, then the reverse step of the
// same gates runs on (psi, lam) and only lam is stored (phi after the
// reverse step equals the loaded tile, which stays in HBM).  RZ gradients of
// the tile qubits are zero here: Im(conj(D_i psi_i) psi_i) = 0.  When this is
// the layer's only pass, the load applies the previous layer's diagonal (or
// generates the first layer's state).
template <typename R, int K, int LOGR, bool CONTIG>
__global__ __launch_bounds__(1 << (K - LOGR)) void k_turn_pass(const void *psi_, void *lam_,
                                                               FusedArgs a)
{
    using T = Tile<K, LOGR>;
    const cx<R> *psi = (const cx<R> *)psi_;
    cx<R> *lam = (cx<R> *)lam_;
    __shared__ cx<R> lds[T::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    RegMap<LOGR, CONTIG> mld, mst;
    mld.init(a.pos + LD);
    mst.init(a.pos + ST);
    P0Diag<R, K, LOGR> pd;
    if (a.in_mode != IN_LOAD) pd.init(a.dt, t);
    double accY[K], accZ[K];
#pragma unroll
    for (int j = 0; j < K; ++j) accY[j] = accZ[j] = 0.0;
    double eacc = 0.0;

    for (u64 tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const u64 base = tile_base(tile, a);
        cx<R> f[T::NR], l[T::NR];
        load_tile<R, K, LOGR, CONTIG>(f, psi, base, toff_ld, mld, a.in_mode, pd, a.dt, t);
        fwd_assign<R, K, LOGR, 0>(f, a);
        if constexpr (T::NA > 1) FwdChain<R, K, LOGR, 1>::run(f, lds, t, a);
        // energy and lam in the last assignment's layout
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            const double d = a.hdiag[base | toff_st | mst.off(r)];
            eacc += d * ((double)f[r].re * f[r].re + (double)f[r].im * f[r].im);
            l[r].re = (R)d * f[r].re;
            l[r].im = (R)d * f[r].im;
        }
        bwd_assign<R, K, LOGR, T::NA - 1>(f, l, accY, a);
        if constexpr (T::NA > 1) BwdChainRev<R, K, LOGR, T::NA - 2>::run(f, l, accY, lds, t, a);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) lam[base | toff_ld | mld.off(r)] = l[r];
    }
    write_partials<R, K>(accY, accZ, true, sh, a);
    const double e = block_sum(eacc, sh);
    if (t == 0) {
        a.epart[blockIdx.x] = e;
        a.epart[a.grid + blockIdx.x] = 0.0;
    }
}


// ------------------------------------------------------- off-diagonal terms

struct OffArgs {
    int n;
    int8_t pos[kMaxTileBits];
    int nruns;
    int8_t run_src[kMaxTileBits + 1], run_w[kMaxTileBits + 1], run_dst[kMaxTileBits + 1];
    u64 ntiles;
    const OffClass *cls;
    int c0, c1;
    const OffTerm *terms;
    double *epart;
    int estride;
};

// One cover pass: the psi tile sits in LDS, so for every class (flip mask x
// inside the tile) each amplitude reads its partner psi_{i^x} there and adds
// F(i^x) psi_{i^x} to lam_i; the class factor F is summed over the class's
// terms in the amplitude precision.  The pass's share of <psi|H|psi> goes to
// FP64 partials.
template <typename R, int K, int LOGR>
__global__ __launch_bounds__(1 << (K - LOGR)) void k_offdiag_pass(const void *psi_, void *lam_,
                                                                  OffArgs a)
{
    using T = Tile<K, LOGR>;
    const cx<R> *psi = (const cx<R> *)psi_;
    cx<R> *lam = (cx<R> *)lam_;
    __shared__ cx<R> lds[T::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0);
    FusedArgs fa;  // only the tile geometry is used
    for (int j = 0; j < K; ++j) fa.pos[j] = a.pos[j];
    fa.nruns = a.nruns;
    for (int k = 0; k < a.nruns; ++k) {
        fa.run_src[k] = a.run_src[k];
        fa.run_w[k] = a.run_w[k];
        fa.run_dst[k] = a.run_dst[k];
    }
    const u64 toff = thread_off<K, LOGR>(t, LD, fa);
    RegMap<LOGR, false> m;
    m.init(a.pos + LD);
    double er = 0.0, ei = 0.0;
    for (u64 tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const u64 base = tile_base(tile, fa);
        cx<R> v[T::NR], acc[T::NR];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            v[r] = psi[base | toff | m.off(r)];
            lds[T::pad(T::u_of(t, r, LD))] = v[r];
            acc[r].re = acc[r].im = R(0);
        }
        __syncthreads();
        for (int c = a.c0; c < a.c1; ++c) {
            const OffClass C = a.cls[c];
            R A[T::NR], B[T::NR];
#pragma unroll
            for (int r = 0; r < T::NR; ++r) A[r] = B[r] = R(0);
            for (int k = C.t0; k < C.t1; ++k) {
                const OffTerm tm = a.terms[k];
                const R cc = (R)tm.c;
#pragma unroll
                for (int r = 0; r < T::NR; ++r) {
                    const u64 ip = (base | toff | m.off(r)) ^ C.x;
                    const R sg = (__popcll(ip & tm.z) & 1) ? -cc : cc;
                    if (tm.ph & 1) B[r] += (tm.ph & 2) ? -sg : sg;
                    else A[r] += (tm.ph & 2) ? -sg : sg;
                }
            }
#pragma unroll
            for (int r = 0; r < T::NR; ++r) {
                const cx<R> pv = lds[T::pad(T::u_of(t, r, LD) ^ (int)C.xu)];
                acc[r].re += A[r] * pv.re - B[r] * pv.im;
                acc[r].im += A[r] * pv.im + B[r] * pv.re;
            }
        }
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            er += (double)v[r].re * acc[r].re + (double)v[r].im * acc[r].im;
            ei += (double)v[r].re * acc[r].im - (double)v[r].im * acc[r].re;
            if (lam) {
                const u64 i = base | toff | m.off(r);
                cx<R> o = lam[i];
                o.re += acc[r].re;
                o.im += acc[r].im;
                lam[i] = o;
            }
        }
    }
    const double tr = block_sum(er, sh);
    const double ti = block_sum(ei, sh);
    if (t == 0) {
        a.epart[blockIdx.x] += tr;
        a.epart[a.estride + blockIdx.x] += ti;
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
    int cz_layers;          // layers that carry the CZ ladder
    int cz;                 // 1 linear CZ, 2 circular CZ, 0 none
    int b[5];               // chunk bounds 0, b1, b2, b3, n
    int off[5];             // entry offsets of the chunks within a table set
    size_t stride;          // bytes per layer
};

__device__ __forceinline__ int chunk_of(const TabArgs &ta, int w)
{
    return w < ta.off[1] ? 0 : (w < ta.off[2] ? 1 : (w < ta.off[3] ? 2 : 3));
}

// in-chunk phase of RZ and CZ for entry v of chunk c in layer l:
// prod_{q in chunk} exp(-+ i phi_q / 2), and the parity of the CZ pairs
// inside the chunk
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
    const int per = ta.off[4];
    const int64_t total = (int64_t)per * ta.rot_layers;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(e / per), w = (int)(e % per);
        const int c = chunk_of(ta, w);
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

// first-layer tables: g0 = prod_{q in chunk} (bit ? sin : cos)(theta_q / 2)
// (the product state R_0|0...0>), g = g0 times the chunk's diagonal phase of
// layer 0 (the state D_0 R_0|0...0>)
template <typename R>
__global__ void k_init_tables(const double *theta, TabArgs ta, cx<R> *gtab, cx<R> *g0tab)
{
    const int per = ta.off[4];
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < per; w += gridDim.x * blockDim.x) {
        const int c = chunk_of(ta, w);
        const u64 v = (u64)(w - ta.off[c]);
        double ang;
        int par;
        chunk_phase(theta, ta, 0, c, v, ang, par);
        double mag = 1.0;
        for (int q = ta.b[c]; q < ta.b[c + 1]; ++q) {
            double s, co;
            sincos(0.5 * theta[q], &s, &co);
            mag *= ((v >> (q - ta.b[c])) & 1) ? s : co;
        }
        cx<R> g0;
        g0.re = (R)mag;
        g0.im = (R)0;
        g0tab[w] = g0;
        if (par) mag = -mag;
        double s, co;
        sincos(ang, &s, &co);
        cx<R> out;
        out.re = (R)(mag * co);
        out.im = (R)(mag * s);
        gtab[w] = out;
    }
}

// psi_i = table product (the first layer's state)
template <typename R>
__global__ void k_table_state(cx<R> *psi, DiagTab d, u64 dim)
{
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x)
        psi[i] = diag_entry<R>(i, d);
}

// v0 (and v1) times the layer diagonal, or its conjugate
template <typename R>
__global__ void k_diag_apply(cx<R> *v0, cx<R> *v1, DiagTab d, u64 dim, int conj)
{
    for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < dim;
         i += (u64)gridDim.x * blockDim.x) {
        cx<R> e = diag_entry<R>(i, d);
        if (conj) e.im = -e.im;
        v0[i] = cmul(v0[i], e);
        if (v1) v1[i] = cmul(v1[i], e);
    }
}

// CNOT ladder as an index permutation, fused with the layer diagonal.
// Forward ladder F = f o g with f = prefix XOR of the index bits (CNOT(q ->
// q+1) for q = 0, 1, ...) and g = CNOT(n-1 -> 0) for the circular form.
// forward:  dst[j] = D(s) src[s], s = g(f^-1(j))  (the state CNOT D psi~)
// inverse:  dst[i] = conj(D(i)) src[f(g(i))]       (undoes both)
template <typename R>
__global__ void k_cnot_gather(const cx<R> *src, cx<R> *dst, int n, int circular, int inverse,
                              DiagTab d, int with_diag)
{
    const u64 dim = 1ull << n, mask = dim - 1;
    for (u64 o = blockIdx.x * (u64)blockDim.x + threadIdx.x; o < dim;
         o += (u64)gridDim.x * blockDim.x) {
        if (!inverse) {
            u64 i = o ^ ((o << 1) & mask);
            if (circular) i ^= (i >> (n - 1)) & 1;
            cx<R> v = src[i];
            if (with_diag) v = cmul(v, diag_entry<R>(i, d));
            dst[o] = v;
        } else {
            u64 v = o;
            if (circular) v ^= (v >> (n - 1)) & 1;
            for (int sh = 1; sh < 64; sh <<= 1) v ^= v << sh;
            cx<R> x = src[v & mask];
            if (with_diag) x = cmul_conj(x, diag_entry<R>(o, d));
            dst[o] = x;
        }
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

// table set at `tab` for a layer (cz_layer: whether it carries the CZ ladder)
DiagTab make_diagtab(const gv_ansatz &an, const Chunks &ch, const void *tab, bool cz_layer)
{
    DiagTab d;
    memset(&d, 0, sizeof(d));
    d.tab = tab;
    d.b1 = ch.b[1];
    d.b2 = ch.b[2];
    d.b3 = ch.b[3];
    d.off1 = ch.off[1];
    d.off2 = ch.off[2];
    d.off3 = ch.off[3];
    d.m0 = (u64)(ch.off[1] - ch.off[0]) - 1;
    d.m1 = (u64)(ch.off[2] - ch.off[1]) - 1;
    d.m2 = (u64)(ch.off[3] - ch.off[2]) - 1;
    d.npair = 0;
    const int n = an.n;
    const bool cz = (an.ent == GV_ENT_CZ_LINEAR || an.ent == GV_ENT_CZ_CIRCULAR) && cz_layer;
    if (!cz) return d;
    // CZ(q-1, q) across every chunk bound q strictly inside [1, n)
    for (int c = 1; c <= 3; ++c) {
        const int q = ch.b[c];
        if (q <= 0 || q >= n) continue;
        bool dup = false;
        for (int k = 0; k < d.npair; ++k) dup |= d.pb[k] == q;
        if (dup) continue;
        d.pa[d.npair] = (int8_t)(q - 1);
        d.pb[d.npair++] = (int8_t)q;
    }
    // the circular pair (n-1, 0) lies inside a chunk only when chunk 0 holds every bit
    if (an.ent == GV_ENT_CZ_CIRCULAR && n > 2 && ch.b[1] < n) {
        d.pa[d.npair] = (int8_t)(n - 1);
        d.pb[d.npair++] = 0;
    }
    return d;
}

DiagTab layer_tab(const gv_ansatz &an, const Chunks &ch, const FusedTables &t, int layer)
{
    return make_diagtab(an, ch, (const char *)t.dtab + (size_t)layer * t.dtab_stride,
                        layer < an.layers);
}

TabArgs make_tab_args(const gv_ansatz &an, const Chunks &ch, size_t stride)
{
    TabArgs ta;
    ta.n = an.n;
    ta.rot_layers = rot_layers(an);
    ta.cz_layers = an.layers;
    ta.cz = an.ent == GV_ENT_CZ_LINEAR ? 1 : (an.ent == GV_ENT_CZ_CIRCULAR ? 2 : 0);
    for (int c = 0; c < 5; ++c) {
        ta.b[c] = ch.b[c];
        ta.off[c] = ch.off[c];
    }
    ta.stride = stride;
    return ta;
}

FusedArgs base_args(const gv_ansatz &an, const TilePlan &plan, int pass, int layer,
                    const FusedTables &t)
{
    FusedArgs a;
    memset(&a, 0, sizeof(a));
    a.n = an.n;
    a.layer = layer;
    a.nparam_layer = 2 * an.n;
    for (int j = 0; j < plan.K; ++j) a.pos[j] = plan.pass[pass].pos[j];
    a.active = plan.pass[pass].active;
    fill_runs(a, plan.pass[pass], plan.K, an.n);
    a.ntiles = 1ull << (an.n - plan.K);
    a.ry = t.ry;
    a.store_phi = a.store_lam = 1;
    return a;
}

inline int elem_grid(u64 dim)
{
    const u64 b = (dim + 255) / 256;
    return (int)(b < 8192 ? b : 8192);
}

#define GV_LAUNCH_K(KERNEL, PREC, GRID, K, ...)                                                   \
    do {                                                                                          \
        switch (K) {                                                                              \
        case 12:                                                                                  \
            if (PREC == GV_C64)                                                                   \
                hipLaunchKernelGGL((KERNEL<float, 12, 4, true>), dim3(GRID), dim3(256), 0, s,     \
                                   __VA_ARGS__);                                                  \
            else                                                                                  \
                hipLaunchKernelGGL((KERNEL<double, 12, 4, true>), dim3(GRID), dim3(256), 0, s,    \
                                   __VA_ARGS__);                                                  \
            break;                                                                                \
        case 10:                                                                                  \
            if (PREC == GV_C64)                                                                   \
                hipLaunchKernelGGL((KERNEL<float, 10, 4, true>), dim3(GRID), dim3(64), 0, s,      \
                                   __VA_ARGS__);                                                  \
            else                                                                                  \
                hipLaunchKernelGGL((KERNEL<double, 10, 4, true>), dim3(GRID), dim3(64), 0, s,     \
                                   __VA_ARGS__);                                                  \
            break;                                                                                \
        case 8:                                                                                   \
            if (PREC == GV_C64)                                                                   \
                hipLaunchKernelGGL((KERNEL<float, 8, 3, false>), dim3(GRID), dim3(32), 0, s,      \
                                   __VA_ARGS__);                                                  \
            else                                                                                  \
                hipLaunchKernelGGL((KERNEL<double, 8, 3, false>), dim3(GRID), dim3(32), 0, s,     \
                                   __VA_ARGS__);                                                  \
            break;                                                                                \
        default: return hipErrorInvalidValue;                                                     \
        }                                                                                         \
    } while (0)

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
    const int64_t total = (int64_t)ta.off[4] * ta.rot_layers;
    const int g = (int)((total + 255) / 256 < 2048 ? (total + 255) / 256 : 2048);
    if (prec == GV_C64) {
        hipLaunchKernelGGL(k_diag_tables<float>, dim3(g), dim3(256), 0, s, theta, ta,
                           (char *)t.dtab);
        hipLaunchKernelGGL(k_init_tables<float>, dim3((ta.off[4] + 255) / 256), dim3(256), 0, s,
                           theta, ta, (cx<float> *)t.gtab, (cx<float> *)t.g0tab);
    } else {
        hipLaunchKernelGGL(k_diag_tables<double>, dim3(g), dim3(256), 0, s, theta, ta,
                           (char *)t.dtab);
        hipLaunchKernelGGL(k_init_tables<double>, dim3((ta.off[4] + 255) / 256), dim3(256), 0, s,
                           theta, ta, (cx<double> *)t.gtab, (cx<double> *)t.g0tab);
    }
    return hipGetLastError();
}

hipError_t fused_init_state(int prec, void *psi, const gv_ansatz &an, const Chunks &ch,
                            const FusedTables &t, hipStream_t s)
{
    // the product state R_0|0...0> (no phases: the first pass of layer 1,
    // or the energy step, applies D_0)
    const DiagTab d = make_diagtab(an, ch, t.g0tab, false);
    const u64 dim = 1ull << an.n;
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_table_state<float>, dim3(elem_grid(dim)), dim3(256), 0, s,
                           (cx<float> *)psi, d, dim);
    else
        hipLaunchKernelGGL(k_table_state<double>, dim3(elem_grid(dim)), dim3(256), 0, s,
                           (cx<double> *)psi, d, dim);
    return hipGetLastError();
}

hipError_t fused_forward_pass(int prec, void *psi, const gv_ansatz &an, const TilePlan &plan,
                              int pass, int layer, int in_mode, const Chunks &ch,
                              const FusedTables &t, hipStream_t s)
{
    if (in_mode != IN_LOAD && pass != 0) return hipErrorInvalidValue;
    FusedArgs a = base_args(an, plan, pass, layer, t);
    a.in_mode = in_mode;
    if (in_mode == IN_LOAD_DIAG) a.dt = layer_tab(an, ch, t, layer - 1);
    if (in_mode == IN_GENERATE) a.dt = make_diagtab(an, ch, t.gtab, 0 < an.layers);
    const int grid = fused_grid(prec, plan, an.n);
    GV_LAUNCH_K(k_fwd_pass, prec, grid, plan.K, psi, a);
    return hipGetLastError();
}

hipError_t fused_backward_pass(int prec, const void *phi_in, void *phi, void *lam,
                               const gv_ansatz &an, const TilePlan &plan, int pass, int layer,
                               const BwdFlags &fl, const Chunks &ch, const FusedTables &t,
                               double *part, int grid, hipStream_t s)
{
    if ((fl.phi_generate || fl.diag_phi || fl.diag_lam) && pass != 0) return hipErrorInvalidValue;
    FusedArgs a = base_args(an, plan, pass, layer, t);
    a.phi_gen = fl.phi_generate;
    if (fl.phi_generate) a.gt = make_diagtab(an, ch, t.g0tab, false);
    a.diag_phi = fl.diag_phi;
    a.diag_lam = fl.diag_lam;
    if (fl.diag_phi || fl.diag_lam) a.dt = layer_tab(an, ch, t, layer);
    a.store_phi = fl.store_phi;
    a.store_lam = fl.store_lam;
    a.part = part;
    a.grid = grid;
    GV_LAUNCH_K(k_bwd_pass, prec, grid, plan.K, phi_in, phi, lam, a);
    return hipGetLastError();
}

hipError_t fused_turnaround(int prec, const void *psi, void *lam, const double *hdiag,
                            const gv_ansatz &an, const TilePlan &plan, int pass, int layer,
                            int in_mode, const Chunks &ch, const FusedTables &t, double *part,
                            double *epart, int grid, hipStream_t s)
{
    if (in_mode != IN_LOAD && pass != 0) return hipErrorInvalidValue;
    FusedArgs a = base_args(an, plan, pass, layer, t);
    a.in_mode = in_mode;
    if (in_mode == IN_LOAD_DIAG) a.dt = layer_tab(an, ch, t, layer - 1);
    if (in_mode == IN_GENERATE) a.dt = make_diagtab(an, ch, t.gtab, 0 < an.layers);
    a.hdiag = hdiag;
    a.part = part;
    a.epart = epart;
    a.grid = grid;
    GV_LAUNCH_K(k_turn_pass, prec, grid, plan.K, psi, lam, a);
    return hipGetLastError();
}

hipError_t fused_diag_apply(int prec, void *v0, void *v1, const gv_ansatz &an, const Chunks &ch,
                            const FusedTables &t, int layer, int conj, hipStream_t s)
{
    const DiagTab d = layer_tab(an, ch, t, layer);
    const u64 dim = 1ull << an.n;
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_diag_apply<float>, dim3(elem_grid(dim)), dim3(256), 0, s,
                           (cx<float> *)v0, (cx<float> *)v1, d, dim, conj);
    else
        hipLaunchKernelGGL(k_diag_apply<double>, dim3(elem_grid(dim)), dim3(256), 0, s,
                           (cx<double> *)v0, (cx<double> *)v1, d, dim, conj);
    return hipGetLastError();
}

hipError_t cnot_ladder_gather(int prec, const void *src, void *dst, const gv_ansatz &an,
                              const Chunks &ch, const FusedTables *t, int layer, int inverse,
                              hipStream_t s)
{
    const int n = an.n;
    const int circular = an.ent == GV_ENT_CNOT_CIRCULAR && n > 2;
    DiagTab d;
    memset(&d, 0, sizeof(d));
    const int with_diag = t != nullptr;
    if (t) d = layer_tab(an, ch, *t, layer);
    const u64 dim = 1ull << n;
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_cnot_gather<float>, dim3(elem_grid(dim)), dim3(256), 0, s,
                           (const cx<float> *)src, (cx<float> *)dst, n, circular, inverse, d,
                           with_diag);
    else
        hipLaunchKernelGGL(k_cnot_gather<double>, dim3(elem_grid(dim)), dim3(256), 0, s,
                           (const cx<double> *)src, (cx<double> *)dst, n, circular, inverse, d,
                           with_diag);
    return hipGetLastError();
}

hipError_t offdiag_pass(int prec, const void *psi, void *lam, int n, int K, const OffPass &op,
                        const OffClass *cls, const OffTerm *terms, double *epart, int estride,
                        hipStream_t s)
{
    OffArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    PassPlan pp;
    for (int j = 0; j < K; ++j) pp.pos[j] = op.pos[j];
    pp.active = 0;
    FusedArgs fa;
    memset(&fa, 0, sizeof(fa));
    fill_runs(fa, pp, K, n);
    for (int j = 0; j < K; ++j) a.pos[j] = op.pos[j];
    a.nruns = fa.nruns;
    for (int k = 0; k < fa.nruns; ++k) {
        a.run_src[k] = fa.run_src[k];
        a.run_w[k] = fa.run_w[k];
        a.run_dst[k] = fa.run_dst[k];
    }
    a.ntiles = 1ull << (n - K);
    a.cls = cls;
    a.c0 = op.c0;
    a.c1 = op.c1;
    a.terms = terms;
    a.epart = epart;
    a.estride = estride;
    const u64 want = prec == GV_C64 ? 1024 : 512;
    const int grid = (int)(a.ntiles < want ? a.ntiles : want);
    if (grid > estride) return hipErrorInvalidValue;
    switch (K) {
    case 12:
        if (prec == GV_C64)
            hipLaunchKernelGGL((k_offdiag_pass<float, 12, 4>), dim3(grid), dim3(256), 0, s, psi, lam, a);
        else
            hipLaunchKernelGGL((k_offdiag_pass<double, 12, 4>), dim3(grid), dim3(256), 0, s, psi, lam, a);
        break;
    case 10:
        if (prec == GV_C64)
            hipLaunchKernelGGL((k_offdiag_pass<float, 10, 4>), dim3(grid), dim3(64), 0, s, psi, lam, a);
        else
            hipLaunchKernelGGL((k_offdiag_pass<double, 10, 4>), dim3(grid), dim3(64), 0, s, psi, lam, a);
        break;
    case 8:
        if (prec == GV_C64)
            hipLaunchKernelGGL((k_offdiag_pass<float, 8, 3>), dim3(grid), dim3(32), 0, s, psi, lam, a);
        else
            hipLaunchKernelGGL((k_offdiag_pass<double, 8, 3>), dim3(grid), dim3(32), 0, s, psi, lam, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gv
