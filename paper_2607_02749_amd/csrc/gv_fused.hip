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
// (DiagTab itself is declared in gv_internal.hpp.)

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
    int nruns;               // tile id -> outside bits, as runs of contiguous bits:
    uint32_t run[kMaxTileBits + 1];  // source bit | width << 8 | destination bit << 16
    u64 ntiles;
    const void *ry;          // [P] shear coefficients (tan(phi/2), sin phi) of the RY gates
    DiagTab dt;              // layer diagonal (or the first layer's generator in forward)
    DiagTab gt;              // reverse: generator of R_0|0...0>
    const double *hdiag;     // turnaround: diagonal of the Hamiltonian
    double *part;            // P x grid gradient partials
    double *epart;           // turnaround: 2 x grid energy partials
    int grid;
    u64 qmask;               // qubits whose gradient rows are written (others get 0)
    int layer2;              // two-layer passes: the second rotation layer
    LDiagTab ld;             // two-layer passes: diagonal of `layer` in the last assignment
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
    // pad(u_of(t, r, l)) = lds_base(t, l) + r * lds_stride(l) whenever the
    // register bits do not straddle the 16-entry padding groups (l = 0 or
    // l >= 4), which lets register r's LDS access use an immediate offset
    static constexpr bool lds_linear(int l) { return l == 0 || l >= 4; }
    static constexpr int lds_stride(int l) { return l == 0 ? 1 : (1 << l) + (1 << (l - 4)); }
    __device__ static __forceinline__ int lds_index(int t, int r, int l)
    {
        return lds_linear(l) ? pad(u_of(t, 0, l)) + r * lds_stride(l) : pad(u_of(t, r, l));
    }
};

template <typename Args>
__device__ __forceinline__ u64 tile_base(u64 tile, const Args &a)
{
    // one word per run keeps the loop on scalar loads
    u64 b = 0;
    for (int i = 0; i < a.nruns; ++i) {
        const uint32_t r = a.run[i];
        b |= ((tile >> (r & 255u)) & ((1ull << ((r >> 8) & 255u)) - 1)) << (r >> 16);
    }
    return b;
}

// physical offset of the thread bits of the assignment with register bits
// [l, l + LOGR) (the other tile bits take thread-id bits in ascending order)
template <int K, int LOGR, typename Args>
__device__ __forceinline__ u64 thread_off(int t, int l, const Args &a)
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

// A tile's element offset, recomputed where the tile is stored: the empty
// asm hides that it equals the load offset, so the compiler does not keep
// one 64-bit address per register live across the whole tile.
__device__ __forceinline__ u64 fresh(u64 o)
{
    asm volatile("" : "+v"(o));
    return o;
}

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

// A layer diagonal in an arbitrary pass layout (LDiagTab): per thread and
// tile the product of the thread and tile-id factors with the signs of the
// straddling CZ pairs, then per register its factor and sign.
template <typename R, int K, int LOGR>
struct LDiag {
    static constexpr int NR = 1 << LOGR;
    cx<R> w;
    uint32_t neg;
    __device__ static __forceinline__ uint32_t reg_pattern(int k)
    {
        constexpr uint32_t P[5] = {0xaaaaaaaau, 0xccccccccu, 0xf0f0f0f0u, 0xff00ff00u, 0xffff0000u};
        constexpr uint32_t ALL = (NR >= 32) ? 0xffffffffu : ((1u << NR) - 1u);
        return P[k] & ALL;
    }
    // idx: the thread's index bits outside the registers (tile base | thread offset)
    __device__ __forceinline__ void tile(const LDiagTab &d, u64 tile_id, u64 idx, int t)
    {
        const cx<R> *T = (const cx<R> *)d.tab;
        w = cmul(T[t], cmul(T[d.offB1 + (tile_id & ((1ull << d.h1) - 1))],
                            T[d.offB2 + (tile_id >> d.h1)]));
        neg = 0;
        int par = 0;
        for (int k = 0; k < d.npair; ++k) {
            const int ka = d.ka[k], kb = d.kb[k];
            if (ka < 0 && kb < 0) par ^= (int)((idx >> d.pa[k]) & (idx >> d.pb[k]) & 1);
            else if (ka >= 0) neg ^= ((idx >> d.pb[k]) & 1) ? reg_pattern(ka) : 0u;
            else neg ^= ((idx >> d.pa[k]) & 1) ? reg_pattern(kb) : 0u;
        }
        if (par) w = cneg(w);
    }
    __device__ __forceinline__ cx<R> at(const LDiagTab &d, int r) const
    {
        const cx<R> v = cmul(w, ((const cx<R> *)d.tab)[d.offR + r]);
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

// The rotation by phi on the pair (x, y), (c x - s y, s x + c y), as three
// shears: x -= t y, y += s x, x -= t y with t = tan(phi / 2), s = sin phi
// (1 - s t = cos phi and t (1 + cos phi) = sin phi).  Three multiply-adds
// per component pair instead of four; the angle's table keeps |phi| <=
// pi / 2, so |t| <= 1.  The inverse is (-t, -s).
template <typename R>
__device__ __forceinline__ void rot_pair(cx<R> &x, cx<R> &y, R t, R sn)
{
    x.re -= t * y.re;
    x.im -= t * y.im;
    y.re += sn * x.re;
    y.im += sn * x.im;
    x.re -= t * y.re;
    x.im -= t * y.im;
}

// Whether tile bit j holds an active gate: from the compile-time mask AM
// when it is set (the kernels compile the two common patterns), else from
// the pass arguments.  AM with kActRuntime still reads the pass arguments
// and only lets the chains skip: the reverse bodies keep fewer registers
// live with the per-gate branches than with straight-line code.
constexpr uint32_t kActRuntime = 1u << 31;
template <uint32_t AM>
__device__ __forceinline__ bool on(const FusedArgs &a, int j)
{
    if constexpr (AM != 0 && !(AM & kActRuntime)) return (AM >> j) & 1;
    else return (a.active >> j) & 1;
}

// Shear coefficients (t, s) of one rotation layer's RY gates on the K tile
// qubits, read once per block: inside the tile loop each gate would
// otherwise wait for its own load.  Only the pass's active qubits are read
// (the gates the assignments apply); the others hold the identity (0, 0).
template <typename R, int K, uint32_t AM = 0>
struct RyC {
    R t[K], s[K];
    __device__ __forceinline__ RyC(const FusedArgs &a, int layer)
    {
        const cx<R> *ry = (const cx<R> *)a.ry + (int64_t)layer * a.nparam_layer;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            t[j] = R(0);
            s[j] = R(0);
            if (on<AM>(a, j)) {
                const cx<R> e = ry[a.pos[j]];
                t[j] = e.re;
                s[j] = e.im;
            }
        }
    }
};

// forward rotations of the tile bits that are new in assignment AI
template <typename R, int K, int LOGR, int AI, uint32_t AM>
__device__ __forceinline__ void fwd_assign(cx<R> (&v)[1 << LOGR], const FusedArgs &a,
                                           const RyC<R, K, AM> &rc)
{
    using T = Tile<K, LOGR>;
    constexpr int LO = T::lo(AI);
    constexpr uint32_t NEW = T::newbits(AI);
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        const int j = LO + k;
        if (!((NEW >> j) & 1) || !on<AM>(a, j)) continue;
        const R tn = rc.t[j], sn = rc.s[j];
#pragma unroll
        for (int r = 0; r < T::NR; ++r)
            if (!(r & (1 << k))) rot_pair(v[r], v[r | (1 << k)], tn, sn);
    }
}

// reverse step of the tile bits new in assignment AI: gradient partial of
// RY (Im<lam|Y_q|phi> = Re(conj(l1) f0) - Re(conj(l0) f1) over the pairs),
// then RY(-theta) on both vectors
template <typename R, int K, int LOGR, int AI, uint32_t AM>
__device__ __forceinline__ void bwd_assign(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR],
                                           double (&accY)[K], const FusedArgs &a,
                                           const RyC<R, K, AM> &rc)
{
    using T = Tile<K, LOGR>;
    constexpr int LO = T::lo(AI);
    constexpr uint32_t NEW = T::newbits(AI);
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        const int j = LO + k;
        if (!((NEW >> j) & 1) || !on<AM>(a, j)) continue;
        const R tn = -rc.t[j], sn = -rc.s[j];
        R g = 0;
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            if (r & (1 << k)) continue;
            const int r1 = r | (1 << k);
            g += (l[r1].re * f[r].re + l[r1].im * f[r].im) - (l[r].re * f[r1].re + l[r].im * f[r1].im);
            rot_pair(f[r], f[r1], tn, sn);
            rot_pair(l[r], l[r1], tn, sn);
        }
        accY[j] += (double)g;
    }
}

// RY partials of the tile bits new in assignment AI from (phi, lam) taken
// at the same point, without rotating: Im<lam|Y_q|phi> over the pairs
template <typename R, int K, int LOGR, int AI, uint32_t AM>
__device__ __forceinline__ void ygrad_assign(const cx<R> (&f)[1 << LOGR], const cx<R> (&l)[1 << LOGR],
                                             double (&accY)[K], const FusedArgs &a)
{
    using T = Tile<K, LOGR>;
    constexpr int LO = T::lo(AI);
    constexpr uint32_t NEW = T::newbits(AI);
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        const int j = LO + k;
        if (!((NEW >> j) & 1) || !on<AM>(a, j)) continue;
        R g = 0;
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            if (r & (1 << k)) continue;
            const int r1 = r | (1 << k);
            g += (l[r1].re * f[r].re + l[r1].im * f[r].im) - (l[r].re * f[r1].re + l[r].im * f[r1].im);
        }
        accY[j] += (double)g;
    }
}

// RY(-theta) of the tile bits new in assignment AI on one vector
template <typename R, int K, int LOGR, int AI, uint32_t AM>
__device__ __forceinline__ void inv_assign(cx<R> (&v)[1 << LOGR], const FusedArgs &a,
                                           const RyC<R, K, AM> &rc)
{
    using T = Tile<K, LOGR>;
    constexpr int LO = T::lo(AI);
    constexpr uint32_t NEW = T::newbits(AI);
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        const int j = LO + k;
        if (!((NEW >> j) & 1) || !on<AM>(a, j)) continue;
        const R tn = -rc.t[j], sn = -rc.s[j];
#pragma unroll
        for (int r = 0; r < T::NR; ++r)
            if (!(r & (1 << k))) rot_pair(v[r], v[r | (1 << k)], tn, sn);
    }
}

template <typename R, int K, int LOGR, int LFROM, int LTO>
__device__ __forceinline__ void exchange(cx<R> (&v)[1 << LOGR], cx<R> *lds, int t)
{
    using T = Tile<K, LOGR>;
    __syncthreads();
    cx<R> *wr = lds + (T::lds_linear(LFROM) ? T::lds_index(t, 0, LFROM) : 0);
#pragma unroll
    for (int r = 0; r < T::NR; ++r) {
        if constexpr (T::lds_linear(LFROM)) wr[r * T::lds_stride(LFROM)] = v[r];
        else lds[T::lds_index(t, r, LFROM)] = v[r];
    }
    __syncthreads();
    const cx<R> *rd = lds + (T::lds_linear(LTO) ? T::lds_index(t, 0, LTO) : 0);
#pragma unroll
    for (int r = 0; r < T::NR; ++r) {
        if constexpr (T::lds_linear(LTO)) v[r] = rd[r * T::lds_stride(LTO)];
        else v[r] = lds[T::lds_index(t, r, LTO)];
    }
}

// The chains below run assignments one after the other, each after an
// exchange into its layout.  With a compile-time active mask AM, an
// assignment in the middle of a chain whose tile bits hold no active gate
// (in every pass after the first, the kept low bits) is skipped, the data
// going straight from the layout it is in (LF) to the next assignment's.
// The first and last layouts never change.

template <typename R, int K, int LOGR, int AI, uint32_t AM, int LF = Tile<K, LOGR>::lo(AI - 1)>
struct FwdChain {
    __device__ static __forceinline__ void run(cx<R> (&v)[1 << LOGR], cx<R> *lds, int t,
                                               const FusedArgs &a, const RyC<R, K, AM> &rc)
    {
        using T = Tile<K, LOGR>;
        if constexpr ((AI + 1 < T::NA) && AM != 0 && !(AM & T::newbits(AI)))
            return FwdChain<R, K, LOGR, AI + 1, AM, LF>::run(v, lds, t, a, rc);
        exchange<R, K, LOGR, LF, T::lo(AI)>(v, lds, t);
        fwd_assign<R, K, LOGR, AI, AM>(v, a, rc);
        if constexpr (AI + 1 < T::NA) FwdChain<R, K, LOGR, AI + 1, AM>::run(v, lds, t, a, rc);
    }
};

// forward assignments in the order AI, AI-1, ..., 0 (each after an exchange
// from AI+1): the second layer of a two-layer pass
template <typename R, int K, int LOGR, int AI, uint32_t AM, int LF = Tile<K, LOGR>::lo(AI + 1)>
struct FwdChainRev {
    __device__ static __forceinline__ void run(cx<R> (&v)[1 << LOGR], cx<R> *lds, int t,
                                               const FusedArgs &a, const RyC<R, K, AM> &rc)
    {
        using T = Tile<K, LOGR>;
        if constexpr ((AI > 0) && AM != 0 && !(AM & T::newbits(AI)))
            return FwdChainRev<R, K, LOGR, AI - 1, AM, LF>::run(v, lds, t, a, rc);
        exchange<R, K, LOGR, LF, T::lo(AI)>(v, lds, t);
        fwd_assign<R, K, LOGR, AI, AM>(v, a, rc);
        if constexpr (AI > 0) FwdChainRev<R, K, LOGR, AI - 1, AM>::run(v, lds, t, a, rc);
    }
};

// reverse assignments AI = 1 .. NA-1, each after an exchange from AI-1
template <typename R, int K, int LOGR, int AI, uint32_t AM, int LF = Tile<K, LOGR>::lo(AI - 1)>
struct BwdChain {
    __device__ static __forceinline__ void run(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR],
                                               double (&accY)[K], cx<R> *lds, int t,
                                               const FusedArgs &a, const RyC<R, K, AM> &rc)
    {
        using T = Tile<K, LOGR>;
        if constexpr ((AI + 1 < T::NA) && AM != 0 && !(AM & T::newbits(AI)))
            return BwdChain<R, K, LOGR, AI + 1, AM, LF>::run(f, l, accY, lds, t, a, rc);
        exchange<R, K, LOGR, LF, T::lo(AI)>(f, lds, t);
        exchange<R, K, LOGR, LF, T::lo(AI)>(l, lds, t);
        bwd_assign<R, K, LOGR, AI, AM>(f, l, accY, a, rc);
        if constexpr (AI + 1 < T::NA)
            BwdChain<R, K, LOGR, AI + 1, AM>::run(f, l, accY, lds, t, a, rc);
    }
};

// reverse assignments in the order AI, AI-1, ..., 0 (each after an exchange
// from AI+1), used where the data ends a forward or reverse part in the last
// assignment
template <typename R, int K, int LOGR, int AI, uint32_t AM, int LF = Tile<K, LOGR>::lo(AI + 1)>
struct BwdChainRev {
    __device__ static __forceinline__ void run(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR],
                                               double (&accY)[K], cx<R> *lds, int t,
                                               const FusedArgs &a, const RyC<R, K, AM> &rc)
    {
        using T = Tile<K, LOGR>;
        if constexpr ((AI > 0) && AM != 0 && !(AM & T::newbits(AI)))
            return BwdChainRev<R, K, LOGR, AI - 1, AM, LF>::run(f, l, accY, lds, t, a, rc);
        exchange<R, K, LOGR, LF, T::lo(AI)>(f, lds, t);
        exchange<R, K, LOGR, LF, T::lo(AI)>(l, lds, t);
        bwd_assign<R, K, LOGR, AI, AM>(f, l, accY, a, rc);
        if constexpr (AI > 0) BwdChainRev<R, K, LOGR, AI - 1, AM>::run(f, l, accY, lds, t, a, rc);
    }
};

// partials of assignments AI .. NA-1, each after an exchange of both vectors
template <typename R, int K, int LOGR, int AI, uint32_t AM, int LF = Tile<K, LOGR>::lo(AI - 1)>
struct GradChain {
    __device__ static __forceinline__ void run(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR],
                                               double (&accY)[K], cx<R> *lds, int t,
                                               const FusedArgs &a)
    {
        using T = Tile<K, LOGR>;
        if constexpr ((AI + 1 < T::NA) && AM != 0 && !(AM & T::newbits(AI)))
            return GradChain<R, K, LOGR, AI + 1, AM, LF>::run(f, l, accY, lds, t, a);
        exchange<R, K, LOGR, LF, T::lo(AI)>(f, lds, t);
        exchange<R, K, LOGR, LF, T::lo(AI)>(l, lds, t);
        ygrad_assign<R, K, LOGR, AI, AM>(f, l, accY, a);
        if constexpr (AI + 1 < T::NA) GradChain<R, K, LOGR, AI + 1, AM>::run(f, l, accY, lds, t, a);
    }
};

// RY(-theta) of assignments AI, AI-1, .., 0 on one vector, each after an
// exchange from AI+1
template <typename R, int K, int LOGR, int AI, uint32_t AM, int LF = Tile<K, LOGR>::lo(AI + 1)>
struct InvChainRev {
    __device__ static __forceinline__ void run(cx<R> (&v)[1 << LOGR], cx<R> *lds, int t,
                                               const FusedArgs &a, const RyC<R, K, AM> &rc)
    {
        using T = Tile<K, LOGR>;
        if constexpr ((AI > 0) && AM != 0 && !(AM & T::newbits(AI)))
            return InvChainRev<R, K, LOGR, AI - 1, AM, LF>::run(v, lds, t, a, rc);
        exchange<R, K, LOGR, LF, T::lo(AI)>(v, lds, t);
        inv_assign<R, K, LOGR, AI, AM>(v, a, rc);
        if constexpr (AI > 0) InvChainRev<R, K, LOGR, AI - 1, AM>::run(v, lds, t, a, rc);
    }
};

// partials of assignments AI, AI-1, .., 0, each after an exchange of both
// vectors from AI+1
template <typename R, int K, int LOGR, int AI, uint32_t AM, int LF = Tile<K, LOGR>::lo(AI + 1)>
struct GradChainRev {
    __device__ static __forceinline__ void run(cx<R> (&f)[1 << LOGR], cx<R> (&l)[1 << LOGR],
                                               double (&accY)[K], cx<R> *lds, int t,
                                               const FusedArgs &a)
    {
        using T = Tile<K, LOGR>;
        if constexpr ((AI > 0) && AM != 0 && !(AM & T::newbits(AI)))
            return GradChainRev<R, K, LOGR, AI - 1, AM, LF>::run(f, l, accY, lds, t, a);
        exchange<R, K, LOGR, LF, T::lo(AI)>(f, lds, t);
        exchange<R, K, LOGR, LF, T::lo(AI)>(l, lds, t);
        ygrad_assign<R, K, LOGR, AI, AM>(f, l, accY, a);
        if constexpr (AI > 0) GradChainRev<R, K, LOGR, AI - 1, AM>::run(f, l, accY, lds, t, a);
    }
};

// RY(-theta) of assignments AI .. NA-1 on one vector, each after an exchange
// from AI-1
template <typename R, int K, int LOGR, int AI, uint32_t AM, int LF = Tile<K, LOGR>::lo(AI - 1)>
struct InvChain {
    __device__ static __forceinline__ void run(cx<R> (&v)[1 << LOGR], cx<R> *lds, int t,
                                               const FusedArgs &a, const RyC<R, K, AM> &rc)
    {
        using T = Tile<K, LOGR>;
        if constexpr ((AI + 1 < T::NA) && AM != 0 && !(AM & T::newbits(AI)))
            return InvChain<R, K, LOGR, AI + 1, AM, LF>::run(v, lds, t, a, rc);
        exchange<R, K, LOGR, LF, T::lo(AI)>(v, lds, t);
        inv_assign<R, K, LOGR, AI, AM>(v, a, rc);
        if constexpr (AI + 1 < T::NA) InvChain<R, K, LOGR, AI + 1, AM>::run(v, lds, t, a, rc);
    }
};

// A tile's registers in the load assignment, plain loads (o: tile base |
// thread offset)
template <typename R, int LOGR, bool CONTIG>
__device__ __forceinline__ void prefetch_tile(cx<R> (&v)[1 << LOGR], const cx<R> *src, u64 o,
                                              const RegMap<LOGR, CONTIG> &m)
{
#pragma unroll
    for (int r = 0; r < (1 << LOGR); ++r) v[r] = ld_amp(src + o + m.off(r));
}

// Load a pass's tile in the load assignment.  In pass 0 the loaded values
// may be multiplied by the layer diagonal (IN_LOAD_DIAG) or replaced by the
// generated first-layer state (IN_GENERATE).
// PL: the caller guarantees mode == IN_LOAD (the common case, compiled
// without the table code).
template <typename R, int K, int LOGR, bool CONTIG, bool PL = false>
__device__ __forceinline__ void load_tile(cx<R> (&v)[1 << LOGR], const cx<R> *src, u64 base,
                                          u64 toff, const RegMap<LOGR, CONTIG> &m, int mode,
                                          P0Diag<R, K, LOGR> &pd, const DiagTab &d, int t)
{
    constexpr int NR = 1 << LOGR;
    const cx<R> *sp = src + (base | toff);
    if constexpr (PL) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = ld_amp(sp + m.off(r));
        return;
    }
    if (mode != IN_LOAD) pd.tile(d, base, t);
    if (mode == IN_GENERATE) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = pd.at(d, r);
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = ld_amp(sp + m.off(r));
        if (mode == IN_LOAD_DIAG) {
#pragma unroll
            for (int r = 0; r < NR; ++r) v[r] = cmul(v[r], pd.at(d, r));
        }
    }
}

// The pass bodies below take the tiles t0, t0 + tstep, ... so that a grid
// of blocks (t0 = blockIdx.x, tstep = gridDim.x) or a single block that owns
// a whole batch instance (t0 = 0, tstep = 1) can run them; col is the
// partial-sum column the block writes.
// The two active masks the kernels compile bodies for: pass 0 (every tile
// bit) and the later passes (all but the kept low bits: 4 for complex64, 3
// for complex128).  Other masks run the generic body (AM = 0).
template <int K>
constexpr uint32_t act_full()
{
    return (1u << K) - 1u;
}
template <typename R, int K>
constexpr uint32_t act_later()
{
    return act_full<K>() & ~((1u << (sizeof(R) == 4 ? 4 : 3)) - 1u);
}

// Each pass kernel is compiled once per mask selector MS, so that every
// variant gets its own register allocation (a kernel holding the three
// bodies would run all of them at the occupancy of the largest): MS_FULL and
// MS_LATER compile the two masks above into the body, MS_ANY reads the
// pass's mask at run time.  RT: the body still reads the mask at run time,
// keeping the chains' per-gate branches (fewer live registers in the
// reverse bodies that rotate both vectors); the whole-assignment skips still
// come from the compiled mask.
enum { MS_ANY = 0, MS_FULL = 1, MS_LATER = 2 };

// The pass kernels, and the waves per SIMD each variant is compiled for
// (its register budget: 4 waves = 128 VGPRs, 3 = 168, 2 = 256).  1 leaves
// the compiler's own choice.  The complex64 two-layer reverse passes are held
// to 3 waves: their bodies want ~175-220 registers, and the third wave hides
// more of the exchanges' barrier waits than the ~30 registers spilled (a few
// scratch accesses per tile) cost.
enum PassKind {
    PK_FWD_PASS, PK_FWD_LOAD_PASS, PK_FWD2_PASS, PK_FWD2_LOAD_PASS, PK_TURN_PASS,
    PK_TURN_LOAD_PASS, PK_BWD_PASS, PK_BWD_LD_PASS, PK_BWD_GF_PASS, PK_BWD_GF_LD_PASS,
    PK_BWD2_PASS, PK_BWD2_PHI_PASS
};
template <typename R>
constexpr int pass_waves(int kind, int ms)
{
    const bool bwd2 = kind == PK_BWD2_PASS || kind == PK_BWD2_PHI_PASS;
    return (sizeof(R) == 4 && ms != MS_ANY && bwd2) ? 3 : 1;
}
template <typename R, int K, int MS, bool RT = false>
constexpr uint32_t pass_mask()
{
    return (MS == MS_FULL ? act_full<K>() : (MS == MS_LATER ? act_later<R, K>() : 0u)) |
           (RT && MS != MS_ANY ? kActRuntime : 0u);
}

template <typename R, int K, int LOGR, bool CONTIG, bool PL = false, uint32_t AM = 0>
__device__ __forceinline__ void fwd_body(cx<R> *psi, const cx<R> *src, const FusedArgs &a,
                                         u64 t0, u64 tstep, cx<R> *lds)
{
    using T = Tile<K, LOGR>;
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    RegMap<LOGR, CONTIG> mld, mst;
    mld.init(a.pos + LD);
    mst.init(a.pos + ST);
    P0Diag<R, K, LOGR> pd;
    if (a.in_mode != IN_LOAD) pd.init(a.dt, t);
    const RyC<R, K, AM> rc(a, a.layer);
    // plain loads: the next tile's loads go out before this tile's chain
    // (the exchange barriers do not wait for them), one tile of registers
    cx<R> nx[T::NR];
    if constexpr (PL)
        if (t0 < a.ntiles) prefetch_tile<R, LOGR, CONTIG>(nx, src, tile_base(t0, a) | toff_ld, mld);
    for (u64 tile = t0; tile < a.ntiles; tile += tstep) {
        const u64 base = tile_base(tile, a);
        cx<R> v[T::NR];
        if constexpr (PL) {
#pragma unroll
            for (int r = 0; r < T::NR; ++r) v[r] = nx[r];
            if (tile + tstep < a.ntiles)
                prefetch_tile<R, LOGR, CONTIG>(nx, src, tile_base(tile + tstep, a) | toff_ld, mld);
        } else {
            load_tile<R, K, LOGR, CONTIG, PL>(v, src, base, toff_ld, mld, a.in_mode, pd, a.dt, t);
        }
        fwd_assign<R, K, LOGR, 0, AM>(v, a, rc);
        if constexpr (T::NA > 1) FwdChain<R, K, LOGR, 1, AM>::run(v, lds, t, a, rc);
        cx<R> *pp = psi + fresh(base | toff_st);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) st_amp(pp + mst.off(r), v[r]);
    }
}

template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_FWD_PASS, MS)) void k_fwd_pass(void *psi_, const void *src_,
                                                              FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    const int b = blockIdx.x, g = gridDim.x;
    fwd_body<R, K, LOGR, CONTIG, false, pass_mask<R, K, MS>()>((cx<R> *)psi_, (const cx<R> *)src_, a, b, g, lds);
}

// the same for a plain load (no diagonal on load, no generated layer)
template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_FWD_LOAD_PASS, MS)) void k_fwd_load_pass(void *psi_, const void *src_,
                                                                   FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    const int b = blockIdx.x, g = gridDim.x;
    fwd_body<R, K, LOGR, CONTIG, true, pass_mask<R, K, MS>()>((cx<R> *)psi_, (const cx<R> *)src_, a, b, g, lds);
}

// Block sums of the gradient partials of the pass's active tile qubits for
// rotation layer `layer`.  The RZ partials come as one accumulator per
// register bit of assignment AZ (accZr) and one per-thread total (ztot)
// whose sign for a thread bit is that bit of the thread id; HAVEZ = false
// writes zeros.
template <typename R, int K, int LOGR, int AZ, bool HAVEZ>
__device__ __forceinline__ void write_partials(const double (&accY)[K], const double (&accZr)[LOGR],
                                               double ztot, double *sh, const FusedArgs &a,
                                               int layer, int col)
{
    constexpr int LZ = Tile<K, LOGR>::lo(AZ);
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!((a.active >> j) & 1)) continue;
        const bool keep = (a.qmask >> a.pos[j]) & 1;
        const int64_t row = (int64_t)layer * a.nparam_layer + a.pos[j];
        const double y = block_sum(accY[j], sh);
        if (t == 0) a.part[row * a.grid + col] = keep ? y : 0.0;
        double z = 0.0;
        if constexpr (HAVEZ) {
            const int tb = j < LZ ? j : j - LOGR;   // thread-id bit of tile bit j
            const bool reg = j >= LZ && j < LZ + LOGR;
            z = block_sum(reg ? accZr[j - LZ] : (((t >> tb) & 1) ? -ztot : ztot), sh);
        }
        if (t == 0) a.part[(row + a.n) * a.grid + col] = keep ? z : 0.0;
    }
}

// RZ partials of the active tile qubits in assignment AI: per register bit
// the signed sum of Im(conj(lam_i) phi_i), and the thread's total (its sign
// per thread bit is applied at the block sum)
template <typename R, int K, int LOGR, int AI, uint32_t AM>
__device__ __forceinline__ void z_partials(const cx<R> (&f)[1 << LOGR], const cx<R> (&l)[1 << LOGR],
                                           double (&accZr)[LOGR], double &ztot, const FusedArgs &a)
{
    constexpr int NR = 1 << LOGR, LZ = Tile<K, LOGR>::lo(AI);
    R tt[NR];
    R tsum = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        tt[r] = l[r].re * f[r].im - l[r].im * f[r].re;
        tsum += tt[r];
    }
    ztot += (double)tsum;
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        if (!on<AM>(a, LZ + k)) continue;
        R s = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) s += ((r >> k) & 1) ? -tt[r] : tt[r];
        accZr[k] += (double)s;
    }
}

// LDG: both vectors first lose the diagonal of `layer` in the load layout
// (a.ld), for the reverse of a two-layer pass.
template <typename R, int K, int LOGR, bool CONTIG, bool LDG, uint32_t AM = 0>
__device__ __forceinline__ void bwd_body(const cx<R> *phi_in, cx<R> *phi, cx<R> *lam,
                                         const FusedArgs &a, u64 t0, u64 tstep, int col,
                                         cx<R> *lds, double *sh)
{
    using T = Tile<K, LOGR>;
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
    LDiag<R, K, LOGR> dg;
    double accY[K], accZr[LOGR], ztot = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) accY[j] = 0.0;
#pragma unroll
    for (int k = 0; k < LOGR; ++k) accZr[k] = 0.0;

    const RyC<R, K, AM> rc(a, a.layer);
    for (u64 tile = t0; tile < a.ntiles; tile += tstep) {
        const u64 base = tile_base(tile, a);
        cx<R> f[T::NR], l[T::NR];
        if (a.phi_gen) {
            pg.tile(a.gt, base, t);
#pragma unroll
            for (int r = 0; r < T::NR; ++r) f[r] = pg.at(a.gt, r);
        } else {
#pragma unroll
            for (int r = 0; r < T::NR; ++r) f[r] = ld_amp(phi_in + (base | toff_ld) + mld.off(r));
        }
#pragma unroll
        for (int r = 0; r < T::NR; ++r) l[r] = ld_amp(lam + (base | toff_ld) + mld.off(r));
        if (any_diag) {
            pd.tile(a.dt, base, t);
#pragma unroll
            for (int r = 0; r < T::NR; ++r) {
                const cx<R> d = pd.at(a.dt, r);
                if (a.diag_phi) f[r] = cmul_conj(f[r], d);
                if (a.diag_lam) l[r] = cmul_conj(l[r], d);
            }
        }
        if constexpr (LDG) {
            dg.tile(a.ld, tile, base | toff_ld, t);
#pragma unroll
            for (int r = 0; r < T::NR; ++r) {
                const cx<R> d = dg.at(a.ld, r);
                f[r] = cmul_conj(f[r], d);
                l[r] = cmul_conj(l[r], d);
            }
        }
        // RZ gradients of the active tile qubits: sum_i z_q(i) Im(conj(lam_i) phi_i)
        z_partials<R, K, LOGR, 0, AM>(f, l, accZr, ztot, a);
        bwd_assign<R, K, LOGR, 0, AM>(f, l, accY, a, rc);
        if constexpr (T::NA > 1) BwdChain<R, K, LOGR, 1, AM>::run(f, l, accY, lds, t, a, rc);
        const u64 o = fresh(base | toff_st);
        cx<R> *pf = phi + o, *pl = lam + o;
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            if (a.store_phi) st_amp(pf + mst.off(r), f[r]);
            if (a.store_lam) st_amp(pl + mst.off(r), l[r]);
        }
    }
    write_partials<R, K, LOGR, 0, true>(accY, accZr, ztot, sh, a, a.layer, col);
}

template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_BWD_PASS, MS)) void k_bwd_pass(const void *phi_in_, void *phi_,
                                                              void *lam_, FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int b = blockIdx.x, g = gridDim.x;
    bwd_body<R, K, LOGR, CONTIG, false, pass_mask<R, K, MS, true>()>((const cx<R> *)phi_in_, (cx<R> *)phi_, (cx<R> *)lam_, a, b, g, b, lds, sh);
}

// the reverse pass that first undoes the layer diagonal given in a.ld
template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_BWD_LD_PASS, MS)) void k_bwd_ld_pass(const void *phi_in_, void *phi_,
                                                                 void *lam_, FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int b = blockIdx.x, g = gridDim.x;
    bwd_body<R, K, LOGR, CONTIG, true, pass_mask<R, K, MS, true>()>((const cx<R> *)phi_in_, (cx<R> *)phi_, (cx<R> *)lam_, a, b, g, b, lds, sh);
}

// Reverse pass that does not write phi back: every RY and RZ partial of the
// pass is taken from (phi, lam) at the pass's end point (the pass's RY gates
// act on distinct qubits, so Y_q and Z_q commute with all of them but RY_q,
// which commutes with Y_q), visiting the assignments 0 .. NA-1 with both
// vectors; then lam alone is rotated back through NA-1 .. 0 and stored in
// the load layout.  phi dies after the partials.
template <typename R, int K, int LOGR, bool CONTIG, bool LDG, uint32_t AM = 0>
__device__ __forceinline__ void bwd_gf_body(const cx<R> *phi_in, cx<R> *lam, const FusedArgs &a,
                                            u64 t0, u64 tstep, int col, cx<R> *lds, double *sh)
{
    using T = Tile<K, LOGR>;
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a);
    RegMap<LOGR, CONTIG> mld;
    mld.init(a.pos + LD);
    P0Diag<R, K, LOGR> pd;
    if (a.diag_lam) pd.init(a.dt, t);
    LDiag<R, K, LOGR> dg;
    double accY[K], accZr[LOGR], ztot = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) accY[j] = 0.0;
#pragma unroll
    for (int k = 0; k < LOGR; ++k) accZr[k] = 0.0;

    const RyC<R, K, AM> rc(a, a.layer);
    for (u64 tile = t0; tile < a.ntiles; tile += tstep) {
        const u64 base = tile_base(tile, a);
        const cx<R> *fp = phi_in + (base | toff_ld);
        const cx<R> *lp = lam + (base | toff_ld);
        cx<R> f[T::NR], l[T::NR];
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            f[r] = ld_amp(fp + mld.off(r));
            l[r] = ld_amp(lp + mld.off(r));
        }
        if (a.diag_lam) {
            pd.tile(a.dt, base, t);
#pragma unroll
            for (int r = 0; r < T::NR; ++r) l[r] = cmul_conj(l[r], pd.at(a.dt, r));
        }
        if constexpr (LDG) {
            dg.tile(a.ld, tile, base | toff_ld, t);
#pragma unroll
            for (int r = 0; r < T::NR; ++r) {
                const cx<R> d = dg.at(a.ld, r);
                f[r] = cmul_conj(f[r], d);
                l[r] = cmul_conj(l[r], d);
            }
        }
        z_partials<R, K, LOGR, 0, AM>(f, l, accZr, ztot, a);
        ygrad_assign<R, K, LOGR, 0, AM>(f, l, accY, a);
        if constexpr (T::NA > 1) GradChain<R, K, LOGR, 1, AM>::run(f, l, accY, lds, t, a);
        inv_assign<R, K, LOGR, T::NA - 1, AM>(l, a, rc);
        if constexpr (T::NA > 1) InvChainRev<R, K, LOGR, T::NA - 2, AM>::run(l, lds, t, a, rc);
        cx<R> *ls = lam + fresh(base | toff_ld);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) st_amp(ls + mld.off(r), l[r]);
    }
    write_partials<R, K, LOGR, 0, true>(accY, accZr, ztot, sh, a, a.layer, col);
}

template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_BWD_GF_PASS, MS)) void k_bwd_gf_pass(const void *phi_in_, void *lam_,
                                                                 FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int b = blockIdx.x, g = gridDim.x;
    bwd_gf_body<R, K, LOGR, CONTIG, false, pass_mask<R, K, MS, true>()>((const cx<R> *)phi_in_, (cx<R> *)lam_, a, b, g, b, lds, sh);
}

template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_BWD_GF_LD_PASS, MS)) void k_bwd_gf_ld_pass(const void *phi_in_,
                                                                    void *lam_, FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int b = blockIdx.x, g = gridDim.x;
    bwd_gf_body<R, K, LOGR, CONTIG, true, pass_mask<R, K, MS, true>()>((const cx<R> *)phi_in_, (cx<R> *)lam_, a, b, g, b, lds, sh);
}

// Reverse of a two-layer pass (rotation layers la = a.layer and lb =
// a.layer2 on the same tile qubits) in one sweep from the pass's end point
// (phi_src, the state the pass wrote, with lam at the same point).  Per tile
// both vectors go back together: the RZ partials of lb there, then through
// RY_lb (assignments 0 .. NA-1, each RY partial taken before its gate is
// undone), the RZ partials of la (the diagonal D_la commutes with Z_q, so
// they can be taken before it is undone), D_la, and RY_la in the order
// NA-1 .. 0.  lam is stored; phi only when the next reverse pass needs it
// (a.store_phi, the modes that keep no copy of the pass's input).  It moves
// 3 A s (4 with phi) where the two single-layer reverse passes move 7 (8).
template <typename R, int K, int LOGR, bool CONTIG, bool SP, uint32_t AM = 0>
__device__ __forceinline__ void bwd2_body(const cx<R> *phi_src, cx<R> *phi, cx<R> *lam,
                                          const FusedArgs &a, u64 t0, u64 tstep, int col,
                                          cx<R> *lds, double *sh)
{
    using T = Tile<K, LOGR>;
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    RegMap<LOGR, CONTIG> mld;
    mld.init(a.pos + LD);
    LDiag<R, K, LOGR> dg;
    double accYa[K], accYb[K], accZa[LOGR], accZb[LOGR], zta = 0.0, ztb = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) accYa[j] = accYb[j] = 0.0;
#pragma unroll
    for (int k = 0; k < LOGR; ++k) accZa[k] = accZb[k] = 0.0;

    const RyC<R, K, AM> rca(a, a.layer), rcb(a, a.layer2);
    for (u64 tile = t0; tile < a.ntiles; tile += tstep) {
        const u64 base = tile_base(tile, a);
        // the diagonal's per-tile factors first: its loop over the straddling
        // pairs placed between the two layers' chains costs ~200 registers
        dg.tile(a.ld, tile, base | toff_st, t);
        cx<R> f[T::NR], l[T::NR];
        {
            const cx<R> *fp = phi_src + (base | toff_ld);
            const cx<R> *lp = lam + (base | toff_ld);
#pragma unroll
            for (int r = 0; r < T::NR; ++r) {
                f[r] = ld_amp(fp + mld.off(r));
                l[r] = ld_amp(lp + mld.off(r));
            }
        }
        // layer lb
        z_partials<R, K, LOGR, 0, AM>(f, l, accZb, ztb, a);
        bwd_assign<R, K, LOGR, 0, AM>(f, l, accYb, a, rcb);
        if constexpr (T::NA > 1) BwdChain<R, K, LOGR, 1, AM>::run(f, l, accYb, lds, t, a, rcb);
        // layer la: RZ partials, D_la undone on both, then the RY gates
        z_partials<R, K, LOGR, T::NA - 1, AM>(f, l, accZa, zta, a);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            const cx<R> d = dg.at(a.ld, r);
            f[r] = cmul_conj(f[r], d);
            l[r] = cmul_conj(l[r], d);
        }
        bwd_assign<R, K, LOGR, T::NA - 1, AM>(f, l, accYa, a, rca);
        if constexpr (T::NA > 1)
            BwdChainRev<R, K, LOGR, T::NA - 2, AM>::run(f, l, accYa, lds, t, a, rca);
        const u64 o = fresh(base | toff_ld);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            if constexpr (SP) st_amp(phi + o + mld.off(r), f[r]);
            st_amp(lam + o + mld.off(r), l[r]);
        }
    }
    write_partials<R, K, LOGR, 0, true>(accYb, accZb, ztb, sh, a, a.layer2, col);
    write_partials<R, K, LOGR, T::NA - 1, true>(accYa, accZa, zta, sh, a, a.layer, col);
}

template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_BWD2_PASS, MS)) void k_bwd2_pass(
    const void *phi_src_, void *phi_, void *lam_, FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int b = blockIdx.x, g = gridDim.x;
    bwd2_body<R, K, LOGR, CONTIG, false, pass_mask<R, K, MS>()>(
        (const cx<R> *)phi_src_, (cx<R> *)phi_, (cx<R> *)lam_, a, b, g, b, lds, sh);
}

// the same, carrying phi back too (a.store_phi)
template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_BWD2_PHI_PASS, MS)) void k_bwd2_phi_pass(
    const void *phi_src_, void *phi_, void *lam_, FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int b = blockIdx.x, g = gridDim.x;
    bwd2_body<R, K, LOGR, CONTIG, true, pass_mask<R, K, MS>()>(
        (const cx<R> *)phi_src_, (cx<R> *)phi_, (cx<R> *)lam_, a, b, g, b, lds, sh);
}

// Last forward pass of the last layer + energy + first reverse pass, for a
// Z-only Hamiltonian with diagonal D: in each tile psi gets the pass's RY
// gates (assignments 0 .. NA-1), E += sum D_i |psi_i|^2 and lam = D psi;
// the RY partials of the pass are taken right there, at the pass's end point
// (assignments NA-1 .. 0 with both vectors), then lam alone is rotated back
// (0 .. NA-1) and stored; psi is not written (it equals the loaded tile's
// source, which stays in HBM).  RZ partials of the tile qubits are zero
// here: Im(conj(D_i psi_i) psi_i) = 0.  When this is the layer's only pass,
// the load applies the previous layer's diagonal (or generates the first
// layer's state).
template <typename R, int K, int LOGR, bool CONTIG, bool PL, uint32_t AM = 0>
__device__ __forceinline__ void turn_body(const cx<R> *psi, cx<R> *lam, const FusedArgs &a,
                                          u64 t0, u64 tstep, int col, cx<R> *lds, double *sh)
{
    using T = Tile<K, LOGR>;
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    RegMap<LOGR, CONTIG> mld, mst;
    mld.init(a.pos + LD);
    mst.init(a.pos + ST);
    P0Diag<R, K, LOGR> pd;
    if (a.in_mode != IN_LOAD) pd.init(a.dt, t);
    double accY[K], accZr[LOGR];
#pragma unroll
    for (int j = 0; j < K; ++j) accY[j] = 0.0;
    double eacc = 0.0;

    const RyC<R, K, AM> rc(a, a.layer);
    for (u64 tile = t0; tile < a.ntiles; tile += tstep) {
        const u64 base = tile_base(tile, a);
        cx<R> f[T::NR], l[T::NR];
        load_tile<R, K, LOGR, CONTIG, PL>(f, psi, base, toff_ld, mld, a.in_mode, pd, a.dt, t);
        fwd_assign<R, K, LOGR, 0, AM>(f, a, rc);
        if constexpr (T::NA > 1) FwdChain<R, K, LOGR, 1, AM>::run(f, lds, t, a, rc);
        // energy and lam in the last assignment's layout
        // E in FP64 from the FP64 diagonal: D_i |psi_i|^2 per amplitude
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            const double d = __builtin_nontemporal_load(a.hdiag + (base | toff_st) + mst.off(r));
            const double fr = (double)f[r].re, fi = (double)f[r].im;
            eacc += d * (fr * fr + fi * fi);
            l[r].re = (R)d * f[r].re;
            l[r].im = (R)d * f[r].im;
        }
        ygrad_assign<R, K, LOGR, T::NA - 1, AM>(f, l, accY, a);
        if constexpr (T::NA > 1)
            GradChainRev<R, K, LOGR, T::NA - 2, AM>::run(f, l, accY, lds, t, a);
        inv_assign<R, K, LOGR, 0, AM>(l, a, rc);
        if constexpr (T::NA > 1) InvChain<R, K, LOGR, 1, AM>::run(l, lds, t, a, rc);
        cx<R> *pl = lam + fresh(base | toff_st);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) st_amp(pl + mst.off(r), l[r]);
    }
    write_partials<R, K, LOGR, 0, false>(accY, accZr, 0.0, sh, a, a.layer, col);
    const double e = block_sum(eacc, sh);
    if (t == 0) {
        a.epart[col] = e;
        a.epart[a.grid + col] = 0.0;
    }
}

template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_TURN_PASS, MS)) void k_turn_pass(const void *psi_, void *lam_,
                                                               FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int b = blockIdx.x, g = gridDim.x;
    turn_body<R, K, LOGR, CONTIG, false, pass_mask<R, K, MS>()>((const cx<R> *)psi_, (cx<R> *)lam_, a, b, g, b, lds, sh);
}

// the same for a plain load (the layer's last pass is not its only one)
template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_TURN_LOAD_PASS, MS)) void k_turn_load_pass(const void *psi_, void *lam_,
                                                                    FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    const int b = blockIdx.x, g = gridDim.x;
    turn_body<R, K, LOGR, CONTIG, true, pass_mask<R, K, MS>()>((const cx<R> *)psi_, (cx<R> *)lam_, a, b, g, b, lds, sh);
}

// ------------------------------------------------------ two-layer passes

// The last pass of rotation layer `layer` and the first of layer2 = layer + 1
// act on the same tile qubits, so one pass does both: the first layer's RY
// gates through the assignments 0 .. NA-1, the first layer's diagonal in
// the last assignment, then the second layer's RY gates back through
// NA-1 .. 0, and the tile is stored in the load layout.
template <typename R, int K, int LOGR, bool CONTIG, bool PL, uint32_t AM = 0>
__device__ __forceinline__ void fwd2_body(cx<R> *psi, const cx<R> *src, const FusedArgs &a,
                                          u64 t0, u64 tstep, cx<R> *lds)
{
    using T = Tile<K, LOGR>;
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0), ST = T::lo(T::NA - 1);
    const u64 toff_ld = thread_off<K, LOGR>(t, LD, a), toff_st = thread_off<K, LOGR>(t, ST, a);
    RegMap<LOGR, CONTIG> mld;
    mld.init(a.pos + LD);
    P0Diag<R, K, LOGR> pd;
    if (a.in_mode != IN_LOAD) pd.init(a.dt, t);
    LDiag<R, K, LOGR> dg;
    const RyC<R, K, AM> rc(a, a.layer);
    const RyC<R, K, AM> rc2(a, a.layer2);
    cx<R> nx[T::NR];   // the next tile, loaded ahead (plain loads)
    if constexpr (PL)
        if (t0 < a.ntiles) prefetch_tile<R, LOGR, CONTIG>(nx, src, tile_base(t0, a) | toff_ld, mld);
    for (u64 tile = t0; tile < a.ntiles; tile += tstep) {
        const u64 base = tile_base(tile, a);
        cx<R> v[T::NR];
        if constexpr (PL) {
#pragma unroll
            for (int r = 0; r < T::NR; ++r) v[r] = nx[r];
            if (tile + tstep < a.ntiles)
                prefetch_tile<R, LOGR, CONTIG>(nx, src, tile_base(tile + tstep, a) | toff_ld, mld);
        } else {
            load_tile<R, K, LOGR, CONTIG, PL>(v, src, base, toff_ld, mld, a.in_mode, pd, a.dt, t);
        }
        fwd_assign<R, K, LOGR, 0, AM>(v, a, rc);
        if constexpr (T::NA > 1) FwdChain<R, K, LOGR, 1, AM>::run(v, lds, t, a, rc);
        dg.tile(a.ld, tile, base | toff_st, t);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) v[r] = cmul(v[r], dg.at(a.ld, r));
        fwd_assign<R, K, LOGR, T::NA - 1, AM>(v, a, rc2);
        if constexpr (T::NA > 1) FwdChainRev<R, K, LOGR, T::NA - 2, AM>::run(v, lds, t, a, rc2);
        cx<R> *pp = psi + fresh(base | toff_ld);
#pragma unroll
        for (int r = 0; r < T::NR; ++r) st_amp(pp + mld.off(r), v[r]);
    }
}

template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_FWD2_PASS, MS)) void k_fwd2_pass(void *psi_, const void *src_,
                                                               FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    const int b = blockIdx.x, g = gridDim.x;
    fwd2_body<R, K, LOGR, CONTIG, false, pass_mask<R, K, MS>()>((cx<R> *)psi_, (const cx<R> *)src_, a, b, g, lds);
}

template <typename R, int K, int LOGR, bool CONTIG, int MS>
__global__ __launch_bounds__(1 << (K - LOGR), pass_waves<R>(PK_FWD2_LOAD_PASS, MS)) void k_fwd2_load_pass(void *psi_, const void *src_,
                                                                    FusedArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    const int b = blockIdx.x, g = gridDim.x;
    fwd2_body<R, K, LOGR, CONTIG, true, pass_mask<R, K, MS>()>((cx<R> *)psi_, (const cx<R> *)src_, a, b, g, lds);
}

// ------------------------------------------------ first-layer gradients

// Arguments of the first-layer gradient kernel.  The state after the first
// layer's RY gates is the product state G = R_0|0...0>, held as chunk tables
// in gt (no CZ pairs); dt is the first layer's diagonal when lam still sits
// after it.
struct Layer0Args {
    int n;
    u64 ntiles;
    int diag_lam;
    DiagTab dt;
    DiagTab gt;
    double *part;
    int grid;
    u64 qmask;
};

// sum over the block of a complex double, returned to every thread
__device__ __forceinline__ void block_sum2_all(double &x, double &y, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        if (o >= (int)blockDim.x) continue;
        x += __shfl_down(x, o, 64);
        y += __shfl_down(y, o, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
        sh[2 * w] = x;
        sh[2 * w + 1] = y;
    }
    __syncthreads();
    x = y = 0.0;
    for (int i = 0; i < nw; ++i) {
        x += sh[2 * i];
        y += sh[2 * i + 1];
    }
}

// Gradients of the first rotation layer (Eq. 11) from lam alone.  With phi
// the product state G after the layer's RY gates, every RY and RZ gradient
// of the layer is Im<lam'|P_q|G> (P = Y or Z, lam' = lam before the layer's
// diagonal), because P_q commutes with the RY gates of the other qubits and
// with the diagonal gates.  G factorises over the index bits, G_i = T0(t)
// T1(r) B(tile) in the coalesced layout (thread bits = index bits 0..K-LOGR-1,
// register bits = the next LOGR bits, tile id = the rest), and
// (Y_q G)_i = (+i if bit q of i is set, else -i) G_{i ^ 2^q}, so per tile a
// thread needs U = sum_r conj(lam'_r) T1(r), the signed sums of the same
// products for the register bits, and the flipped-partner sums W_k; the
// thread and tile factors multiply in afterwards.  One read of lam replaces
// the layer's reverse passes.
template <typename R, int K, int LOGR>
__global__ __launch_bounds__(1 << (K - LOGR), sizeof(R) == 4 ? 3 : 1) void k_layer0_grad(const void *lam_, Layer0Args a)
{
    constexpr int NR = 1 << LOGR, LD = K - LOGR;
    __shared__ double sh[2 * ((1 << (K - LOGR)) / 64 + 1)];
    const cx<R> *lam = (const cx<R> *)lam_;
    const int t = threadIdx.x;
    const cx<R> *G = (const cx<R> *)a.gt.tab;
    P0Diag<R, K, LOGR> pd;
    if (a.diag_lam) pd.init(a.dt, t);
    const int nb = a.n - K;            // tile-id qubits K .. n-1
    double Vre = 0, Vim = 0;
    double Wre[LOGR], Wim[LOGR], Zre[LOGR], Zim[LOGR];
#pragma unroll
    for (int k = 0; k < LOGR; ++k) Wre[k] = Wim[k] = Zre[k] = Zim[k] = 0.0;
    double bY = 0, bZ = 0;             // thread t < nb: qubit K + t
    const cx<R> g0 = G[t];

    for (u64 tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const u64 base = tile << K;
        cx<R> c[NR];                   // conj(lam'_r)
#pragma unroll
        for (int r = 0; r < NR; ++r) c[r] = lam[base | ((u64)r << LD) | (u64)t];
        if (a.diag_lam) {
            pd.tile(a.dt, base, t);
#pragma unroll
            for (int r = 0; r < NR; ++r) c[r] = cmul_conj(c[r], pd.at(a.dt, r));
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) c[r].im = -c[r].im;
        R ure = 0, uim = 0;
        R zr[LOGR], zi[LOGR], wr[LOGR], wi[LOGR];
#pragma unroll
        for (int k = 0; k < LOGR; ++k) zr[k] = zi[k] = wr[k] = wi[k] = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const cx<R> p = cmul(c[r], G[a.gt.off1 + r]);
            ure += p.re;
            uim += p.im;
#pragma unroll
            for (int k = 0; k < LOGR; ++k) {
                const bool b = (r >> k) & 1;
                zr[k] += b ? -p.re : p.re;
                zi[k] += b ? -p.im : p.im;
                const cx<R> q = cmul(c[r], G[a.gt.off1 + (r ^ (1 << k))]);
                // (+-i) q: +i q = (-q.im, q.re), -i q = (q.im, -q.re)
                wr[k] += b ? -q.im : q.im;
                wi[k] += b ? q.re : -q.re;
            }
        }
        const cx<R> b2 = G[a.gt.off2 + ((base >> a.gt.b2) & a.gt.m2)];
        const cx<R> b3 = G[a.gt.off3 + (base >> a.gt.b3)];
        const double Bre = (double)b2.re * b3.re - (double)b2.im * b3.im;
        const double Bim = (double)b2.re * b3.im + (double)b2.im * b3.re;
        Vre += Bre * ure - Bim * uim;
        Vim += Bre * uim + Bim * ure;
#pragma unroll
        for (int k = 0; k < LOGR; ++k) {
            Wre[k] += Bre * wr[k] - Bim * wi[k];
            Wim[k] += Bre * wi[k] + Bim * wr[k];
            Zre[k] += Bre * zr[k] - Bim * zi[k];
            Zim[k] += Bre * zi[k] + Bim * zr[k];
        }
        // tile-id qubits: S = sum over the tile of conj(lam'_i) T0(t) T1(r)
        if (nb > 0) {
            double Sre = (double)g0.re * ure - (double)g0.im * uim;
            double Sim = (double)g0.re * uim + (double)g0.im * ure;
            block_sum2_all(Sre, Sim, sh);
            if (t < nb) {
                const int q = K + t;
                const bool bit = (base >> q) & 1;
                // Z: sign * Im(B S)
                const double im_bs = Bre * Sim + Bim * Sre;
                bZ += bit ? -im_bs : im_bs;
                // Y: Im((+-i) B' S) with B' the factor of the partner tile
                const u64 fb = base ^ (1ull << q);
                const cx<R> f2 = G[a.gt.off2 + ((fb >> a.gt.b2) & a.gt.m2)];
                const cx<R> f3 = G[a.gt.off3 + (fb >> a.gt.b3)];
                const double Fre = (double)f2.re * f3.re - (double)f2.im * f3.im;
                const double Fim = (double)f2.re * f3.im + (double)f2.im * f3.re;
                const double re_fs = Fre * Sre - Fim * Sim;
                bY += bit ? re_fs : -re_fs;
            }
        }
    }

    const int col = blockIdx.x;
    auto put = [&](int q, double y, double z, bool lane0) {
        if (!lane0) return;
        const bool keep = (a.qmask >> q) & 1;
        a.part[(int64_t)q * a.grid + col] = keep ? y : 0.0;
        a.part[(int64_t)(a.n + q) * a.grid + col] = keep ? z : 0.0;
    };
    // thread bits j: Z = sum_t sign_j(t) Im(T0(t) V), Y = sum_t Im((+-i) T0(t^2^j) V)
    for (int j = 0; j < LD; ++j) {
        const bool bit = (t >> j) & 1;
        const double im_tv = (double)g0.re * Vim + (double)g0.im * Vre;
        const cx<R> gf = G[t ^ (1 << j)];
        const double re_fv = (double)gf.re * Vre - (double)gf.im * Vim;
        const double z = block_sum(bit ? -im_tv : im_tv, sh);
        const double y = block_sum(bit ? re_fv : -re_fv, sh);
        put(j, y, z, t == 0);
    }
    // register bits k: Y = sum_t Im(T0(t) W_k), Z = sum_t Im(T0(t) Z_k)
#pragma unroll
    for (int k = 0; k < LOGR; ++k) {
        const double y = block_sum((double)g0.re * Wim[k] + (double)g0.im * Wre[k], sh);
        const double z = block_sum((double)g0.re * Zim[k] + (double)g0.im * Zre[k], sh);
        put(LD + k, y, z, t == 0);
    }
    // tile-id qubits: accumulated whole by thread t
    if (t < nb) put(K + t, bY, bZ, true);
}

// ------------------------------------------------------- off-diagonal terms

struct OffArgs {
    int n;
    int8_t pos[kMaxTileBits];
    int nruns;
    uint32_t run[kMaxTileBits + 1];
    u64 ntiles;
    const OffClass *cls;
    int c0, c1;
    const OffTerm *terms;
    double *epart;
    int estride;
};

// The pass's classes and terms are read through the scalar unit's cache:
// every lane reads the same entry (constant address space, read only).
typedef __attribute__((address_space(4))) const OffTerm ScalarTerm;
typedef __attribute__((address_space(4))) const OffClass ScalarClass;

__device__ __forceinline__ float term_cf(ScalarTerm &q, float) { return q.cf32; }
__device__ __forceinline__ double term_cf(ScalarTerm &q, double) { return q.cf; }

// Signed sum over terms [k0, k1) of a class for this thread: the tile
// base's share of each term's sign on the scalar unit, the thread's through
// tz.
template <typename R>
__device__ __forceinline__ R off_term(ScalarTerm &q, u64 base, uint32_t tid)
{
    R cf = term_cf(q, R(0));
    if (__popcll(base & q.z) & 1) cf = -cf;
    return (__popc(tid & q.tz) & 1) ? -cf : cf;
}
template <typename R>
__device__ __forceinline__ R off_sum(ScalarTerm *q, int k0, int k1, u64 base, uint32_t tid)
{
    R w = 0;
    for (int k = k0; k < k1; ++k) w += off_term<R>(q[k], base, tid);
    return w;
}
// The same per group (its terms share their register signs; every class
// side ends with a group end), each group's sum spread over X once.
template <typename R, int NR>
__device__ __forceinline__ void off_groups(R (&X)[NR], ScalarTerm *q, int k0, int k1, u64 base,
                                           uint32_t tid)
{
    for (int k = k0; k < k1;) {
        R w = 0;
        uint32_t sig;
        do {
            w += off_term<R>(q[k], base, tid);
            sig = q[k].sig;
            ++k;
        } while (!(sig & kOffGroupEnd));
#pragma unroll
        for (int r = 0; r < NR; ++r) X[r] += ((sig >> r) & 1) ? -w : w;
    }
}

// One class on a thread's 16 registers: partner reads from the LDS tile (pb:
// the partner thread's register 0; XH: the flip also touches register
// bits, xh), the real and imaginary sums, their products into acc.
template <typename R, int NR, int STRIDE, bool XH>
__device__ __forceinline__ void off_class(cx<R> (&acc)[NR], const cx<R> *pb, uint32_t xh,
                                          uint32_t xu, int t0, int ti, int t1, ScalarTerm *q,
                                          u64 base, uint32_t tid)
{
    typedef R r2 __attribute__((ext_vector_type(2)));
    cx<R> pv[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const r2 v = *(const r2 *)(pb + (XH ? (int)((uint32_t)r ^ xh) : r) * STRIDE);
        pv[r] = cx<R>{v.x, v.y};
    }
    R A[NR];
    if (ti > t0) {
        if (xu & kOffReFlat) {
            const R w = off_sum<R>(q, t0, ti, base, tid);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                acc[r].re += w * pv[r].re;
                acc[r].im += w * pv[r].im;
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) A[r] = R(0);
            off_groups<R, NR>(A, q, t0, ti, base, tid);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                acc[r].re += A[r] * pv[r].re;
                acc[r].im += A[r] * pv[r].im;
            }
        }
    }
    if (t1 > ti) {
        if (xu & kOffImFlat) {
            const R w = off_sum<R>(q, ti, t1, base, tid);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                acc[r].re -= w * pv[r].im;
                acc[r].im += w * pv[r].re;
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) A[r] = R(0);
            off_groups<R, NR>(A, q, ti, t1, base, tid);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                acc[r].re -= A[r] * pv[r].im;
                acc[r].im += A[r] * pv[r].re;
            }
        }
    }
}

// One cover pass: the psi tile sits in LDS, so for every class (flip mask x
// inside the tile) each amplitude reads its partner psi_{i^x} there and adds
// F(i^x) psi_{i^x} to lam_i, where F(i^x) = sum_k c_k i^{ph_k}
// (-1)^{popcount((i^x) & z_k)}: the real part from the class's real terms,
// the imaginary part from the others (a side without terms skips its
// products, a side without register signs uses one factor for all of the
// thread's registers).  The pass's share of <psi|H|psi> goes to FP64
// partials.
template <typename R, int K, int LOGR>
__device__ __forceinline__ void off_body(const cx<R> *psi, cx<R> *lam, const OffArgs &a, u64 t0,
                                         u64 tstep, int col, cx<R> *lds, double *sh)
{
    using T = Tile<K, LOGR>;
    const int t = threadIdx.x;
    constexpr int LD = T::lo(0);
    constexpr int STRIDE = T::lds_stride(LD);
    static_assert(T::lds_linear(LD), "load layout");
    const u64 toff = thread_off<K, LOGR>(t, LD, a);
    RegMap<LOGR, false> m;
    m.init(a.pos + LD);
    ScalarTerm *q = (ScalarTerm *)a.terms;
    ScalarClass *cls = (ScalarClass *)a.cls;
    constexpr uint32_t TMASK = (1u << LD) - 1u;   // tile bits held by the thread id
    double er = 0.0, ei = 0.0;
    for (u64 tile = t0; tile < a.ntiles; tile += tstep) {
        const u64 base = tile_base(tile, a);
        const u64 bt = base | toff;
        cx<R> v[T::NR], acc[T::NR];
        __syncthreads();
        const cx<R> *pt = psi + bt;
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            v[r] = ld_amp(pt + m.off(r));
            lds[T::lds_index(t, r, LD)] = v[r];
            acc[r].re = acc[r].im = R(0);
        }
        __syncthreads();
        for (int c = a.c0; c < a.c1; ++c) {
            const uint32_t xu = cls[c].xu;
            // partners: thread t ^ xl, register r ^ xh (immediate offsets when xh = 0)
            const uint32_t xl = xu & TMASK, xh = (xu & 0xffffu) >> LD;
            const cx<R> *pb = lds + T::pad(t ^ (int)xl);
            if (xh == 0)
                off_class<R, T::NR, STRIDE, false>(acc, pb, 0, xu, cls[c].t0, cls[c].ti, cls[c].t1,
                                                   q, base, (uint32_t)t);
            else
                off_class<R, T::NR, STRIDE, true>(acc, pb, xh, xu, cls[c].t0, cls[c].ti, cls[c].t1,
                                                  q, base, (uint32_t)t);
        }
        cx<R> *lt = lam ? lam + fresh(bt) : nullptr;
#pragma unroll
        for (int r = 0; r < T::NR; ++r) {
            er += (double)v[r].re * acc[r].re + (double)v[r].im * acc[r].im;
            ei += (double)v[r].re * acc[r].im - (double)v[r].im * acc[r].re;
            if (lt) {
                cx<R> o = ld_amp(lt + m.off(r));
                o.re += acc[r].re;
                o.im += acc[r].im;
                st_amp(lt + m.off(r), o);
            }
        }
    }
    const double tr = block_sum(er, sh);
    const double ti = block_sum(ei, sh);
    if (t == 0) {
        a.epart[col] += tr;
        a.epart[a.estride + col] += ti;
    }
    __syncthreads();
}

// W: waves per SIMD the kernel is compiled for (1: the compiler's choice).
// Large complex64 states run the W = 4 variant (128 VGPRs; the LDS tile
// allows 4 blocks per CU): the fourth wave hides more of the per-term scalar
// loads; small grids, where no CU gets a fourth block, keep the other.
template <typename R, int K, int LOGR, int W = 1>
__global__ __launch_bounds__(1 << (K - LOGR), W) void k_offdiag_pass(const void *psi_, void *lam_,
                                                                     OffArgs a)
{
    __shared__ cx<R> lds[Tile<K, LOGR>::LDS];
    __shared__ double sh[(1 << (K - LOGR)) / 64 + 1];
    off_body<R, K, LOGR>((const cx<R> *)psi_, (cx<R> *)lam_, a, blockIdx.x, gridDim.x, blockIdx.x,
                         lds, sh);
}

// ------------------------------------------------------------ table kernels
// RY(theta) rotates each pair by phi = theta / 2.  Where cos phi < 0 the
// passes rotate by phi - pi instead, the same gate times -1, so that the
// shear coefficients stay bounded: ry[p] = (tan(phi' / 2), sin phi') of that
// angle, computed in FP64 (tan(phi' / 2) = sin phi' / (1 + cos phi'), no
// cancellation for cos phi' >= 0) and rounded once to the amplitude
// precision (so the passes read them as scalar operands).
__device__ __forceinline__ bool ry_flipped(double theta, double &sn, double &cs)
{
    sincos(0.5 * theta, &sn, &cs);
    if (cs >= 0.0) return false;
    sn = -sn;
    cs = -cs;
    return true;
}
template <typename R>
__device__ __forceinline__ void ry_entry(double theta, cx<R> *e)
{
    double sn, cs;
    ry_flipped(theta, sn, cs);
    *e = cx<R>{(R)(sn / (1.0 + cs)), (R)sn};
}
// The -1 of every RY gate the passes rotate by phi - pi (those of rotation
// layers 1 .. rot-1; the first layer is generated from its tables, never
// rotated): their product S goes into the first chunk of the first layer's
// tables, so the generated state is S R_0|0..0>, every later state carries
// the product of the flips still to come (the state after the last layer is
// exact), and in the reverse sweep phi and lam carry the same sign.  Called
// by every thread of the block (each tests a share of the gates, the
// parities meet in LDS); each gets S.
__device__ __forceinline__ double ry_flip_sign(const double *theta, int n, int rot)
{
    __shared__ int par;
    if (threadIdx.x == 0) par = 0;
    __syncthreads();
    int p = 0;
    for (int i = threadIdx.x; i < (rot - 1) * n; i += blockDim.x) {
        double sn, cs;
        p ^= (int)ry_flipped(theta[(int64_t)(1 + i / n) * 2 * n + i % n], sn, cs);
    }
    if (p) atomicXor(&par, 1);
    __syncthreads();
    return par ? -1.0 : 1.0;
}

template <typename R>
__global__ void k_ry_table(const double *theta, int64_t np, cx<R> *ry)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x)
        ry_entry<R>(theta[p], ry + p);
}


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
// layer 0 (the state D_0 R_0|0...0>); the first chunk also carries the sign
// S of the flipped RY gates
template <typename R>
__global__ void k_init_tables(const double *theta, TabArgs ta, cx<R> *gtab, cx<R> *g0tab)
{
    const double S = ry_flip_sign(theta, ta.n, ta.rot_layers);
    const int per = ta.off[4];
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < per; w += gridDim.x * blockDim.x) {
        const int c = chunk_of(ta, w);
        const u64 v = (u64)(w - ta.off[c]);
        double ang;
        int par;
        chunk_phase(theta, ta, 0, c, v, ang, par);
        double mag = c == 0 ? S : 1.0;
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
// A CNOT network layer as an index gather.  The network sends basis index
// b to M b (M linear over GF(2), given by its columns), so
//   forward:  dst[o] = D(s) src[s], s = M^-1 o   (the state CNOT D psi~)
//   inverse:  dst[i] = conj(D(i)) src[M i]       (undoes both)
// with `map` holding the columns of M^-1 (forward) or M (inverse).  The
// map of an index is the XOR of five byte-table entries built in LDS.
template <typename R>
__global__ __launch_bounds__(256) void k_linmap_gather(const cx<R> *src, cx<R> *dst, LinMap map,
                                                       int inverse, DiagTab d, int with_diag)
{
    __shared__ u64 tab[5][256];
    for (int e = threadIdx.x; e < 5 * 256; e += blockDim.x) {
        const int k = e >> 8, v = e & 255;
        u64 acc = 0;
        for (int b = 0; b < 8; ++b) {
            const int q = 8 * k + b;
            if (((v >> b) & 1) && q < map.n) acc ^= map.col[q];
        }
        tab[k][v] = acc;
    }
    __syncthreads();
    const u64 dim = 1ull << map.n;
    for (u64 o = blockIdx.x * (u64)blockDim.x + threadIdx.x; o < dim;
         o += (u64)gridDim.x * blockDim.x) {
        const u64 s = tab[0][o & 255] ^ tab[1][(o >> 8) & 255] ^ tab[2][(o >> 16) & 255] ^
                      tab[3][(o >> 24) & 255] ^ tab[4][(o >> 32) & 255];
        cx<R> v = src[s];
        if (with_diag) v = inverse ? cmul_conj(v, diag_entry<R>(o, d)) : cmul(v, diag_entry<R>(s, d));
        dst[o] = v;
    }
}

// Entries of one LDiagTab: entry m of a group is the product over the
// group's qubits of the RZ factor e^{-i phi_q/2} (bit clear) or e^{+i phi_q/2}
// (bit set), times -1 per CZ pair inside the group with both bits set.  The
// phase is summed in FP64 and rounded once.
template <typename R>
__global__ void k_ldiag_table(const double *theta, LDiagBuild b, cx<R> *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= b.total) return;
    int first, count, m;
    if (e < b.offR) { first = 0; count = b.nt; m = e; }
    else if (e < b.offB1) { first = b.nt; count = b.nr; m = e - b.offR; }
    else if (e < b.offB2) { first = b.nt + b.nr; count = b.h1; m = e - b.offB1; }
    else { first = b.nt + b.nr + b.h1; count = b.h2; m = e - b.offB2; }
    const double *phi = theta + (int64_t)b.layer * 2 * b.n + b.n;
    double ph = 0.0;
    int par = 0;
    for (int j = 0; j < count; ++j) {
        const int q = b.q[first + j];
        const bool set = (m >> j) & 1;
        ph += set ? 0.5 * phi[q] : -0.5 * phi[q];
        if (!set || b.cz == 0) continue;
        // partner of q in the ladder: q + 1, and n-1 -> 0 when circular
        int p = q + 1;
        if (p == b.n) p = (b.cz == 2 && b.n > 2) ? 0 : -1;
        if (p < 0) continue;
        for (int i = 0; i < count; ++i)
            if (b.q[first + i] == p && ((m >> i) & 1)) par ^= 1;
    }
    double sn, cs;
    sincos(ph, &sn, &cs);
    if (par) {
        sn = -sn;
        cs = -cs;
    }
    out[e] = cx<R>{(R)cs, (R)sn};
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
        a.run[a.nruns] = (uint32_t)src | (uint32_t)w << 8 | (uint32_t)q << 16;
        ++a.nruns;
        src += w;
        q += w;
    }
}

DiagTab layer_tab(const gv_ansatz &an, const Chunks &ch, const FusedTables &t, int layer)
{
    return make_diagtab(an, ch, (const char *)t.dtab + (size_t)layer * t.dtab_stride,
                        layer < an.layers);
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
    a.qmask = ~0ull;
    return a;
}

inline int elem_grid(u64 dim)
{
    const u64 b = (dim + 255) / 256;
    return (int)(b < 8192 ? b : 8192);
}

#define GV_LAUNCH_KS(KERNEL, MS, PREC, GRID, K, ...)                                                   \
    do {                                                                                          \
        switch (K) {                                                                              \
        case 12:                                                                                  \
            if (PREC == GV_C64)                                                                   \
                hipLaunchKernelGGL((KERNEL<float, 12, 4, true, MS>), dim3(GRID), dim3(256), 0, s,     \
                                   __VA_ARGS__);                                                  \
            else                                                                                  \
                hipLaunchKernelGGL((KERNEL<double, 12, 4, true, MS>), dim3(GRID), dim3(256), 0, s,    \
                                   __VA_ARGS__);                                                  \
            break;                                                                                \
        case 10:                                                                                  \
            if (PREC == GV_C64)                                                                   \
                hipLaunchKernelGGL((KERNEL<float, 10, 4, true, MS>), dim3(GRID), dim3(64), 0, s,  \
                                   __VA_ARGS__);                                                  \
            else                                                                                  \
                hipLaunchKernelGGL((KERNEL<double, 10, 4, true, MS>), dim3(GRID), dim3(64), 0, s, \
                                   __VA_ARGS__);                                                  \
            break;                                                                                \
        case 8:                                                                                   \
            if (PREC == GV_C64)                                                                   \
                hipLaunchKernelGGL((KERNEL<float, 8, 3, false, MS>), dim3(GRID), dim3(32), 0, s,  \
                                   __VA_ARGS__);                                                  \
            else                                                                                  \
                hipLaunchKernelGGL((KERNEL<double, 8, 3, false, MS>), dim3(GRID), dim3(32), 0, s, \
                                   __VA_ARGS__);                                                  \
            break;                                                                                \
        default: return hipErrorInvalidValue;                                                     \
        }                                                                                         \
    } while (0)

// the selector of a pass's active mask (the kernels' pass_mask, on the host)
static int mask_sel(int prec, int K, uint32_t active)
{
    const uint32_t full = (1u << K) - 1u;
    const uint32_t later = full & ~((1u << (prec == GV_C64 ? 4 : 3)) - 1u);
    return active == full ? MS_FULL : (active == later ? MS_LATER : MS_ANY);
}

#define GV_LAUNCH_KM(KERNEL, PREC, GRID, K, ACTIVE, ...)                                          \
    do {                                                                                          \
        switch (mask_sel(PREC, K, ACTIVE)) {                                                      \
        case MS_FULL: GV_LAUNCH_KS(KERNEL, MS_FULL, PREC, GRID, K, __VA_ARGS__); break;           \
        case MS_LATER: GV_LAUNCH_KS(KERNEL, MS_LATER, PREC, GRID, K, __VA_ARGS__); break;         \
        default: GV_LAUNCH_KS(KERNEL, MS_ANY, PREC, GRID, K, __VA_ARGS__); break;                 \
        }                                                                                         \
    } while (0)


// ---------------------------------------------------------------- batching
//
// Many independent instances (their own n, layers, angles, Hamiltonian and
// qubit block) in one persistent kernel: each block takes the next instance
// from an atomic queue (in the order the host gives, largest first by
// default) and runs that instance's whole evaluation -- the same tile passes
// as the single-instance engine, over all of the instance's tiles, with block
// barriers between passes.  One block owns an instance, so its energy and
// gradient block sums are the final, fixed-order FP64 results.

// tables of every instance: blockIdx.y is the instance
template <typename R>
__global__ void k_batch_tables(const BatchInst *insts)
{
    const BatchInst &I = insts[blockIdx.y];
    const TabArgs &ta = I.ta;
    const double S = ry_flip_sign(I.theta, ta.n, ta.rot_layers);
    const int per = ta.off[4];
    const int64_t np = 2ll * I.n * I.rot;
    const int64_t nd = (int64_t)per * I.rot;
    const int64_t total = np + nd + per;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < np) {
            ry_entry<R>(I.theta[e], (cx<R> *)I.ry + e);
            continue;
        }
        const int64_t f = e - np;
        const bool init = f >= nd;
        const int l = init ? 0 : (int)(f / per);
        const int w = init ? (int)(f - nd) : (int)(f % per);
        const int c = chunk_of(ta, w);
        const u64 v = (u64)(w - ta.off[c]);
        double ang;
        int par;
        chunk_phase(I.theta, ta, l, c, v, ang, par);
        double sn, cs;
        sincos(ang, &sn, &cs);
        if (!init) {
            if (par) {
                sn = -sn;
                cs = -cs;
            }
            cx<R> out;
            out.re = (R)cs;
            out.im = (R)sn;
            ((cx<R> *)(I.dtab + (size_t)l * I.dtab_stride))[w] = out;
        } else {
            double mag = c == 0 ? S : 1.0;
            for (int q = ta.b[c]; q < ta.b[c + 1]; ++q) {
                double s2, c2;
                sincos(0.5 * I.theta[q], &s2, &c2);
                mag *= ((v >> (q - ta.b[c])) & 1) ? s2 : c2;
            }
            cx<R> g0;
            g0.re = (R)mag;
            g0.im = (R)0;
            ((cx<R> *)I.g0tab)[w] = g0;
            if (par) mag = -mag;
            cx<R> g;
            g.re = (R)(mag * cs);
            g.im = (R)(mag * sn);
            ((cx<R> *)I.gtab)[w] = g;
        }
    }
}

// the batch's two queue counters (a fill kernel: capturable in a HIP graph)
__global__ void k_zero_u32(unsigned *p)
{
    if (threadIdx.x < 2 && blockIdx.x == 0) p[threadIdx.x] = 0u;
}

__device__ __forceinline__ void batch_fill_pass(FusedArgs &a, const BatchInst &I, int p, int layer)
{
    a.n = I.n;
    a.layer = layer;
    a.nparam_layer = 2 * I.n;
    for (int j = 0; j < kMaxTileBits; ++j) a.pos[j] = I.pass[p].pos[j];
    a.active = I.pass[p].active;
    a.nruns = I.pass[p].nruns;
    for (int k = 0; k <= kMaxTileBits; ++k) a.run[k] = I.pass[p].run[k];
    a.ntiles = I.ntiles;
    a.ry = I.ry;
    a.in_mode = IN_LOAD;
    a.diag_phi = a.diag_lam = a.phi_gen = 0;
    a.store_phi = a.store_lam = 1;
    a.part = I.grad;
    a.grid = 1;
    a.qmask = I.qmask;
}

__device__ __forceinline__ DiagTab batch_layer_tab(const BatchInst &I, int layer)
{
    DiagTab d = (I.cz && layer < I.layers) ? I.dt_cz : I.dt_plain;
    d.tab = I.dtab + (size_t)layer * I.dtab_stride;
    return d;
}

template <typename R>
// fa / oa: the pass arguments in LDS (written by thread 0 before each body;
// as a local array they would live in per-lane scratch memory)
__device__ void batch_instance(const BatchInst &I, cx<R> *lds, double *sh, FusedArgs &a,
                               OffArgs &oa, cx<R> *psi_lds = nullptr, cx<R> *lam_lds = nullptr)
{
    constexpr int K = 12, LOGR = 4;
    const int t = threadIdx.x, nt = blockDim.x;
    // psi_lds / lam_lds: the instance's vectors live in the block's LDS
    cx<R> *psi = psi_lds ? psi_lds : (cx<R> *)I.psi, *lam = lam_lds ? lam_lds : (cx<R> *)I.lam;
    const u64 dim = 1ull << I.n;
    const int R_ = I.rot, np = I.np;
    // forward: R_0|0..0> (generated inside layer 1's first pass), then the layers
    if (R_ == 1) {
        for (u64 i = t; i < dim; i += nt) psi[i] = diag_entry<R>(i, I.g0);
        __syncthreads();
    }
    for (int l = 1; l < R_; ++l) {
        for (int p = 0; p < np; ++p) {
            if (t == 0) {
                batch_fill_pass(a, I, p, l);
                if (p == 0) {
                    a.in_mode = l == 1 ? IN_GENERATE : IN_LOAD_DIAG;
                    a.dt = l == 1 ? I.gt : batch_layer_tab(I, l - 1);
                }
            }
            __syncthreads();
            fwd_body<R, K, LOGR, true>(psi, psi, a, 0, 1, lds);
            __syncthreads();
        }
    }
    // psi = D psi~ of the last layer unless H is diagonal (then they commute)
    if (!I.zonly) {
        const DiagTab d = batch_layer_tab(I, R_ - 1);
        for (u64 i = t; i < dim; i += nt) psi[i] = cmul(psi[i], diag_entry<R>(i, d));
        __syncthreads();
    }
    // an empty qubit block asks for the energy alone: no lam, no reverse
    // sweep, a zero gradient
    const bool eonly = I.qmask == 0;
    // energy: diagonal part with lam = D psi, then the off-diagonal cover passes
    {
        double e = 0.0;
        for (u64 i = t; i < dim; i += nt) {
            const cx<R> v = psi[i];
            const double d = I.hdiag[i];
            e += d * ((double)v.re * v.re + (double)v.im * v.im);
            if (eonly) continue;
            cx<R> o;
            o.re = (R)d * v.re;
            o.im = (R)d * v.im;
            lam[i] = o;
        }
        const double tot = block_sum(e, sh);
        if (t == 0) {
            I.energy[0] = tot;
            I.energy[1] = 0.0;
        }
        __syncthreads();
    }
    for (int k = 0; k < I.noff; ++k) {
        if (t == 0) {
            const BatchOffPass &op = I.offp[k];
            oa.n = I.n;
            for (int j = 0; j < kMaxTileBits; ++j) oa.pos[j] = op.tile.pos[j];
            oa.nruns = op.tile.nruns;
            for (int q = 0; q <= kMaxTileBits; ++q) oa.run[q] = op.tile.run[q];
            oa.ntiles = I.ntiles;
            oa.cls = I.cls;
            oa.c0 = op.c0;
            oa.c1 = op.c1;
            oa.terms = I.terms;
            oa.epart = I.energy;
            oa.estride = 1;
        }
        __syncthreads();
        off_body<R, K, LOGR>(psi, eonly ? nullptr : lam, oa, 0, 1, 0, lds, sh);
        __syncthreads();
    }
    if (eonly) {
        for (int64_t p = t; p < 2ll * I.n * R_; p += nt) I.grad[p] = 0.0;
        return;
    }
    // reverse sweep
    bool post = !I.zonly;
    for (int l = R_ - 1; l >= 0; --l) {
        for (int p = 0; p < np; ++p) {
            const bool last = p == np - 1;
            if (t == 0) {
                batch_fill_pass(a, I, p, l);
                if (p == 0) {
                    a.phi_gen = l == 0;
                    if (a.phi_gen) a.gt = I.g0;
                    a.diag_phi = post && l > 0;
                    a.diag_lam = post;
                    if (a.diag_phi || a.diag_lam) a.dt = batch_layer_tab(I, l);
                }
                a.store_phi = !last || l - 1 >= 1;
                a.store_lam = !(l == 0 && last);
            }
            __syncthreads();
            bwd_body<R, K, LOGR, true, false>(psi, psi, lam, a, 0, 1, 0, lds, sh);
            __syncthreads();
        }
        post = true;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_batch(const BatchInst *insts, const int *order, int count,
                                               unsigned *counter)
{
    __shared__ cx<R> lds[Tile<12, 4>::LDS];
    __shared__ double sh[8];
    __shared__ FusedArgs fa;
    __shared__ OffArgs oa;
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int idx = next;
        __syncthreads();
        if (idx >= count) break;   // every block leaves once the queue is empty
        batch_instance<R>(insts[order[idx]], lds, sh, fa, oa);
    }
}

// The same for instances small enough to keep psi and lam in the block's
// LDS for the whole evaluation (kBatchLdsAmps amplitudes each, next to the
// tile exchange buffer: 2 x 32 KB + 34 KB of the 160 KB in complex64).
template <typename R>
__global__ __launch_bounds__(256) void k_batch_lds(const BatchInst *insts, const int *order,
                                                   int count, unsigned *counter)
{
    __shared__ cx<R> lds[Tile<12, 4>::LDS];
    __shared__ cx<R> vpsi[kBatchLdsAmps], vlam[kBatchLdsAmps];
    __shared__ double sh[8];
    __shared__ FusedArgs fa;
    __shared__ OffArgs oa;
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int idx = next;
        __syncthreads();
        if (idx >= count) break;   // every block leaves once the queue is empty
        batch_instance<R>(insts[order[idx]], lds, sh, fa, oa, vpsi, vlam);
    }
}

}  // namespace

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
        d.pa[d.npair] = q - 1;
        d.pb[d.npair++] = q;
    }
    // the circular pair (n-1, 0) lies inside a chunk only when chunk 0 holds every bit
    if (an.ent == GV_ENT_CZ_CIRCULAR && n > 2 && ch.b[1] < n) {
        d.pa[d.npair] = n - 1;
        d.pb[d.npair++] = 0;
    }
    return d;
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

void pass_runs(const int8_t *pos, int K, int n, BatchPass *out)
{
    PassPlan pp;
    for (int j = 0; j < K; ++j) pp.pos[j] = pos[j];
    pp.active = 0;
    FusedArgs fa;
    memset(&fa, 0, sizeof(fa));
    fill_runs(fa, pp, K, n);
    for (int j = 0; j < K; ++j) out->pos[j] = pos[j];
    out->nruns = fa.nruns;
    for (int k = 0; k < fa.nruns; ++k) out->run[k] = fa.run[k];
}


int fused_grid(int prec, const TilePlan &plan, int n)
{
    // persistent blocks: four rounds of three resident blocks on each of the
    // 256 CUs, which also balances the kernels that keep four resident
    const u64 ntiles = 1ull << (n - plan.K);
    const u64 want = prec == GV_C64 ? 3072 : 512;
    return (int)(ntiles < want ? ntiles : want);
}

hipError_t fused_build_tables(int prec, const gv_ansatz &an, const Chunks &ch,
                              const double *theta, const FusedTables &t, hipStream_t s)
{
    const int64_t np = nparams(an);
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_ry_table<float>, dim3((int)((np + 255) / 256)), dim3(256), 0, s,
                           theta, np, (cx<float> *)t.ry);
    else
        hipLaunchKernelGGL(k_ry_table<double>, dim3((int)((np + 255) / 256)), dim3(256), 0, s,
                           theta, np, (cx<double> *)t.ry);
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
                              const FusedTables &t, hipStream_t s, const void *src)
{
    if (!src) src = psi;
    if (in_mode != IN_LOAD && pass != 0) return hipErrorInvalidValue;
    FusedArgs a = base_args(an, plan, pass, layer, t);
    a.in_mode = in_mode;
    if (in_mode == IN_LOAD_DIAG) a.dt = layer_tab(an, ch, t, layer - 1);
    if (in_mode == IN_GENERATE) a.dt = make_diagtab(an, ch, t.gtab, 0 < an.layers);
    const int grid = fused_grid(prec, plan, an.n);
    if (in_mode == IN_LOAD) GV_LAUNCH_KM(k_fwd_load_pass, prec, grid, plan.K, a.active, psi, src, a);
    else GV_LAUNCH_KM(k_fwd_pass, prec, grid, plan.K, a.active, psi, src, a);
    return hipGetLastError();
}

hipError_t fused_backward_pass(int prec, const void *phi_in, void *phi, void *lam,
                               const gv_ansatz &an, const TilePlan &plan, int pass, int layer,
                               const BwdFlags &fl, const Chunks &ch, const FusedTables &t,
                               double *part, int grid, hipStream_t s, const LDiagTab *ld_load)
{
    if ((fl.phi_generate || fl.diag_phi || fl.diag_lam) && pass != 0) return hipErrorInvalidValue;
    if (ld_load && (fl.phi_generate || fl.diag_phi || fl.diag_lam)) return hipErrorInvalidValue;
    if (fl.grad_first && (fl.store_phi || !fl.store_lam || fl.phi_generate || fl.diag_phi))
        return hipErrorInvalidValue;
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
    if (ld_load) a.ld = *ld_load;
    if (fl.grad_first) {
        if (ld_load) GV_LAUNCH_KM(k_bwd_gf_ld_pass, prec, grid, plan.K, a.active, phi_in, lam, a);
        else GV_LAUNCH_KM(k_bwd_gf_pass, prec, grid, plan.K, a.active, phi_in, lam, a);
    } else if (ld_load) {
        GV_LAUNCH_KM(k_bwd_ld_pass, prec, grid, plan.K, a.active, phi_in, phi, lam, a);
    } else {
        GV_LAUNCH_KM(k_bwd_pass, prec, grid, plan.K, a.active, phi_in, phi, lam, a);
    }
    return hipGetLastError();
}

hipError_t fused_backward2_pass(int prec, const void *phi_src, void *phi, void *lam,
                                const gv_ansatz &an, const TilePlan &plan, int pass, int layer,
                                int store_phi, const LDiagTab &ld_last, const FusedTables &t,
                                double *part, int grid, hipStream_t s)
{
    FusedArgs a = base_args(an, plan, pass, layer, t);
    a.layer2 = layer + 1;
    a.ld = ld_last;
    a.store_phi = store_phi;
    a.part = part;
    a.grid = grid;
    if (store_phi) GV_LAUNCH_KM(k_bwd2_phi_pass, prec, grid, plan.K, a.active, phi_src, phi, lam, a);
    else GV_LAUNCH_KM(k_bwd2_pass, prec, grid, plan.K, a.active, phi_src, phi, lam, a);
    return hipGetLastError();
}

hipError_t fused_layer0_grad(int prec, const void *lam, const gv_ansatz &an, const TilePlan &plan,
                             int diag_lam, const Chunks &ch, const FusedTables &t, double *part,
                             int grid, hipStream_t s)
{
    Layer0Args a;
    memset(&a, 0, sizeof(a));
    a.n = an.n;
    a.ntiles = 1ull << (an.n - plan.K);
    a.diag_lam = diag_lam;
    if (diag_lam) a.dt = layer_tab(an, ch, t, 0);
    a.gt = make_diagtab(an, ch, t.g0tab, false);
    a.part = part;
    a.grid = grid;
    a.qmask = ~0ull;
    switch (plan.K) {
    case 12:
        if (prec == GV_C64)
            hipLaunchKernelGGL((k_layer0_grad<float, 12, 4>), dim3(grid), dim3(256), 0, s, lam, a);
        else
            hipLaunchKernelGGL((k_layer0_grad<double, 12, 4>), dim3(grid), dim3(256), 0, s, lam, a);
        break;
    case 10:
        if (prec == GV_C64)
            hipLaunchKernelGGL((k_layer0_grad<float, 10, 4>), dim3(grid), dim3(64), 0, s, lam, a);
        else
            hipLaunchKernelGGL((k_layer0_grad<double, 10, 4>), dim3(grid), dim3(64), 0, s, lam, a);
        break;
    case 8:
        if (prec == GV_C64)
            hipLaunchKernelGGL((k_layer0_grad<float, 8, 3>), dim3(grid), dim3(32), 0, s, lam, a);
        else
            hipLaunchKernelGGL((k_layer0_grad<double, 8, 3>), dim3(grid), dim3(32), 0, s, lam, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int ldiag_entries(int n, int K, int LOGR)
{
    const int nb = n - K, h1 = nb - nb / 2, h2 = nb / 2;
    return (1 << (K - LOGR)) + (1 << LOGR) + (1 << h1) + (1 << h2);
}

static int assign_lo(int K, int LOGR, int a)
{
    return a == 0 ? K - LOGR : std::min((a - 1) * LOGR, K - LOGR);
}

hipError_t make_ldiag(int prec, const gv_ansatz &an, const TilePlan &plan, int pass, int last,
                      int layer, const double *theta, void *tab, LDiagTab *out, hipStream_t s)
{
    const int n = an.n, K = plan.K, LOGR = K == 8 ? 3 : 4;
    const int NA = 1 + (K - LOGR + LOGR - 1) / LOGR;
    const int lo = assign_lo(K, LOGR, last ? NA - 1 : 0);
    const PassPlan &pp = plan.pass[pass];
    LDiagBuild b;
    memset(&b, 0, sizeof(b));
    b.n = n;
    b.layer = layer;
    b.nt = K - LOGR;
    b.nr = LOGR;
    const int nb = n - K;
    b.h1 = nb - nb / 2;
    b.h2 = nb / 2;
    int group[64];   // 0 thread, 1 register, 2 B1, 3 B2
    int regbit[64];
    int c = 0;
    bool in_tile[64] = {false};
    for (int j = 0; j < K; ++j) in_tile[pp.pos[j]] = true;
    for (int j = 0; j < K; ++j)
        if (j < lo || j >= lo + LOGR) {
            b.q[c++] = pp.pos[j];
            group[pp.pos[j]] = 0;
            regbit[pp.pos[j]] = -1;
        }
    for (int k = 0; k < LOGR; ++k) {
        b.q[c++] = pp.pos[lo + k];
        group[pp.pos[lo + k]] = 1;
        regbit[pp.pos[lo + k]] = k;
    }
    int m = 0;
    for (int q = 0; q < n; ++q) {
        if (in_tile[q]) continue;
        b.q[c++] = (int8_t)q;
        group[q] = m < b.h1 ? 2 : 3;
        regbit[q] = -1;
        ++m;
    }
    const bool cz_layer = layer < an.layers;
    b.cz = !cz_layer ? 0 : (an.ent == GV_ENT_CZ_LINEAR ? 1 : (an.ent == GV_ENT_CZ_CIRCULAR ? 2 : 0));
    b.offR = 1 << b.nt;
    b.offB1 = b.offR + (1 << b.nr);
    b.offB2 = b.offB1 + (1 << b.h1);
    b.total = b.offB2 + (1 << b.h2);

    LDiagTab d;
    memset(&d, 0, sizeof(d));
    d.tab = tab;
    d.offR = b.offR;
    d.offB1 = b.offB1;
    d.offB2 = b.offB2;
    d.h1 = b.h1;
    auto add = [&](int qa, int qb) {
        if (group[qa] == group[qb]) return true;
        if (d.npair >= kMaxLPairs) return false;
        d.pa[d.npair] = qa;
        d.pb[d.npair] = qb;
        d.ka[d.npair] = regbit[qa];
        d.kb[d.npair] = regbit[qb];
        ++d.npair;
        return true;
    };
    if (b.cz != 0) {
        for (int q = 0; q + 1 < n; ++q)
            if (!add(q, q + 1)) return hipErrorInvalidValue;
        if (b.cz == 2 && n > 2 && !add(n - 1, 0)) return hipErrorInvalidValue;
    }
    *out = d;
    const int grid = (b.total + 255) / 256;
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_ldiag_table<float>, dim3(grid), dim3(256), 0, s, theta, b,
                           (cx<float> *)tab);
    else
        hipLaunchKernelGGL(k_ldiag_table<double>, dim3(grid), dim3(256), 0, s, theta, b,
                           (cx<double> *)tab);
    return hipGetLastError();
}

hipError_t fused_forward2_pass(int prec, void *psi, const gv_ansatz &an, const TilePlan &plan,
                               int pass, int layer, int in_mode, const Chunks &ch,
                               const FusedTables &t, const LDiagTab &ld, hipStream_t s,
                               const void *src)
{
    if (!src) src = psi;
    if (in_mode != IN_LOAD && pass != 0) return hipErrorInvalidValue;
    if (layer + 1 >= an.layers + an.final_rotation) return hipErrorInvalidValue;
    FusedArgs a = base_args(an, plan, pass, layer, t);
    a.layer2 = layer + 1;
    a.ld = ld;
    a.in_mode = in_mode;
    if (in_mode == IN_LOAD_DIAG) a.dt = layer_tab(an, ch, t, layer - 1);
    if (in_mode == IN_GENERATE) a.dt = make_diagtab(an, ch, t.gtab, 0 < an.layers);
    const int grid = fused_grid(prec, plan, an.n);
    if (in_mode == IN_LOAD) GV_LAUNCH_KM(k_fwd2_load_pass, prec, grid, plan.K, a.active, psi, src, a);
    else GV_LAUNCH_KM(k_fwd2_pass, prec, grid, plan.K, a.active, psi, src, a);
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
    if (in_mode == IN_LOAD) GV_LAUNCH_KM(k_turn_load_pass, prec, grid, plan.K, a.active, psi, lam, a);
    else GV_LAUNCH_KM(k_turn_pass, prec, grid, plan.K, a.active, psi, lam, a);
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
    if (n > 40) return hipErrorInvalidValue;
    const LinMap map = cnot_linmap(n, an.ent, layer, !inverse);
    DiagTab d;
    memset(&d, 0, sizeof(d));
    const int with_diag = t != nullptr;
    if (t) d = layer_tab(an, ch, *t, layer);
    const u64 dim = 1ull << n;
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_linmap_gather<float>, dim3(elem_grid(dim)), dim3(256), 0, s,
                           (const cx<float> *)src, (cx<float> *)dst, map, inverse, d, with_diag);
    else
        hipLaunchKernelGGL(k_linmap_gather<double>, dim3(elem_grid(dim)), dim3(256), 0, s,
                           (const cx<double> *)src, (cx<double> *)dst, map, inverse, d, with_diag);
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
    for (int k = 0; k < fa.nruns; ++k) a.run[k] = fa.run[k];
    a.ntiles = 1ull << (n - K);
    a.cls = cls;
    a.c0 = op.c0;
    a.c1 = op.c1;
    a.terms = terms;
    a.epart = epart;
    a.estride = estride;
    // three resident blocks per CU, four rounds (as the fused passes)
    const u64 want = prec == GV_C64 ? 3072 : 512;
    const int grid = (int)(a.ntiles < want ? a.ntiles : want);
    if (grid > estride) return hipErrorInvalidValue;
    switch (K) {
    case 12:
        if (prec == GV_C64 && a.ntiles >= (1ull << 16)) {
            hipLaunchKernelGGL((k_offdiag_pass<float, 12, 4, 4>), dim3(grid), dim3(256), 0, s, psi, lam, a);
        } else if (prec == GV_C64) {
            hipLaunchKernelGGL((k_offdiag_pass<float, 12, 4>), dim3(grid), dim3(256), 0, s, psi, lam, a);
        } else {
            hipLaunchKernelGGL((k_offdiag_pass<double, 12, 4>), dim3(grid), dim3(256), 0, s, psi, lam, a);
        }
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

hipError_t batch_tables(int prec, const BatchInst *dev_insts, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const dim3 grid(64, (unsigned)count);
    if (prec == GV_C64)
        hipLaunchKernelGGL(k_batch_tables<float>, grid, dim3(256), 0, s, dev_insts);
    else
        hipLaunchKernelGGL(k_batch_tables<double>, grid, dim3(256), 0, s, dev_insts);
    return hipGetLastError();
}

hipError_t batch_zero(unsigned *counter, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t batch_run(int prec, const BatchInst *dev_insts, const int *order, int count,
                     unsigned *counter, int grid, bool lds_resident, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (lds_resident) {
        if (prec != GV_C64) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_batch_lds<float>, dim3(grid), dim3(256), 0, s, dev_insts, order,
                           count, counter);
    } else if (prec == GV_C64) {
        hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(256), 0, s, dev_insts, order, count,
                           counter);
    } else {
        hipLaunchKernelGGL(k_batch<double>, dim3(grid), dim3(256), 0, s, dev_insts, order, count,
                           counter);
    }
    return hipGetLastError();
}

}  // namespace gv
