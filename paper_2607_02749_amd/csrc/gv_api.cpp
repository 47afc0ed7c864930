// gv_api.cpp -- the C ABI (include/gv.h): validation, Hamiltonian ingest and
// canonicalisation (Eq. 6), planning, and the launch sequences of the energy
// (Eq. 4) and its gradient.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "gv_internal.hpp"

namespace gv {

static thread_local std::string g_last_error;

gv_status set_error(gv_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

// Error-path test hook: when >= 0, the number of HIP status checks that
// still pass before one reports an injected failure (then it turns off).
static std::atomic<int64_t> g_inject_after{-1};

gv_status check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) {
        if (g_inject_after.load(std::memory_order_relaxed) < 0) return GV_OK;
        if (g_inject_after.fetch_sub(1) != 0) return GV_OK;
        return set_error(GV_EHIP, "%s: injected HIP error (test hook)", what);
    }
    return set_error(GV_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static hipEvent_t take_event(gv_state_s *st)
{
    if (!st->event_pool.empty()) {
        hipEvent_t e = st->event_pool.back();
        st->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(gv_state_s *st, int kind, double bytes) : st_(st), kind_(kind), bytes_(bytes)
{
    if (!st_ || !st_->profiling) return;
    start_ = take_event(st_);
    if (start_ && hipEventRecord(start_, st_->stream) != hipSuccess) {
        st_->event_pool.push_back(start_);
        start_ = nullptr;
    }
}

ProfScope::~ProfScope()
{
    if (!start_) return;
    hipEvent_t stop = take_event(st_);
    if (!stop || hipEventRecord(stop, st_->stream) != hipSuccess) {
        st_->event_pool.push_back(start_);
        if (stop) st_->event_pool.push_back(stop);
        return;
    }
    st_->records.push_back({kind_, start_, stop, bytes_});
}

int rot_layers(const gv_ansatz &a) { return a.layers + a.final_rotation; }
int64_t nparams(const gv_ansatz &a) { return 2ll * a.n * rot_layers(a); }

// Tile passes of one layer: pass 0 takes bits 0..K-1; later passes keep the C
// low bits (for contiguous runs) and take the next K-C unprocessed bits,
// topping up with the already-processed bits just below them so every tile
// has K bits and the tile's top bits stay at consecutive positions.
bool make_tile_plan(int n, int K, int C, TilePlan *out)
{
    if (K < 1 || K > kMaxTileBits || K > n || C < 0 || C > K) return false;
    TilePlan p;
    p.K = K;
    p.C = C;
    p.npass = 0;
    int next = K;
    {
        PassPlan &pp = p.pass[p.npass++];
        for (int j = 0; j < K; ++j) pp.pos[j] = (int8_t)j;
        pp.active = (K >= 32) ? 0xffffffffu : ((1u << K) - 1u);
    }
    while (next < n) {
        if (p.npass >= kMaxPasses || K - C < 1) return false;
        const int m = std::min(K - C, n - next);
        std::vector<int> bits;
        for (int j = 0; j < C; ++j) bits.push_back(j);
        const int fill = K - C - m;
        for (int j = 0; j < fill; ++j) bits.push_back(next - fill + j);  // next - fill >= C
        for (int j = 0; j < m; ++j) bits.push_back(next + j);
        std::sort(bits.begin(), bits.end());
        PassPlan &pp = p.pass[p.npass++];
        pp.active = 0;
        for (int j = 0; j < K; ++j) {
            pp.pos[j] = (int8_t)bits[j];
            if (bits[j] >= next) pp.active |= 1u << j;
        }
        next += m;
    }
    *out = p;
    return true;
}

Chunks make_chunks(int n, int K, int LOGR)
{
    // chunk 0: the thread bits and chunk 1: the register bits of pass 0's load
    // assignment; chunks 2 and 3 split the remaining bits in halves
    Chunks c;
    c.b[0] = 0;
    c.b[1] = std::min(n, K - LOGR);
    c.b[2] = std::min(n, K);
    c.b[3] = std::min(n, K + (n - K + 1) / 2);
    c.b[4] = n;
    c.off[0] = 0;
    for (int k = 0; k < 4; ++k) c.off[k + 1] = c.off[k] + (1 << (c.b[k + 1] - c.b[k]));
    return c;
}

static const int kEnergyGrid = 3072;  // blocks of the energy and off-diagonal kernels
static const int kPartCols = 4096;    // energy-partial columns the work buffer holds
static_assert(kEnergyGrid <= kPartCols, "energy partials must fit the work buffer");

static int choose_K(int n) { return n >= 12 ? 12 : (n >= 10 ? 10 : 8); }
static int choose_logr(int K) { return K == 8 ? 3 : 4; }
static int choose_C(gv_precision p, int K) { return std::min(K - 1, p == GV_C64 ? 4 : 3); }
static bool fused_ok(gv_engine e, int n) { return e == GV_ENGINE_FUSED && n >= 8; }

// One tile pass of the forward sweep in snake order: group g (a pass of the
// tile plan) for rotation layer la, and, when lb >= 0, also for layer
// lb = la + 1 (a two-layer pass).  slot >= 0: the state after the pass is a
// checkpoint slot.
struct FwdOp {
    int g, la, lb, in_mode, slot;
};

// Snake order for diagonal entanglers: layer l runs the plan's passes
// forward when l is odd and backward when l is even, so the last pass of a
// layer and the first of the next act on the same tile qubits and fuse into
// one two-layer pass (the layer diagonal between them is applied in
// registers).  Layer 0 (the product state) is generated inside layer 1's
// first pass.  keep_last_single keeps the last layer's pass out of a
// two-layer pass (the turnaround takes it).  Checkpoint slots go to the
// states after two-layer passes (every pass when the plan has one pass).
static std::vector<FwdOp> snake_ops(int np, int upto, bool keep_last_single, bool ckpt)
{
    std::vector<FwdOp> ops;
    for (int l = 1; l <= upto; ++l)
        for (int i = 0; i < np; ++i) {
            const int g = (l & 1) ? i : np - 1 - i;
            if (i == 0 && l >= 2) {
                FwdOp &pv = ops.back();
                const bool hold = keep_last_single && l == upto && np == 1;
                if (pv.lb < 0 && pv.g == g && !hold) {
                    pv.lb = l;
                    continue;
                }
                ops.push_back({g, l, -1, FWD_LOAD_DIAG, -1});  // np == 1: g == 0
                continue;
            }
            ops.push_back({g, l, -1, (l == 1 && i == 0) ? FWD_GENERATE : FWD_LOAD, -1});
        }
    if (ckpt) {
        int slot = 0;
        const int last = (int)ops.size() - (keep_last_single ? 2 : 1);
        for (int k = 0; k < last; ++k)
            if (ops[k].lb >= 0 || np == 1) ops[k].slot = slot++;
    }
    return ops;
}

// buffers the STORE mode needs: one per pass output except the last
static int store_slots(const gv_ansatz &a, int np)
{
    const bool cnot = ent_is_cnot(a.ent);
    const int R = rot_layers(a);
    if (cnot || R < 2) return std::max(0, R - 2);
    const size_t m = std::max(snake_ops(np, R - 1, false, false).size(),
                              snake_ops(np, R - 1, true, false).size());
    return (int)m - 1;
}

gv_status work_layout(const gv_ansatz &a, gv_precision prec, gv_engine eng, gv_grad_mode mode,
                      WorkLayout *out)
{
    WorkLayout w;
    const size_t s = amp_bytes(prec);
    const size_t A = (size_t)1 << a.n;
    const int64_t P = nparams(a);
    const int R = rot_layers(a);
    size_t off = 0;
    TilePlan plan;
    if (fused_ok(eng, a.n)) {
        if (!make_tile_plan(a.n, choose_K(a.n), choose_C(prec, choose_K(a.n)), &plan))
            return set_error(GV_EUNSUPPORTED, "no tile plan for n=%d", a.n);
        w.grid = fused_grid(prec, plan, a.n);
    } else {
        w.grid = kPlainGrid;
    }
    // energy partials: 2 rows of max(kPartCols, grid) columns (the fused
    // turnaround writes one column per block)
    w.epart = off;
    off += align_up(2 * (size_t)std::max(kPartCols, w.grid) * sizeof(double));
    if (fused_ok(eng, a.n)) {
        const int K = choose_K(a.n);
        const Chunks ch = make_chunks(a.n, K, choose_logr(K));
        w.dtab_stride = align_up((size_t)ch.off[4] * s);
        w.ry_tab = off;
        off += align_up((size_t)P * 2 * sizeof(double) + 8);
        w.dtab = off;
        off += w.dtab_stride * (size_t)(R > 0 ? R : 1);
        w.gtab = off;
        off += w.dtab_stride;
        w.g0tab = off;
        off += w.dtab_stride;
        w.ldtab_stride = align_up((size_t)ldiag_entries(a.n, K, choose_logr(K)) * s);
        w.ldtab = off;
        off += w.ldtab_stride * (size_t)(R > 0 ? 2 * R : 1);
    }
    w.part = off;
    off += align_up((size_t)P * w.grid * sizeof(double) + 8);
    w.lam = off;
    off += align_up(A * s);
    const bool cnot = ent_is_cnot(a.ent);
    if (fused_ok(eng, a.n) && cnot) {
        w.scratch = off;
        off += align_up(A * s);
    }
    if (mode == GV_GRAD_CHECKPOINT && fused_ok(eng, a.n) && R > 2) {
        w.ckpt = off;  // states at the inner layer boundaries
        off += align_up(A * s) * (size_t)(R - 2);
    }
    if (mode == GV_GRAD_STORE && fused_ok(eng, a.n)) {
        w.ckpt = off;  // the output of every pass but the last
        off += align_up(A * s) * (size_t)store_slots(a, plan.npass);
    }
    w.total = off;
    *out = w;
    return GV_OK;
}

// ----------------------------------------------------------------- validation

static gv_status check_ansatz(const gv_ansatz *a)
{
    if (!a) return set_error(GV_EINVAL, "ansatz is NULL");
    if (a->n < 1 || a->n > kMaxQubits)
        return set_error(GV_EINVAL, "n=%d outside 1..%d", a->n, kMaxQubits);
    if (a->layers < 0 || a->layers > 4096) return set_error(GV_EINVAL, "layers=%d", a->layers);
    if (a->final_rotation != 0 && a->final_rotation != 1)
        return set_error(GV_EINVAL, "final_rotation must be 0 or 1");
    if (a->ent < GV_ENT_NONE || a->ent > GV_ENT_CNOT_SCA)
        return set_error(GV_EINVAL, "unknown entangler %d", a->ent);
    return GV_OK;
}

static bool aligned(const void *p) { return ((uintptr_t)p % kAlign) == 0; }

// ------------------------------------------------------------------ gate list
struct Gate {
    int kind;  // 0 RY, 1 RZ, 2 CZ, 3 CNOT
    int a, b;
    int64_t p;
};

static std::vector<Gate> gate_list(const gv_ansatz &an)
{
    std::vector<Gate> g;
    const int n = an.n;
    for (int l = 0; l < rot_layers(an); ++l) {
        const int64_t base = (int64_t)l * 2 * n;
        for (int q = 0; q < n; ++q) g.push_back({0, q, -1, base + q});
        for (int q = 0; q < n; ++q) g.push_back({1, q, -1, base + n + q});
        if (l >= an.layers) break;
        if (an.ent == GV_ENT_CZ_LINEAR || an.ent == GV_ENT_CZ_CIRCULAR) {
            for (int q = 0; q + 1 < n; ++q) g.push_back({2, q, q + 1, -1});
            if (an.ent == GV_ENT_CZ_CIRCULAR && n > 2) g.push_back({2, n - 1, 0, -1});
        } else if (ent_is_cnot(an.ent)) {
            for (const auto &ct : cnot_network(n, an.ent, l)) g.push_back({3, ct.first, ct.second, -1});
        }
    }
    return g;
}

// ------------------------------------------------------------- launch chains

static gv_status plain_forward(gv_state st, const gv_ansatz &an, const double *theta)
{
    const int prec = st->prec;
    hipStream_t s = st->stream;
    if (gv_status e = check_hip(plain_set_zero_state(prec, st->amps, an.n, s), "zero state"))
        return e;
    const double A = (double)(1ull << an.n), sb = (double)amp_bytes(st->prec);
    for (const Gate &g : gate_list(an)) {
        hipError_t e;
        ProfScope ps(st, GV_PROF_PLAIN_GATE, g.kind == 2 ? 0.5 * A * sb : (g.kind == 3 ? A * sb : 2 * A * sb));
        switch (g.kind) {
        case 0: e = plain_ry(prec, st->amps, an.n, g.a, theta, g.p, 0, s); break;
        case 1: e = plain_rz(prec, st->amps, an.n, g.a, theta, g.p, 0, s); break;
        case 2: e = plain_cz(prec, st->amps, an.n, g.a, g.b, s); break;
        default: e = plain_cnot(prec, st->amps, an.n, g.a, g.b, s); break;
        }
        if (gv_status r = check_hip(e, "plain gate")) return r;
    }
    return GV_OK;
}

struct FusedCtx {
    TilePlan plan;
    Chunks ch;
    FusedTables tabs;
    WorkLayout w;
    std::vector<FwdOp> ops;          // snake order (diagonal entanglers)
    std::vector<LDiagTab> ld;        // per rotation layer: its diagonal in the last assignment
    std::vector<LDiagTab> ld0;       // ... and in the load assignment of the same pass
};

static bool is_cnot(const gv_ansatz &a) { return ent_is_cnot(a.ent); }

}  // namespace gv

std::vector<std::pair<int, int>> gv::cnot_network(int n, int ent, int layer)
{
    std::vector<std::pair<int, int>> g;
    switch (ent) {
    case GV_ENT_CNOT_LINEAR:
    case GV_ENT_CNOT_CIRCULAR:
        if (ent == GV_ENT_CNOT_CIRCULAR && n > 2) g.push_back({n - 1, 0});
        for (int q = 0; q + 1 < n; ++q) g.push_back({q, q + 1});
        break;
    case GV_ENT_CNOT_FULL:
        for (int i = 0; i + 1 < n; ++i)
            for (int j = i + 1; j < n; ++j) g.push_back({i, j});
        break;
    case GV_ENT_CNOT_REVERSE_LINEAR:
        for (int q = n - 2; q >= 0; --q) g.push_back({q, q + 1});
        break;
    case GV_ENT_CNOT_PAIRWISE:
        for (int start = 0; start < 2; ++start)
            for (int q = start; q + 1 < n; q += 2) g.push_back({q, q + 1});
        break;
    case GV_ENT_CNOT_SCA: {
        // the circular list, entry 0 = (n-1, 0) and entry e = (e-1, e), rotated
        // right by the layer index; odd layers exchange control and target
        std::vector<std::pair<int, int>> ring;
        if (n > 2) ring.push_back({n - 1, 0});
        for (int q = 0; q + 1 < n; ++q) ring.push_back({q, q + 1});
        const int m = (int)ring.size();
        for (int e = 0; e < m; ++e) {
            std::pair<int, int> ct = n > 2 ? ring[(size_t)(((e - layer) % m + m) % m)] : ring[(size_t)e];
            if (layer & 1) std::swap(ct.first, ct.second);
            g.push_back(ct);
        }
        break;
    }
    default:
        break;
    }
    return g;
}

gv::LinMap gv::cnot_linmap(int n, int ent, int layer, bool inverse)
{
    LinMap m;
    memset(&m, 0, sizeof(m));
    m.n = n;
    for (int q = 0; q < n; ++q) m.col[q] = 1ull << q;
    // CNOT(c -> t) sends v to v ^ (bit c of v) << t; the map of the whole
    // network is the product of the gates (applied to every column), in
    // order for the network and in reverse order for its inverse
    std::vector<std::pair<int, int>> g = cnot_network(n, ent, layer);
    if (inverse) std::reverse(g.begin(), g.end());
    for (const auto &ct : g)
        for (int q = 0; q < n; ++q) m.col[q] ^= ((m.col[q] >> ct.first) & 1ull) << ct.second;
    return m;
}

namespace gv {

static gv_status fused_setup(gv_state st, const gv_ansatz &an, const double *theta,
                             gv_grad_mode mode, FusedCtx *c)
{
    if (gv_status r = work_layout(an, st->prec, st->engine, mode, &c->w)) return r;
    if (c->w.total > st->work_bytes)
        return set_error(GV_ESIZE, "work buffer %zu bytes < %zu needed", st->work_bytes,
                         c->w.total);
    const int K = choose_K(an.n);
    make_tile_plan(an.n, K, choose_C(st->prec, K), &c->plan);
    c->ch = make_chunks(an.n, K, choose_logr(K));
    char *w = (char *)st->work;
    c->tabs.ry = w + c->w.ry_tab;
    c->tabs.dtab = w + c->w.dtab;
    c->tabs.dtab_stride = c->w.dtab_stride;
    c->tabs.gtab = w + c->w.gtab;
    c->tabs.g0tab = w + c->w.g0tab;
    c->tabs.ldtab = w + c->w.ldtab;
    c->tabs.ldtab_stride = c->w.ldtab_stride;
    ProfScope ps(st, GV_PROF_OTHER, 0.0);
    return check_hip(fused_build_tables(st->prec, an, c->ch, theta, c->tabs, st->stream), "tables");
}

// psi <- CNOT D_layer psi (forward) or its inverse, through the scratch vector
static gv_status cnot_step(gv_state st, const gv_ansatz &an, const FusedCtx &c, int layer,
                           void *v, int inverse)
{
    const size_t vb = ((size_t)1 << an.n) * amp_bytes(st->prec);
    void *scratch = (char *)st->work + c.w.scratch;
    ProfScope ps(st, GV_PROF_OTHER, 4.0 * vb);
    hipError_t e = cnot_ladder_gather(st->prec, v, scratch, an, c.ch, &c.tabs, layer, inverse,
                                      st->stream);
    if (e == hipSuccess) e = copy_vector(v, scratch, vb, st->stream);
    return check_hip(e, "cnot ladder");
}

// Forward from |0...0> to psi~_upto, the state after the RY gates of layer
// `upto` and before its diagonal.  skip_last leaves out layer upto's last
// pass (the turnaround applies it).  ckpt (may be NULL) receives psi~_l in
// slot l-1 for l = 1 .. R-2.
static gv_status fused_forward(gv_state st, const gv_ansatz &an, const FusedCtx &c, int upto,
                               bool skip_last, void *psi, char *ckpt, size_t vb)
{
    const int np = c.plan.npass, R = rot_layers(an);
    const bool cnot = is_cnot(an);
    const bool gen_first = !cnot && upto >= 1;  // R_0|0..0> generated inside layer 1's pass 0
    hipStream_t s = st->stream;
    if (!gen_first) {
        ProfScope ps(st, GV_PROF_INIT, (double)vb);
        if (gv_status r = check_hip(fused_init_state(st->prec, psi, an, c.ch, c.tabs, s), "init"))
            return r;
    }
    for (int l = 1; l <= upto; ++l) {
        int in_mode = FWD_LOAD_DIAG;
        if (cnot) {
            if (gv_status r = cnot_step(st, an, c, l - 1, psi, 0)) return r;
            in_mode = FWD_LOAD;
        } else if (l == 1) {
            in_mode = FWD_GENERATE;
        }
        for (int p = 0; p < np; ++p) {
            if (skip_last && l == upto && p == np - 1) break;
            const int mode = p == 0 ? in_mode : FWD_LOAD;
            ProfScope ps(st, GV_PROF_FORWARD_PASS, mode == FWD_GENERATE ? (double)vb : 2.0 * vb);
            if (gv_status r = check_hip(fused_forward_pass(st->prec, psi, an, c.plan, p, l, mode,
                                                           c.ch, c.tabs, s),
                                        "forward pass"))
                return r;
        }
        if (ckpt && l <= R - 2) {
            ProfScope ps(st, GV_PROF_OTHER, 2.0 * vb);
            if (gv_status r = check_hip(copy_vector(ckpt + (size_t)(l - 1) * vb, psi, vb, s),
                                        "checkpoint"))
                return r;
        }
    }
    return GV_OK;
}

// psi~ of the last layer -> psi (its diagonal, and the CNOT ladder when the
// layer carries one), or back on both vectors
static gv_status last_layer_transform(gv_state st, const gv_ansatz &an, const FusedCtx &c,
                                      void *psi, void *lam, int inverse)
{
    const int l = rot_layers(an) - 1;
    const size_t vb = ((size_t)1 << an.n) * amp_bytes(st->prec);
    if (is_cnot(an) && l < an.layers) {
        if (gv_status r = cnot_step(st, an, c, l, psi, inverse)) return r;
        if (lam)
            if (gv_status r = cnot_step(st, an, c, l, lam, inverse)) return r;
        return GV_OK;
    }
    ProfScope ps(st, GV_PROF_OTHER, (lam ? 4.0 : 2.0) * vb);
    return check_hip(fused_diag_apply(st->prec, psi, lam, an, c.ch, c.tabs, l, inverse, st->stream),
                     "diagonal");
}

static bool use_snake(const gv_ansatz &an) { return !is_cnot(an) && rot_layers(an) >= 2; }

// op list and the two-layer passes' diagonal tables
static gv_status snake_setup(gv_state st, const gv_ansatz &an, const double *theta,
                             bool keep_last_single, bool ckpt, FusedCtx *c)
{
    const int R = rot_layers(an);
    c->ops = snake_ops(c->plan.npass, R - 1, keep_last_single, ckpt);
    c->ld.assign(R, LDiagTab{});
    c->ld0.assign(R, LDiagTab{});
    ProfScope ps(st, GV_PROF_OTHER, 0.0);
    for (const FwdOp &op : c->ops) {
        if (op.lb < 0) continue;
        for (int last = 0; last < 2; ++last) {
            void *tab = (char *)c->tabs.ldtab + (size_t)(2 * op.la + last) * c->tabs.ldtab_stride;
            LDiagTab *out = last ? &c->ld[op.la] : &c->ld0[op.la];
            if (gv_status r = check_hip(make_ldiag(st->prec, an, c->plan, op.g, last, op.la, theta,
                                                   tab, out, st->stream),
                                        "layout diagonal tables"))
                return r;
        }
    }
    return GV_OK;
}

// Where the STORE mode keeps the output of pass k: its own buffer, except
// the last pass, which writes the state buffer.
static void *store_out(const FusedCtx &c, int k, void *psi, char *bufs, size_t vb)
{
    return k == (int)c.ops.size() - 1 ? psi : bufs + (size_t)k * vb;
}

// The first `count` passes of the snake order, from |0...0>: in place on
// psi (copying checkpoint slots out of it when ckpt is set), or with
// store = true from each pass's buffer to the next.
static gv_status snake_forward(gv_state st, const gv_ansatz &an, const FusedCtx &c, size_t count,
                               void *psi, char *ckpt, size_t vb, bool store = false)
{
    hipStream_t s = st->stream;
    for (size_t k = 0; k < count; ++k) {
        const FwdOp &op = c.ops[k];
        void *dst = store ? store_out(c, (int)k, psi, ckpt, vb) : psi;
        const void *src = (store && k > 0) ? store_out(c, (int)k - 1, psi, ckpt, vb) : dst;
        ProfScope ps(st, op.lb >= 0 ? GV_PROF_FORWARD_PASS2 : GV_PROF_FORWARD_PASS,
                     op.in_mode == FWD_GENERATE ? (double)vb : 2.0 * vb);
        hipError_t e = op.lb >= 0
                           ? fused_forward2_pass(st->prec, dst, an, c.plan, op.g, op.la, op.in_mode,
                                                 c.ch, c.tabs, c.ld[op.la], s, src)
                           : fused_forward_pass(st->prec, dst, an, c.plan, op.g, op.la, op.in_mode,
                                                c.ch, c.tabs, s, src);
        if (gv_status r = check_hip(e, "forward pass")) return r;
        if (!store && ckpt && op.slot >= 0) {
            ProfScope pc(st, GV_PROF_OTHER, 2.0 * vb);
            if (gv_status r = check_hip(copy_vector(ckpt + (size_t)op.slot * vb, psi, vb, s),
                                        "checkpoint"))
                return r;
        }
    }
    return GV_OK;
}

static gv_status energy_chain(gv_state st, gv_pauli_sum h, void *lam, double *epart,
                              double *energy)
{
    hipStream_t s = st->stream;
    const double vb = (double)((size_t)1 << st->n) * amp_bytes(st->prec);
    {
        ProfScope ps(st, GV_PROF_ENERGY, (lam ? 2 * vb : vb) + (double)((size_t)1 << st->n) * 8);
        if (gv_status r = check_hip(energy_diag(st->prec, st->amps, h->diag, lam, st->n, epart,
                                                kEnergyGrid, s),
                                    "energy diag"))
            return r;
    }
    const bool cover = !h->off_passes.empty() && fused_ok(st->engine, st->n) &&
                       h->cover_K == choose_K(st->n) &&
                       h->cover_C == choose_C(st->prec, choose_K(st->n));
    if (!h->off_passes.empty() && !cover)
        return set_error(GV_ESTATE, "pauli sum was prepared for another precision or engine");
    for (const OffPass &op : h->off_passes) {
        ProfScope ps(st, GV_PROF_OFFDIAG, (lam ? 3.0 : 1.0) * vb);
        if (gv_status r = check_hip(offdiag_pass(st->prec, st->amps, lam, st->n, h->cover_K, op,
                                                 h->dev_cls, h->dev_terms, epart, kEnergyGrid, s),
                                    "off-diagonal pass"))
            return r;
    }
    if (!h->loose_terms.empty()) {
        std::vector<uint64_t> lx, lz;
        std::vector<double> lc;
        for (int64_t k : h->loose_terms) {
            lx.push_back(h->ox[k]);
            lz.push_back(h->oz[k]);
            lc.push_back(h->oc[k]);
        }
        ProfScope ps(st, GV_PROF_OFFDIAG, (double)lx.size() * (lam ? 3 : 1) * vb);
        if (gv_status r = check_hip(energy_offdiag_terms(st->prec, st->amps, lam, st->n,
                                                         (int64_t)lx.size(), lx.data(), lz.data(),
                                                         lc.data(), epart, kEnergyGrid, s),
                                    "energy off-diagonal"))
            return r;
    }
    return check_hip(reduce_energy(epart, kEnergyGrid, energy, s), "energy reduce");
}

}  // namespace gv

using namespace gv;

// ======================================================================= ABI

extern "C" {

const char *gv_version(void) { return "gv 0.1 (gfx950)"; }

const char *gv_last_error(void) { return g_last_error.c_str(); }

gv_status gv_debug_inject_hip_error(int64_t after)
{
    g_inject_after.store(after < 0 ? -1 : after);
    return GV_OK;
}

int64_t gv_num_params(const gv_ansatz *a)
{
    if (check_ansatz(a) != GV_OK) return -1;
    return nparams(*a);
}

gv_status gv_query_sizes(const gv_ansatz *a, gv_precision prec, gv_engine engine,
                         gv_grad_mode mode, size_t *state_bytes, size_t *work_bytes,
                         size_t *diag_bytes)
{
    if (gv_status r = check_ansatz(a)) return r;
    if (prec != GV_C64 && prec != GV_C128) return set_error(GV_EINVAL, "precision");
    if (engine != GV_ENGINE_FUSED && engine != GV_ENGINE_PLAIN) return set_error(GV_EINVAL, "engine");
    if (mode < GV_GRAD_UNCOMPUTE || mode > GV_GRAD_STORE) return set_error(GV_EINVAL, "mode");
    WorkLayout w;
    if (gv_status r = work_layout(*a, prec, engine, mode, &w)) return r;
    if (state_bytes) *state_bytes = ((size_t)1 << a->n) * amp_bytes(prec);
    if (work_bytes) *work_bytes = w.total;
    if (diag_bytes) *diag_bytes = ((size_t)1 << a->n) * sizeof(double);
    return GV_OK;
}

gv_status gv_state_create(int32_t n, gv_precision prec, gv_engine engine, void *amps,
                          size_t amps_bytes, void *work, size_t work_bytes, void *stream,
                          gv_state *out)
{
    if (!out) return set_error(GV_EINVAL, "out is NULL");
    if (n < 1 || n > kMaxQubits) return set_error(GV_EINVAL, "n=%d outside 1..%d", n, kMaxQubits);
    if (prec != GV_C64 && prec != GV_C128) return set_error(GV_EINVAL, "precision %d", prec);
    if (engine != GV_ENGINE_FUSED && engine != GV_ENGINE_PLAIN)
        return set_error(GV_EINVAL, "engine %d", engine);
    if (!amps) return set_error(GV_EINVAL, "amplitude buffer is NULL");
    const size_t need = ((size_t)1 << n) * amp_bytes(prec);
    if (amps_bytes < need)
        return set_error(GV_ESIZE, "amplitude buffer %zu bytes < %zu", amps_bytes, need);
    if (!aligned(amps) || (work && !aligned(work)))
        return set_error(GV_EINVAL, "device buffers must be %zu-byte aligned", kAlign);
    gv_state st = new (std::nothrow) gv_state_s;
    if (!st) return set_error(GV_EINVAL, "out of host memory");
    st->n = n;
    st->prec = prec;
    st->engine = engine;
    st->amps = amps;
    st->amps_bytes = amps_bytes;
    st->work = work;
    st->work_bytes = work ? work_bytes : 0;
    st->stream = (hipStream_t)stream;
    *out = st;
    return GV_OK;
}

gv_status gv_state_destroy(gv_state st)
{
    if (st) {
        gv_profile_reset(st);
        for (hipEvent_t e : st->event_pool) (void)hipEventDestroy(e);
    }
    delete st;
    return GV_OK;
}

gv_status gv_state_set_stream(gv_state st, void *stream)
{
    if (!st) return set_error(GV_EINVAL, "state is NULL");
    st->stream = (hipStream_t)stream;
    return GV_OK;
}

gv_status gv_apply_ansatz(gv_state st, const double *theta, const gv_ansatz *a)
{
    if (!st) return set_error(GV_EINVAL, "state is NULL");
    if (gv_status r = check_ansatz(a)) return r;
    if (a->n != st->n) return set_error(GV_ESTATE, "ansatz n=%d but state n=%d", a->n, st->n);
    if (!theta) return set_error(GV_EINVAL, "params is NULL");
    if (rot_layers(*a) == 0) {
        if (gv_status r = check_hip(plain_set_zero_state(st->prec, st->amps, a->n, st->stream),
                                    "zero state"))
            return r;
    } else if (fused_ok(st->engine, a->n)) {
        FusedCtx c;
        if (gv_status r = fused_setup(st, *a, theta, GV_GRAD_UNCOMPUTE, &c)) return r;
        const size_t vb = ((size_t)1 << a->n) * amp_bytes(st->prec);
        if (use_snake(*a)) {
            if (gv_status r = snake_setup(st, *a, theta, false, false, &c)) return r;
            if (gv_status r = snake_forward(st, *a, c, c.ops.size(), st->amps, nullptr, vb))
                return r;
        } else if (gv_status r = fused_forward(st, *a, c, rot_layers(*a) - 1, false, st->amps,
                                               nullptr, vb)) {
            return r;
        }
        if (gv_status r = last_layer_transform(st, *a, c, st->amps, nullptr, 0)) return r;
    } else {
        if (gv_status r = plain_forward(st, *a, theta)) return r;
    }
    st->has_psi = true;
    return GV_OK;
}

gv_status gv_pauli_sum_create(int32_t n, int64_t m, const uint64_t *x, const uint64_t *z,
                              const double *c, gv_pauli_sum *out)
{
    if (!out) return set_error(GV_EINVAL, "out is NULL");
    if (n < 1 || n > kMaxQubits) return set_error(GV_EINVAL, "n=%d outside 1..%d", n, kMaxQubits);
    if (m < 0) return set_error(GV_EINVAL, "m < 0");
    if (m > 0 && (!x || !z || !c)) return set_error(GV_EINVAL, "term arrays are NULL");
    const uint64_t valid = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    std::map<std::pair<uint64_t, uint64_t>, double> merged;
    for (int64_t k = 0; k < m; ++k) {
        if ((x[k] | z[k]) & ~valid)
            return set_error(GV_EINVAL, "term %lld has a mask bit >= n", (long long)k);
        if (!isfinite(c[k]))
            return set_error(GV_EINVAL, "term %lld has a non-finite coefficient", (long long)k);
        merged[std::make_pair(x[k], z[k])] += c[k];
    }
    gv_pauli_sum h = new (std::nothrow) gv_pauli_s;
    if (!h) return set_error(GV_EINVAL, "out of host memory");
    h->n = n;
    for (const auto &kv : merged) {
        if (kv.second == 0.0) continue;
        if (kv.first.first == 0) {
            h->dz.push_back(kv.first.second);
            h->dc.push_back(kv.second);
        } else {
            h->ox.push_back(kv.first.first);
            h->oz.push_back(kv.first.second);
            h->oc.push_back(kv.second);
        }
    }
    // greedy qubit-wise-commuting groups of the off-diagonal terms: every
    // qubit carries one letter (X, Y or Z) per group
    for (size_t k = 0; k < h->ox.size(); ++k) {
        const uint64_t xk = h->ox[k], zk = h->oz[k];
        const uint64_t X = xk & ~zk, Y = xk & zk, Z = zk & ~xk;
        bool placed = false;
        for (QwcGroup &g : h->groups) {
            const uint64_t gsup = g.xmask | g.ymask | g.zmask, ksup = xk | zk;
            const uint64_t both = gsup & ksup;
            if (((g.xmask ^ X) & both) || ((g.ymask ^ Y) & both) || ((g.zmask ^ Z) & both))
                continue;
            g.xmask |= X;
            g.ymask |= Y;
            g.zmask |= Z;
            g.terms.push_back((int64_t)k);
            placed = true;
            break;
        }
        if (!placed) {
            QwcGroup g;
            g.xmask = X;
            g.ymask = Y;
            g.zmask = Z;
            g.terms.push_back((int64_t)k);
            h->groups.push_back(g);
        }
    }
    *out = h;
    return GV_OK;
}

gv_status gv_pauli_sum_destroy(gv_pauli_sum h)
{
    delete h;
    return GV_OK;
}

gv_status gv_pauli_sum_info(gv_pauli_sum h, int64_t *n_diag, int64_t *n_offdiag, int64_t *n_groups)
{
    if (!h) return set_error(GV_EINVAL, "pauli sum is NULL");
    if (n_diag) *n_diag = (int64_t)h->dz.size();
    if (n_offdiag) *n_offdiag = (int64_t)h->ox.size();
    if (n_groups) *n_groups = (int64_t)h->groups.size();
    return GV_OK;
}

static void pauli_layout(const gv_pauli_s *h, size_t *diag, size_t *cls, size_t *terms,
                         size_t *sz, size_t *sc, size_t *total, size_t *gmask = nullptr,
                         size_t *gcoef = nullptr)
{
    size_t off = 0;
    *diag = off;
    off += align_up(((size_t)1 << h->n) * sizeof(double));
    *cls = off;
    off += align_up(h->ox.size() * sizeof(OffClass) + 8);
    *terms = off;
    off += align_up(h->ox.size() * sizeof(OffTerm) + 8);
    *sz = off;
    off += align_up(h->dz.size() * 8 + 8);
    *sc = off;
    off += align_up(h->dc.size() * 8 + 8);
    if (gmask) *gmask = off;
    off += align_up(h->ox.size() * 8 + 8);
    if (gcoef) *gcoef = off;
    off += align_up(h->ox.size() * 8 + 8);
    *total = off;
}

// Bits of the tile a cover pass should take next: grown from `seed` one bit
// at a time, each time the bit that completes the most pending classes
// (weighted by their terms), ties broken by the number of pending classes
// the bit could still complete with the free slots left, then by the bit.
static uint64_t grow_tile(uint64_t tile, int K, int n, const std::vector<uint64_t> &hx,
                          const std::vector<int64_t> &wt, const std::vector<char> &done)
{
    while (__builtin_popcountll(tile) < K) {
        const int free_after = K - __builtin_popcountll(tile) - 1;
        int best_q = -1;
        int64_t best_gain = -1, best_part = -1;
        for (int q = 0; q < n; ++q) {
            const uint64_t b = 1ull << q;
            if (tile & b) continue;
            int64_t gain = 0, part = 0;
            for (size_t c = 0; c < hx.size(); ++c) {
                if (done[c] || !(hx[c] & b)) continue;
                const uint64_t miss = hx[c] & ~(tile | b);
                if (!miss) gain += wt[c];
                else if (__builtin_popcountll(miss) <= free_after) part += 1;
            }
            if (gain > best_gain || (gain == best_gain && part > best_part)) {
                best_q = q;
                best_gain = gain;
                best_part = part;
            }
        }
        if (best_q < 0) break;
        tile |= 1ull << best_q;
    }
    return tile;
}

// Group the off-diagonal terms by flip mask (classes) and cover the classes
// with tiles of K index bits that keep bits 0..C-1: a class goes to a tile
// that holds its flip bits, and every class sits in exactly one tile.  The
// tiles are chosen greedily to cover as many pending terms as possible
// (several seeds per pass, the best kept), with at most kOffPassTerms terms
// per pass so the pass stages all of them in LDS.  Within a class the terms
// are ordered by (real / imaginary phase, z restricted to the register bits
// of the pass's load layout), and the last term of each such group is
// flagged: the kernel sums a group's signed coefficients per thread and
// applies the group's register sign pattern once.  Classes whose flip bits
// cannot fit any tile are applied term by term.
static void build_cover(gv_pauli_s *h, int K, int C, int logr)
{
    h->classes.clear();
    h->class_terms.clear();
    h->off_passes.clear();
    h->loose_terms.clear();
    h->cover_K = K;
    h->cover_C = C;
    const int n = h->n;
    std::map<uint64_t, std::vector<int64_t>> by_x;
    for (size_t k = 0; k < h->ox.size(); ++k) by_x[h->ox[k]].push_back((int64_t)k);
    const uint64_t low = (C >= 64) ? ~0ull : ((1ull << C) - 1);
    // classes, a class of more than kOffPassTerms terms split into several
    // with the same flip mask (their factors add on the same pairs)
    std::vector<uint64_t> xs, hx;
    std::vector<int64_t> wt;
    std::vector<std::vector<int64_t>> cterms;
    for (const auto &kv : by_x) {
        if (__builtin_popcountll(kv.first & ~low) > K - C) {
            for (int64_t k : kv.second) h->loose_terms.push_back(k);
            continue;
        }
        for (size_t i0 = 0; i0 < kv.second.size(); i0 += kOffPassTerms) {
            const size_t i1 = std::min(kv.second.size(), i0 + (size_t)kOffPassTerms);
            xs.push_back(kv.first);
            hx.push_back(kv.first & ~low);
            wt.push_back((int64_t)(i1 - i0));
            cterms.emplace_back(kv.second.begin() + i0, kv.second.begin() + i1);
        }
    }
    std::vector<char> done(xs.size(), 0);
    size_t left = xs.size();
    while (left > 0) {
        // seeds: the low bits alone, and the low bits plus each flip bit of
        // the pending classes with the most terms
        std::vector<uint64_t> seeds{low};
        {
            std::vector<size_t> idx;
            for (size_t c = 0; c < xs.size(); ++c)
                if (!done[c]) idx.push_back(c);
            std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return wt[a] > wt[b]; });
            for (size_t i = 0; i < idx.size() && seeds.size() < 9; ++i)
                if (__builtin_popcountll(low | hx[idx[i]]) <= K) seeds.push_back(low | hx[idx[i]]);
        }
        uint64_t best_tile = 0;
        int64_t best_cov = -1;
        for (uint64_t seed : seeds) {
            const uint64_t t = grow_tile(seed, K, n, hx, wt, done);
            int64_t cov = 0, nt = 0;
            for (size_t c = 0; c < xs.size(); ++c)
                if (!done[c] && !(hx[c] & ~t) && nt + wt[c] <= kOffPassTerms) {
                    cov += wt[c];
                    nt += wt[c];
                }
            if (cov > best_cov) {
                best_cov = cov;
                best_tile = t;
            }
        }
        uint64_t tile = best_tile;
        for (int q = 0; q < n && __builtin_popcountll(tile) < K; ++q) tile |= 1ull << q;
        OffPass op;
        int j = 0;
        int8_t where[64];
        for (int q = 0; q < n; ++q)
            if ((tile >> q) & 1) {
                where[q] = (int8_t)j;
                op.pos[j++] = (int8_t)q;
            }
        // register bits of the load layout: tile bits K - logr .. K - 1
        uint64_t regmask = 0;
        for (int r = K - logr; r < K; ++r) regmask |= 1ull << op.pos[r];
        op.c0 = (int)h->classes.size();
        int64_t nt = 0;
        for (size_t c = 0; c < xs.size(); ++c) {
            if (done[c] || (hx[c] & ~tile) || nt + wt[c] > kOffPassTerms) continue;
            done[c] = 1;
            --left;
            nt += wt[c];
            const uint64_t x = xs[c];
            OffClass cl;
            cl.x = x;
            cl.xu = 0;
            for (int q = 0; q < n; ++q)
                if ((x >> q) & 1) cl.xu |= 1u << where[q];
            cl.t0 = (int32_t)h->class_terms.size();
            std::vector<int64_t> ks = cterms[c];
            auto key = [&](int64_t k) {
                const int imag = __builtin_popcountll(h->ox[k] & h->oz[k]) & 1;
                return std::make_pair(imag, h->oz[k] & regmask);
            };
            std::stable_sort(ks.begin(), ks.end(), [&](int64_t a, int64_t b) { return key(a) < key(b); });
            cl.ti = cl.t0 + (int32_t)ks.size();
            uint32_t flat_off = 0;   // sides with a register sign
            for (size_t i = 0; i < ks.size(); ++i) {
                const int64_t k = ks[i];
                const uint64_t z = h->oz[k];
                const int ph = __builtin_popcountll(x & z) & 3;
                if ((ph & 1) && cl.ti == cl.t0 + (int32_t)ks.size())
                    cl.ti = (int32_t)h->class_terms.size();
                OffTerm tm;
                tm.z = z;
                // i^ph = +-1 or +-i; the -1 of ph & 2 and of the parity of
                // x & z (the flipped bits' share of (i ^ x) & z) go into cf
                const bool neg = ((ph >> 1) & 1) ^ (__builtin_popcountll(x & z) & 1);
                tm.cf = neg ? -h->oc[k] : h->oc[k];
                tm.tz = 0;
                for (int j = 0; j < K - logr; ++j)
                    if ((z >> op.pos[j]) & 1) tm.tz |= 1u << j;
                tm.sig = 0;
                for (int r = 0; r < (1 << logr); ++r) {
                    int par = 0;
                    for (int b = 0; b < logr; ++b)
                        if ((r >> b) & 1) par ^= (int)((z >> op.pos[K - logr + b]) & 1);
                    tm.sig |= (uint32_t)par << r;
                }
                if (i + 1 == ks.size() || key(ks[i + 1]) != key(k)) tm.sig |= kOffGroupEnd;
                tm.cf32 = (float)tm.cf;
                tm.pad = 0;
                if (tm.sig & 0xffffu) flat_off |= (ph & 1) ? kOffImFlat : kOffReFlat;
                h->class_terms.push_back(tm);
            }
            cl.t1 = (int32_t)h->class_terms.size();
            cl.xu |= (kOffReFlat | kOffImFlat) & ~flat_off;
            h->classes.push_back(cl);
        }
        op.c1 = (int)h->classes.size();
        // every pass takes a class: the seeded tiles each cover the class
        // they were seeded with, which holds at most kOffPassTerms terms
        if (op.c1 == op.c0) {   // (defensive) apply what is left term by term
            for (size_t c = 0; c < xs.size(); ++c)
                if (!done[c]) {
                    done[c] = 1;
                    --left;
                    for (int64_t k : cterms[c]) h->loose_terms.push_back(k);
                }
            break;
        }
        h->off_passes.push_back(op);
    }
}

gv_status gv_pauli_sum_plan(gv_pauli_sum h, int32_t n_state, gv_precision prec, gv_engine engine,
                            int64_t *passes, int64_t *max_pass_terms, int64_t *loose_terms)
{
    if (!h) return set_error(GV_EINVAL, "pauli sum is NULL");
    if (prec != GV_C64 && prec != GV_C128) return set_error(GV_EINVAL, "precision %d", prec);
    if (engine != GV_ENGINE_FUSED && engine != GV_ENGINE_PLAIN) return set_error(GV_EINVAL, "engine");
    if (n_state != h->n) return set_error(GV_ESTATE, "pauli sum n=%d but n=%d", h->n, n_state);
    gv_pauli_s tmp;
    tmp.n = h->n;
    tmp.ox = h->ox;
    tmp.oz = h->oz;
    tmp.oc = h->oc;
    int64_t np = 0, mx = 0, lo = (int64_t)h->ox.size();
    if (fused_ok(engine, h->n)) {
        const int K = choose_K(h->n);
        build_cover(&tmp, K, choose_C(prec, K), choose_logr(K));
        np = (int64_t)tmp.off_passes.size();
        for (const OffPass &op : tmp.off_passes)
            mx = std::max<int64_t>(mx, tmp.classes[op.c1 - 1].t1 - tmp.classes[op.c0].t0);
        lo = (int64_t)tmp.loose_terms.size();
    }
    if (passes) *passes = np;
    if (max_pass_terms) *max_pass_terms = mx;
    if (loose_terms) *loose_terms = lo;
    return GV_OK;
}

gv_status gv_pauli_sum_device_bytes(gv_pauli_sum h, size_t *bytes)
{
    if (!h || !bytes) return set_error(GV_EINVAL, "NULL argument");
    size_t a, b, c, d, e;
    pauli_layout(h, &a, &b, &c, &d, &e, bytes);
    return GV_OK;
}

static gv_status prepare_impl(gv_pauli_sum h, gv_precision prec, gv_engine engine, hipStream_t s,
                              void *dev, size_t bytes)
{
    if (!dev) return set_error(GV_EINVAL, "NULL buffer");
    if (prec != GV_C64 && prec != GV_C128) return set_error(GV_EINVAL, "precision %d", prec);
    if (engine != GV_ENGINE_FUSED && engine != GV_ENGINE_PLAIN) return set_error(GV_EINVAL, "engine");
    if (!aligned(dev)) return set_error(GV_EINVAL, "buffer must be %zu-byte aligned", kAlign);
    size_t odiag, ocls, oterms, osz, osc, total, ogm, ogc;
    pauli_layout(h, &odiag, &ocls, &oterms, &osz, &osc, &total, &ogm, &ogc);
    if (bytes < total) return set_error(GV_ESIZE, "buffer %zu bytes < %zu", bytes, total);
    char *base = (char *)dev;
    h->dev_gmask = (uint64_t *)(base + ogm);
    h->dev_gcoef = (double *)(base + ogc);
    h->prep_gen++;
    h->dev = dev;
    h->dev_bytes = bytes;
    h->diag = (double *)(base + odiag);
    h->dev_cls = (OffClass *)(base + ocls);
    h->dev_terms = (OffTerm *)(base + oterms);
    h->prepared = false;
    const int n = h->n;
    if (fused_ok(engine, n)) {
        const int K = choose_K(n);
        build_cover(h, K, choose_C(prec, K), choose_logr(K));
    } else {
        h->classes.clear();
        h->class_terms.clear();
        h->off_passes.clear();
        h->loose_terms.clear();
        for (size_t k = 0; k < h->ox.size(); ++k) h->loose_terms.push_back((int64_t)k);
        h->cover_K = h->cover_C = 0;
    }
    if (!h->classes.empty()) {
        if (gv_status r = check_hip(hipMemcpyAsync(h->dev_cls, h->classes.data(),
                                                   h->classes.size() * sizeof(OffClass),
                                                   hipMemcpyHostToDevice, s), "copy"))
            return r;
        if (gv_status r = check_hip(hipMemcpyAsync(h->dev_terms, h->class_terms.data(),
                                                   h->class_terms.size() * sizeof(OffTerm),
                                                   hipMemcpyHostToDevice, s), "copy"))
            return r;
    }
    // off-diagonal terms in group order: support masks and coefficients
    std::vector<uint64_t> gm;
    std::vector<double> gc;
    for (const QwcGroup &g : h->groups)
        for (int64_t k : g.terms) {
            gm.push_back(h->ox[(size_t)k] | h->oz[(size_t)k]);
            gc.push_back(h->oc[(size_t)k]);
        }
    if (!gm.empty()) {
        if (gv_status r = check_hip(hipMemcpyAsync(h->dev_gmask, gm.data(), gm.size() * 8,
                                                   hipMemcpyHostToDevice, s), "copy"))
            return r;
        if (gv_status r = check_hip(hipMemcpyAsync(h->dev_gcoef, gc.data(), gc.size() * 8,
                                                   hipMemcpyHostToDevice, s), "copy"))
            return r;
    }
    uint64_t *sz = (uint64_t *)(base + osz);
    double *sc = (double *)(base + osc);
    if (!h->dz.empty()) {
        if (gv_status r = check_hip(hipMemcpyAsync(sz, h->dz.data(), h->dz.size() * 8,
                                                   hipMemcpyHostToDevice, s), "copy"))
            return r;
        if (gv_status r = check_hip(hipMemcpyAsync(sc, h->dc.data(), h->dc.size() * 8,
                                                   hipMemcpyHostToDevice, s), "copy"))
            return r;
    }
    if (gv_status r = check_hip(fill_zero_f64(h->diag, 1ull << n, s), "zero diag")) return r;
    if (gv_status r = check_hip(scatter_coeffs(h->diag, sz, sc, (int64_t)h->dz.size(), s), "scatter"))
        return r;
    if (gv_status r = check_hip(fwht_inplace(h->diag, n, s), "fwht")) return r;
    if (gv_status r = check_hip(hipStreamSynchronize(s), "prepare sync")) return r;
    h->prepared = true;
    return GV_OK;
}

gv_status gv_pauli_sum_prepare(gv_pauli_sum h, gv_state st, void *dev, size_t bytes)
{
    if (!h || !st) return set_error(GV_EINVAL, "NULL argument");
    if (h->n != st->n) return set_error(GV_ESTATE, "pauli sum n=%d but state n=%d", h->n, st->n);
    return prepare_impl(h, st->prec, st->engine, st->stream, dev, bytes);
}

gv_status gv_pauli_sum_prepare_for(gv_pauli_sum h, gv_precision prec, gv_engine engine,
                                   void *stream, void *dev, size_t bytes)
{
    if (!h) return set_error(GV_EINVAL, "NULL argument");
    return prepare_impl(h, prec, engine, (hipStream_t)stream, dev, bytes);
}

gv_status gv_energy(gv_state st, gv_pauli_sum h, double *energy)
{
    if (!st || !h || !energy) return set_error(GV_EINVAL, "NULL argument");
    if (!h->prepared) return set_error(GV_ESTATE, "pauli sum not prepared");
    if (h->n != st->n) return set_error(GV_ESTATE, "pauli sum n=%d but state n=%d", h->n, st->n);
    if (!st->has_psi) return set_error(GV_ESTATE, "no state: call gv_apply_ansatz first");
    if (st->work_bytes < align_up(2 * kEnergyGrid * sizeof(double)))
        return set_error(GV_ESIZE, "energy needs >= %zu work bytes",
                         align_up(2 * kEnergyGrid * sizeof(double)));
    return energy_chain(st, h, nullptr, (double *)st->work, energy);
}

gv_status gv_energy_grad(gv_state st, gv_pauli_sum h, const double *theta, const gv_ansatz *a,
                         const uint8_t *mask, gv_grad_mode mode, double *energy, double *grad)
{
    if (!st || !h || !theta || !energy || !grad) return set_error(GV_EINVAL, "NULL argument");
    if (gv_status r = check_ansatz(a)) return r;
    if (a->n != st->n) return set_error(GV_ESTATE, "ansatz n=%d but state n=%d", a->n, st->n);
    if (!h->prepared) return set_error(GV_ESTATE, "pauli sum not prepared");
    if (h->n != st->n) return set_error(GV_ESTATE, "pauli sum n=%d but state n=%d", h->n, st->n);
    if (mode < GV_GRAD_UNCOMPUTE || mode > GV_GRAD_STORE) return set_error(GV_EINVAL, "mode");
    const int64_t P = nparams(*a);
    const int n = a->n;
    const size_t vb = ((size_t)1 << n) * amp_bytes(st->prec);
    hipStream_t s = st->stream;
    char *w = (char *)st->work;

    if (!fused_ok(st->engine, n)) {
        if (mode != GV_GRAD_UNCOMPUTE)
            return set_error(GV_EUNSUPPORTED, "the plain engine runs the uncompute sweep only");
        WorkLayout L;
        if (gv_status r = work_layout(*a, st->prec, st->engine, mode, &L)) return r;
        if (L.total > st->work_bytes)
            return set_error(GV_ESIZE, "work buffer %zu bytes < %zu needed", st->work_bytes, L.total);
        void *lam = w + L.lam;
        double *part = (double *)(w + L.part);
        if (gv_status r = plain_forward(st, *a, theta)) return r;
        if (gv_status r = energy_chain(st, h, lam, (double *)(w + L.epart), energy)) return r;
        const std::vector<Gate> g = gate_list(*a);
        for (size_t k = g.size(); k-- > 0;) {
            const Gate &G = g[k];
            hipError_t e;
            const double A = (double)(1ull << n), sb = (double)amp_bytes(st->prec);
            ProfScope ps(st, GV_PROF_PLAIN_GATE,
                         G.kind == 2 ? A * sb : (G.kind == 3 ? 2 * A * sb : 4 * A * sb));
            switch (G.kind) {
            case 0:
                e = plain_adj_ry(st->prec, st->amps, lam, n, G.a, theta, G.p, part + G.p * L.grid, s);
                break;
            case 1:
                e = plain_adj_rz(st->prec, st->amps, lam, n, G.a, theta, G.p, part + G.p * L.grid, s);
                break;
            case 2:
                e = plain_cz(st->prec, st->amps, n, G.a, G.b, s);
                if (e == hipSuccess) e = plain_cz(st->prec, lam, n, G.a, G.b, s);
                break;
            default:
                e = plain_cnot(st->prec, st->amps, n, G.a, G.b, s);
                if (e == hipSuccess) e = plain_cnot(st->prec, lam, n, G.a, G.b, s);
                break;
            }
            if (gv_status r = check_hip(e, "reverse step")) return r;
        }
        st->has_psi = false;
        ProfScope ps(st, GV_PROF_OTHER, 0.0);
        return check_hip(reduce_rows(part, P, L.grid, mask, grad, s), "grad reduce");
    }

    const int R = rot_layers(*a);
    if (R == 0) {  // no parameters: psi = |0...0>
        if (st->work_bytes < align_up(2 * kEnergyGrid * sizeof(double)))
            return set_error(GV_ESIZE, "work buffer too small");
        if (gv_status r = check_hip(plain_set_zero_state(st->prec, st->amps, n, s), "zero"))
            return r;
        st->has_psi = true;
        return energy_chain(st, h, nullptr, (double *)w, energy);
    }
    FusedCtx c;
    if (gv_status r = fused_setup(st, *a, theta, mode, &c)) return r;
    void *psi = st->amps;
    void *lam = w + c.w.lam;
    // the layer-by-layer path keeps layer boundaries for STORE as CHECKPOINT does
    const gv_grad_mode lmode = mode == GV_GRAD_STORE ? GV_GRAD_CHECKPOINT : mode;
    char *ckpt = (lmode == GV_GRAD_CHECKPOINT && R > 2) ? w + c.w.ckpt : nullptr;
    double *part = (double *)(w + c.w.part);
    double *epart = (double *)(w + c.w.epart);
    const bool cnot = is_cnot(*a);
    const int np = c.plan.npass;
    const bool zonly = h->oc.empty();
    // the turnaround fuses the last forward pass, the energy and the first
    // reverse pass; it needs a diagonal H that commutes with the last layer
    const bool turn = zonly && !cnot && R >= 2;

    if (use_snake(*a)) {
        const bool store = mode == GV_GRAD_STORE;
        // checkpoint slots mark the states that CHECKPOINT keeps and RECOMPUTE rebuilds
        const bool slots = mode == GV_GRAD_CHECKPOINT || mode == GV_GRAD_RECOMPUTE;
        if (gv_status r = snake_setup(st, *a, theta, turn, slots, &c)) return r;
        const std::vector<FwdOp> &ops = c.ops;
        const int nops = (int)ops.size();
        for (const FwdOp &op : ops)
            if (op.slot >= R - 2) return set_error(GV_EUNSUPPORTED, "checkpoint slot %d", op.slot);
        if (store && nops - 1 > store_slots(*a, np))
            return set_error(GV_EUNSUPPORTED, "%d passes need more buffers than reserved", nops);
        char *ck = (mode == GV_GRAD_CHECKPOINT || store) ? w + c.w.ckpt : nullptr;
        int kstart;
        if (turn) {
            if (gv_status r = snake_forward(st, *a, c, nops - 1, psi, ck, vb, store)) return r;
            const FwdOp &op = ops[nops - 1];
            const void *tin = (store && nops >= 2) ? store_out(c, nops - 2, psi, ck, vb) : psi;
            ProfScope ps(st, GV_PROF_TURNAROUND, 2.0 * vb + 8.0 * (double)((size_t)1 << n));
            if (gv_status r = check_hip(fused_turnaround(st->prec, tin, lam, h->diag, *a, c.plan,
                                                         op.g, op.la, op.in_mode, c.ch, c.tabs,
                                                         part, epart, c.w.grid, s),
                                        "turnaround"))
                return r;
            if (gv_status r = check_hip(reduce_energy(epart, c.w.grid, energy, s), "energy reduce"))
                return r;
            kstart = nops - 2;
        } else {
            // psi~ -> psi (the last layer's diagonal), E and lam = H psi, then
            // both vectors back to the point before that diagonal
            if (gv_status r = snake_forward(st, *a, c, nops, psi, ck, vb, store)) return r;
            if (gv_status r = last_layer_transform(st, *a, c, psi, nullptr, 0)) return r;
            if (gv_status r = energy_chain(st, h, lam, epart, energy)) return r;
            if (gv_status r = last_layer_transform(st, *a, c, psi, lam, 1)) return r;
            kstart = nops - 1;
        }
        for (int k = kstart; k >= 0; --k) {
            const FwdOp &op = ops[k];
            // phi comes from the previous reverse pass (uncompute), from the
            // turnaround's untouched input, from a checkpoint or recomputed;
            // the last three have not been through the next pass's load diagonal
            const void *phi_src = store ? store_out(c, k, psi, ck, vb) : psi;
            bool fresh = store || (turn && k == kstart);
            if (!store && k != kstart && op.slot >= 0) {
                if (mode == GV_GRAD_CHECKPOINT) {
                    phi_src = ck + (size_t)op.slot * vb;
                    fresh = true;
                } else if (mode == GV_GRAD_RECOMPUTE) {
                    if (gv_status r = snake_forward(st, *a, c, k + 1, psi, nullptr, vb)) return r;
                    fresh = true;
                }
            }
            const bool next_diag = k + 1 < nops && ops[k + 1].in_mode == FWD_LOAD_DIAG;
            const bool prev_fresh =
                store || (k >= 1 && ops[k - 1].slot >= 0 && mode != GV_GRAD_UNCOMPUTE);
            BwdFlags fl;
            fl.diag_lam = next_diag;
            fl.diag_phi = next_diag && !fresh;
            fl.store_phi = k >= 1 && !prev_fresh;
            fl.store_lam = 1;
            fl.grad_first = !fl.store_phi && !fl.diag_phi;
            // a two-layer pass is undone in one sweep from its output (3 A s,
            // 4 when phi must be carried back, instead of 7 or 8)
            if (op.lb >= 0 && k >= 1 && !fl.diag_lam) {
                ProfScope ps(st, GV_PROF_BACKWARD2, (fl.store_phi ? 4.0 : 3.0) * vb);
                if (gv_status r = check_hip(
                        fused_backward2_pass(st->prec, phi_src, psi, lam, *a, c.plan, op.g, op.la,
                                             fl.store_phi, c.ld[op.la], c.tabs, part, c.w.grid, s),
                        "two-layer backward pass"))
                    return r;
                continue;
            }
            // otherwise a two-layer pass is undone by two reverse passes: layer
            // lb's RY gates, then layer la's diagonal (on load) and RY gates
            if (op.lb >= 0) {
                BwdFlags fa = fl;
                fa.store_phi = 1;
                fa.grad_first = 0;
                ProfScope ps(st, GV_PROF_BACKWARD_PASS, 4.0 * vb);
                if (gv_status r = check_hip(
                        fused_backward_pass(st->prec, phi_src, psi, lam, *a, c.plan, op.g, op.lb,
                                            fa, c.ch, c.tabs, part, c.w.grid, s),
                        "backward pass"))
                    return r;
                phi_src = psi;
                fl.diag_phi = fl.diag_lam = 0;
            }
            const double bytes = (3.0 + (fl.store_phi ? 1.0 : 0.0)) * vb;
            const bool ldl = op.lb >= 0;
            ProfScope ps(st,
                         fl.grad_first ? (ldl ? GV_PROF_BACKWARD_GF_LD : GV_PROF_BACKWARD_GF)
                                       : (ldl ? GV_PROF_BACKWARD_LD : GV_PROF_BACKWARD_PASS),
                         bytes);
            hipError_t e = fused_backward_pass(st->prec, phi_src, psi, lam, *a, c.plan, op.g, op.la,
                                               fl, c.ch, c.tabs, part, c.w.grid, s,
                                               op.lb >= 0 ? &c.ld0[op.la] : nullptr);
            if (gv_status r = check_hip(e, "backward pass")) return r;
        }
        {   // layer 0: lam now sits after the first layer's diagonal
            ProfScope ps(st, GV_PROF_FIRST_LAYER, (double)vb);
            if (gv_status r = check_hip(fused_layer0_grad(st->prec, lam, *a, c.plan, 1, c.ch,
                                                          c.tabs, part, c.w.grid, s),
                                        "first-layer gradients"))
                return r;
        }
        st->has_psi = false;
        ProfScope ps(st, GV_PROF_OTHER, 0.0);
        return check_hip(reduce_rows(part, P, c.w.grid, mask, grad, s), "grad reduce");
    }

    // What the state and lam buffers hold at the start of a layer's reverse
    // sweep: the point before the layer's diagonal (PRE) or after it (POST).
    bool phi_post, lam_post;
    if (turn) {
        if (gv_status r = fused_forward(st, *a, c, R - 1, true, psi, ckpt, vb)) return r;
        const int l = R - 1, p = np - 1;
        const int in_mode = np > 1 ? FWD_LOAD : (l == 1 ? FWD_GENERATE : FWD_LOAD_DIAG);
        ProfScope ps(st, GV_PROF_TURNAROUND, 2.0 * vb + 8.0 * (double)((size_t)1 << n));
        if (gv_status r = check_hip(fused_turnaround(st->prec, psi, lam, h->diag, *a, c.plan, p, l,
                                                     in_mode, c.ch, c.tabs, part, epart,
                                                     c.w.grid, s),
                                    "turnaround"))
            return r;
        if (gv_status r = check_hip(reduce_energy(epart, c.w.grid, energy, s), "energy reduce"))
            return r;
        phi_post = lam_post = false;
    } else {
        if (gv_status r = fused_forward(st, *a, c, R - 1, false, psi, ckpt, vb)) return r;
        // a diagonal H commutes with a diagonal last layer: then psi~ serves as psi
        const bool need_t = !zonly || (cnot && R - 1 < a->layers);
        if (need_t)
            if (gv_status r = last_layer_transform(st, *a, c, psi, nullptr, 0)) return r;
        if (gv_status r = energy_chain(st, h, lam, epart, energy)) return r;
        phi_post = lam_post = need_t;
    }

    for (int l = R - 1; l >= 0; --l) {
        // passes of this layer still to undo (the turnaround did the last one)
        const int npl = (turn && l == R - 1) ? np - 1 : np;
        const bool cnot_layer = cnot && l < a->layers;
        const bool phi_gen = l == 0;
        const void *phi_src = psi;
        if (!phi_gen && l <= R - 2 && npl > 0) {
            if (lmode == GV_GRAD_CHECKPOINT) {
                phi_src = ckpt + (size_t)(l - 1) * vb;
                phi_post = false;
            } else if (lmode == GV_GRAD_RECOMPUTE) {
                if (gv_status r = fused_forward(st, *a, c, l, false, psi, nullptr, vb)) return r;
                phi_post = false;
            }
        }
        if (phi_gen) phi_post = false;
        if (cnot_layer && npl > 0) {  // undo the ladder (and the diagonal) by gathers
            if (lam_post)
                if (gv_status r = cnot_step(st, *a, c, l, lam, 1)) return r;
            if (phi_post)
                if (gv_status r = cnot_step(st, *a, c, l, psi, 1)) return r;
            phi_post = lam_post = false;
        }
        if (phi_gen && npl > 0) {  // layer 0: one read of lam gives every gradient of the layer
            ProfScope ps(st, GV_PROF_FIRST_LAYER, (double)vb);
            if (gv_status r = check_hip(fused_layer0_grad(st->prec, lam, *a, c.plan, lam_post ? 1 : 0,
                                                          c.ch, c.tabs, part, c.w.grid, s),
                                        "first-layer gradients"))
                return r;
            break;
        }
        // does layer l-1 read phi from the state buffer?
        const bool next_phi_needed = l - 1 >= 1 && lmode == GV_GRAD_UNCOMPUTE;
        for (int p = 0; p < npl; ++p) {
            const bool last = p == npl - 1;
            BwdFlags fl;
            fl.phi_generate = phi_gen && p == 0;
            fl.diag_phi = p == 0 && phi_post;
            fl.diag_lam = p == 0 && lam_post;
            fl.store_phi = !last || next_phi_needed;
            fl.store_lam = !(l == 0 && last);
            const double bytes = (fl.phi_generate ? 1.0 : 2.0) * vb +
                                 ((fl.store_phi ? 1.0 : 0.0) + (fl.store_lam ? 1.0 : 0.0)) * vb;
            ProfScope ps(st, GV_PROF_BACKWARD_PASS, bytes);
            hipError_t e = fused_backward_pass(st->prec, p == 0 ? phi_src : psi, psi, lam, *a,
                                               c.plan, p, l, fl, c.ch, c.tabs, part, c.w.grid, s);
            if (gv_status r = check_hip(e, "backward pass")) return r;
        }
        // after undoing layer l's RY gates both vectors sit after layer l-1's
        // diagonal, except phi when the turnaround was layer l's only pass
        // (the state buffer then still holds the layer's input, before it)
        lam_post = true;
        phi_post = npl > 0;
    }
    st->has_psi = false;
    ProfScope ps(st, GV_PROF_OTHER, 0.0);
    return check_hip(reduce_rows(part, P, c.w.grid, mask, grad, s), "grad reduce");
}

gv_status gv_profile_enable(gv_state st, int32_t enable)
{
    if (!st) return set_error(GV_EINVAL, "state is NULL");
    st->profiling = enable != 0;
    return GV_OK;
}

gv_status gv_profile_reset(gv_state st)
{
    if (!st) return set_error(GV_EINVAL, "state is NULL");
    for (const gv_prof_record &r : st->records) {
        st->event_pool.push_back(r.start);
        st->event_pool.push_back(r.stop);
    }
    st->records.clear();
    return GV_OK;
}

gv_status gv_profile_read(gv_state st, int32_t kind, int64_t *launches, double *ms, double *bytes)
{
    if (!st) return set_error(GV_EINVAL, "state is NULL");
    if (kind < 0 || kind >= GV_PROF_KINDS) return set_error(GV_EINVAL, "kind %d", kind);
    int64_t cnt = 0;
    double tot = 0.0, b = 0.0;
    for (const gv_prof_record &r : st->records) {
        if (r.kind != kind) continue;
        if (gv_status e = check_hip(hipEventSynchronize(r.stop), "event sync")) return e;
        float t = 0.0f;
        if (gv_status e = check_hip(hipEventElapsedTime(&t, r.start, r.stop), "event time"))
            return e;
        ++cnt;
        tot += t;
        b += r.bytes;
    }
    if (launches) *launches = cnt;
    if (ms) *ms = tot;
    if (bytes) *bytes = b;
    return GV_OK;
}

size_t gv_sample_work_bytes(int32_t n)
{
    if (n < 1 || n > kMaxQubits) return 0;
    return sample_work_bytes(n);
}

static gv_status check_amps(int32_t n, gv_precision prec, const void *amps, void *work,
                            size_t work_bytes, size_t need)
{
    if (n < 1 || n > kMaxQubits) return set_error(GV_EINVAL, "n=%d outside 1..%d", n, kMaxQubits);
    if (prec != GV_C64 && prec != GV_C128) return set_error(GV_EINVAL, "precision %d", prec);
    if (!amps || !work) return set_error(GV_EINVAL, "NULL buffer");
    if (!aligned(amps) || !aligned(work))
        return set_error(GV_EINVAL, "buffers must be %zu-byte aligned", kAlign);
    if (work_bytes < need) return set_error(GV_ESIZE, "work buffer %zu bytes < %zu", work_bytes, need);
    return GV_OK;
}

gv_status gv_sample(int32_t n, gv_precision prec, const void *amps, const double *u,
                    int64_t shots, void *work, size_t work_bytes, uint64_t *out, void *stream)
{
    if (gv_status r = check_amps(n, prec, amps, work, work_bytes, sample_work_bytes(n))) return r;
    if (shots < 0) return set_error(GV_EINVAL, "shots < 0");
    if (shots > 0 && (!u || !out)) return set_error(GV_EINVAL, "NULL draws or output");
    return check_hip(sample_born(prec, amps, n, u, shots, work, out, (hipStream_t)stream),
                     "sample");
}

gv_status gv_argmax(int32_t n, gv_precision prec, const void *amps, void *work, size_t work_bytes,
                    uint64_t *index, double *prob, void *stream)
{
    if (gv_status r = check_amps(n, prec, amps, work, work_bytes, sample_work_bytes(n))) return r;
    if (!index) return set_error(GV_EINVAL, "index is NULL");
    return check_hip(argmax_prob(prec, amps, n, work, index, prob, (hipStream_t)stream), "argmax");
}

static size_t shots_work_bytes(const gv_pauli_s *h, gv_precision prec, int64_t shots)
{
    const size_t A = (size_t)1 << h->n;
    return sample_work_bytes(h->n) + align_up(A * amp_bytes(prec)) +
           align_up((size_t)shots * 8 + 8) + align_up((h->ox.size() + 1) * 8);
}

size_t gv_energy_shots_work_bytes(gv_pauli_sum h, gv_precision prec, int64_t shots)
{
    if (!h || shots < 0 || (prec != GV_C64 && prec != GV_C128)) return 0;
    return shots_work_bytes(h, prec, shots);
}

gv_status gv_pauli_sum_group(gv_pauli_sum h, int64_t g, uint64_t *xmask, uint64_t *ymask,
                             uint64_t *zmask, int64_t *nterms)
{
    if (!h) return set_error(GV_EINVAL, "pauli sum is NULL");
    if (g < 0 || g >= (int64_t)h->groups.size()) return set_error(GV_EINVAL, "group %lld", (long long)g);
    const QwcGroup &q = h->groups[(size_t)g];
    if (xmask) *xmask = q.xmask;
    if (ymask) *ymask = q.ymask;
    if (zmask) *zmask = q.zmask;
    if (nterms) *nterms = (int64_t)q.terms.size();
    return GV_OK;
}

gv_status gv_energy_shots(gv_pauli_sum h, int32_t n, gv_precision prec, const void *amps,
                          const double *u, int64_t shots, void *work, size_t work_bytes,
                          double *energy, void *stream)
{
    if (!h || !energy) return set_error(GV_EINVAL, "NULL argument");
    if (!h->prepared) return set_error(GV_ESTATE, "pauli sum not prepared");
    if (h->n != n) return set_error(GV_ESTATE, "pauli sum n=%d but n=%d", h->n, n);
    if (shots < 1 || !u) return set_error(GV_EINVAL, "need shots >= 1 and the draws");
    if (gv_status r = check_amps(n, prec, amps, work, work_bytes, shots_work_bytes(h, prec, shots)))
        return r;
    hipStream_t s = (hipStream_t)stream;
    const size_t A = (size_t)1 << n;
    char *w = (char *)work;
    void *swork = w;
    void *rot = w + sample_work_bytes(n);
    uint64_t *idx = (uint64_t *)((char *)rot + align_up(A * amp_bytes(prec)));
    double *vals = (double *)((char *)idx + align_up((size_t)shots * 8 + 8));
    double *dpart = vals + h->ox.size();
    // the Z-only terms (and the identity) from shots of psi: mean of D(b)
    if (gv_status r = check_hip(sample_born(prec, amps, n, u, shots, swork, idx, s), "sample"))
        return r;
    if (gv_status r = check_hip(diag_mean(idx, shots, h->diag, dpart, s), "diagonal mean")) return r;
    // every qubit-wise-commuting group from shots of psi in its eigenbasis
    int64_t t0 = 0;
    for (size_t g = 0; g < h->groups.size(); ++g) {
        const QwcGroup &q = h->groups[g];
        const int64_t m = (int64_t)q.terms.size();
        if (gv_status r = check_hip(basis_rotate(prec, amps, rot, n, q.xmask, q.ymask, s), "basis"))
            return r;
        if (gv_status r = check_hip(sample_born(prec, rot, n, u + (size_t)(g + 1) * shots, shots,
                                                swork, idx, s),
                                    "sample"))
            return r;
        if (gv_status r = check_hip(parity_means(idx, shots, h->dev_gmask + t0, h->dev_gcoef + t0,
                                                 m, vals + t0, s),
                                    "parity means"))
            return r;
        t0 += m;
    }
    return check_hip(sum_terms(vals, (int64_t)h->ox.size(), dpart, energy, s), "sum");
}

gv_status gv_stream_probe(int32_t kind, int32_t width, int32_t unroll, int32_t nontemporal,
                          int32_t grid, int32_t tile_shift, void *dst, const void *src0,
                          const void *src1, size_t bytes, void *stream)
{
    if (kind < GV_STREAM_READ || kind > GV_STREAM_TRIAD) return set_error(GV_EINVAL, "kind %d", kind);
    if (width != 4 && width != 8 && width != 16) return set_error(GV_EINVAL, "width %d", width);
    if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8 && unroll != 16)
        return set_error(GV_EINVAL, "unroll %d", unroll);
    if (grid < 0) return set_error(GV_EINVAL, "grid %d", grid);
    if (bytes == 0 || bytes % 65536 != 0)
        return set_error(GV_EINVAL, "bytes must be a positive multiple of 64 KiB");
    if (tile_shift != 0) {
        const size_t nvec = bytes / (size_t)width;
        if (tile_shift < 4 || tile_shift > 40 || (nvec & (nvec - 1)) != 0 ||
            nvec < ((size_t)1 << (tile_shift + 8)))
            return set_error(GV_EINVAL, "tile_shift %d needs a power-of-two count >= 2^%d",
                             tile_shift, tile_shift + 8);
    }
    if (!dst) return set_error(GV_EINVAL, "dst is NULL");
    if (kind != GV_STREAM_WRITE && !src0) return set_error(GV_EINVAL, "src0 is NULL");
    if (kind == GV_STREAM_TRIAD && !src1) return set_error(GV_EINVAL, "src1 is NULL");
    if (!aligned(dst) || (src0 && !aligned(src0)) || (src1 && !aligned(src1)))
        return set_error(GV_EINVAL, "buffers must be %zu-byte aligned", kAlign);
    return check_hip(stream_probe(kind, width, unroll, nontemporal != 0, dst, src0, src1, bytes,
                                  grid, tile_shift, (hipStream_t)stream),
                     "stream probe");
}

}  // extern "C"
