// gv_internal.hpp -- host-side structures and kernel launcher declarations.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gv.h"

namespace gv {

typedef uint64_t u64;

constexpr int kMaxQubits = 34;
constexpr int kPlainGrid = 1024;       // blocks of every reducing plain kernel
constexpr int kPlainBlock = 256;
constexpr int kMaxTileBits = 12;
constexpr int kMaxPasses = 8;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
inline size_t amp_bytes(gv_precision p) { return p == GV_C64 ? 8 : 16; }

// ---------------------------------------------------------------- Hamiltonian
struct QwcGroup {
    u64 xmask = 0, ymask = 0, zmask = 0;  // per-qubit basis letters of the group
    std::vector<int64_t> terms;            // indices into the off-diagonal arrays
};

// Off-diagonal terms that flip the same index bits x form a class: on the
// amplitude pair (i, i ^ x) their sum acts as one complex factor
// F(i ^ x) = sum_k c_k i^{ph_k} (-1)^{popcount((i ^ x) & z_k)}.  A class's
// terms with a real i^{ph} come first ([t0, ti)), the imaginary ones after
// ([ti, t1)).
struct OffClass {
    u64 x;          // flip mask
    uint32_t xu;    // the same mask in the tile-local bits of its cover pass
                    // (bits 0..15), plus kOffReFlat / kOffImFlat
    int32_t t0, t1; // its terms [t0, t1) in the term table
    int32_t ti;     // first term with an imaginary i^{ph}
};
// the class's real (imaginary) terms carry no register signs: their sum is
// the same for all of a thread's registers
constexpr uint32_t kOffReFlat = 1u << 16;
constexpr uint32_t kOffImFlat = 1u << 17;
// A term as the cover pass's kernel applies it (everything that depends
// only on the pass's tile layout is folded in on the host): the sign of
// term k at amplitude i ^ x is cf times (-1) to the parities of z & the
// tile base, tz & the thread id (the thread bits of the load layout) and
// the register bits (sig bit r for register r).
struct OffTerm {
    u64 z;
    double cf;      // c_k times -1 for ph & 2 and for the parity of x & z
    float cf32;     // the same in single precision
    uint32_t tz;    // z on the load layout's thread bits, as thread-id bits
    uint32_t sig;   // bits 0..15: register signs; kOffGroupEnd: last term of
                    // its group (same register signs and phase parity)
    uint32_t pad;
};
constexpr uint32_t kOffGroupEnd = 1u << 30;
constexpr int kOffPassTerms = 512;   // terms one cover pass stages in LDS
// A cover pass: a tile whose bits hold every flip bit of its classes.
struct OffPass {
    int8_t pos[kMaxTileBits];
    int c0, c1;     // classes [c0, c1)
};

}  // namespace gv

struct gv_pauli_s {
    int n = 0;
    // Z-only terms after merging (identity included as z = 0)
    std::vector<uint64_t> dz;
    std::vector<double> dc;
    // off-diagonal terms after merging
    std::vector<uint64_t> ox, oz;
    std::vector<double> oc;
    std::vector<gv::QwcGroup> groups;
    // off-diagonal classes in cover-pass order (built by prepare for a tile
    // size) and the terms no cover pass holds (applied one by one)
    std::vector<gv::OffClass> classes;
    std::vector<gv::OffTerm> class_terms;
    std::vector<gv::OffPass> off_passes;
    std::vector<int64_t> loose_terms;
    int cover_K = 0, cover_C = 0;
    gv::OffClass *dev_cls = nullptr;
    gv::OffTerm *dev_terms = nullptr;
    // the off-diagonal terms in qubit-wise-commuting group order: support
    // masks and coefficients (for the finite-shot estimate)
    uint64_t *dev_gmask = nullptr;
    double *dev_gcoef = nullptr;
    // device form (borrowed caller memory)
    void *dev = nullptr;
    size_t dev_bytes = 0;
    double *diag = nullptr;         // 2^n doubles
    bool prepared = false;
    uint64_t prep_gen = 0;          // bumped by every prepare (batches check it)
};

struct gv_prof_record {
    int kind;
    hipEvent_t start, stop;
    double bytes;
};

struct gv_state_s {
    int n = 0;
    gv_precision prec = GV_C64;
    gv_engine engine = GV_ENGINE_FUSED;
    void *amps = nullptr;
    size_t amps_bytes = 0;
    void *work = nullptr;
    size_t work_bytes = 0;
    hipStream_t stream = nullptr;
    bool has_psi = false;
    // per-kernel-class timing (gv_profile_*)
    bool profiling = false;
    std::vector<hipEvent_t> event_pool;
    std::vector<gv_prof_record> records;
};

namespace gv {

// ------------------------------------------------------------- error plumbing
gv_status set_error(gv_status s, const char *fmt, ...);
gv_status check_hip(hipError_t e, const char *what);

// Brackets the launches made during its lifetime with events when the state
// is profiling.
class ProfScope {
public:
    ProfScope(gv_state_s *st, int kind, double bytes);
    ~ProfScope();
private:
    gv_state_s *st_;
    int kind_;
    double bytes_;
    hipEvent_t start_ = nullptr;
};

// ------------------------------------------------------------------- planning
struct PassPlan {
    int8_t pos[kMaxTileBits];   // physical bit of tile bit j, ascending
    uint32_t active;            // tile bits whose qubit gets its gate in this pass
};

struct TilePlan {
    int K = 0;        // tile bits
    int C = 0;        // contiguous low bits kept in every pass (coalescing)
    int npass = 0;
    PassPlan pass[kMaxPasses];
};

bool make_tile_plan(int n, int K, int C, TilePlan *out);

// Diagonal tables of one layer over four chunks of the amplitude index (see
// gv_fused.hip): T0 | T1 | T2 | T3 and the CZ pairs that straddle chunks.
struct DiagTab {
    const void *tab;
    int b1, b2, b3;
    int off1, off2, off3;
    u64 m0, m1, m2;
    int npair;
    int pa[4], pb[4];        // 32-bit so the per-tile loop reads them with scalar loads
};

// Diagonal of one rotation layer (its RZ gates and CZ ladder) in the register
// layout of one assignment of a tile pass: the entry of index i is
// T[thread id] R[register] B1[tile id & (2^h1 - 1)] B2[tile id >> h1], times
// -1 for every CZ pair whose two qubits sit in different groups and are
// both set.  ka / kb give the register bit of such a pair's qubits (-1 when
// the qubit is a thread or tile-id bit).
constexpr int kMaxLPairs = 36;
struct LDiagTab {
    const void *tab;
    int offR, offB1, offB2;
    int h1;
    int npair;
    // 32-bit entries: the per-tile loop over the pairs then reads them with
    // scalar loads (byte entries go through vector loads and a wait each)
    int pa[kMaxLPairs], pb[kMaxLPairs];
    int ka[kMaxLPairs], kb[kMaxLPairs];
};

// What the table kernel needs to fill one LDiagTab: the qubit of every
// index bit of the four groups, in order (thread bits, register bits, B1
// bits, B2 bits).
struct LDiagBuild {
    int n, layer;
    int nt, nr, h1, h2;
    int8_t q[40];
    int cz;                 // 0 none, 1 linear, 2 circular
    int offR, offB1, offB2, total;
};

// What the table kernels need to fill one ansatz's tables.
struct TabArgs {
    int n;
    int rot_layers;
    int cz_layers;          // layers that carry the CZ ladder
    int cz;                 // 1 linear CZ, 2 circular CZ, 0 none
    int b[5];               // chunk bounds 0, b1, b2, b3, n
    int off[5];             // entry offsets of the chunks within a table set
    size_t stride;          // bytes per layer
};

// Diagonal-table chunks: chunk c covers index bits [b[c], b[c+1]); its
// entries start at off[c] (off[4] = entries per layer)
struct Chunks {
    int b[5];
    int off[5];
};
Chunks make_chunks(int n, int K, int LOGR);

// Work-buffer layout for gv_energy_grad / gv_energy.
struct WorkLayout {
    size_t lam = 0;          // adjoint vector
    size_t ckpt = 0;         // stored states: L-2 boundaries (CHECKPOINT) or pass outputs (STORE)
    size_t scratch = 0;      // one vector (CNOT gather)
    size_t ry_tab = 0;       // per parameter: RY shear coefficients, amplitude precision
    size_t dtab = 0;         // per rotation layer: diagonal tables in pass 0's load layout
    size_t gtab = 0;         // first-layer tables D_0 R_0|0..0>
    size_t g0tab = 0;        // first-layer tables R_0|0..0>
    size_t part = 0;         // gradient partials: P rows x grid columns
    size_t epart = 0;        // energy partials: 2 x grid
    size_t total = 0;
    int grid = 0;            // columns of the partial arrays
    size_t dtab_stride = 0;  // bytes per layer of diagonal tables (fwd + bwd)
    size_t ldtab = 0;        // per rotation layer: layout diagonal of a two-layer pass
    size_t ldtab_stride = 0;
};
gv_status work_layout(const gv_ansatz &a, gv_precision prec, gv_engine eng, gv_grad_mode mode,
                      WorkLayout *out);

int rot_layers(const gv_ansatz &a);
int64_t nparams(const gv_ansatz &a);

// CNOT networks: whether the entangler is one, and the (control, target)
// list of its layer `layer` in application order
inline bool ent_is_cnot(int ent) { return ent >= GV_ENT_CNOT_LINEAR && ent <= GV_ENT_CNOT_SCA; }
std::vector<std::pair<int, int>> cnot_network(int n, int ent, int layer);

// A CNOT network as a GF(2)-linear map of the amplitude index: col[q] is
// the image of the index with only bit q set; index i goes to the XOR of the
// columns of its set bits.
struct LinMap {
    u64 col[40];
    int n;
};
// the map of layer `layer`'s network (inverse = its inverse)
LinMap cnot_linmap(int n, int ent, int layer, bool inverse);

// ------------------------------------------------------------------ launchers
// All launchers enqueue on `s` and return the launch status.

// plain engine (one kernel per gate), prec selects float / double amplitudes
hipError_t plain_set_zero_state(int prec, void *psi, int n, hipStream_t s);
hipError_t plain_ry(int prec, void *psi, int n, int q, const double *theta, int64_t p, int inv,
                    hipStream_t s);
hipError_t plain_rz(int prec, void *psi, int n, int q, const double *theta, int64_t p, int inv,
                    hipStream_t s);
hipError_t plain_cz(int prec, void *psi, int n, int a, int b, hipStream_t s);
hipError_t plain_cnot(int prec, void *psi, int n, int ctl, int tgt, hipStream_t s);
// adjoint step of a rotation gate: gradient partial row + inverse gate on phi and lam
hipError_t plain_adj_ry(int prec, void *phi, void *lam, int n, int q, const double *theta,
                        int64_t p, double *part_row, hipStream_t s);
hipError_t plain_adj_rz(int prec, void *phi, void *lam, int n, int q, const double *theta,
                        int64_t p, double *part_row, hipStream_t s);

// Hamiltonian
hipError_t fill_zero_f64(double *d, u64 count, hipStream_t s);
hipError_t scatter_coeffs(double *h, const uint64_t *z, const double *c, int64_t m, hipStream_t s);
hipError_t fwht_inplace(double *d, int n, hipStream_t s);
// lam = D psi (lam may be null), energy partials (re, im) = sum conj(psi) D psi
hipError_t energy_diag(int prec, const void *psi, const double *diag, void *lam, int n,
                       double *epart, int grid, hipStream_t s);
// lam += c P psi for every off-diagonal term, energy partials accumulated
hipError_t energy_offdiag_terms(int prec, const void *psi, void *lam, int n, int64_t m,
                                const uint64_t *ox, const uint64_t *oz, const double *oc,
                                double *epart, int grid, hipStream_t s);
// out[r] = sum_c part[r*cols + c] (masked rows -> 0), optionally scaled
hipError_t reduce_rows(const double *part, int64_t rows, int cols, const uint8_t *mask,
                       double *out, hipStream_t s);
// energy_dev[0..1] = column sums of the 2 x grid energy partials
hipError_t reduce_energy(const double *epart, int grid, double *energy, hipStream_t s);

hipError_t copy_vector(void *dst, const void *src, size_t bytes, hipStream_t s);

// measurement (gv_sample.hip): Born-rule samples, the most probable index,
// the basis change of a qubit-wise-commuting group, shot averages
size_t sample_work_bytes(int n);
hipError_t sample_born(int prec, const void *psi, int n, const double *u, int64_t shots,
                       void *work, uint64_t *out, hipStream_t s);
hipError_t argmax_prob(int prec, const void *psi, int n, void *work, uint64_t *idx, double *p,
                       hipStream_t s);
hipError_t basis_rotate(int prec, const void *src, void *dst, int n, u64 xmask, u64 ymask,
                        hipStream_t s);
hipError_t parity_means(const uint64_t *b, int64_t shots, const uint64_t *mask, const double *c,
                        int64_t m, double *term_out, hipStream_t s);
hipError_t diag_mean(const uint64_t *b, int64_t shots, const double *diag, double *out,
                     hipStream_t s);
hipError_t sum_terms(const double *term, int64_t m, const double *diag_part, double *out,
                     hipStream_t s);

// streaming-bandwidth probe (gv_stream.hip): kind is a gv_stream_kind
enum { STREAM_READ = 0, STREAM_WRITE = 1, STREAM_COPY = 2, STREAM_RMW = 3, STREAM_TRIAD = 4 };
hipError_t stream_probe(int kind, int width, int unroll, int nt, void *dst, const void *s0,
                        const void *s1, size_t bytes, int grid, int shift, hipStream_t s);

// one cover pass of off-diagonal classes: lam += (sum of the classes) psi
// (lam may be NULL); energy partials epart[b], epart[estride + b] += the
// pass's contribution to <psi|H|psi>
hipError_t offdiag_pass(int prec, const void *psi, void *lam, int n, int K, const OffPass &op,
                        const OffClass *cls, const OffTerm *terms, double *epart, int estride,
                        hipStream_t s);

// fused engine
struct FusedTables {
    const void *ry;      // [P]: RY shear coefficients in the amplitude precision
    void *dtab;          // per rotation layer diagonal tables (RZ phases, CZ signs)
    size_t dtab_stride;
    void *gtab;          // D_0 R_0|0...0> tables
    void *g0tab;         // R_0|0...0> tables
    void *ldtab;         // per rotation layer: its diagonal in a two-layer pass's layout
    size_t ldtab_stride;
};
struct BwdFlags {
    int phi_generate = 0;   // phi = R_0|0...0> from tables instead of a load (pass 0)
    int diag_phi = 0;       // undo the layer's diagonal on phi as it loads (pass 0)
    int diag_lam = 0;       // undo the layer's diagonal on lam as it loads (pass 0)
    int store_phi = 1, store_lam = 1;
    // phi is not written back (store_phi = 0): take every partial at the pass's
    // end point and rotate lam alone
    int grad_first = 0;
};
// forward pass input modes
enum { FWD_LOAD = 0, FWD_LOAD_DIAG = 1, FWD_GENERATE = 2 };
hipError_t fused_build_tables(int prec, const gv_ansatz &a, const Chunks &ch, const double *theta,
                              const FusedTables &t, hipStream_t s);
hipError_t fused_init_state(int prec, void *psi, const gv_ansatz &a, const Chunks &ch,
                            const FusedTables &t, hipStream_t s);
// src (NULL: psi) is where the pass reads its input; it writes psi
hipError_t fused_forward_pass(int prec, void *psi, const gv_ansatz &a, const TilePlan &plan,
                              int pass, int layer, int in_mode, const Chunks &ch,
                              const FusedTables &t, hipStream_t s,
                              const void *src = nullptr);
// ld_load (may be NULL): both vectors first lose `layer`'s diagonal in the
// pass's load layout (the second half of a two-layer pass's reverse)
hipError_t fused_backward_pass(int prec, const void *phi_in, void *phi, void *lam,
                               const gv_ansatz &a, const TilePlan &plan, int pass, int layer,
                               const BwdFlags &fl, const Chunks &ch, const FusedTables &t,
                               double *part, int grid, hipStream_t s,
                               const LDiagTab *ld_load = nullptr);
// Gradients of rotation layer 0 from lam alone (one read), lam before
// (diag_lam = 0) or after (1) the layer's diagonal; qubits of layer 0 only.
hipError_t fused_layer0_grad(int prec, const void *lam, const gv_ansatz &an, const TilePlan &plan,
                             int diag_lam, const Chunks &ch, const FusedTables &t, double *part,
                             int grid, hipStream_t s);
// Two-layer passes (the last pass of `layer` and the first of layer + 1 on
// the same tile qubits).  make_ldiag fills `tab` (device, ldiag_entries
// entries of the precision's complex type) for layer's diagonal in the last
// (last = 1) or the load (last = 0) assignment of plan pass `pass`; the
// table kernel runs on `s`.
int ldiag_entries(int n, int K, int LOGR);
hipError_t make_ldiag(int prec, const gv_ansatz &an, const TilePlan &plan, int pass, int last,
                      int layer, const double *theta, void *tab, LDiagTab *out, hipStream_t s);
hipError_t fused_forward2_pass(int prec, void *psi, const gv_ansatz &an, const TilePlan &plan,
                               int pass, int layer, int in_mode, const Chunks &ch,
                               const FusedTables &t, const LDiagTab &ld, hipStream_t s,
                               const void *src = nullptr);
// Reverse of a two-layer pass (layers `layer` and layer + 1 on plan pass
// `pass`) in one sweep from the state the pass wrote (phi_src) and lam at
// the same point: lam is rewritten in place, the partials of both layers
// written, and with store_phi the state before the pass goes to phi (which
// may be phi_src).
hipError_t fused_backward2_pass(int prec, const void *phi_src, void *phi, void *lam,
                                const gv_ansatz &an, const TilePlan &plan, int pass, int layer,
                                int store_phi, const LDiagTab &ld_last, const FusedTables &t,
                                double *part, int grid, hipStream_t s);
hipError_t fused_turnaround(int prec, const void *psi, void *lam, const double *hdiag,
                            const gv_ansatz &a, const TilePlan &plan, int pass, int layer,
                            int in_mode, const Chunks &ch, const FusedTables &t, double *part,
                            double *epart, int grid, hipStream_t s);
hipError_t fused_diag_apply(int prec, void *v0, void *v1, const gv_ansatz &a, const Chunks &ch,
                            const FusedTables &t, int layer, int conj, hipStream_t s);
// CNOT ladder gather; with t != NULL the layer diagonal is fused in
hipError_t cnot_ladder_gather(int prec, const void *src, void *dst, const gv_ansatz &a,
                              const Chunks &ch, const FusedTables *t, int layer, int inverse,
                              hipStream_t s);
int fused_grid(int prec, const TilePlan &plan, int n);

// ---------------------------------------------------------------- batching
// One tile pass of a batch instance (pass 0 of the plan, or a later one).
struct BatchPass {
    int8_t pos[kMaxTileBits];
    uint32_t active;
    int nruns;
    uint32_t run[kMaxTileBits + 1];   // source bit | width << 8 | destination bit << 16
};
struct BatchOffPass {
    BatchPass tile;
    int c0, c1;
};
// Everything the persistent batch kernel needs about one instance.
struct BatchInst {
    int n, layers, rot, np, noff, zonly;
    int cz;                   // 1 linear CZ, 2 circular CZ, 0 no entangler
    u64 ntiles;
    u64 qmask;                // gradient written for these qubits' parameters
    const double *theta;
    double *energy, *grad;
    const double *hdiag;
    const OffClass *cls;
    const OffTerm *terms;
    const BatchOffPass *offp;
    void *psi, *lam;
    void *ry;            // [P] RY shear coefficients, amplitude precision
    char *dtab;
    size_t dtab_stride;
    void *gtab, *g0tab;
    DiagTab dt_cz, dt_plain;  // layer tables (tab = layer 0's; layer l adds l * stride)
    DiagTab gt, g0;           // D_0 R_0|0..0> and R_0|0..0>
    TabArgs ta;
    BatchPass pass[kMaxPasses];
};
// tables of every instance (one launch), then the queue counter reset and the
// persistent kernel; grid = persistent blocks
hipError_t batch_tables(int prec, const BatchInst *dev_insts, int count, hipStream_t s);
// The batch's two queue counters (persistent kernel, LDS-resident kernel)
// reset to zero, then one persistent kernel over order[0 .. count): the
// LDS-resident one (complex64 instances of at most kBatchLdsAmps
// amplitudes, their vectors in the block's LDS) or the plain one.
constexpr int kBatchLdsAmps = 4096;
hipError_t batch_zero(unsigned *counter, hipStream_t s);
hipError_t batch_run(int prec, const BatchInst *dev_insts, const int *order, int count,
                     unsigned *counter, int grid, bool lds_resident, hipStream_t s);
// host helpers shared with gv_batch.cpp
DiagTab make_diagtab(const gv_ansatz &an, const Chunks &ch, const void *tab, bool cz_layer);
TabArgs make_tab_args(const gv_ansatz &an, const Chunks &ch, size_t stride);
void pass_runs(const int8_t *pos, int K, int n, BatchPass *out);

}  // namespace gv
