/*
 * gv.h -- C ABI of the MI355X (gfx950) state-vector energy / gradient engine
 * for Graph-VQE's hot path.
 *
 * What the library computes (Graph-VQE, Sec. IV):
 *   psi(theta) = U(theta)|0...0>  -- hardware-efficient ansatz: per layer RY on
 *                                    every qubit, RZ on every qubit, then an
 *                                    entangler ladder (Sec. IV-B, Eq. 7, Eq. 8)
 *   H = sum_k c_k P_k             -- real coefficients, Pauli strings (Eq. 6)
 *   E(theta) = <psi|H|psi>        -- the VQE objective (Eq. 4)
 *   dE/dtheta                     -- exact gradient (Eq. 13 gives one way to get
 *                                    it; this library uses a reverse sweep)
 *   restricted gradient           -- only the parameters of a qubit block
 *                                    (Eq. 11 and the block gradient of Sec. IV-D)
 *
 * Conventions:
 *   - qubit q is bit q of an amplitude index (little endian);
 *   - amplitudes are interleaved complex (re, im): float pairs for GV_C64,
 *     double pairs for GV_C128, 2^n of them, index-ordered;
 *   - parameters are doubles, index l*2n + g*n + q for layer l, gate g
 *     (0 = RY, 1 = RZ) and qubit q; P = 2 n (layers + final_rotation);
 *   - RY(t) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]],
 *     RZ(t) = diag(exp(-i t/2), exp(i t/2))  (Eq. 7);
 *   - a Pauli string is the pair of bit masks (x, z) with
 *     P(x, z) = i^{popcount(x & z)} X^x Z^z, so Y on qubit q is x_q = z_q = 1.
 *
 * Memory ownership: every device buffer (state, workspace, Hamiltonian
 * buffer, parameters, outputs) belongs to the caller and is borrowed for the
 * lifetime of the handle that was given it.  Compute calls allocate no device
 * memory.  Host-side handles are owned by the library and released by the
 * matching *_destroy call.
 *
 * Streams: compute calls enqueue work on the state's stream (a hipStream_t
 * passed as void*, NULL = the default stream) and return without waiting.
 * Outputs are valid once that stream reaches the point of the call.
 *
 * Errors: every call returns a gv_status.  Arguments are validated before any
 * work is enqueued; on a non-OK status nothing has been enqueued and no output
 * is written.  GV_EHIP means the HIP runtime reported an error while
 * enqueueing; state contents are then undefined but the handle stays valid.
 * gv_last_error() returns a thread-local description of the last failure.
 * Handles are not thread-safe; distinct handles may be used from distinct
 * threads.
 */
#ifndef GV_H
#define GV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GV_OK = 0,
    GV_EINVAL = 1,        /* bad argument (null pointer, range, mask bit >= n, non-finite) */
    GV_ESIZE = 2,         /* a caller buffer is smaller than required */
    GV_EUNSUPPORTED = 3,  /* valid request this build does not handle */
    GV_ESTATE = 4,        /* call order (e.g. energy before any ansatz) or handle mismatch */
    GV_EHIP = 5           /* HIP runtime error while enqueueing */
} gv_status;

typedef enum { GV_C64 = 0, GV_C128 = 1 } gv_precision;

/* Entangler of each repeated layer (Sec. IV-B lists linear, circular and
 * full patterns; Sec. V-A also runs reverse-linear, pairwise and
 * shifted-circular-alternating ones).  CNOT networks apply their gates in
 * the order listed. */
typedef enum {
    GV_ENT_NONE = 0,
    GV_ENT_CZ_LINEAR = 1,     /* CZ(q, q+1), q = 0..n-2 (all commute) */
    GV_ENT_CZ_CIRCULAR = 2,   /* linear plus CZ(n-1, 0) when n > 2 */
    GV_ENT_CNOT_LINEAR = 3,   /* CNOT(q -> q+1) applied for q = 0, 1, ..., n-2 */
    GV_ENT_CNOT_CIRCULAR = 4, /* CNOT(n-1 -> 0) first (n > 2), then the linear ladder */
    GV_ENT_CNOT_FULL = 5,     /* CNOT(i -> j) for every i < j, i the outer loop */
    GV_ENT_CNOT_REVERSE_LINEAR = 6, /* CNOT(q -> q+1) for q = n-2 down to 0 */
    GV_ENT_CNOT_PAIRWISE = 7, /* CNOT(q -> q+1) for even q, then for odd q */
    GV_ENT_CNOT_SCA = 8       /* layer l: the circular list (n-1 -> 0), (0 -> 1), ...,
                                 (n-2 -> n-1) rotated right by l mod n, control and
                                 target exchanged in odd layers (n <= 2: linear) */
} gv_entangler;

/* How the reverse sweep recovers the forward states at large n. */
typedef enum {
    GV_GRAD_UNCOMPUTE = 0,    /* undo gates on the final state; no extra memory */
    GV_GRAD_CHECKPOINT = 1,   /* store the state at the layers-2 inner layer boundaries
                                 (the first layer is regenerated) */
    GV_GRAD_RECOMPUTE = 2,    /* re-run the forward from |0> to each of those boundaries */
    GV_GRAD_STORE = 3         /* keep the state after every fused tile pass (each pass
                                 writes its own buffer); the reverse sweep reads them back
                                 and writes only lambda.  Most memory, least traffic.
                                 Ansatze with a CNOT ladder store the layer boundaries
                                 only, as CHECKPOINT does. */
} gv_grad_mode;

/* Kernel family.  FUSED: tile passes that apply many gates per HBM sweep.
 * PLAIN: one kernel per gate (the straightforward reference GPU path). */
typedef enum { GV_ENGINE_FUSED = 0, GV_ENGINE_PLAIN = 1 } gv_engine;

typedef struct {
    int32_t n;               /* qubits, 1..34 */
    int32_t layers;          /* repeated [RY all, RZ all, entangler] layers, >= 0 */
    int32_t ent;             /* gv_entangler */
    int32_t final_rotation;  /* 1: one more RY/RZ layer without entangler
                                (EfficientSU2 of Eq. 8: P = 2 n (layers + 1)) */
} gv_ansatz;

typedef struct gv_state_s *gv_state;
typedef struct gv_pauli_s *gv_pauli_sum;

/* Library version string. */
const char *gv_version(void);

/* Thread-local text of the last non-OK status ("" if none). */
const char *gv_last_error(void);

/* Test hook for the error paths: after `after` more successful HIP status
 * checks (process-wide), the next one reports GV_EHIP ("injected HIP
 * error") as if the runtime had failed, then the hook turns itself off;
 * after < 0 turns it off.  The work already enqueued runs normally; the
 * failing call returns at that point like on a real HIP error. */
gv_status gv_debug_inject_hip_error(int64_t after);

/* Number of ansatz parameters, 2 n (layers + final_rotation), or -1 if the
 * ansatz is invalid. */
int64_t gv_num_params(const gv_ansatz *ansatz);

/* Buffer sizes for a state that will run `ansatz` (Sec. IV-B, Eq. 8) in
 * `prec` with gradient mode `mode` on `engine`: state_bytes = 2^n
 * amplitudes; work_bytes = the workspace gv_energy_grad needs (adjoint
 * vector, stored states of the mode, tables, reduction partials);
 * diag_bytes = the FP64 diagonal of a Hamiltonian's Z-only part on n qubits
 * (2^n doubles; gv_pauli_sum_device_bytes adds the off-diagonal tables of a
 * given Hamiltonian).  Any output pointer may be NULL. */
gv_status gv_query_sizes(const gv_ansatz *ansatz, gv_precision prec, gv_engine engine,
                         gv_grad_mode mode, size_t *state_bytes, size_t *work_bytes,
                         size_t *diag_bytes);

/* Create a state of n qubits (the register the ansatz of Sec. IV-B acts on)
 * over caller-owned device memory.
 *   amps_dev / amps_bytes: >= 2^n amplitudes of `prec`, 256-byte aligned;
 *   work_dev / work_bytes: workspace (may be NULL/0 when only gv_apply_ansatz
 *                          and gv_energy are used with the PLAIN engine);
 *   stream: hipStream_t (as void*), NULL for the default stream.
 * The state starts "empty": gv_energy before gv_apply_ansatz is GV_ESTATE. */
gv_status gv_state_create(int32_t n, gv_precision prec, gv_engine engine,
                          void *amps_dev, size_t amps_bytes,
                          void *work_dev, size_t work_bytes,
                          void *stream, gv_state *out);
gv_status gv_state_destroy(gv_state st);
gv_status gv_state_set_stream(gv_state st, void *stream);

/* psi <- U(theta)|0...0> (Eq. 7, Eq. 8).  params_dev: device doubles, P of
 * them.  ansatz->n must equal the state's n. */
gv_status gv_apply_ansatz(gv_state st, const double *params_dev, const gv_ansatz *ansatz);

/* Build a Pauli sum from host arrays (copied; Eq. 6).  Terms with the same
 * (x, z) are merged by adding coefficients; zero coefficients are dropped.
 * Mask bits >= n and non-finite coefficients are GV_EINVAL. */
gv_status gv_pauli_sum_create(int32_t n, int64_t m, const uint64_t *x, const uint64_t *z,
                              const double *c, gv_pauli_sum *out);
gv_status gv_pauli_sum_destroy(gv_pauli_sum h);

/* Counts after merging: diagonal (Z-only, incl. identity) terms, off-diagonal
 * terms, qubit-wise-commuting groups of the off-diagonal terms.  Any output
 * pointer may be NULL. */
gv_status gv_pauli_sum_info(gv_pauli_sum h, int64_t *n_diag, int64_t *n_offdiag,
                            int64_t *n_groups);

/* How the off-diagonal terms (Eq. 6) would be applied to a state of n_state
 * qubits in `prec` on `engine` (host-side planning only, no device work):
 * the number of cover passes (each one sweep over psi and lambda), the most
 * terms one pass holds, and the terms applied one by one (flip masks too wide
 * for a tile; every term on the plain engine).  Any output pointer may be
 * NULL. */
gv_status gv_pauli_sum_plan(gv_pauli_sum h, int32_t n_state, gv_precision prec, gv_engine engine,
                            int64_t *passes, int64_t *max_pass_terms, int64_t *loose_terms);

/* Device bytes the Hamiltonian needs: the FP64 diagonal of its Z-only part
 * (2^n doubles) followed by the off-diagonal term tables. */
gv_status gv_pauli_sum_device_bytes(gv_pauli_sum h, size_t *bytes);

/* Build the device form of H (Eq. 6) into caller memory `dev` (>= device_bytes,
 * 256-byte aligned): the diagonal D_i = sum_{k: x_k = 0} c_k (-1)^{|i & z_k|}
 * by an in-place fast Walsh-Hadamard transform, and the off-diagonal terms
 * grouped by flip mask into the tile passes of the state's engine and
 * precision (states of another precision or engine then get GV_ESTATE).
 * Runs on the state's stream and waits for it (a setup call).  `dev` is
 * borrowed until gv_pauli_sum_destroy or the next prepare. */
gv_status gv_pauli_sum_prepare(gv_pauli_sum h, gv_state st, void *dev, size_t bytes);

/* The same without a state: build the device form for states of precision
 * `prec` on `engine` (and for batches), on `stream`. */
gv_status gv_pauli_sum_prepare_for(gv_pauli_sum h, gv_precision prec, gv_engine engine,
                                   void *stream, void *dev, size_t bytes);

/* E = <psi|H|psi> of the state's current psi (Eq. 4).  energy_dev: 2 device doubles
 * (real part, imaginary part; the latter is rounding noise for real c_k).
 * Needs work memory for reduction partials (FUSED: always; PLAIN: >= 1 MiB). */
gv_status gv_energy(gv_state st, gv_pauli_sum h, double *energy_dev);

/* Energy and gradient at params_dev (Eq. 4; gradient as Eq. 13 defines it).
 *   grad_mask_dev: NULL = every parameter; else P device bytes, nonzero where
 *                  the gradient is wanted (restricted update of Eq. 11); other
 *                  entries of grad_dev are written as 0;
 *   mode: how forward states are recovered in the reverse sweep;
 *   energy_dev: 2 device doubles (re, im); grad_dev: P device doubles.
 * The reverse sweep uses the state's amplitude buffer as scratch: afterwards
 * it does not hold psi(theta) (gv_apply_ansatz recomputes it). */
gv_status gv_energy_grad(gv_state st, gv_pauli_sum h, const double *params_dev,
                         const gv_ansatz *ansatz, const uint8_t *grad_mask_dev,
                         gv_grad_mode mode, double *energy_dev, double *grad_dev);

/* ------------------------------------------------------------------------
 * Batches: Graph-VQE optimises qubit blocks concurrently, each block's
 * restricted cost being the full energy with only that block's parameters
 * free (Sec. IV-D, Eq. 11), and computes gradients only for a block's
 * parameters.  A batch runs many such independent evaluations -- each with
 * its own ansatz size, angles, Hamiltonian and qubit block -- in one
 * persistent kernel: each block of the grid takes whole instances from an
 * atomic queue (largest first by default) and runs their forward sweep,
 * energy and reverse sweep.  Instances with n >= split_n instead run as
 * whole-GPU tile passes (the path of gv_energy_grad, store mode) on
 * side streams forked from and joined back to the batch's stream, alongside
 * the persistent kernel, so one large instance is not left to a single
 * compute unit.  Grid, order and split come from gv_batch_tuning (an
 * autotuner picks them; see paper_2607_02749_amd/autotune.py).
 * Limits: 12 <= n <= 30; CZ or no entangler; every Hamiltonian prepared with
 * gv_pauli_sum_prepare_for(h, prec, GV_ENGINE_FUSED, ...).
 */
/* One instance: an ansatz, its angles and its Hamiltonian (the Hamiltonian's
 * FP64 diagonal and off-diagonal tables live in the device buffer it was
 * prepared into).  The block it updates is its gv_cluster. */
typedef struct {
    gv_ansatz ansatz;
    const double *params_dev;  /* P = 2 n (layers + final_rotation) device doubles */
    gv_pauli_sum h;            /* prepared for the batch precision, fused engine */
} gv_instance;

/* Restricted update of Eq. 11: the gradient is computed for the RY and RZ
 * angles of these qubits in every layer (2 |B| (layers + final_rotation)
 * entries) and written as 0 elsewhere.  An empty block (qubit_mask = 0)
 * asks for the energy alone: no reverse sweep runs and the gradient is all
 * zeros (the shifted evaluations of the parameter-shift rule, Eq. 13). */
typedef struct {
    uint64_t qubit_mask;
} gv_cluster;

typedef struct {
    int32_t blocks_per_cu;     /* persistent blocks per compute unit, 1..8 (default 2) */
    int32_t order;             /* 0: largest instance first (default), 1: input order */
    int32_t split_n;           /* n from which instances run as whole-GPU passes;
                                  0: default (17), > 30: never */
    int32_t lds_n;             /* instances with n <= lds_n keep psi and lam in the
                                  workgroup's LDS for the whole evaluation (own
                                  persistent kernel, one block per compute unit):
                                  complex64 only, at most 12 (the two 32 KB vectors
                                  and the 34 KB tile exchange buffer fill most of
                                  the 160 KB); 0: default (12), -1: never */
} gv_batch_tuning;

typedef struct gv_batch_s *gv_batch;

/* Workspace bytes for a batch (per-instance states, tables, descriptors,
 * and the work regions of the whole-GPU instances, which depend on
 * tuning->split_n; tuning may be NULL for the defaults). */
gv_status gv_batch_query(int32_t count, const gv_instance *inst, gv_precision prec,
                         const gv_batch_tuning *tuning, size_t *work_bytes);
/* Plan a batch over caller memory `work_dev` (256-byte aligned, >= query)
 * (Sec. IV-D, Eq. 11).
 *   clusters: count entries, or NULL for unrestricted gradients;
 *   energies_dev: out, 2 * count device doubles, (re, im) of instance i at 2 i;
 *   grads_dev: out, sum_i P_i device doubles, instance i's gradient at offset
 *              sum_{j<i} P_j (0 outside its cluster).
 * tuning may be NULL.  use_graph != 0 records the launches once as a HIP
 * graph that gv_batch_run replays; between runs the caller may rewrite the
 * parameter arrays in place.  Waits for the stream (it stages the instance
 * records into work_dev).  The instance and cluster arrays are copied; the
 * device pointers, the Hamiltonian handles and their prepared device buffers
 * must stay valid -- and the Hamiltonians must not be prepared again -- for
 * the batch's lifetime (gv_batch_run checks the last point and returns
 * GV_ESTATE). */
gv_status gv_batch_create(int32_t count, const gv_instance *inst, const gv_cluster *clusters,
                          gv_precision prec, const gv_batch_tuning *tuning, void *work_dev,
                          size_t work_bytes, void *stream, int32_t use_graph,
                          double *energies_dev, double *grads_dev, gv_batch *out);
/* Enqueue one evaluation of every instance on the batch's stream. */
gv_status gv_batch_run(gv_batch b);
gv_status gv_batch_destroy(gv_batch b);
/* One evaluation of every instance with the default tuning and no graph
 * (Sec. IV-D, Eq. 11; arguments as gv_batch_create): waits for work already
 * on `stream` while it stages the instance records, then enqueues the
 * evaluation on `stream` and returns.  The whole-GPU instances run one after
 * another on `stream` (no side streams), so nothing the call creates outlives
 * it. */
gv_status gv_batch_energy_grad(int32_t count, const gv_instance *inst, const gv_cluster *clusters,
                               gv_precision prec, void *work_dev, size_t work_bytes, void *stream,
                               double *energies_dev, double *grads_dev);

/* ------------------------------------------------------------------------
 * Per-kernel-class timing.  While enabled, every launch of the state's
 * compute calls is bracketed by HIP events recorded on the state's stream,
 * and the algorithmic bytes of the launch (the reads and writes the step
 * must make, e.g. read + write of psi and lambda for a reverse pass) are
 * recorded with it.  Events are host-side objects created on demand; no
 * device memory is allocated.  gv_profile_read waits for the recorded events.
 */
typedef enum {
    GV_PROF_FORWARD_PASS = 0,   /* fused ansatz tile pass (one layer) */
    GV_PROF_BACKWARD_PASS = 1,  /* reverse tile pass rotating phi and lambda */
    GV_PROF_ENERGY = 2,         /* diagonal energy and lambda = H psi */
    GV_PROF_INIT = 3,           /* first-layer product state */
    GV_PROF_PLAIN_GATE = 4,     /* plain engine gate or reverse step */
    GV_PROF_OTHER = 5,          /* tables, reductions, copies, gathers */
    GV_PROF_OFFDIAG = 6,        /* off-diagonal terms: lambda += H_off psi */
    GV_PROF_FIRST_LAYER = 7,    /* first rotation layer's gradients from lambda */
    GV_PROF_FORWARD_PASS2 = 8,  /* two-layer forward tile pass */
    GV_PROF_BACKWARD_LD = 9,    /* reverse pass undoing a layer diagonal on load */
    GV_PROF_BACKWARD_GF = 10,   /* reverse pass rotating lambda alone (phi not kept) */
    GV_PROF_BACKWARD_GF_LD = 11,/* the same, undoing a layer diagonal on load */
    GV_PROF_TURNAROUND = 12,    /* last forward pass + energy + first reverse pass */
    GV_PROF_BACKWARD2 = 13,     /* reverse of a two-layer pass in one sweep (STORE mode) */
    GV_PROF_KINDS = 14
} gv_prof_kind;

gv_status gv_profile_enable(gv_state st, int32_t enable);
gv_status gv_profile_reset(gv_state st);
/* launches, total milliseconds and total algorithmic bytes of one kind since
 * the last reset.  Any output pointer may be NULL. */
gv_status gv_profile_read(gv_state st, int32_t kind, int64_t *launches, double *ms,
                          double *bytes);

/* ------------------------------------------------------------------------
 * Measurement (Sec. IV-F, Sec. V-A).  The paper estimates energies from 8192
 * shots and decodes the most probable bitstring; these calls do both on a
 * state vector in device memory (amps_dev: 2^n amplitudes of `prec`, e.g. a
 * state's buffer after gv_apply_ansatz), enqueued on `stream`.  Random
 * numbers are the caller's: u_dev holds uniform draws in [0, 1).
 *
 * gv_sample: shots indices drawn from the Born distribution |psi_i|^2 by
 *   inverse-CDF sampling (out_dev[j] = the i with cdf(i-1) <= u_j * total <
 *   cdf(i), cumulative sums in FP64).  work_dev: gv_sample_work_bytes(n).
 * gv_argmax: the index of the largest |psi_i|^2 (ties: the smallest index)
 *   and that probability (prob_dev may be NULL).  Same work size.
 * gv_energy_shots: the finite-shot estimate of <psi|H|psi> for a prepared
 *   Hamiltonian: the Z-only part as the mean of the FP64 diagonal D(b) over
 *   `shots` samples of psi (draws u_dev[0 .. shots)), each qubit-wise-
 *   commuting group g (gv_pauli_sum_group order) from `shots` samples of psi
 *   in the group's eigenbasis (H on X qubits, H S^dagger on Y qubits; draws
 *   u_dev[(g+1) shots ..)), term k contributing c_k times the mean of
 *   (-1)^{popcount(b & support_k)}.  u_dev: (1 + groups) * shots doubles;
 *   energy_dev: 2 doubles (estimate, 0); work_dev:
 *   gv_energy_shots_work_bytes(h, prec, shots). */
size_t gv_sample_work_bytes(int32_t n);
gv_status gv_sample(int32_t n, gv_precision prec, const void *amps_dev, const double *u_dev,
                    int64_t shots, void *work_dev, size_t work_bytes, uint64_t *out_dev,
                    void *stream);
gv_status gv_argmax(int32_t n, gv_precision prec, const void *amps_dev, void *work_dev,
                    size_t work_bytes, uint64_t *index_dev, double *prob_dev, void *stream);
/* Group g of the Hamiltonian's qubit-wise-commuting grouping of its
 * off-diagonal terms (greedy first fit over the merged terms in (x, z)
 * order): the qubits carrying X, Y and Z in the group, and its term count. */
gv_status gv_pauli_sum_group(gv_pauli_sum h, int64_t g, uint64_t *xmask, uint64_t *ymask,
                             uint64_t *zmask, int64_t *nterms);
size_t gv_energy_shots_work_bytes(gv_pauli_sum h, gv_precision prec, int64_t shots);
gv_status gv_energy_shots(gv_pauli_sum h, int32_t n, gv_precision prec, const void *amps_dev,
                          const double *u_dev, int64_t shots, void *work_dev, size_t work_bytes,
                          double *energy_dev, void *stream);

/* ------------------------------------------------------------------------
 * Streaming-bandwidth probe (measurement only; no part of the method).
 * Runs one perfectly coalesced streaming kernel over `bytes` bytes so the
 * state-vector passes can be compared with what the device's HBM delivers to
 * plain streams:
 *   kind GV_STREAM_READ   reads src0;
 *        GV_STREAM_WRITE  writes dst;
 *        GV_STREAM_COPY   dst = src0;
 *        GV_STREAM_RMW    dst = src0 + dst (two streams read, one written back,
 *                         the pattern of a reverse pass over phi and lambda);
 *        GV_STREAM_TRIAD  dst = src0 + src1.
 *   width: bytes per lane per access, 4, 8 or 16; unroll: accesses in flight
 *   per lane, 1, 2, 4 or 8; nontemporal != 0 uses non-temporal loads/stores;
 *   grid: blocks of 256 lanes, 0 = one block per 256 * unroll accesses;
 *   tile_shift: 0 = linear order; s in 4..40 = the layout of a state-vector
 *   tile pass: bits 0..3 of an access's index stay, bits 4..11 move to bits
 *   s..s+7 and the other bits fill the rest in order (runs of 16 accesses lie
 *   2^s accesses apart); then bytes / width must be a power of two >= 2^(s+8).
 * unroll may also be 16.  bytes must be a positive multiple of 64 KiB; every
 * buffer the kind uses must hold `bytes` device bytes (READ writes at most
 * 4 KiB of dst, never in practice), 256-byte aligned.  Enqueues on `stream`
 * and returns. */
typedef enum {
    GV_STREAM_READ = 0, GV_STREAM_WRITE = 1, GV_STREAM_COPY = 2, GV_STREAM_RMW = 3,
    GV_STREAM_TRIAD = 4
} gv_stream_kind;
gv_status gv_stream_probe(int32_t kind, int32_t width, int32_t unroll, int32_t nontemporal,
                          int32_t grid, int32_t tile_shift, void *dst, const void *src0,
                          const void *src1, size_t bytes, void *stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: energy and
 * gradient like gv_energy_grad in GV_GRAD_UNCOMPUTE mode, without a state or
 * a caller workspace.  The state vector, the adjoint vector and every table
 * and partial sum live in one library-owned static device array of
 * gv_noalloc_scratch_bytes() (64 MiB) per GPU, held from the library's load
 * until the process ends: n <= 21 in GV_C64, n <= 20 in GV_C128 (larger
 * requests return GV_ESIZE before any work).  The call allocates nothing
 * (no hipMalloc, no allocating library routine); it enqueues on `stream` and
 * returns.  Arguments as gv_energy_grad; h must be prepared for `prec` on the
 * fused engine (gv_pauli_sum_prepare_for).  Every call on one GPU shares the
 * array: calls that overlap on one GPU (other streams, other threads) race.
 * Nothing has to be cleared between calls (every scratch entry a call reads
 * it has written first). */
gv_status gv_energy_grad_noalloc(int32_t n, gv_precision prec, gv_pauli_sum h,
                                 const double *params_dev, const gv_ansatz *ansatz,
                                 const uint8_t *grad_mask_dev, double *energy_dev,
                                 double *grad_dev, void *stream);
size_t gv_noalloc_scratch_bytes(void);

#ifdef __cplusplus
}
#endif
#endif /* GV_H */
