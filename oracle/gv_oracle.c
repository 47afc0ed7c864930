/*
 * gv_oracle.c -- CPU oracle for the Graph-VQE energy / gradient hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path loads this file or
 * its library; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU library.
 *
 * What it computes, in the plainest form (complex128 amplitudes, every sum in
 * double precision, one gate at a time, no fusion or reordering):
 *
 *   psi(theta) = U(theta)|0...0>            ansatz, Sec. IV-B, Eq. 7 and Eq. 8
 *   H = sum_k c_k P_k, c_k real             Eq. 6
 *   E(theta) = <psi|H|psi>                  Eq. 4
 *   dE/dtheta_j                             (exact; Eq. 13 is one way to get it)
 *
 * Conventions (readings of points the paper leaves open):
 *   - qubit q is bit q of the amplitude index;
 *   - a layer applies RY(theta) to every qubit, then RZ(phi) to every qubit,
 *     then the entangler; an optional final layer applies only RY, RZ
 *     (EfficientSU2 of Eq. 8: L repeated layers plus one rotation layer);
 *   - parameter index of layer l, gate g (0 = RY, 1 = RZ), qubit q is
 *     l*2n + g*n + q;
 *   - RY(t) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]],
 *     RZ(t) = diag(exp(-i t/2), exp(+i t/2))            (Eq. 7);
 *   - entanglers: CZ on (q, q+1) for q = 0..n-2 (circular adds (n-1, 0));
 *     CNOT networks (Sec. IV-B names linear, circular and full patterns;
 *     Sec. V-A also uses reverse-linear, pairwise and shifted-circular-
 *     alternating ones), each a list of CNOT(control -> target) applied in
 *     order:
 *       linear          (q, q+1) for q = 0, 1, ..., n-2
 *       circular        (n-1, 0) first (n > 2), then linear
 *       full            (i, j) for i = 0..n-2, j = i+1..n-1, i outer
 *       reverse linear  (q, q+1) for q = n-2 down to 0
 *       pairwise        (q, q+1) for even q, then for odd q
 *       sca             in layer l the circular list [(n-1, 0), (0, 1), ...,
 *                       (n-2, n-1)] rotated right by l mod n, with control
 *                       and target exchanged in the odd layers (for n <= 2
 *                       the linear list);
 *   - Pauli string P(x, z) = i^{|x & z|} X^x Z^z over bit masks x, z, so that
 *     (P psi)_i = i^{|x & z|} (-1)^{popcount((i ^ x) & z)} psi_{i ^ x}.
 *
 * Gradient: reverse-mode ("adjoint") sweep, gate by gate.  With phi the
 * state after gate k and lambda = (gates after k)^dagger H psi, the
 * derivative of E by the angle of exp(-i t G / 2) is Im <lambda|G|phi>.
 * The parameter-shift rule of Eq. 13 checks it in the tests.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* loops shorter than this run on one thread (thread start-up would dominate) */
#define OMP_MIN 16384

enum { G_RY = 0, G_RZ = 1, G_CZ = 2, G_CNOT = 3 };
enum { ENT_NONE = 0, ENT_CZ_LINEAR = 1, ENT_CZ_CIRCULAR = 2,
       ENT_CNOT_LINEAR = 3, ENT_CNOT_CIRCULAR = 4, ENT_CNOT_FULL = 5,
       ENT_CNOT_REVERSE_LINEAR = 6, ENT_CNOT_PAIRWISE = 7, ENT_CNOT_SCA = 8 };

typedef struct {
    int kind;
    int a, b;      /* qubit (RY/RZ); CZ pair; CNOT control a, target b */
    int64_t p;     /* parameter index, -1 for fixed gates */
} gate_t;

int gvo_num_params(int n, int layers, int final_rotation)
{
    return 2 * n * (layers + final_rotation);
}

/* Upper bound on the number of gates of the circuit. */
static int64_t max_gates(int n, int layers, int final_rotation)
{
    return (int64_t)(layers + final_rotation) * (2 * (int64_t)n + (int64_t)n * n + 1);
}

/* Gate list of the circuit in application order. Returns the count, or -1. */
static int64_t build_circuit(int n, int layers, int ent, int final_rotation, gate_t *g)
{
    int64_t k = 0;
    for (int l = 0; l < layers + final_rotation; ++l) {
        int64_t base = (int64_t)l * 2 * n;
        for (int q = 0; q < n; ++q) {
            gate_t t = { G_RY, q, -1, base + q };
            g[k++] = t;
        }
        for (int q = 0; q < n; ++q) {
            gate_t t = { G_RZ, q, -1, base + n + q };
            g[k++] = t;
        }
        if (l >= layers) break;  /* the final rotation layer has no entangler */
        switch (ent) {
        case ENT_NONE:
            break;
        case ENT_CZ_LINEAR:
        case ENT_CZ_CIRCULAR:
            for (int q = 0; q + 1 < n; ++q) {
                gate_t t = { G_CZ, q, q + 1, -1 };
                g[k++] = t;
            }
            if (ent == ENT_CZ_CIRCULAR && n > 2) {
                gate_t t = { G_CZ, n - 1, 0, -1 };
                g[k++] = t;
            }
            break;
        case ENT_CNOT_LINEAR:
        case ENT_CNOT_CIRCULAR:
            if (ent == ENT_CNOT_CIRCULAR && n > 2) {
                gate_t t = { G_CNOT, n - 1, 0, -1 };
                g[k++] = t;
            }
            for (int q = 0; q + 1 < n; ++q) {
                gate_t t = { G_CNOT, q, q + 1, -1 };
                g[k++] = t;
            }
            break;
        case ENT_CNOT_FULL:
            for (int i = 0; i + 1 < n; ++i)
                for (int j = i + 1; j < n; ++j) {
                    gate_t t = { G_CNOT, i, j, -1 };
                    g[k++] = t;
                }
            break;
        case ENT_CNOT_REVERSE_LINEAR:
            for (int q = n - 2; q >= 0; --q) {
                gate_t t = { G_CNOT, q, q + 1, -1 };
                g[k++] = t;
            }
            break;
        case ENT_CNOT_PAIRWISE:
            for (int start = 0; start < 2; ++start)
                for (int q = start; q + 1 < n; q += 2) {
                    gate_t t = { G_CNOT, q, q + 1, -1 };
                    g[k++] = t;
                }
            break;
        case ENT_CNOT_SCA: {
            /* circular list: entry 0 is (n-1, 0), entry e >= 1 is (e-1, e) */
            const int m = n > 2 ? n : n - 1;
            for (int e = 0; e < m; ++e) {
                int src = n > 2 ? ((e - l) % m + m) % m : e;
                int c = n > 2 ? (src == 0 ? n - 1 : src - 1) : src;
                int t = n > 2 ? (src == 0 ? 0 : src) : src + 1;
                if (l & 1) {
                    int tmp = c;
                    c = t;
                    t = tmp;
                }
                gate_t gt = { G_CNOT, c, t, -1 };
                g[k++] = gt;
            }
            break;
        }
        default:
            return -1;
        }
    }
    return k;
}

/* index with a zero bit inserted at position q */
static inline uint64_t insert0(uint64_t k, int q)
{
    uint64_t lo = k & ((1ULL << q) - 1);
    return ((k >> q) << (q + 1)) | lo;
}

static void apply_ry(int n, int q, double t, cplx *psi)
{
    const double c = cos(0.5 * t), s = sin(0.5 * t);
    const uint64_t half = 1ULL << (n - 1), bit = 1ULL << q;
#pragma omp parallel for schedule(static) if (half > OMP_MIN)
    for (int64_t k = 0; k < (int64_t)half; ++k) {
        uint64_t i = insert0((uint64_t)k, q), j = i | bit;
        cplx a = psi[i], b = psi[j];
        psi[i] = c * a - s * b;
        psi[j] = s * a + c * b;
    }
}

static void apply_rz(int n, int q, double t, cplx *psi)
{
    const cplx e0 = cexp(-0.5 * I * t), e1 = cexp(0.5 * I * t);
    const uint64_t half = 1ULL << (n - 1), bit = 1ULL << q;
#pragma omp parallel for schedule(static) if (half > OMP_MIN)
    for (int64_t k = 0; k < (int64_t)half; ++k) {
        uint64_t i = insert0((uint64_t)k, q), j = i | bit;
        psi[i] *= e0;
        psi[j] *= e1;
    }
}

static void apply_cz(int n, int a, int b, cplx *psi)
{
    const uint64_t dim = 1ULL << n, m = (1ULL << a) | (1ULL << b);
#pragma omp parallel for schedule(static) if (dim > OMP_MIN)
    for (int64_t i = 0; i < (int64_t)dim; ++i)
        if (((uint64_t)i & m) == m) psi[i] = -psi[i];
}

static void apply_cnot(int n, int ctl, int tgt, cplx *psi)
{
    const uint64_t half = 1ULL << (n - 1), cb = 1ULL << ctl, tb = 1ULL << tgt;
#pragma omp parallel for schedule(static) if (half > OMP_MIN)
    for (int64_t k = 0; k < (int64_t)half; ++k) {
        uint64_t i = insert0((uint64_t)k, tgt);   /* target bit 0 */
        if (i & cb) {
            uint64_t j = i | tb;
            cplx t = psi[i];
            psi[i] = psi[j];
            psi[j] = t;
        }
    }
}

/* gate, or its inverse when inv != 0 */
static void apply_gate(int n, const gate_t *g, const double *theta, int inv, cplx *psi)
{
    double t = g->p >= 0 ? theta[g->p] : 0.0;
    if (inv) t = -t;
    switch (g->kind) {
    case G_RY: apply_ry(n, g->a, t, psi); break;
    case G_RZ: apply_rz(n, g->a, t, psi); break;
    case G_CZ: apply_cz(n, g->a, g->b, psi); break;
    case G_CNOT: apply_cnot(n, g->a, g->b, psi); break;
    }
}

/* Im <lam| Y_q |phi> */
static double im_expect_y(int n, int q, const cplx *lam, const cplx *phi)
{
    const uint64_t half = 1ULL << (n - 1), bit = 1ULL << q;
    double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+:acc) if (half > OMP_MIN)
    for (int64_t k = 0; k < (int64_t)half; ++k) {
        uint64_t i = insert0((uint64_t)k, q), j = i | bit;
        /* (Y phi)_i = -i phi_j, (Y phi)_j = +i phi_i */
        cplx v = conj(lam[i]) * (-I * phi[j]) + conj(lam[j]) * (I * phi[i]);
        acc += cimag(v);
    }
    return acc;
}

/* Im <lam| Z_q |phi> */
static double im_expect_z(int n, int q, const cplx *lam, const cplx *phi)
{
    const uint64_t dim = 1ULL << n, bit = 1ULL << q;
    double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+:acc) if (dim > OMP_MIN)
    for (int64_t i = 0; i < (int64_t)dim; ++i) {
        double s = ((uint64_t)i & bit) ? -1.0 : 1.0;
        acc += s * cimag(conj(lam[i]) * phi[i]);
    }
    return acc;
}

/* ---------------------------------------------------------------- exports */

/* psi <- U(theta)|0...0>.  psi holds 2^n complex128 (interleaved re, im). */
int gvo_prepare(int n, int layers, int ent, int final_rotation,
                const double *theta, double *psi_out)
{
    if (n < 1 || n > 40 || layers < 0) return 1;
    cplx *psi = (cplx *)psi_out;
    const uint64_t dim = 1ULL << n;
    memset(psi, 0, dim * sizeof(cplx));
    psi[0] = 1.0;
    gate_t *g = (gate_t *)malloc(sizeof(gate_t) * (size_t)max_gates(n, layers, final_rotation));
    if (!g) return 2;
    int64_t ng = build_circuit(n, layers, ent, final_rotation, g);
    if (ng < 0) { free(g); return 1; }
    for (int64_t k = 0; k < ng; ++k) apply_gate(n, &g[k], theta, 0, psi);
    free(g);
    return 0;
}

/* Apply gates [first, first + count) of the circuit (inverse gates in reverse
 * order when inverse != 0) to psi in place.  Returns the number applied. */
int64_t gvo_apply_gates(int n, int layers, int ent, int final_rotation,
                        const double *theta, int64_t first, int64_t count,
                        int inverse, double *psi_io)
{
    gate_t *g = (gate_t *)malloc(sizeof(gate_t) * (size_t)max_gates(n, layers, final_rotation));
    if (!g) return -1;
    int64_t ng = build_circuit(n, layers, ent, final_rotation, g);
    if (ng < 0) { free(g); return -1; }
    if (first < 0) first = 0;
    if (first > ng) first = ng;
    if (count > ng - first) count = ng - first;
    cplx *psi = (cplx *)psi_io;
    if (!inverse)
        for (int64_t k = first; k < first + count; ++k) apply_gate(n, &g[k], theta, 0, psi);
    else
        for (int64_t k = first + count - 1; k >= first; --k) apply_gate(n, &g[k], theta, 1, psi);
    free(g);
    return count;
}

int64_t gvo_num_gates(int n, int layers, int ent, int final_rotation)
{
    gate_t *g = (gate_t *)malloc(sizeof(gate_t) * (size_t)max_gates(n, layers, final_rotation));
    if (!g) return -1;
    int64_t ng = build_circuit(n, layers, ent, final_rotation, g);
    free(g);
    return ng;
}

/* Diagonal of the Z-only part (terms with x = 0), by direct summation:
 * D_i = sum_{k : x_k = 0} c_k (-1)^{popcount(i & z_k)}. */
void gvo_diag(int n, int64_t m, const uint64_t *x, const uint64_t *z,
              const double *c, double *d)
{
    const uint64_t dim = 1ULL << n;
#pragma omp parallel for schedule(static) if (dim > OMP_MIN)
    for (int64_t i = 0; i < (int64_t)dim; ++i) {
        double acc = 0.0;
        for (int64_t k = 0; k < m; ++k) {
            if (x[k]) continue;
            acc += (__builtin_popcountll((uint64_t)i & z[k]) & 1) ? -c[k] : c[k];
        }
        d[i] = acc;
    }
}

/* One diagonal entry D_i (same definition). */
double gvo_diag_at(int64_t m, const uint64_t *x, const uint64_t *z,
                   const double *c, uint64_t i)
{
    double acc = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        if (x[k]) continue;
        acc += (__builtin_popcountll(i & z[k]) & 1) ? -c[k] : c[k];
    }
    return acc;
}

/* out <- H psi.  Z-only terms use d when it is given (d from gvo_diag);
 * with d == NULL every term is applied one by one. */
void gvo_apply_h(int n, int64_t m, const uint64_t *x, const uint64_t *z,
                 const double *c, const double *d, const double *psi_in,
                 double *out_)
{
    const uint64_t dim = 1ULL << n;
    const cplx *psi = (const cplx *)psi_in;
    cplx *out = (cplx *)out_;
    static const double complex ipow[4] = { 1.0, I, -1.0, -I };
#pragma omp parallel for schedule(static) if (dim > OMP_MIN)
    for (int64_t i = 0; i < (int64_t)dim; ++i) {
        cplx acc = d ? d[i] * psi[i] : 0.0;
        for (int64_t k = 0; k < m; ++k) {
            if (d && !x[k]) continue;
            uint64_t j = (uint64_t)i ^ x[k];
            int ph = __builtin_popcountll(x[k] & z[k]) & 3;
            double s = (__builtin_popcountll(j & z[k]) & 1) ? -1.0 : 1.0;
            acc += c[k] * s * ipow[ph] * psi[j];
        }
        out[i] = acc;
    }
}

/* <a|b> */
void gvo_inner(int n, const double *a_, const double *b_, double *re, double *im)
{
    const uint64_t dim = 1ULL << n;
    const cplx *a = (const cplx *)a_, *b = (const cplx *)b_;
    double sr = 0.0, si = 0.0;
#pragma omp parallel for schedule(static) reduction(+:sr, si) if (dim > OMP_MIN)
    for (int64_t i = 0; i < (int64_t)dim; ++i) {
        cplx v = conj(a[i]) * b[i];
        sr += creal(v);
        si += cimag(v);
    }
    *re = sr;
    *im = si;
}

/* Energy and gradient.  energy_out[0..1] = Re, Im of <psi|H|psi>.
 * grad_out[P]: entries with mask[j] == 0 are set to 0 (mask may be NULL).
 * d: diagonal from gvo_diag, or NULL (then every term is applied directly). */
int gvo_energy_grad(int n, int layers, int ent, int final_rotation,
                    const double *theta, int64_t m, const uint64_t *x,
                    const uint64_t *z, const double *c, const double *d,
                    const uint8_t *mask, double *energy_out, double *grad_out)
{
    if (n < 1 || n > 40) return 1;
    const uint64_t dim = 1ULL << n;
    const int np = gvo_num_params(n, layers, final_rotation);
    cplx *phi = (cplx *)malloc(dim * sizeof(cplx));
    cplx *lam = (cplx *)malloc(dim * sizeof(cplx));
    gate_t *g = (gate_t *)malloc(sizeof(gate_t) * (size_t)max_gates(n, layers, final_rotation));
    if (!phi || !lam || !g) { free(phi); free(lam); free(g); return 2; }
    int64_t ng = build_circuit(n, layers, ent, final_rotation, g);
    if (ng < 0) { free(phi); free(lam); free(g); return 1; }

    memset(phi, 0, dim * sizeof(cplx));
    phi[0] = 1.0;
    for (int64_t k = 0; k < ng; ++k) apply_gate(n, &g[k], theta, 0, phi);

    gvo_apply_h(n, m, x, z, c, d, (const double *)phi, (double *)lam);
    gvo_inner(n, (const double *)phi, (const double *)lam, &energy_out[0], &energy_out[1]);

    for (int j = 0; j < np; ++j) grad_out[j] = 0.0;
    for (int64_t k = ng - 1; k >= 0; --k) {
        const gate_t *gk = &g[k];
        if (gk->p >= 0 && (!mask || mask[gk->p])) {
            grad_out[gk->p] = gk->kind == G_RY ? im_expect_y(n, gk->a, lam, phi)
                                               : im_expect_z(n, gk->a, lam, phi);
        }
        apply_gate(n, gk, theta, 1, phi);
        apply_gate(n, gk, theta, 1, lam);
    }
    free(phi);
    free(lam);
    free(g);
    return 0;
}

/* Adjoint steps for gates [first, first + count) in reverse order, on given
 * phi and lam (both updated in place); gradient entries written to grad.
 * This is the inner loop of gvo_energy_grad, exposed so that a bounded part
 * of a large evaluation can be timed. */
int64_t gvo_adjoint_gates(int n, int layers, int ent, int final_rotation,
                          const double *theta, int64_t first, int64_t count,
                          double *phi_, double *lam_, double *grad)
{
    gate_t *g = (gate_t *)malloc(sizeof(gate_t) * (size_t)max_gates(n, layers, final_rotation));
    if (!g) return -1;
    int64_t ng = build_circuit(n, layers, ent, final_rotation, g);
    if (ng < 0) { free(g); return -1; }
    if (first < 0) first = 0;
    if (first > ng) first = ng;
    if (count > ng - first) count = ng - first;
    cplx *phi = (cplx *)phi_, *lam = (cplx *)lam_;
    for (int64_t k = first + count - 1; k >= first; --k) {
        const gate_t *gk = &g[k];
        if (gk->p >= 0)
            grad[gk->p] = gk->kind == G_RY ? im_expect_y(n, gk->a, lam, phi)
                                           : im_expect_z(n, gk->a, lam, phi);
        apply_gate(n, gk, theta, 1, phi);
        apply_gate(n, gk, theta, 1, lam);
    }
    free(g);
    return count;
}

/* Threads the OpenMP loops use (1 without OpenMP), and a way to change it
 * (for timing the oracle on a given number of host cores). */
int gvo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void gvo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
