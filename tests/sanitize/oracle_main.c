/* Drives the CPU oracle under AddressSanitizer / UndefinedBehaviorSanitizer:
 * every entry point on small circuits (all entanglers, a final rotation,
 * duplicate and off-diagonal terms), checking the results stay finite.
 * Exit status 0 when every call succeeded. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int gvo_num_params(int n, int layers, int final_rotation);
int64_t gvo_num_gates(int n, int layers, int ent, int final_rotation);
int gvo_prepare(int n, int layers, int ent, int final_rotation, const double *theta,
                double *psi);
int64_t gvo_apply_gates(int n, int layers, int ent, int final_rotation, const double *theta,
                        int64_t first, int64_t count, int inverse, double *psi);
void gvo_diag(int n, int64_t m, const uint64_t *x, const uint64_t *z, const double *c, double *d);
void gvo_apply_h(int n, int64_t m, const uint64_t *x, const uint64_t *z, const double *c,
                 const double *d, const double *psi, double *out);
int gvo_energy_grad(int n, int layers, int ent, int final_rotation, const double *theta,
                    int64_t m, const uint64_t *x, const uint64_t *z, const double *c,
                    const double *d, const uint8_t *mask, double *e, double *g);

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) / 9007199254740992.0;
}

int main(void)
{
    uint64_t seed = 7;
    int fails = 0;
    for (int n = 1; n <= 7; n += 2)
        for (int ent = 0; ent <= 8; ++ent)
            for (int fr = 0; fr <= 1; ++fr) {
                const int L = 2, P = gvo_num_params(n, L, fr);
                const int64_t m = 3 * n + 2;
                double *th = malloc(sizeof(double) * P), *g = malloc(sizeof(double) * P);
                uint64_t *x = malloc(sizeof(uint64_t) * m), *z = malloc(sizeof(uint64_t) * m);
                double *c = malloc(sizeof(double) * m), *d = malloc(sizeof(double) << n);
                /* complex128 amplitudes, interleaved (re, im) */
                double *psi = malloc((2 * sizeof(double)) << n);
                double *out = malloc((2 * sizeof(double)) << n);
                uint8_t *mask = malloc(P);
                for (int p = 0; p < P; ++p) {
                    th[p] = 6.283185307179586 * urand(&seed) - 3.141592653589793;
                    mask[p] = (uint8_t)(p % 3 != 0);
                }
                const uint64_t all = (1ull << n) - 1;
                for (int64_t k = 0; k < m; ++k) {
                    x[k] = (k % 3 == 0) ? ((uint64_t)(urand(&seed) * 1e9) & all) : 0;
                    z[k] = (uint64_t)(urand(&seed) * 1e9) & all;
                    c[k] = urand(&seed) - 0.5;
                }
                x[m - 1] = x[0];   /* a duplicate term */
                z[m - 1] = z[0];
                double e[2];
                if (gvo_prepare(n, L, ent, fr, th, psi)) ++fails;
                gvo_diag(n, m, x, z, c, d);
                gvo_apply_h(n, m, x, z, c, d, psi, out);
                const int64_t ng = gvo_num_gates(n, L, ent, fr);
                gvo_apply_gates(n, L, ent, fr, th, 0, ng, 1, psi);
                if (gvo_energy_grad(n, L, ent, fr, th, m, x, z, c, d, mask, e, g)) ++fails;
                if (!isfinite(e[0]) || !isfinite(e[1])) ++fails;
                for (int p = 0; p < P; ++p)
                    if (!isfinite(g[p])) ++fails;
                free(th); free(g); free(x); free(z); free(c); free(d); free(psi); free(out);
                free(mask);
            }
    printf("oracle sanitizer run: %d failures\n", fails);
    return fails != 0;
}
