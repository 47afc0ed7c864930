// Drives the library's host-side code under AddressSanitizer /
// UndefinedBehaviorSanitizer (host code only; no GPU is touched): Pauli-sum
// ingest with duplicates, zeros and bad input, the off-diagonal cover
// planner on wide random sums, group queries, and the size queries of every
// ansatz shape, engine, precision and gradient mode.  Exit status 0 when
// every status is the expected one.
#include <stdint.h>
#include <stdio.h>
#include <vector>

#include "gv.h"

static uint64_t rnd(uint64_t &s)
{
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return s >> 11;
}

int main()
{
    int fails = 0;
    uint64_t seed = 11;
    for (int n : {1, 5, 8, 12, 20, 28, 32, 34}) {
        for (int m : {0, 1, 7, 300, 2500}) {
            std::vector<uint64_t> x(m), z(m);
            std::vector<double> c(m);
            const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
            for (int k = 0; k < m; ++k) {
                const int a = (int)(rnd(seed) % n), b = (int)(rnd(seed) % n);
                x[k] = (k % 2) ? ((1ull << a) | (1ull << b)) & all : 0;
                z[k] = rnd(seed) & all;
                c[k] = (k % 11 == 0) ? 0.0 : (double)(rnd(seed) % 1000) / 999.0 - 0.5;
            }
            if (m > 3) {   // a duplicate of term 1
                x[m - 1] = x[1];
                z[m - 1] = z[1];
            }
            gv_pauli_sum h = nullptr;
            if (gv_pauli_sum_create(n, m, m ? x.data() : nullptr, m ? z.data() : nullptr,
                                    m ? c.data() : nullptr, &h) != GV_OK) {
                ++fails;
                printf("create n=%d m=%d: %s\n", n, m, gv_last_error());
                continue;
            }
            int64_t nd = 0, no = 0, ng = 0;
            if (gv_pauli_sum_info(h, &nd, &no, &ng) != GV_OK) ++fails;
            for (int64_t g = 0; g < ng; ++g) {
                uint64_t xm, ym, zm;
                int64_t nt;
                if (gv_pauli_sum_group(h, g, &xm, &ym, &zm, &nt) != GV_OK) ++fails;
            }
            for (gv_precision p : {GV_C64, GV_C128})
                for (gv_engine e : {GV_ENGINE_FUSED, GV_ENGINE_PLAIN}) {
                    int64_t passes, mx, loose;
                    if (gv_pauli_sum_plan(h, n, p, e, &passes, &mx, &loose) != GV_OK) ++fails;
                }
            size_t db = 0;
            if (gv_pauli_sum_device_bytes(h, &db) != GV_OK) ++fails;
            gv_pauli_sum_destroy(h);
        }
        for (int ent = 0; ent <= 8; ++ent)
            for (int layers : {0, 1, 6})
                for (int fr : {0, 1}) {
                    gv_ansatz a = {n, layers, ent, fr};
                    if (gv_num_params(&a) < 0) ++fails;
                    for (gv_precision p : {GV_C64, GV_C128})
                        for (gv_engine e : {GV_ENGINE_FUSED, GV_ENGINE_PLAIN})
                            for (int mode = 0; mode < 4; ++mode) {
                                size_t sb, wb, dbb;
                                const gv_status r = gv_query_sizes(
                                    &a, p, e, (gv_grad_mode)mode, &sb, &wb, &dbb);
                                if (r != GV_OK && r != GV_EUNSUPPORTED) ++fails;
                            }
                }
    }
    // invalid input must be refused with a message, not read out of bounds
    {
        const uint64_t x = 1ull << 40, z = 0;
        const double c = 1.0;
        gv_pauli_sum h = nullptr;
        if (gv_pauli_sum_create(8, 1, &x, &z, &c, &h) != GV_EINVAL) ++fails;
        const double bad = 0.0 / 0.0;
        const uint64_t x1 = 1;
        if (gv_pauli_sum_create(8, 1, &x1, &z, &bad, &h) != GV_EINVAL) ++fails;
        gv_ansatz a = {0, 1, 0, 0};
        size_t sb, wb, dbb;
        if (gv_query_sizes(&a, GV_C64, GV_ENGINE_FUSED, GV_GRAD_STORE, &sb, &wb, &dbb) == GV_OK)
            ++fails;
        if (gv_query_sizes(nullptr, GV_C64, GV_ENGINE_FUSED, GV_GRAD_STORE, &sb, &wb, &dbb) == GV_OK)
            ++fails;
    }
    printf("host sanitizer run: %d failures\n", fails);
    return fails != 0;
}
