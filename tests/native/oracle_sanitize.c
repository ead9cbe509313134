/* A small driver of the oracle for the sanitizer build (AddressSanitizer and
   UndefinedBehaviorSanitizer, host code only): a coarse table grid, then lepton and photon
   steps in a plane wave and on a grid, with pairs, the optical-depth decision, sub-cycling,
   a full photon store (capacity overflow), compaction and non-finite inputs.  It checks only
   that every call completes; the sanitizers report any out-of-bounds access, use after free,
   leak or undefined operation. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/qed_oracle.h"

static double urand(unsigned *st)
{
    *st = *st * 1664525u + 1013904223u;
    return (*st >> 8) * (1.0 / 16777216.0);
}

static double *dalloc(size_t n) { return (double *)calloc(n, sizeof(double)); }

int main(void)
{
    orc_table_spec spec;
    memset(&spec, 0, sizeof(spec));
    spec.n_chi[0] = 21; spec.n_chi[1] = 15;                     /* 4 nodes per decade */
    spec.lnchi0[0] = log(1e-3); spec.lnchi0[1] = log(0.05);
    spec.dlnchi[0] = spec.dlnchi[1] = log(10.0) / 4.0;
    spec.n_rho = 24; spec.rho0 = -37.5; spec.drho = 75.0 / 23.0;
    orc_tables T;
    if (orc_tables_build(&T, &spec, 2) != 0) return 1;

    const int n = 200, capg = 300;                               /* a photon store that fills up */
    orc_leptons L, P;
    orc_photons G;
    memset(&L, 0, sizeof(L)); memset(&P, 0, sizeof(P)); memset(&G, 0, sizeof(G));
    L.cap = P.cap = 2 * n; L.species = 0; P.species = 1;
    G.cap = capg;
    for (int i = 0; i < 3; ++i) {
        L.x[i] = dalloc(L.cap); L.p[i] = dalloc(L.cap); L.s[i] = dalloc(L.cap);
        P.x[i] = dalloc(P.cap); P.p[i] = dalloc(P.cap); P.s[i] = dalloc(P.cap);
        G.x[i] = dalloc(G.cap); G.k[i] = dalloc(G.cap); G.P[i] = dalloc(G.cap);
    }
    G.id = (uint64_t *)calloc(G.cap, sizeof(uint64_t));
    L.near = (uint8_t *)calloc(L.cap, 1); P.near = (uint8_t *)calloc(P.cap, 1); G.near = (uint8_t *)calloc(G.cap, 1);
    L.cond = dalloc(L.cap); P.cond = dalloc(P.cap); G.cond = dalloc(G.cap);
    L.tau = dalloc(L.cap); L.tau_target = dalloc(L.cap); P.tau = dalloc(P.cap); P.tau_target = dalloc(P.cap);
    unsigned st = 7;
    for (int j = 0; j < n; ++j) {
        double g = 500.0 + 4000.0 * urand(&st);
        L.p[0][j] = sqrt(g * g - 1.0);
        L.s[1][j] = urand(&st) < 0.5 ? 1.0 : -1.0;
        L.x[0][j] = -6.0 * urand(&st);
    }
    L.n = n;
    L.p[1][5] = NAN;                                             /* a non-finite lepton */

    float *grid[6];
    const int nx = 16, ny = 8;
    for (int c = 0; c < 6; ++c) {
        grid[c] = (float *)calloc((size_t)nx * ny, sizeof(float));
        for (int i = 0; i < nx * ny; ++i) grid[c][i] = (float)(200.0 * (urand(&st) - 0.5));
    }
    orc_fields f[2];
    memset(f, 0, sizeof(f));
    f[0].kind = 1; f[0].a0 = 300.0; f[0].phase_len = 60.0;
    f[1].kind = 2; f[1].nx = nx; f[1].ny = ny; f[1].dx = f[1].dy = 0.2;
    for (int c = 0; c < 6; ++c) f[1].grid[c] = grid[c];

    orc_counters ctr;
    memset(&ctr, 0, sizeof(ctr));
    const uint32_t base = (1u << 0) | (1u << 1) | (1u << 2) | (1u << 3) | (1u << 4) | (1u << 5) | (1u << 6) |
                          (1u << 8) | (1u << 9) | (1u << 10);
    const uint32_t variants[4] = {base, base | (1u << 11), base | (1u << 12), base | (1u << 14) | (1u << 13)};
    for (int k = 0; k < 120; ++k) {
        orc_params prm;
        memset(&prm, 0, sizeof(prm));
        prm.t = 0.06 * k; prm.dt = 0.06; prm.a_e = 1.16e-3; prm.eps_r = 3.03e-6;
        prm.chi_e_min = 1e-3; prm.chi_e_max = 1e2; prm.chi_g_min = 0.05; prm.chi_g_max = 1e2;
        prm.k_retire = 10.0; prm.near_tol = 1e-10; prm.step = k; prm.seed = 3;
        prm.flags = variants[(k / 30) % 4]; prm.u24 = k & 1;
        const orc_fields *fk = &f[(k / 15) & 1];
        orc_lepton_step(&T, &prm, fk, &L, &G, &ctr, 2);
        orc_lepton_step(&T, &prm, fk, &P, &G, &ctr, 2);
        orc_photon_step(&T, &prm, fk, &G, &L, &P, &ctr, 2);
        if (k % 10 == 9) orc_compact(&G);
    }
    printf("sanitized run: %lld emissions, %lld pairs, %lld overflow, %lld non-finite, %lld photons stored\n",
           (long long)ctr.n_emit, (long long)ctr.n_pair, (long long)ctr.n_capacity_overflow,
           (long long)ctr.n_nonfinite, (long long)G.n);
    for (int i = 0; i < 3; ++i) {
        free(L.x[i]); free(L.p[i]); free(L.s[i]); free(P.x[i]); free(P.p[i]); free(P.s[i]);
        free(G.x[i]); free(G.k[i]); free(G.P[i]);
    }
    free(G.id); free(L.near); free(P.near); free(G.near); free(L.cond); free(P.cond); free(G.cond);
    free(L.tau); free(L.tau_target); free(P.tau); free(P.tau_target);
    for (int c = 0; c < 6; ++c) free(grid[c]);
    orc_tables_free(&T);
    return ctr.n_emit > 0 && ctr.n_capacity_overflow > 0 ? 0 : 2;
}
