/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE: calls every routine of the oracle on small inputs
 * (periodic, open, diluted and thin lattices, fields, colour maps, 1, 2 and 4 labels, one or
 * two ICM moves, odd and even Trotter rings), so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks the oracle's memory accesses and arithmetic.  Prints a
 * checksum of everything computed; exits 0.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sg_oracle.h"

static uint64_t mix(uint64_t h, int64_t v) { return (h ^ (uint64_t)v) * 1099511628211ull; }

static void couplings(int Lx, int Ly, int Lz, uint32_t seed, int dilute, int8_t *J)
{
    uint32_t s = seed * 2654435761u + 1u;
    for (int i = 0; i < 3 * Lx * Ly * Lz; ++i) {
        s = s * 1664525u + 1013904223u;
        J[i] = (s >> 31) ? 1 : -1;
        if (dilute && ((s >> 20) & 7u) == 0u) J[i] = 0;
    }
}

static uint64_t run_case(int Lx, int Ly, int Lz, uint32_t periodic, int dilute, int hmax, int R_lab,
                         uint64_t h)
{
    const int n = Lx * Ly * Lz;
    int8_t *J = malloc((size_t)3 * n), *hf = NULL;
    couplings(Lx, Ly, Lz, (uint32_t)(n + periodic), dilute, J);
    if (hmax) {
        hf = malloc((size_t)n);
        for (int j = 0; j < n; ++j) hf[j] = (int8_t)((j * 7) % (2 * hmax + 1) - hmax);
    }
    sgo_lattice lat = {Lx, Ly, Lz, periodic, J, hf, NULL, 0};
    const int nb = 5, slots = nb * R_lab;
    double beta[5] = {0.3, 0.7, 1.0, 1.6, 2.4}, sb[20];
    for (int s = 0; s < slots; ++s) sb[s] = beta[s / R_lab];
    int8_t *sp = malloc((size_t)slots * n);
    int64_t E[20] = {0}, best = INT64_MAX, trace[8] = {0}, accc[4 * 4] = {0};
    int32_t info[5 * 2 * 4], acc[4 * 4] = {0};
    uint32_t ctr[3] = {0, 0, 0};
    sgo_apt_init(&lat, 1, slots, 77, 1, sp);
    for (int t = 0; t < 3; ++t) sgo_apt_sweep(&lat, 1, slots, sb, 77, 2, (uint32_t)t, sp);
    for (int s = 0; s < slots; ++s) {
        E[s] = sgo_energy(&lat, sp + (int64_t)s * n);
        h = mix(h, E[s]);
        for (int j = 0; j < n; ++j) h = mix(h, sgo_local_field(&lat, sp + (int64_t)s * n, j));
    }
    for (int pairs = 1; pairs <= 2; ++pairs) {
        for (int i = 0; i < 5 * 2 * 4; ++i) info[i] = -7;   /* one label: the call writes none */
        int32_t rc = sgo_apt_icm(&lat, 1, nb, R_lab, beta, 0.9, pairs, 77, (uint32_t)pairs, sp, info);
        h = mix(h, rc);
        for (int i = 0; i < nb * (R_lab / 2 > 0 ? R_lab / 2 : 1) * 4; ++i) h = mix(h, info[i]);
    }
    for (int s = 0; s < slots; ++s) E[s] = sgo_energy(&lat, sp + (int64_t)s * n);
    sgo_apt_swap(1, nb, R_lab, beta, 77, 1, n, sp, E, acc);
    memset(accc, 0, sizeof accc);
    int32_t rc = sgo_apt_run(&lat, 1, nb, R_lab, beta, 77, 8, 2, hmax ? 1e300 : 1.0, 2, 1, ctr, sp, E,
                             &best, trace, accc);
    h = mix(h, rc);
    h = mix(h, best);
    for (int i = 0; i < 8; ++i) h = mix(h, trace[i]);
    /* colour map and the Trotter direction */
    int8_t *cmap = malloc((size_t)n);
    for (int j = 0; j < n; ++j) cmap[j] = (int8_t)sgo_colour(&lat, 0, j, 0);
    sgo_lattice lc = lat;
    lc.colour = cmap;
    lc.n_map_colours = sgo_n_colours(&lat, 0);
    for (int M = 3; M <= 4; ++M) {
        const int Rq = 2;
        int8_t *q = malloc((size_t)Rq * M * n);
        int64_t slE[2 * 4], bE;
        int8_t *bs = malloc((size_t)n);
        int32_t agree[2 * 4];
        double g[4] = {3.0, 2.0, 1.0, 0.01};
        const sgo_lattice *use = (M == 4) ? &lc : &lat;
        sgo_sqa_init(use, 2, M, 0, Rq, 78, q);
        sgo_sqa_anneal(use, 2, M, 0, Rq, 2.0, g, 4, 78, 0, q, slE, &bE, bs);
        sgo_trotter_agreement(use, M, Rq, q, agree);
        h = mix(h, bE);
        for (int i = 0; i < Rq * M; ++i) h = mix(mix(h, slE[i]), agree[i]);
        for (int k = 0; k < M; ++k)
            for (int j = 0; j < n; ++j) h = mix(h, sgo_colour(use, M, j, k));
        free(q);
        free(bs);
    }
    if (!hmax) {
        sgo_adaptive_params p = {0.5, 1.25, 0.5, 3, 40, 20, 6};
        double bo[6], so[6];
        int64_t mo[6 * 3 * 2];
        int32_t len = sgo_adaptive_ladder(&lat, 3, &p, 79, bo, so, mo);
        h = mix(h, len);
        double f[4];
        sgo_instance_features(&lat, f);
        for (int k = 0; k < 4; ++k) h = mix(h, (int64_t)(f[k] * 1e9));
    }
    free(cmap);
    free(sp);
    free(J);
    free(hf);
    return h;
}

int main(void)
{
    uint64_t h = 1469598103934665603ull;
    h = run_case(4, 4, 4, 7, 0, 0, 2, h);
    h = run_case(5, 3, 2, 5, 1, 0, 4, h);
    h = run_case(3, 4, 5, 0, 0, 3, 2, h);
    h = run_case(2, 2, 2, 7, 0, 0, 1, h);
    h = run_case(1, 1, 6, 4, 0, 0, 4, h);
    h = run_case(6, 5, 1, 3, 1, 2, 2, h);
    /* thresholds, swap rule, Philox, MLP */
    for (int I = -8; I <= 8; ++I) h = mix(h, sgo_heat_threshold(0.7, I));
    for (int s = -6; s <= 6; ++s)
        for (int t = -2; t <= 2; t += 2) h = mix(h, sgo_sqa_threshold(4.0, 8, 1.3, s, t));
    h = mix(h, sgo_swap_accept(0.5, 0.9, -100, -90, 123456789u));
    uint32_t c[4] = {1, 2, 3, 4}, k[2] = {5, 6}, o[4];
    sgo_philox4x32_10(c, k, o);
    h = mix(mix(h, o[0]), o[3]);
    static double P[6625], G[6625], x[3 * 4], y[3 * 33], out[3 * 33];
    for (int i = 0; i < 6625; ++i) P[i] = ((i * 37) % 101 - 50) * 1e-3;
    for (int i = 0; i < 12; ++i) x[i] = (i % 5) * 0.3 - 0.5;
    for (int i = 0; i < 99; ++i) y[i] = -0.2 + 0.01 * i;
    double loss = sgo_mlp_loss_grad(P, x, y, 3, G, out);
    h = mix(h, (int64_t)(loss * 1e12));
    h = mix(h, (int64_t)(sgo_sigma_from_moments(10, 30, 5) * 1e12));
    printf("oracle checksum %016llx\n", (unsigned long long)h);
    return 0;
}
