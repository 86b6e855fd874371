/*
 * Host-side paths of libsg under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * TEST INFRASTRUCTURE: built and run by tests/test_host_sanitizers.py on a machine without a
 * GPU.  It calls every entry point whose work is host code: the DSATUR colouring (checked
 * proper here), the instance features, the ladder repair, and context creation for both
 * methods with valid and invalid configurations.  Without a device a valid configuration
 * builds every host-side table (site records, colour classes, heat-bath and swap thresholds)
 * and stops at the first device call with SG_EHIP; invalid ones stop at their check.  The
 * outputs and status codes are folded into a checksum, printed on the last line, which must
 * equal that of the same driver linked against the ordinary build.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sg.h"

static uint64_t g_state = 0x2545F4914F6CDD1Dull;
static uint64_t g_sum = 0xCBF29CE484222325ull;   /* FNV-1a */

static uint32_t next_u32(void)
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (uint32_t)(g_state >> 32);
}

static void fold(const void *p, size_t n)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        g_sum ^= b[i];
        g_sum *= 0x100000001B3ull;
    }
}

static void fold_status(int32_t st)
{
    fold(&st, sizeof st);
    const char *msg = sg_last_error(NULL);
    if (msg) fold(msg, strlen(msg));
}

typedef struct {
    int Lx, Ly, Lz;
    unsigned periodic;
    double p_absent;
    int hmax;
} geom;

/* +-1 couplings (bonds across open boundaries and a fraction p_absent removed), fields in
 * [-hmax, hmax] when hmax > 0. */
static void make_lattice(const geom *g, int8_t **J, int8_t **h, sg_lattice *L)
{
    const int n = g->Lx * g->Ly * g->Lz;
    *J = (int8_t *)malloc((size_t)n * 3);
    *h = g->hmax > 0 ? (int8_t *)malloc((size_t)n) : NULL;
    for (int z = 0; z < g->Lz; ++z)
        for (int y = 0; y < g->Ly; ++y)
            for (int x = 0; x < g->Lx; ++x) {
                const int j = (z * g->Ly + y) * g->Lx + x;
                const int last[3] = {x == g->Lx - 1, y == g->Ly - 1, z == g->Lz - 1};
                const int len[3] = {g->Lx, g->Ly, g->Lz};
                for (int a = 0; a < 3; ++a) {
                    int8_t v = (next_u32() & 1u) ? 1 : -1;
                    if ((last[a] && !((g->periodic >> a) & 1u)) || len[a] < 2) v = 0;
                    if ((double)next_u32() / 4294967296.0 < g->p_absent) v = 0;
                    (*J)[3 * j + a] = v;
                }
                if (*h) (*h)[j] = (int8_t)((int)(next_u32() % (uint32_t)(2 * g->hmax + 1)) - g->hmax);
            }
    L->Lx = g->Lx;
    L->Ly = g->Ly;
    L->Lz = g->Lz;
    L->periodic = g->periodic;
    L->J = *J;
    L->h = *h;
}

static int neighbour(const sg_lattice *L, int j, int a)
{
    int c[3] = {j % L->Lx, (j / L->Lx) % L->Ly, j / (L->Lx * L->Ly)};
    const int len[3] = {L->Lx, L->Ly, L->Lz};
    c[a] = (c[a] + 1) % len[a];
    return (c[2] * L->Ly + c[1]) * L->Lx + c[0];
}

static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "host driver: %s\n", what);
        exit(1);
    }
}

int main(void)
{
    const geom geoms[] = {{4, 4, 4, 7, 0.0, 0},  {5, 5, 5, 7, 0.0, 0},   {6, 5, 4, 6, 0.0, 2},
                          {3, 2, 5, 0, 0.2, 0},  {15, 15, 12, 4, 0.0, 0}, {7, 6, 5, 7, 0.25, 0},
                          {1, 1, 1, 7, 0.0, 0},  {2, 1, 1, 1, 0.0, 3},   {15, 15, 15, 7, 0.0, 0}};
    const int ng = (int)(sizeof geoms / sizeof geoms[0]);
    sg_lattice lat[16];
    int8_t *Js[16], *hs[16], *cols[16];
    for (int g = 0; g < ng; ++g) {
        make_lattice(&geoms[g], &Js[g], &hs[g], &lat[g]);
        const int n = lat[g].Lx * lat[g].Ly * lat[g].Lz;
        cols[g] = (int8_t *)malloc((size_t)n);
        int32_t nc = 0;
        const int32_t st = sg_dsatur_colouring(&lat[g], cols[g], &nc);
        fold_status(st);
        check(st == SG_OK, "dsatur failed");
        for (int j = 0; j < n; ++j)
            for (int a = 0; a < 3; ++a)
                if (Js[g][3 * j + a] != 0)
                    check(cols[g][j] != cols[g][neighbour(&lat[g], j, a)], "dsatur colouring not proper");
        fold(cols[g], (size_t)n);
        fold(&nc, sizeof nc);
        double f[4];
        fold_status(sg_instance_features(&lat[g], 1, f));
        fold(f, sizeof f);
    }
    /* the ladder repair, in place and out of place, and its refusals */
    double beta[32], acc[31], lo[31], hi[31], out[32];
    for (int k = 0; k < 32; ++k) beta[k] = 0.4 * pow(8.0, k / 31.0);
    for (int b = 0; b < 31; ++b) {
        acc[b] = (double)(next_u32() % 1001u) / 1000.0;
        lo[b] = 0.15 + 0.001 * b;
        hi[b] = 0.45 + 0.001 * b;
    }
    fold_status(sg_ladder_repair(beta, acc, lo, hi, 32, 1.0, out));
    fold(out, sizeof out);
    fold_status(sg_ladder_repair(beta, acc, lo, hi, 32, 0.5, out));
    fold(out, sizeof out);
    memcpy(out, beta, sizeof beta);
    fold_status(sg_ladder_repair(out, acc, lo, hi, 32, 1.0, out));
    fold(out, sizeof out);
    fold_status(sg_ladder_repair(beta, acc, lo, hi, 1, 1.0, out));
    fold_status(sg_ladder_repair(beta, acc, hi, lo, 32, 1.0, out));
    fold_status(sg_ladder_repair(beta, acc, lo, hi, 32, 0.0, out));
    acc[3] = 2.0;
    fold_status(sg_ladder_repair(beta, acc, lo, hi, 32, 1.0, out));

    /* APT contexts: every instance, three per context in turn, closed-form and DSATUR colours */
    double ladder[3 * 32];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 32; ++k) ladder[32 * i + k] = 0.2 * pow(15.0, k / 31.0) + 0.01 * i;
    for (int g = 0; g + 2 < ng; ++g) {
        sg_config cfg;
        memset(&cfg, 0, sizeof cfg);
        cfg.mode = SG_APT;
        cfg.n_inst = 3;
        cfg.inst = &lat[g];
        cfg.n_beta = 32;
        cfg.beta = ladder;
        cfg.reps_per_beta = (g % 3 == 0) ? 4 : 2;
        cfg.seed = 1234u + (uint64_t)g;
        sg_ctx *ctx = NULL;
        const int8_t *const cm[3] = {cols[g], NULL, cols[g + 2]};
        int32_t st = sg_create_ex(&cfg, (g & 1) ? cm : NULL, &ctx);
        fold_status(st);
        if (st == SG_OK) sg_destroy(ctx);
        check(st == SG_EHIP || st == SG_OK || st == SG_EUNSUPPORTED, "APT create: unexpected status");
    }
    {   /* invalid APT configurations */
        sg_config cfg;
        memset(&cfg, 0, sizeof cfg);
        cfg.mode = SG_APT;
        cfg.n_inst = 1;
        cfg.inst = &lat[0];
        cfg.n_beta = 32;
        cfg.beta = ladder;
        cfg.reps_per_beta = 3;
        sg_ctx *ctx = NULL;
        fold_status(sg_create(&cfg, &ctx));
        cfg.reps_per_beta = 2;
        double bad[32];
        memcpy(bad, ladder, sizeof bad);
        bad[5] = bad[4];
        cfg.beta = bad;
        fold_status(sg_create(&cfg, &ctx));
        cfg.beta = ladder;
        int8_t *improper = (int8_t *)calloc(64, 1);   /* every site colour 0 */
        const int8_t *const cm[1] = {improper};
        fold_status(sg_create_ex(&cfg, cm, &ctx));
        improper[0] = 7;                               /* a value outside 0..3 */
        fold_status(sg_create_ex(&cfg, cm, &ctx));
        free(improper);
        cfg.n_inst = 0;
        fold_status(sg_create(&cfg, &ctx));
        fold_status(sg_create(NULL, &ctx));
        cfg.mode = 9;
        cfg.n_inst = 1;
        fold_status(sg_create(&cfg, &ctx));
    }
    /* DT-SQA contexts, valid and invalid */
    const int Ms[] = {2, 6, 16, 32, 60, 64};
    for (int q = 0; q < 6; ++q) {
        const int g = q % (ng - 2);
        sg_config cfg;
        memset(&cfg, 0, sizeof cfg);
        cfg.mode = SG_SQA;
        cfg.n_inst = 3;
        cfg.inst = &lat[g];
        cfg.M = Ms[q];
        cfg.R = 1 + 7 * q;
        cfg.sqa_beta = 0.5 * Ms[q];
        cfg.seed = 99u + (uint64_t)q;
        sg_ctx *ctx = NULL;
        const int8_t *const cm[3] = {NULL, cols[g + 1], NULL};
        int32_t st = sg_create_ex(&cfg, (q & 1) ? cm : NULL, &ctx);
        fold_status(st);
        if (st == SG_OK) sg_destroy(ctx);
        check(st == SG_EHIP || st == SG_OK, "SQA create: unexpected status");
    }
    {
        sg_config cfg;
        memset(&cfg, 0, sizeof cfg);
        cfg.mode = SG_SQA;
        cfg.n_inst = 1;
        cfg.inst = &lat[0];
        cfg.sqa_beta = 4.0;
        sg_ctx *ctx = NULL;
        cfg.R = 4;
        cfg.M = 66;
        fold_status(sg_create(&cfg, &ctx));
        cfg.M = 16;
        cfg.R = 0;
        fold_status(sg_create(&cfg, &ctx));
        cfg.R = 4;
        cfg.sqa_beta = -1.0;
        fold_status(sg_create(&cfg, &ctx));
    }
    for (int g = 0; g < ng; ++g) {
        free(Js[g]);
        free(hs[g]);
        free(cols[g]);
    }
    printf("libsg host checksum %016llx\n", (unsigned long long)g_sum);
    return 0;
}
