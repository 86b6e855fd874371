/*
 * sg_oracle.c -- plain CPU oracle (TEST INFRASTRUCTURE ONLY; see sg_oracle.h).
 *
 * Slow on purpose: loops in the order the paper describes them, no blocking,
 * no fusion, no bit tricks.  Compile with -O2 -ffp-contract=off (no fast-math).
 */
#include "sg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, as published by Salmon, Moraes, Dror and Shaw (SC'11):     */
/* ten rounds of two 32x32->64 multiplies with the two round multipliers,    */
/* the Weyl key schedule between rounds.                                     */
/* ------------------------------------------------------------------------- */
void sgo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One 32-bit word of the stream: key = (seed lo, seed hi),
 * counter = (c0, c1, c2, inst << 4 | tag). */
uint32_t sgo_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                  uint32_t inst, uint32_t tag, int word)
{
    uint32_t ctr[4] = {c0, c1, c2, (inst << 4) | (tag & 15u)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    sgo_philox4x32_10(ctr, key, out);
    return out[word & 3];
}

/* ------------------------------------------------------------------------- */
/* Geometry: site j = x + Lx*(y + Ly*z); J[3*j+a] couples j to its +a        */
/* neighbour.  Open axes have no bond across the boundary; an axis of length */
/* one has no neighbours at all.                                             */
/* ------------------------------------------------------------------------- */
int32_t sgo_n_sites(const sgo_lattice *lat) { return lat->Lx * lat->Ly * lat->Lz; }

static int32_t axis_len(const sgo_lattice *lat, int32_t a)
{
    return a == 0 ? lat->Lx : (a == 1 ? lat->Ly : lat->Lz);
}

static int32_t axis_coord(const sgo_lattice *lat, int32_t j, int32_t a)
{
    if (a == 0) return j % lat->Lx;
    if (a == 1) return (j / lat->Lx) % lat->Ly;
    return j / (lat->Lx * lat->Ly);
}

static int32_t axis_stride(const sgo_lattice *lat, int32_t a)
{
    return a == 0 ? 1 : (a == 1 ? lat->Lx : lat->Lx * lat->Ly);
}

int32_t sgo_neighbour(const sgo_lattice *lat, int32_t j, int32_t a, int32_t dir)
{
    int32_t L = axis_len(lat, a);
    if (L < 2) return -1;
    int32_t c = axis_coord(lat, j, a);
    int32_t c2 = c + dir;
    if (c2 < 0 || c2 >= L) {
        if (!((lat->periodic >> a) & 1u)) return -1;
        c2 = (c2 + L) % L;
    }
    return j + (c2 - c) * axis_stride(lat, a);
}

/* Coupling on the bond from j towards direction dir along axis a (0 if absent). */
int32_t sgo_bond(const sgo_lattice *lat, int32_t j, int32_t a, int32_t dir)
{
    int32_t nb = sgo_neighbour(lat, j, a, dir);
    if (nb < 0) return 0;
    return dir > 0 ? lat->J[3 * j + a] : lat->J[3 * nb + a];
}

/* ------------------------------------------------------------------------- */
/* Colouring (Methods, "Graph Coloring"): neighbours must differ in colour.  */
/* Every neighbour relation changes exactly one coordinate, so a colour that */
/* is a sum of per-axis labels modulo C is proper when each axis label       */
/* changes between neighbours modulo C.  With every periodic axis of even    */
/* length (the Trotter ring of M slices counts as a periodic axis) the       */
/* lattice is bipartite and C = 2 with label i mod 2.  Otherwise C = 3 with  */
/* label i mod 2, except 2 at the last site of an odd periodic axis.         */
/* M = 0 means no Trotter axis (APT).                                        */
/* ------------------------------------------------------------------------- */
static int odd_ring(const sgo_lattice *lat, int32_t a)
{
    int32_t L = axis_len(lat, a);
    return ((lat->periodic >> a) & 1u) && L >= 3 && (L & 1);
}

/* With a given colour map c(j) (a proper colouring of the coupled sites, e.g. DSATUR's for an
 * irregular graph, Methods "Graph Coloring") the Trotter label t(k) is added modulo
 * C = max(map colours, 2 for an even ring, 3 for an odd one): spatial neighbours share t
 * and differ in c; Trotter neighbours share c and differ in t by 1 or 2. */
static int32_t trotter_label(int32_t M, int32_t k)
{
    if (M <= 0) return 0;
    return ((M & 1) && k == M - 1) ? 2 : (k & 1);
}

int32_t sgo_n_colours(const sgo_lattice *lat, int32_t M)
{
    if (lat->colour) {
        int32_t C = lat->n_map_colours;
        if (M > 0 && C < ((M & 1) ? 3 : 2)) C = (M & 1) ? 3 : 2;
        return C;
    }
    int three = odd_ring(lat, 0) || odd_ring(lat, 1) || odd_ring(lat, 2);
    if (M > 0 && (M & 1)) three = 1;
    return three ? 3 : 2;
}

int32_t sgo_colour(const sgo_lattice *lat, int32_t M, int32_t j, int32_t k)
{
    int32_t C = sgo_n_colours(lat, M);
    if (lat->colour) return (lat->colour[j] + trotter_label(M, k)) % C;
    int32_t sum = 0;
    for (int32_t a = 0; a < 3; ++a) {
        int32_t c = axis_coord(lat, j, a);
        if (C == 3 && odd_ring(lat, a) && c == axis_len(lat, a) - 1) sum += 2;
        else sum += c & 1;
    }
    if (M > 0) {
        if (C == 3 && (M & 1) && k == M - 1) sum += 2;
        else sum += k & 1;
    }
    return sum % C;
}

/* Eq. (5): I_j = sum over neighbours of J_jk s_k, plus h_j. */
int32_t sgo_local_field(const sgo_lattice *lat, const int8_t *s, int32_t j)
{
    int32_t I = lat->h ? lat->h[j] : 0;
    for (int32_t a = 0; a < 3; ++a) {
        for (int32_t dir = -1; dir <= 1; dir += 2) {
            int32_t nb = sgo_neighbour(lat, j, a, dir);
            if (nb >= 0) I += sgo_bond(lat, j, a, dir) * s[nb];
        }
    }
    return I;
}

/* Eq. (1) / Eq. (8): E = - sum over bonds J s s - sum h s (each bond once). */
int64_t sgo_energy(const sgo_lattice *lat, const int8_t *s)
{
    int64_t E = 0;
    int32_t n = sgo_n_sites(lat);
    for (int32_t j = 0; j < n; ++j) {
        for (int32_t a = 0; a < 3; ++a) {
            int32_t nb = sgo_neighbour(lat, j, a, +1);
            if (nb >= 0) E -= (int64_t)lat->J[3 * j + a] * s[j] * s[nb];
        }
        if (lat->h) E -= (int64_t)lat->h[j] * s[j];
    }
    return E;
}

/* ------------------------------------------------------------------------- */
/* Thresholds.  Eq. (6): s = sgn(tanh(beta I) - r), r uniform in [-1,1], so  */
/* P(s = +1) = (1 + tanh(beta I))/2.  With u a uniform 32-bit word the       */
/* update is s = +1 iff u < T, T = floor(P * 2^32) (saturated at 2^32 - 1).  */
/* ------------------------------------------------------------------------- */
static uint32_t prob_to_threshold(double p)
{
    if (p >= 1.0) return 0xFFFFFFFFu;
    return (uint32_t)(p * 4294967296.0);
}

uint32_t sgo_heat_threshold(double beta, int32_t I)
{
    double x = beta * (double)I;
    double p = 0.5 * (1.0 + tanh(x));
    return prob_to_threshold(p);
}

/* Supplementary Eq. S.3 with M Trotter slices: J_par = J/M, h/M per slice,
 * J_perp = -(1/(2 beta)) ln tanh(beta Gamma / M).  The Gibbs argument for a
 * spin with spatial field s (J/M and h/M folded in as beta/M) and Trotter sum
 * tau = s(k-1) + s(k+1) is (beta/M) s + K tau with K = beta J_perp. */
uint32_t sgo_sqa_threshold(double beta, int32_t M, double gamma, int32_t s, int32_t tau)
{
    double K = -0.5 * log(tanh(beta * gamma / (double)M));
    double x = (beta / (double)M) * (double)s + K * (double)tau;
    double p = 0.5 * (1.0 + tanh(x));
    return prob_to_threshold(p);
}

/* Eq. (4): accept with probability min(1, exp(dbeta * dE)),
 * dbeta = beta_hi - beta_lo > 0, dE = E_hi - E_lo. */
int32_t sgo_swap_accept(double beta_lo, double beta_hi, int64_t E_lo, int64_t E_hi, uint32_t u)
{
    double x = (beta_hi - beta_lo) * (double)(E_hi - E_lo);
    if (x >= 0.0) return 1;
    double e = exp(x) * 4294967296.0;
    uint32_t T = (uint32_t)e;
    return u < T;
}

/* ------------------------------------------------------------------------- */
/* APT replicas.  Slot s = b * R_lab + l holds the replica at inverse        */
/* temperature index b with ICM label l.                                     */
/* ------------------------------------------------------------------------- */
void sgo_apt_init(const sgo_lattice *lat, uint32_t inst, int32_t n_slots, uint64_t seed,
                  uint32_t tag, int8_t *spins)
{
    int32_t n = sgo_n_sites(lat);
    for (int32_t s = 0; s < n_slots; ++s)
        for (int32_t j = 0; j < n; ++j) {
            uint32_t w = sgo_word(seed, (uint32_t)j, 0u, (uint32_t)s >> 2, inst, tag, s & 3);
            spins[(int64_t)s * n + j] = (w < 0x80000000u) ? 1 : -1;
        }
}

/* One sweep (Algorithm S2, "p-computer"): for each colour, every p-bit of
 * that colour solves Eqs. (5)-(6) using the current state of the others. */
void sgo_apt_sweep(const sgo_lattice *lat, uint32_t inst, int32_t n_slots,
                   const double *slot_beta, uint64_t seed, uint32_t tag, uint32_t t,
                   int8_t *spins)
{
    int32_t n = sgo_n_sites(lat);
    int32_t C = sgo_n_colours(lat, 0);
    for (int32_t c = 0; c < C; ++c)
        for (int32_t j = 0; j < n; ++j) {
            if (sgo_colour(lat, 0, j, 0) != c) continue;
            for (int32_t s = 0; s < n_slots; ++s) {
                int8_t *x = spins + (int64_t)s * n;
                int32_t I = sgo_local_field(lat, x, j);
                uint32_t T = sgo_heat_threshold(slot_beta[s], I);
                uint32_t u = sgo_word(seed, (uint32_t)j, t, (uint32_t)s >> 2, inst, tag, s & 3);
                x[j] = (u < T) ? 1 : -1;
            }
        }
}

/* ICMop (Algorithm S2): overlap, one cluster of overlap -1 chosen through a
 * uniformly drawn seed site, then either the cluster is flipped in both
 * replicas or, when it holds more than half of the sites, one replica chosen
 * at random is flipped entirely.  Pairs: 2 labels -> (0,1); 4 labels -> one
 * of the three perfect matchings drawn at random (Methods, "APT details").
 * pairs_per_call (4 labels): 2 moves both pairs of the matching, 1 moves one of
 * the two, drawn at random (the Supplementary comparison of one and two ICMs per
 * sweep); the pair not moved gets the "not applied" record.
 * info[(b * npair + pi) * 4 + {0..3}] = (m, seed site, |C|, branch) with
 * branch 0 = cluster, 1 = whole first replica, 2 = whole second; -1 when the
 * temperature is below the cutoff.  Returns 0, or -5 when some pair would be
 * moved and h is non-zero (the whole-replica branch keeps the energy only for
 * h = 0); with no temperature at or above the cutoff the call is a no-op. */
static const int32_t PAIRINGS[3][2][2] = {{{0, 1}, {2, 3}}, {{0, 2}, {1, 3}}, {{0, 3}, {1, 2}}};

int32_t sgo_apt_icm(const sgo_lattice *lat, uint32_t inst, int32_t n_beta, int32_t R_lab,
                    const double *beta, double cutoff, int32_t pairs_per_call, uint64_t seed,
                    uint32_t a, int8_t *spins, int32_t *info)
{
    int32_t n = sgo_n_sites(lat);
    if (R_lab != 2 && R_lab != 4) return 0;
    int32_t applies = 0;
    for (int32_t b = 0; b < n_beta; ++b) applies |= beta[b] >= cutoff;
    if (lat->h && applies)
        for (int32_t j = 0; j < n; ++j)
            if (lat->h[j] != 0) return -5;
    int32_t npair = R_lab / 2;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    char *inC = (char *)malloc((size_t)n);
    for (int32_t b = 0; b < n_beta; ++b) {
        int32_t pairing = 0, only = -1;
        if (R_lab == 4) {
            uint32_t w = sgo_word(seed, (uint32_t)b, a, 0u, inst, SGO_TAG_ICM_PAIR, 0);
            pairing = (int32_t)(((uint64_t)w * 3u) >> 32);
            if (pairs_per_call == 1)
                only = (int32_t)(sgo_word(seed, (uint32_t)b, a, 0u, inst, SGO_TAG_ICM_PAIR, 1) >> 31);
        }
        for (int32_t pi = 0; pi < npair; ++pi) {
            int32_t *rec = info ? info + ((int64_t)b * npair + pi) * 4 : NULL;
            if (!(beta[b] >= cutoff) || (only >= 0 && pi != only)) {
                if (rec) rec[0] = rec[1] = rec[2] = rec[3] = -1;
                continue;
            }
            int32_t la = PAIRINGS[pairing][pi][0], lb = PAIRINGS[pairing][pi][1];
            int8_t *A = spins + (int64_t)(b * R_lab + la) * n;
            int8_t *B = spins + (int64_t)(b * R_lab + lb) * n;
            uint32_t pick = (uint32_t)(b * npair + pi);
            uint32_t w0 = sgo_word(seed, pick, a, 0u, inst, SGO_TAG_ICM_PICK, 0);
            uint32_t w1 = sgo_word(seed, pick, a, 0u, inst, SGO_TAG_ICM_PICK, 1);
            /* overlap q_j = A_j B_j; m = number of sites with q = -1 */
            int32_t m = 0;
            for (int32_t j = 0; j < n; ++j) m += (A[j] != B[j]);
            if (m == 0) {
                if (rec) { rec[0] = 0; rec[1] = -1; rec[2] = 0; rec[3] = 0; }
                continue;
            }
            int32_t k = (int32_t)(((uint64_t)w0 * (uint64_t)m) >> 32);
            int32_t seed_site = -1;
            for (int32_t j = 0, cnt = 0; j < n; ++j)
                if (A[j] != B[j]) {
                    if (cnt == k) { seed_site = j; break; }
                    ++cnt;
                }
            /* breadth-first search over present bonds inside q = -1 */
            memset(inC, 0, (size_t)n);
            int32_t head = 0, tail = 0;
            queue[tail++] = seed_site;
            inC[seed_site] = 1;
            while (head < tail) {
                int32_t j = queue[head++];
                for (int32_t ax = 0; ax < 3; ++ax)
                    for (int32_t dir = -1; dir <= 1; dir += 2) {
                        int32_t nb = sgo_neighbour(lat, j, ax, dir);
                        if (nb < 0 || sgo_bond(lat, j, ax, dir) == 0) continue;
                        if (inC[nb] || A[nb] == B[nb]) continue;
                        inC[nb] = 1;
                        queue[tail++] = nb;
                    }
            }
            int32_t size = tail, branch;
            if (2 * size > n) {
                int8_t *X = ((w1 >> 31) == 0) ? A : B;
                branch = ((w1 >> 31) == 0) ? 1 : 2;
                for (int32_t j = 0; j < n; ++j) X[j] = (int8_t)-X[j];
            } else {
                branch = 0;
                for (int32_t q = 0; q < size; ++q) {
                    int32_t j = queue[q];
                    A[j] = (int8_t)-A[j];
                    B[j] = (int8_t)-B[j];
                }
            }
            if (rec) { rec[0] = m; rec[1] = seed_site; rec[2] = size; rec[3] = branch; }
        }
    }
    free(queue);
    free(inC);
    return 0;
}

/* Replica exchange (Eq. 4; Methods "APT details"): attempt a = 1, 2, ...;
 * odd a tries index pairs (0,1),(2,3),..., even a tries (1,2),(3,4),...;
 * each label is its own tempering chain.  accepted[b * R_lab + l] is 1 / 0
 * for an attempted pair (b, b+1) and -1 when the pair was not attempted. */
void sgo_apt_swap(uint32_t inst, int32_t n_beta, int32_t R_lab, const double *beta,
                  uint64_t seed, uint32_t a, int32_t n, int8_t *spins, int64_t *E,
                  int32_t *accepted)
{
    if (accepted)
        for (int32_t i = 0; i < (n_beta - 1) * R_lab; ++i) accepted[i] = -1;
    int32_t first = (a & 1u) ? 0 : 1;
    int8_t *tmp = (int8_t *)malloc((size_t)n);
    for (int32_t b = first; b + 1 < n_beta; b += 2)
        for (int32_t l = 0; l < R_lab; ++l) {
            int32_t s0 = b * R_lab + l, s1 = (b + 1) * R_lab + l;
            uint32_t u = sgo_word(seed, (uint32_t)(b * R_lab + l), a, 0u, inst, SGO_TAG_SWAP, 0);
            int32_t acc = sgo_swap_accept(beta[b], beta[b + 1], E[s0], E[s1], u);
            if (acc) {
                memcpy(tmp, spins + (int64_t)s0 * n, (size_t)n);
                memcpy(spins + (int64_t)s0 * n, spins + (int64_t)s1 * n, (size_t)n);
                memcpy(spins + (int64_t)s1 * n, tmp, (size_t)n);
                int64_t e = E[s0]; E[s0] = E[s1]; E[s1] = e;
            }
            if (accepted) accepted[b * R_lab + l] = acc;
        }
    free(tmp);
}

/* APT main loop of Algorithm S2 for one instance.  One cycle =
 * sweeps_per_swap sweeps, one ICM call (pairs at beta >= cutoff, icm_pairs as
 * in sgo_apt_icm), energies,
 * one swap attempt, then the running minimum energy.  counters =
 * {sweeps done, ICM calls done, swap attempts done} are read and advanced.
 * accept_count[(n_beta-1) * R_lab] accumulates accepted swaps (nullable). */
int32_t sgo_apt_run(const sgo_lattice *lat, uint32_t inst, int32_t n_beta, int32_t R_lab,
                    const double *beta, uint64_t seed, int64_t n_cycles,
                    int32_t sweeps_per_swap, double icm_cutoff, int32_t icm_pairs,
                    int32_t record_every, uint32_t *counters, int8_t *spins, int64_t *E,
                    int64_t *best, int64_t *best_trace, int64_t *accept_count)
{
    int32_t n = sgo_n_sites(lat);
    int32_t n_slots = n_beta * R_lab;
    double *slot_beta = (double *)malloc(sizeof(double) * (size_t)n_slots);
    int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * (size_t)((n_beta - 1) * R_lab + 1));
    for (int32_t s = 0; s < n_slots; ++s) slot_beta[s] = beta[s / R_lab];
    int32_t rc = 0;
    for (int64_t cyc = 0; cyc < n_cycles; ++cyc) {
        for (int32_t i = 0; i < sweeps_per_swap; ++i)
            sgo_apt_sweep(lat, inst, n_slots, slot_beta, seed, SGO_TAG_APT_SWEEP,
                          counters[0]++, spins);
        rc = sgo_apt_icm(lat, inst, n_beta, R_lab, beta, icm_cutoff, icm_pairs, seed,
                         ++counters[1], spins, NULL);
        if (rc) break;
        for (int32_t s = 0; s < n_slots; ++s) E[s] = sgo_energy(lat, spins + (int64_t)s * n);
        sgo_apt_swap(inst, n_beta, R_lab, beta, seed, ++counters[2], n, spins, E, acc);
        for (int32_t s = 0; s < n_slots; ++s)
            if (E[s] < *best) *best = E[s];
        if (accept_count)
            for (int32_t i = 0; i < (n_beta - 1) * R_lab; ++i) accept_count[i] += (acc[i] == 1);
        if (record_every > 0 && best_trace && (cyc + 1) % record_every == 0)
            best_trace[(cyc + 1) / record_every - 1] = *best;
    }
    free(slot_beta);
    free(acc);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* DT-SQA (Algorithm S1).  Spins [r][k][n]: replica r0 + r, Trotter slice k.  */
/* Slice k = 2 hh + p at site j draws word (hh & 3) of the block with        */
/* counter words 0 and 2 equal to 2 j + p and (r << 16) | (hh >> 2).         */
/* ------------------------------------------------------------------------- */
static uint32_t sqa_c0(int32_t j, int32_t k) { return ((uint32_t)j << 1) | ((uint32_t)k & 1u); }

static uint32_t sqa_c2(int32_t r, int32_t k)
{
    uint32_t hh = (uint32_t)k >> 1;
    return ((uint32_t)r << 16) | (hh >> 2);
}

void sgo_sqa_init(const sgo_lattice *lat, uint32_t inst, int32_t M, int32_t r0, int32_t R,
                  uint64_t seed, int8_t *spins)
{
    int32_t n = sgo_n_sites(lat);
    for (int32_t r = 0; r < R; ++r)
        for (int32_t k = 0; k < M; ++k)
            for (int32_t j = 0; j < n; ++j) {
                uint32_t w = sgo_word(seed, sqa_c0(j, k), 0u, sqa_c2(r0 + r, k), inst,
                                      SGO_TAG_SQA_INIT, (k >> 1) & 3);
                spins[((int64_t)r * M + k) * n + j] = (w < 0x80000000u) ? 1 : -1;
            }
}

/* One annealing step: the transverse coupling follows Gamma, then one
 * coloured sweep of the (d+1)-dimensional lattice. */
void sgo_sqa_step(const sgo_lattice *lat, uint32_t inst, int32_t M, int32_t r0, int32_t R,
                  double beta, double gamma, uint64_t seed, uint32_t t, int8_t *spins)
{
    int32_t n = sgo_n_sites(lat);
    int32_t C = sgo_n_colours(lat, M);
    for (int32_t c = 0; c < C; ++c)
        for (int32_t k = 0; k < M; ++k)
            for (int32_t j = 0; j < n; ++j) {
                if (sgo_colour(lat, M, j, k) != c) continue;
                for (int32_t r = 0; r < R; ++r) {
                    int8_t *slice = spins + ((int64_t)r * M + k) * n;
                    int8_t up = spins[((int64_t)r * M + (k + M - 1) % M) * n + j];
                    int8_t dn = spins[((int64_t)r * M + (k + 1) % M) * n + j];
                    int32_t s = sgo_local_field(lat, slice, j);
                    uint32_t T = sgo_sqa_threshold(beta, M, gamma, s, up + dn);
                    uint32_t u = sgo_word(seed, sqa_c0(j, k), t, sqa_c2(r0 + r, k), inst,
                                          SGO_TAG_SQA_SWEEP, (k >> 1) & 3);
                    slice[j] = (u < T) ? 1 : -1;
                }
            }
}

/* Algorithm S1 main loop, then the energy of every slice under the original
 * couplings and the minimum (ties -> lowest r*M + k). */
void sgo_sqa_anneal(const sgo_lattice *lat, uint32_t inst, int32_t M, int32_t r0, int32_t R,
                    double beta, const double *gamma, int32_t n_steps, uint64_t seed, uint32_t t0,
                    int8_t *spins, int64_t *slice_E, int64_t *best_E, int8_t *best_state)
{
    int32_t n = sgo_n_sites(lat);
    for (int32_t t = 0; t < n_steps; ++t)
        sgo_sqa_step(lat, inst, M, r0, R, beta, gamma[t], seed, t0 + (uint32_t)t, spins);
    int64_t best = 0;
    int64_t arg = -1;
    for (int64_t q = 0; q < (int64_t)R * M; ++q) {
        int64_t e = sgo_energy(lat, spins + q * n);
        if (slice_E) slice_E[q] = e;
        if (arg < 0 || e < best) { best = e; arg = q; }
    }
    if (best_E) *best_E = best;
    if (best_state) memcpy(best_state, spins + arg * n, (size_t)n);
}

/* Correlation along the Trotter direction (Supplementary, correlation-length
 * figure): C_r = (1/n) sum_i s_{i,0} s_{i,r}.  Returned exactly as the number of
 * sites where slice r agrees with slice 0, agree[r][k] for replica r, slice k
 * (C_k = (2 agree - n) / n). */
void sgo_trotter_agreement(const sgo_lattice *lat, int32_t M, int32_t R, const int8_t *spins,
                           int32_t *agree)
{
    int32_t n = sgo_n_sites(lat);
    for (int32_t r = 0; r < R; ++r)
        for (int32_t k = 0; k < M; ++k) {
            const int8_t *s0 = spins + ((int64_t)r * M) * n;
            const int8_t *sk = spins + ((int64_t)r * M + k) * n;
            int32_t a = 0;
            for (int32_t i = 0; i < n; ++i) a += (s0[i] * sk[i] > 0);
            agree[r * M + k] = a;
        }
}

/* ------------------------------------------------------------------------- */
/* Adaptive inverse-temperature ladder (Algorithm S2 preprocessing; Methods  */
/* "APT details"): chains run at beta_t, each chain's energy spread over the */
/* last `tail` sweeps, sigma_E = mean over chains, beta_{t+1} = beta_t +     */
/* alpha / sigma_E, stop once sigma_E < tol.  The spread is the sample       */
/* standard deviation, formed from exact integer moments.                    */
/* ------------------------------------------------------------------------- */
double sgo_sigma_from_moments(int64_t S1, int64_t S2, int64_t N)
{
    int64_t num = N * S2 - S1 * S1;
    double var = (double)num / ((double)N * (double)(N - 1));
    return sqrt(var);
}

int32_t sgo_adaptive_ladder(const sgo_lattice *lat, uint32_t inst, const sgo_adaptive_params *p,
                            uint64_t seed, double *beta_out, double *sigma_out,
                            int64_t *moments_out)
{
    int32_t n = sgo_n_sites(lat);
    int32_t nc = p->n_chains;
    int8_t *spins = (int8_t *)malloc((size_t)nc * (size_t)n);
    double *cb = (double *)malloc(sizeof(double) * (size_t)nc);
    int64_t *S1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    int64_t *S2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    sgo_apt_init(lat, inst, nc, seed, SGO_TAG_ADAPT_INIT, spins);
    double beta_t = p->beta0;
    uint32_t tglob = 0;
    int32_t len = 0;
    for (int32_t step = 0; step < p->max_steps; ++step) {
        for (int32_t c = 0; c < nc; ++c) { cb[c] = beta_t; S1[c] = 0; S2[c] = 0; }
        for (int32_t i = 0; i < p->sweeps; ++i) {
            sgo_apt_sweep(lat, inst, nc, cb, seed, SGO_TAG_ADAPT_SWEEP, tglob++, spins);
            if (i >= p->sweeps - p->tail)
                for (int32_t c = 0; c < nc; ++c) {
                    int64_t e = sgo_energy(lat, spins + (int64_t)c * n);
                    S1[c] += e;
                    S2[c] += e * e;
                }
        }
        double sum = 0.0;
        for (int32_t c = 0; c < nc; ++c) sum += sgo_sigma_from_moments(S1[c], S2[c], p->tail);
        double sigma = sum / (double)nc;
        if (moments_out)
            for (int32_t c = 0; c < nc; ++c) {
                moments_out[((int64_t)step * nc + c) * 2 + 0] = S1[c];
                moments_out[((int64_t)step * nc + c) * 2 + 1] = S2[c];
            }
        beta_out[step] = beta_t;
        if (sigma_out) sigma_out[step] = sigma;
        len = step + 1;
        if (sigma < p->tol) break;
        beta_t = beta_t + p->alpha / sigma;
    }
    free(spins); free(cb); free(S1); free(S2);
    return len;
}

/* ------------------------------------------------------------------------- */
/* Ladder-predictor network (not part of the paper; a project component):    */
/* 4 instance features -> 64 -> 64 (ReLU) -> 33 outputs o.  Predicted log   */
/* betas: y_0 = o_0, y_k = y_{k-1} + softplus(o_k) for k = 1..31; y_32 =     */
/* o_32 is the log ICM cutoff.  Loss = mean squared error over the 33 values.*/
/* Parameter layout: W1[64][4] b1[64] W2[64][64] b2[64] W3[33][64] b3[33].   */
/* ------------------------------------------------------------------------- */
void sgo_instance_features(const sgo_lattice *lat, double *f)
{
    int32_t n = sgo_n_sites(lat);
    double sum = 0.0, sum2 = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        int32_t c = 0;
        for (int32_t a = 0; a < 3; ++a)
            for (int32_t dir = -1; dir <= 1; dir += 2) c += sgo_bond(lat, j, a, dir);
        double v = fabs((double)c);
        sum += v;
        sum2 += v * v;
    }
    double mean = sum / (double)n;
    double var = sum2 / (double)n - mean * mean;
    int64_t plaq = 0, frus = 0;
    for (int32_t j = 0; j < n; ++j)
        for (int32_t a = 0; a < 3; ++a)
            for (int32_t b = a + 1; b < 3; ++b) {
                int32_t ja = sgo_neighbour(lat, j, a, +1);
                int32_t jb = sgo_neighbour(lat, j, b, +1);
                if (ja < 0 || jb < 0) continue;
                int32_t p1 = sgo_bond(lat, j, a, +1), p2 = sgo_bond(lat, ja, b, +1);
                int32_t p3 = sgo_bond(lat, jb, a, +1), p4 = sgo_bond(lat, j, b, +1);
                if (!p1 || !p2 || !p3 || !p4) continue;
                ++plaq;
                if (p1 * p2 * p3 * p4 < 0) ++frus;
            }
    f[0] = cbrt((double)n);
    f[1] = mean;
    f[2] = var;
    f[3] = plaq ? (double)frus / (double)plaq : 0.0;
}

static double softplus(double x) { return x > 30.0 ? x : log1p(exp(x)); }
static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

double sgo_mlp_loss_grad(const double *P, const double *x, const double *y, int32_t batch,
                         double *grad, double *out)
{
    enum { NI = 4, NH = 64, NO = 33 };
    const double *W1 = P, *b1 = W1 + NH * NI, *W2 = b1 + NH, *b2 = W2 + NH * NH;
    const double *W3 = b2 + NH, *b3 = W3 + NO * NH;
    double *gW1 = grad, *gb1 = gW1 + NH * NI, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH;
    double *gW3 = gb2 + NH, *gb3 = gW3 + NO * NH;
    if (grad) memset(grad, 0, sizeof(double) * (NH * NI + NH + NH * NH + NH + NO * NH + NO));
    double loss = 0.0;
    for (int32_t b = 0; b < batch; ++b) {
        const double *xb = x + b * NI;
        double z1[NH], a1[NH], z2[NH], a2[NH], o[NO], yp[NO];
        for (int i = 0; i < NH; ++i) {
            double acc = b1[i];
            for (int k = 0; k < NI; ++k) acc += W1[i * NI + k] * xb[k];
            z1[i] = acc;
            a1[i] = acc > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < NH; ++i) {
            double acc = b2[i];
            for (int k = 0; k < NH; ++k) acc += W2[i * NH + k] * a1[k];
            z2[i] = acc;
            a2[i] = acc > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < NO; ++i) {
            double acc = b3[i];
            for (int k = 0; k < NH; ++k) acc += W3[i * NH + k] * a2[k];
            o[i] = acc;
        }
        yp[0] = o[0];
        for (int i = 1; i < 32; ++i) yp[i] = yp[i - 1] + softplus(o[i]);
        yp[32] = o[32];
        if (out)
            for (int i = 0; i < NO; ++i) out[b * NO + i] = yp[i];
        if (!y) continue;
        double dy[NO];
        for (int i = 0; i < NO; ++i) {
            double d = yp[i] - y[b * NO + i];
            loss += d * d;
            dy[i] = 2.0 * d / (double)(batch * NO);
        }
        if (!grad) continue;
        double dO[NO];
        double suffix = 0.0;
        for (int i = 31; i >= 1; --i) {
            suffix += dy[i];
            dO[i] = sigmoid(o[i]) * suffix;
        }
        dO[0] = suffix + dy[0];
        dO[32] = dy[32];
        double da2[NH], dz2[NH], da1[NH], dz1[NH];
        for (int k = 0; k < NH; ++k) da2[k] = 0.0;
        for (int i = 0; i < NO; ++i) {
            gb3[i] += dO[i];
            for (int k = 0; k < NH; ++k) {
                gW3[i * NH + k] += dO[i] * a2[k];
                da2[k] += dO[i] * W3[i * NH + k];
            }
        }
        for (int k = 0; k < NH; ++k) { dz2[k] = z2[k] > 0.0 ? da2[k] : 0.0; da1[k] = 0.0; }
        for (int i = 0; i < NH; ++i) {
            gb2[i] += dz2[i];
            for (int k = 0; k < NH; ++k) {
                gW2[i * NH + k] += dz2[i] * a1[k];
                da1[k] += dz2[i] * W2[i * NH + k];
            }
        }
        for (int k = 0; k < NH; ++k) dz1[k] = z1[k] > 0.0 ? da1[k] : 0.0;
        for (int i = 0; i < NH; ++i) {
            gb1[i] += dz1[i];
            for (int k = 0; k < NI; ++k) gW1[i * NI + k] += dz1[i] * xb[k];
        }
    }
    return y ? loss / (double)(batch * NO) : 0.0;
}
