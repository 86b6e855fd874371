/*
 * sg_oracle.h -- plain CPU oracle for the spin-glass Monte Carlo hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no source with the HIP path.
 *
 * Every routine here is the slow, literal form of a step of the method in
 * "Pushing the Boundary of Quantum Advantage in Hard Combinatorial
 * Optimization with Probabilistic Computers" (arXiv:2503.10302):
 *   - p-bit synapse and neuron, Eqs. (5)-(6); Boltzmann law, Eqs. (7)-(8);
 *   - graph-coloured parallel update, Methods "Graph Coloring";
 *   - DT-SQA, Supplementary Eqs. S.1-S.3 and Algorithm S1;
 *   - APT + ICM, Eq. (4), Methods "APT details", Algorithm S2.
 * Points the paper leaves open are fixed by the readings listed with each
 * function (the same list is kept in the design notes of the repository).
 *
 * Floating point: every threshold is built in FP64 from libm tanh/exp/log;
 * this file must be compiled with -ffp-contract=off and without fast-math.
 */
#ifndef SG_ORACLE_H
#define SG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Random-stream tags (low 4 bits of counter word 3). */
enum {
    SGO_TAG_APT_INIT = 1,
    SGO_TAG_APT_SWEEP = 2,
    SGO_TAG_SWAP = 3,
    SGO_TAG_ICM_PAIR = 4,
    SGO_TAG_ICM_PICK = 5,
    SGO_TAG_SQA_INIT = 6,
    SGO_TAG_SQA_SWEEP = 7,
    SGO_TAG_ADAPT_INIT = 8,
    SGO_TAG_ADAPT_SWEEP = 9
};

typedef struct {
    int32_t Lx, Ly, Lz;
    uint32_t periodic;   /* bit0 = x, bit1 = y, bit2 = z */
    const int8_t *J;     /* [Lz][Ly][Lx][3]: bond from site j to its +x,+y,+z neighbour */
    const int8_t *h;     /* [n] or NULL (all zero) */
    const int8_t *colour;   /* [n] colour of every site (a proper colouring of the bonds with
                               J != 0, values 0 .. n_map_colours - 1), or NULL: closed form */
    int32_t n_map_colours;
} sgo_lattice;

/* ---- random numbers: Philox4x32-10 (Salmon et al., SC'11) ---- */
void sgo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t sgo_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                  uint32_t inst, uint32_t tag, int word);

/* ---- lattice geometry ---- */
int32_t sgo_n_sites(const sgo_lattice *lat);
int32_t sgo_neighbour(const sgo_lattice *lat, int32_t j, int32_t axis, int32_t dir);
int32_t sgo_bond(const sgo_lattice *lat, int32_t j, int32_t axis, int32_t dir);
int32_t sgo_n_colours(const sgo_lattice *lat, int32_t M);
int32_t sgo_colour(const sgo_lattice *lat, int32_t M, int32_t j, int32_t k);
int32_t sgo_local_field(const sgo_lattice *lat, const int8_t *spins, int32_t j);
int64_t sgo_energy(const sgo_lattice *lat, const int8_t *spins);

/* ---- acceptance thresholds (FP64 -> uint32) ---- */
uint32_t sgo_heat_threshold(double beta, int32_t I);
uint32_t sgo_sqa_threshold(double beta, int32_t M, double gamma, int32_t s, int32_t tau);
int32_t sgo_swap_accept(double beta_lo, double beta_hi, int64_t E_lo, int64_t E_hi, uint32_t u);

/* ---- APT (one instance, n_slots = n_beta * R_lab replicas, spins [slot][n]) ---- */
void sgo_apt_init(const sgo_lattice *lat, uint32_t inst, int32_t n_slots, uint64_t seed,
                  uint32_t tag, int8_t *spins);
void sgo_apt_sweep(const sgo_lattice *lat, uint32_t inst, int32_t n_slots,
                   const double *slot_beta, uint64_t seed, uint32_t tag, uint32_t t,
                   int8_t *spins);
int32_t sgo_apt_icm(const sgo_lattice *lat, uint32_t inst, int32_t n_beta, int32_t R_lab,
                    const double *beta, double cutoff, int32_t pairs_per_call, uint64_t seed,
                    uint32_t a, int8_t *spins, int32_t *info);
void sgo_apt_swap(uint32_t inst, int32_t n_beta, int32_t R_lab, const double *beta,
                  uint64_t seed, uint32_t a, int32_t n, int8_t *spins, int64_t *E,
                  int32_t *accepted);
int32_t sgo_apt_run(const sgo_lattice *lat, uint32_t inst, int32_t n_beta, int32_t R_lab,
                    const double *beta, uint64_t seed, int64_t n_cycles,
                    int32_t sweeps_per_swap, double icm_cutoff, int32_t icm_pairs,
                    int32_t record_every, uint32_t *counters, int8_t *spins, int64_t *E,
                    int64_t *best, int64_t *best_trace, int64_t *accept_count);

/* ---- DT-SQA (one instance, replicas r0 .. r0+R-1, spins [R][M][n]) ---- */
void sgo_sqa_init(const sgo_lattice *lat, uint32_t inst, int32_t M, int32_t r0, int32_t R,
                  uint64_t seed, int8_t *spins);
void sgo_sqa_step(const sgo_lattice *lat, uint32_t inst, int32_t M, int32_t r0, int32_t R,
                  double beta, double gamma, uint64_t seed, uint32_t t, int8_t *spins);
void sgo_sqa_anneal(const sgo_lattice *lat, uint32_t inst, int32_t M, int32_t r0, int32_t R,
                    double beta, const double *gamma, int32_t n_steps, uint64_t seed, uint32_t t0,
                    int8_t *spins, int64_t *slice_E, int64_t *best_E, int8_t *best_state);

/* Trotter-direction correlation: agree[r][k] = #{i : s_{i,0} = s_{i,k}} in replica r. */
void sgo_trotter_agreement(const sgo_lattice *lat, int32_t M, int32_t R, const int8_t *spins,
                           int32_t *agree);

/* ---- adaptive beta ladder (Algorithm S2, preprocessing loop) ---- */
typedef struct {
    double beta0, alpha, tol;
    int32_t n_chains, sweeps, tail, max_steps;
} sgo_adaptive_params;
int32_t sgo_adaptive_ladder(const sgo_lattice *lat, uint32_t inst, const sgo_adaptive_params *p,
                            uint64_t seed, double *beta_out, double *sigma_out,
                            int64_t *moments_out);
double sgo_sigma_from_moments(int64_t S1, int64_t S2, int64_t N);

/* ---- ladder-predictor MLP, FP64 reference ---- */
void sgo_instance_features(const sgo_lattice *lat, double *f4);
double sgo_mlp_loss_grad(const double *params, const double *x, const double *y, int32_t batch,
                         double *grad, double *out);

#ifdef __cplusplus
}
#endif
#endif
