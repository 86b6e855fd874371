/*
 * sg.h -- C ABI of the MI355X spin-glass Monte Carlo library (libsg.so).
 *
 * The library runs the data-parallel hot path of the probabilistic-computer
 * solvers of arXiv:2503.10302 on one AMD Instinct MI355X (gfx950):
 *   - graph-coloured p-bit (Gibbs) sweeps, Eqs. (5)-(6), over many replicas
 *     and inverse temperatures (Methods, "Graph Coloring");
 *   - replica-exchange swaps, Eq. (4), with the alternating pair schedule and
 *     per-label chains of Methods, "APT details";
 *   - Houdayer isoenergetic cluster moves, Algorithm S2 (ICMop);
 *   - discrete-time simulated quantum annealing, Supplementary Eqs. S.1-S.3
 *     and Algorithm S1;
 *   - the adaptive inverse-temperature ladder of Algorithm S2 and a learned
 *     ladder predictor that replaces it (with the adaptive stage as fallback).
 *
 * Conventions shared by every entry point
 *   - Every function returns sg_status: SG_OK (0) or a negative error code.
 *     Nothing aborts or exits.  sg_last_error() gives a message.
 *   - Host pointers only.  The caller owns every array it passes; sg_create
 *     copies what it needs.  The context owns all device memory it allocates
 *     and frees it in sg_destroy.
 *   - All work of one context is ordered on one HIP stream (given in the
 *     config, or created by the library when NULL).  Functions that write
 *     host arrays synchronise that stream before returning.
 *   - A context is not thread-safe; use one per thread.
 *   - On SG_EINVAL / SG_EUNSUPPORTED the context is left unchanged.
 *
 * Data layout
 *   - Site index j = x + Lx*(y + Ly*z), n = Lx*Ly*Lz <= 32767.
 *   - J[3*j + a] (int8, -1, 0 or +1) is the coupling between site j and its
 *     +a neighbour (a = 0,1,2 for x,y,z).  Along a periodic axis the last site
 *     couples to the first; across an open boundary the stored value is
 *     ignored.  0 means no bond.  h[j] (int8, |h| <= 31) or NULL.
 *   - Spins are exchanged as int8 +1/-1.
 *   - APT replica slot s = b*reps_per_beta + l: inverse temperature index b,
 *     ICM label l.  DT-SQA slot (r, k): independent replica r, Trotter slice k.
 *
 * Random numbers: Philox4x32-10 keyed by the 64-bit seed; each update draws
 * from a counter made of (site, sweep index, slot group, instance, purpose), so
 * results do not depend on the launch configuration and checkpoints resume
 * exactly.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sg_status;
#define SG_OK 0
#define SG_EINVAL (-1)         /* invalid argument */
#define SG_ENOMEM (-2)         /* device or host allocation failed */
#define SG_EHIP (-3)           /* HIP runtime error (no device, launch failure) */
#define SG_ESTATE (-4)         /* call does not fit the context's mode or state */
#define SG_EUNSUPPORTED (-5)   /* valid input this implementation does not handle */

#define SG_APT 1
#define SG_SQA 2

typedef struct sg_ctx sg_ctx;

/* One problem instance (Eq. 1 with fields, Eq. 8). */
typedef struct {
    int32_t Lx, Ly, Lz;
    uint32_t periodic;   /* bit0 = x, bit1 = y, bit2 = z */
    const int8_t *J;     /* [Lz][Ly][Lx][3] */
    const int8_t *h;     /* [n] or NULL */
} sg_lattice;

typedef struct {
    int32_t mode;              /* SG_APT or SG_SQA */
    int32_t n_inst;            /* >= 1; lattice sizes may differ (batched form) */
    const sg_lattice *inst;    /* [n_inst] */
    /* APT (Algorithm S2): */
    int32_t n_beta;            /* >= 2 inverse temperatures per instance */
    const double *beta;        /* [n_inst][n_beta], strictly ascending, >= 0 */
    int32_t reps_per_beta;     /* ICM labels per temperature: 1, 2 or 4 */
    /* DT-SQA (Algorithm S1): */
    int32_t M;                 /* Trotter slices, 2..64 (an odd ring takes a third colour) */
    int32_t R;                 /* independent replicas per instance, 1..65535 */
    double sqa_beta;           /* inverse temperature beta > 0 */
    uint64_t seed;
    void *hip_stream;          /* hipStream_t borrowed from the caller, or NULL */
} sg_config;

/* Validate, copy the instances, build colour classes and acceptance tables,
 * allocate device memory and draw the random initial spins (Algorithm S1 and
 * S2: random initial states for all replicas).  *out is NULL on error.  The
 * per-instance tables are built on up to 16 host threads, all ended before the call
 * returns; when several instances are invalid, the error names the lowest of them. */
sg_status sg_create(const sg_config *cfg, sg_ctx **out);
/* sg_create with a colour map per instance (Methods, "Graph Coloring": the p-bits of one
 * colour share no bond and are updated in parallel).  colour (nullable) [n_inst], colour[i]
 * (nullable: the closed-form colouring) [n] int8 in 0..3, copied.  APT sweeps colour classes
 * 0, 1, ... in turn; DT-SQA colours site j of slice k with (colour[j] + t(k)) mod C, where
 * t(k) = k mod 2 except t(M - 1) = 2 when M is odd, and C = max(colours, 2, 3 if M is odd).  SG_EINVAL when two sites joined by a bond with J != 0 share a colour
 * or a value is outside 0..3.  Any proper map gives a valid sampler; the oracle takes the
 * same map.  sg_create(cfg, out) = sg_create_ex(cfg, NULL, out). */
sg_status sg_create_ex(const sg_config *cfg, const int8_t *const *colour, sg_ctx **out);
/* DSATUR colouring (Brelaz) of one instance's interaction graph (sites joined by bonds with
 * J != 0): colour_out [n] in 0..*n_colours - 1.  It uses two colours on every bipartite
 * graph (all lattices without an odd periodic axis, diluted or not), three or more where an
 * odd cycle remains.  SG_EUNSUPPORTED if more than four colours would be needed. */
sg_status sg_dsatur_colouring(const sg_lattice *inst, int8_t *colour_out, int32_t *n_colours);
void sg_destroy(sg_ctx *ctx);
const char *sg_last_error(const sg_ctx *ctx);

/* APT: n_sweeps coloured Gibbs sweeps of every replica (Eqs. 5-6): for each
 * colour, every p-bit of that colour in every slot is resampled at its slot's
 * inverse temperature. */
sg_status sg_sweep(sg_ctx *ctx, int32_t n_sweeps);

/* APT: one ICMop per replica pair at every inverse temperature >= beta_cutoff
 * (Algorithm S2; 2 labels -> one pair, 4 labels -> a random matching).
 * info_host (nullable) [n_inst][n_beta][max(1, reps/2)][4] receives
 * (m, seed site, cluster size, branch) per pair, -1 where not applied.
 * SG_EUNSUPPORTED when an instance has a non-zero field (the whole-replica
 * branch is isoenergetic only for h = 0). */
sg_status sg_icm(sg_ctx *ctx, double beta_cutoff, int32_t *info_host);

/* Energies (Eq. 8) of every slot.  E_host: APT [n_inst][n_beta*reps] in slot
 * order, DT-SQA [n_inst][R][M] per slice under the original couplings. */
sg_status sg_energy(sg_ctx *ctx, int64_t *E_host);

/* APT: one replica-exchange attempt (Eq. 4).  Attempts are numbered from 1;
 * odd attempts try temperature pairs (0,1),(2,3),..., even ones (1,2),...;
 * each label decides on its own.  accepted_host (nullable)
 * [n_inst][(n_beta-1)*reps]: 1 accepted, 0 rejected, -1 not attempted. */
sg_status sg_swap(sg_ctx *ctx, int32_t *accepted_host);

/* APT main loop (Algorithm S2), n_cycles times: sweeps_per_swap sweeps, one
 * ICM call at beta >= icm_cutoff (pass +inf for none), energies, one swap
 * attempt, running minimum energy per instance.  Runs as device-resident
 * cycles replayed from a captured HIP graph.  best_trace (nullable)
 * [n_inst][n_cycles / record_every] receives the running minimum. */
sg_status sg_run_apt(sg_ctx *ctx, int64_t n_cycles, int32_t sweeps_per_swap, double icm_cutoff,
                     int32_t record_every, int64_t *best_trace);

/* Options of the APT main loop and of the ICM call beyond those of sg_run_apt / sg_icm:
 * per-instance ICM cutoffs (a learned ladder predicts one per instance) and the number
 * of Houdayer moves per temperature per call with four labels (Supplementary comparison
 * of APT with zero, one and two ICMs per sweep: two moves both pairs of the drawn
 * matching, one moves one of them, chosen at random).  With two labels there is one
 * pair and both values give one move; no ICM is icm_cutoff = +inf. */
typedef struct {
    int32_t sweeps_per_swap;            /* >= 1 (sg_run_apt_ex only) */
    int32_t icm_pairs;                  /* 2 or 1 */
    double icm_cutoff;                  /* ICM at beta >= icm_cutoff, all instances ... */
    const double *icm_cutoff_per_inst;  /* ... or [n_inst] per instance (nullable) */
    int32_t record_every;               /* as in sg_run_apt (sg_run_apt_ex only) */
} sg_apt_options;
/* sg_run_apt with these options; sg_run_apt(c, n, s, cut, r, t) equals sg_run_apt_ex with
 * {s, 2, cut, NULL, r}.  SG_EINVAL for icm_pairs outside {1, 2} or a NaN cutoff. */
sg_status sg_run_apt_ex(sg_ctx *ctx, int64_t n_cycles, const sg_apt_options *opt,
                        int64_t *best_trace);
/* sg_icm with these options (sweeps_per_swap and record_every are ignored). */
sg_status sg_icm_ex(sg_ctx *ctx, const sg_apt_options *opt, int32_t *info_host);

/* APT: running minimum energy per instance since creation [n_inst]. */
sg_status sg_best(sg_ctx *ctx, int64_t *best_host);

/* APT: accepted-swap counts since creation [n_inst][(n_beta-1)*reps]. */
sg_status sg_swap_counts(sg_ctx *ctx, int64_t *counts_host);

/* DT-SQA (Algorithm S1): for t = 0..n_steps-1, J_perp follows gamma[t]
 * (Supplementary Eq. S.3) and every slice of every replica gets one coloured
 * sweep of the (d+1)-dimensional lattice.  Then the energy of every slice
 * under the original couplings; best_E[n_inst] and best_state[n_inst][n_max]
 * (nullable) receive the minimum and its slice (ties: lowest r*M + k). */
sg_status sg_sqa_anneal(sg_ctx *ctx, const double *gamma, int32_t n_steps, int64_t *best_E,
                        int8_t *best_state);

/* DT-SQA: correlation along the Trotter direction of the current state (Supplementary
 * correlation-length figure, C_k = (1/n) sum_i s_{i,0} s_{i,k} measured from slice 0),
 * exactly: agree_host [n_inst][R][M] = number of sites where slice k of replica r agrees with
 * its slice 0 (C_k = (2 agree - n) / n). */
sg_status sg_sqa_trotter_agreement(sg_ctx *ctx, int32_t *agree_host);

/* ---- acceptance thresholds ----
 * The FP64-built thresholds the kernels compare their uniform 32-bit words with, computed by
 * the same host code that fills the contexts' tables, so that the builders can be checked
 * against an independent implementation.  Heat bath (Eq. 6): T = floor(2^32 (1 + tanh(beta
 * I)) / 2), saturated at 2^32 - 1, s = +1 iff u < T.  DT-SQA (Supplementary Eq. S.3): the same
 * with the argument (beta / M) s + K tau, K = -ln tanh(beta gamma / M) / 2, s the spatial
 * field and tau the sum of the two Trotter neighbours.  Swap (Eq. 4): an exchange of
 * inverse temperatures beta_lo < beta_hi whose energy change is unfavourable by d >= 1
 * (Delta beta Delta E = -(beta_hi - beta_lo) d) is accepted iff u < T = floor(exp(-(beta_hi -
 * beta_lo) d) 2^32).  SG_EINVAL (message in sg_last_error(NULL)) for invalid arguments. */
sg_status sg_threshold_heat_bath(double beta, int32_t I, uint32_t *T);
sg_status sg_threshold_sqa(double beta, int32_t M, double gamma, int32_t s, int32_t tau, uint32_t *T);
sg_status sg_threshold_swap(double beta_lo, double beta_hi, int64_t d, uint32_t *T);

/* ---- device outputs ----
 * The same results as sg_energy, sg_get_spins, sg_best and sg_sqa_anneal, written to memory
 * the caller allocated on the context's device with the HIP runtime the library uses, in the same
 * layouts (E_dev int64 [n_inst][n_beta * reps] or [n_inst][R][M]; spins_dev int8 +1/-1
 * [n_inst][slots][n_max] or [n_inst][R][M][n_max], 0 past an instance's n; best_dev int64
 * [n_inst]; best_E_dev int64 [n_inst], best_state_dev int8 [n_inst][n_max]).  The work is
 * queued on the context's stream and nothing is copied to the host: the results are there once
 * that stream reaches them (create the context on the consumer's stream, or call
 * sg_synchronize).  sg_sqa_anneal_dev still waits for the stream between 256-step chunks of a
 * longer schedule, whose threshold tables it rebuilds on the host.  The caller provides buffers
 * of the sizes above; a pointer that is not device memory of the context's device gives
 * SG_EINVAL before any work is queued. */
sg_status sg_energy_dev(sg_ctx *ctx, int64_t *E_dev);
sg_status sg_get_spins_dev(sg_ctx *ctx, int8_t *spins_dev);
sg_status sg_best_dev(sg_ctx *ctx, int64_t *best_dev);
sg_status sg_sqa_anneal_dev(sg_ctx *ctx, const double *gamma, int32_t n_steps, int64_t *best_E_dev,
                            int8_t *best_state_dev);

/* Launch configuration (an implementation choice; results do not depend on it).
 * DT-SQA contexts: the work-group size, a multiple of 64 in 128..1024.  The first
 * sg_sqa_anneal of a context whose size is unset (0) times 256, 512, 768 and 1024 for a few
 * steps on a scratch copy of the replicas and keeps the fastest.
 * APT contexts: a code 1..12 = 1 + order + 6 * (8 waves per SIMD ? 1 : 0), order 0..5 the
 * dispatch order of the replica kernel's work-groups (0-3: instances spread over the eight
 * XCDs, quads sorted by estimated cost with cluster-move weight 3, 1, 2, 4; 4: one global cost
 * sort; 5: instance-major), and at least 7 or 8 waves per SIMD (the kernel's register
 * budget).  Codes 13..15: order 0 at 7 waves, with the cycles of sg_run_apt / sg_run_apt_ex
 * split into two launch groups that run side by side on the context's stream and a second
 * stream the library creates (joined back before the call's later work): the largest
 * instances up to 65, 75 or 85 % of all sites, and the rest (one group if that leaves the
 * second empty).  The first sg_run_apt / sg_run_apt_ex of a context whose code is unset (0)
 * times all fifteen on its own shape (sweeps per swap, cluster moves) and keeps the fastest,
 * leaving the context's state as it was; other calls use code 1 until then.
 * Both tuners cache their pick per workload shape for the process and in the file named by
 * the environment variable SG_TUNE_CACHE (default ~/.cache/libsg_tune.txt; best effort).
 * get: 0 while unset.  set: 0 re-enables the autotuner; any other value outside the allowed
 * set gives SG_EINVAL. */
sg_status sg_get_launch_config(sg_ctx *ctx, int32_t *config);
sg_status sg_set_launch_config(sg_ctx *ctx, int32_t config);

/* Spins in logical order, +1/-1.  APT [n_inst][n_beta*reps][n_max];
 * DT-SQA [n_inst][R][M][n_max]; n_max = largest n, unused tail zero. */
sg_status sg_get_spins(sg_ctx *ctx, int8_t *spins_host);
/* A part of one instance's state, for sampling large contexts: APT logical slots
 * [first, first + count) as [count][n], DT-SQA replicas [first, first + count) as
 * [count][M][n] (n = that instance's site count), +1/-1.  SG_EINVAL when the
 * instance or the range is outside the context. */
sg_status sg_get_spins_range(sg_ctx *ctx, int32_t inst, int32_t first, int32_t count,
                             int8_t *spins_host);
sg_status sg_set_spins(sg_ctx *ctx, const int8_t *spins_host);

/* Counters {sweeps or SQA steps done, ICM calls, swap attempts}. */
sg_status sg_get_counters(sg_ctx *ctx, uint32_t *counters3);

/* Checkpoint: spins, counters and running minima in one opaque blob.
 * sg_get_state with blob == NULL sets *len to the size needed. */
sg_status sg_get_state(sg_ctx *ctx, void *blob, size_t *len);
sg_status sg_set_state(sg_ctx *ctx, const void *blob, size_t len);

/* Stream-ordered timing: record a HIP event on the context's stream now
 * (sg_timer_start) and the elapsed milliseconds at the matching stop. */
sg_status sg_timer_start(sg_ctx *ctx);
sg_status sg_timer_stop(sg_ctx *ctx, float *ms);
sg_status sg_synchronize(sg_ctx *ctx);

/* Kernel timing: while enabled, every main kernel launch (one DT-SQA kernel
 * per chunk of at most 256 steps, one captured graph of 32 APT cycles) is
 * bracketed by HIP events on the context's stream.  sg_kernel_time returns
 * the summed milliseconds and the number of launches since the last call
 * (or since enabling), and resets the tally. */
sg_status sg_kernel_timing(sg_ctx *ctx, int32_t enable);
sg_status sg_kernel_time(sg_ctx *ctx, float *ms, int32_t *launches);

/* ---- adaptive ladder (Algorithm S2 preprocessing; Methods "APT details") ----
 * Chains start random at beta0; each step runs `sweeps` sweeps per chain at
 * beta_t, takes each chain's sample standard deviation of the energy over the
 * last `tail` sweeps (exact integer moments, FP64 on the host), averages it
 * over chains (sigma_E), appends beta_t and stops once sigma_E < tol,
 * otherwise beta_{t+1} = beta_t + alpha / sigma_E.  All instances run as one
 * batch.  beta_out [n_inst][max_steps], sigma_out (nullable) same shape,
 * len_out [n_inst]. */
typedef struct {
    double beta0, alpha, tol;
    int32_t n_chains, sweeps, tail, max_steps;
} sg_adaptive_params;
sg_status sg_adaptive_ladder(const sg_lattice *inst, int32_t n_inst, const sg_adaptive_params *p,
                             uint64_t seed, void *hip_stream, double *beta_out, double *sigma_out,
                             int32_t *len_out);

/* ---- learned ladder predictor (project component, not in the paper) ----
 * Features per instance: cube root of n, mean and variance over sites of the
 * absolute sum of the couplings at the site, and the frustrated-plaquette
 * fraction.  Network 4 -> 64 -> 64 -> 33 (ReLU, FP32) on standardised
 * features; outputs log beta_0, softplus increments of log beta_1..31, and
 * the log ICM cutoff.  Parameters: W1[64][4] b1[64] W2[64][64] b2[64]
 * W3[33][64] b3[33] (6625 floats) followed by the feature mean[4] and std[4]. */
#define SG_MLP_NPARAM 6625
typedef struct sg_mlp sg_mlp;
sg_status sg_mlp_create(const float *params /* nullable: random init from seed */, uint64_t seed,
                        void *hip_stream, sg_mlp **out);
void sg_mlp_destroy(sg_mlp *m);
sg_status sg_instance_features(const sg_lattice *inst, int32_t n_inst, double *features /*[n_inst][4]*/);
sg_status sg_mlp_set_standardisation(sg_mlp *m, const float *mean4, const float *std4);
/* Mean-squared-error loss and its gradient over a batch (raw features and
 * targets [B][33] = log betas and log cutoff); FP32 kernels. */
sg_status sg_mlp_loss_grad(sg_mlp *m, const float *x, const float *y, int32_t batch, float *loss,
                           float *grad /* nullable [6625] */);
/* Adam training: epochs over the data set in minibatches (lr, betas 0.9/0.999). */
sg_status sg_mlp_train(sg_mlp *m, const float *x, const float *y, int32_t n, int32_t batch,
                       int32_t epochs, float lr, float *loss_per_epoch);
sg_status sg_mlp_get_params(sg_mlp *m, float *params /*[6625 + 8]*/);
/* Predicted ladders: beta_out [n_inst][32] ascending, cutoff_out [n_inst]. */
sg_status sg_ladder_predict(sg_mlp *m, const sg_lattice *inst, int32_t n_inst, double *beta_out,
                            double *cutoff_out);

/* One repair step of a 32-rung (any n_beta >= 2) ladder from a pilot's swap acceptance, for
 * a ladder that failed its band.  With the acceptance of a pair at inverse temperatures
 * spaced dbeta read as erfc(dbeta sigma / 2) (Gaussian energies of spread sigma; the adaptive
 * stage's rule beta + alpha / sigma_E gives erfc(alpha / 2), Methods "APT details"), each pair
 * has a length 2 erfc^-1(a): measured from acc, wanted from the band's midpoint.  Rung k moves
 * to where the measured length, interpolated linearly in log beta between the old rungs,
 * reaches the share of the total that the wanted lengths give it; the end rungs stay.  With
 * damping d in (0, 1] the result is exp((1 - d) log beta + d log beta_new) rung by rung.
 * Acceptances are clamped to [1e-3, 1 - 1e-3].  beta [n_beta] strictly ascending, positive;
 * acc, band_lo, band_hi [n_beta - 1]; beta_out [n_beta] (may alias beta), strictly ascending.
 * Host arithmetic only.  SG_EINVAL (message in sg_last_error(NULL)) for invalid arguments. */
sg_status sg_ladder_repair(const double *beta, const double *acc, const double *band_lo,
                           const double *band_hi, int32_t n_beta, double damping, double *beta_out);

/* The judge of candidate 32-rung ladders, with the adaptive stage as fallback:
 *   1. a pilot APT+ICM run of pilot_cycles cycles on the candidates (2 labels, one sweep per
 *      attempt, each instance at its own ICM cutoff, seed) and the swap acceptance of every
 *      adjacent pair (accepted / attempted exchanges) against [band_lo, band_hi];
 *   2. up to repair_rounds rounds on the instances outside the band: sg_ladder_repair from the
 *      last pilot's acceptance (damping 1 in the first round, 0.5 after), a pilot of the
 *      repaired ladders of those instances alone (seed + 2 + round), the band check;
 *   3. for every instance still outside, the adaptive stage (fallback parameters, seed + 1)
 *      resampled to 32 rungs by linear interpolation in the normalised rung index, its cutoff
 *      the first rung >= 1.
 * beta_io [n_inst][32] and cutoff_io [n_inst]: the candidates in, the judged ladders out.
 * band_lo, band_hi [n_inst][31].  status [n_inst]: 0 the candidate passed, 2 a repaired
 * ladder passed, 1 the adaptive stage's ladder.  acc_out (nullable) [n_inst][31]: the
 * acceptance of the last pilot run on the instance (status 1: of its last rejected ladder). */
sg_status sg_judge_ladders(const sg_lattice *inst, int32_t n_inst, const double *band_lo,
                           const double *band_hi, const sg_adaptive_params *fallback,
                           int32_t pilot_cycles, int32_t repair_rounds, uint64_t seed,
                           double *beta_io, double *cutoff_io, int32_t *status, double *acc_out);

/* The learned-ladder flow: the network's ladders and per-instance ICM cutoffs
 * (sg_ladder_predict) put through sg_judge_ladders with the same arguments. */
sg_status sg_learned_ladders(sg_mlp *m, const sg_lattice *inst, int32_t n_inst, const double *band_lo,
                             const double *band_hi, const sg_adaptive_params *fallback,
                             int32_t pilot_cycles, int32_t repair_rounds, uint64_t seed,
                             double *beta_out, double *cutoff_out, int32_t *status, double *acc_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sg_ladder_predict without any
 * allocation.  Same arguments, same results bit for bit.  The network inputs and outputs
 * are staged in a static device array of the library (one per GPU, about 0.6 MB, held until
 * the process ends, its address resolved by sg_mlp_create on the network's device) and, on
 * the host, inside beta_out itself; the call allocates nothing, host or device.
 * n_inst must be 1..SG_PREDICT_NOALLOC_MAX, otherwise SG_EINVAL with a message in
 * sg_last_error(NULL).  Every call on one GPU shares that GPU's array: calls that overlap
 * in time on one GPU (two threads, two streams) race and must be serialised by the caller.
 * The call synchronises the network's stream before returning. */
#define SG_PREDICT_NOALLOC_MAX 4096
sg_status sg_ladder_predict_noalloc(sg_mlp *m, const sg_lattice *inst, int32_t n_inst,
                                    double *beta_out, double *cutoff_out);

#ifdef __cplusplus
}
#endif
#endif
