// sg_internal.h -- structures shared by the host side (sg_api.cpp) and the
// device kernels (sg_kernels.hip) of libsg.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

// Random-stream purposes (low 4 bits of Philox counter word 3; word 3 is
// instance << 4 | purpose).
enum : uint32_t {
    TAG_APT_INIT = 1,
    TAG_APT_SWEEP = 2,
    TAG_SWAP = 3,
    TAG_ICM_PAIR = 4,
    TAG_ICM_PICK = 5,
    TAG_SQA_INIT = 6,
    TAG_SQA_SWEEP = 7,
    TAG_ADAPT_INIT = 8,
    TAG_ADAPT_SWEEP = 9,
};

constexpr int kMaxColours = 4;   // colour classes of a given colour map
constexpr int kMaxH = 31;      // |h| bound, so that h + 32 fits 6 bits of a site record
constexpr int kMaxN = 32767;   // sites per instance (16-bit site and neighbour indices)
constexpr int kMaxByteOffsetSites = 16383;   // neighbour byte offsets (4 x index) fit 16 bits
constexpr int kQuadThreads = 256;
constexpr int kSqaThreads = 512;
constexpr int kSqaTabWords = 976;        // static LDS of the DT-SQA kernel (tables)
constexpr size_t kMaxLds = 160 * 1024;   // LDS per CU on gfx950

// Site record (uint4), one per site:
//   x: j | d << 16 | jneg << 19 | (h + 32) << 25 | p << 31
//      d    = number of bonds with J != 0 (0..6)
//      jneg = bit a set when the bond to neighbour a has J = -1
//      p    = (DT-SQA phase lists only) parity of the Trotter slices updated
//   y: nb[0] | nb[1] << 16   (+x, -x)
//   z: nb[2] | nb[3] << 16   (+y, -y)
//   w: nb[4] | nb[5] << 16   (+z, -z)
// An absent bond (open boundary, axis of length one, or J = 0) points at the
// dummy index n, whose spin word is kept zero.  The DT-SQA phase lists hold, in
// place of each nb, the word offset 2 nb + p of the neighbour's spin word of
// parity p.

// Per-instance geometry and buffer offsets on the device.
struct InstDev {
    int32_t n;           // sites
    int32_t npad;        // sites rounded up to a multiple of 16
    int32_t n_colours;   // colour classes (APT) or phases (DT-SQA), at most kMaxColours
    int32_t n_slots;     // APT: n_beta * reps; DT-SQA: M
    int32_t col_off[4];  // first record of each colour class / phase (relative)
    int32_t col_cnt[4];  // records in each class / phase
    int32_t col_p1[4];   // DT-SQA: records of parity 0 at the start of each phase, then
                         // those of parity 1 up to col_p2
    int32_t col_p2[4];   // DT-SQA, odd M: start of the records that update the last slice
                         // M - 1 alone (bit H - 1 of word 0); col_cnt when M is even
    int64_t rec_off;     // colour-sorted (or phase) records
    int64_t recj_off;    // site-ordered records
    int64_t spin_off;    // APT: byte offset of replica buffer 0; DT-SQA: word offset
    int32_t slot_off;    // APT: first entry in perm / E / slot_lut / swap arrays
    int32_t swap_off;    // APT: first pair entry of swap tables
    int32_t info_off;    // APT: first ICM info record
    int32_t lx;          // row length (x extent)
    int32_t n_rows;      // Ly * Lz
    int32_t row_off;     // first entry of the row tables, -1 when lx > 32
    int32_t ly, lz;      // y and z extents (rows are r = y + ly z)
    int32_t planes;      // 1: every y-z plane's rows fit one per lane in one wave and all
                         //    planes in the work-group's waves (wave-local cluster search)
    int32_t n_bonds;     // bonds with J != 0 (each counted once)
};

// Row tables of an instance for the cluster search (rows of lx <= 32 sites):
//   rowA[r] = {bond to +x present (bit x), bond to -x, bond to +y, bond to -y}
//   rowB[r] = {bond to +z, bond to -z, row(+y) | row(-y) << 16, row(+z) | row(-z) << 16}
//   rowC[r] = {J = -1 on the bond to +x, to +y, to +z, 0}
// "present" means the neighbour exists and J != 0.

// One work-group task of the APT replica kernel: instance and group of four
// consecutive logical slots.  inst < 0 = idle filler.
struct QuadDesc {
    int32_t inst;
    int32_t quad;
};

// Replica exchange of one instance (also run at the end of a fused cycle).
struct SwapArgs {
    const InstDev *inst;
    const int32_t *perm_in;    // state before the exchange (may equal perm / E)
    const int32_t *E_in;
    int32_t *perm;             // state after it
    int32_t *E;
    const uint32_t *tab;       // swap thresholds, per pair: T[d] for |dE| = d
    const int32_t *tab_off;    // per (instance, pair)
    const int32_t *tab_len;
    int64_t *best;             // per instance
    int64_t *trace;            // [inst][trace_cap] or null
    int32_t trace_cap;
    int32_t record_every;
    int64_t *acc_count;        // per (instance, pair, label)
    int32_t *acc_out;          // per (instance, pair, label) or null
    uint32_t *ctr;
    uint32_t key0, key1;
    int32_t n_beta;
    int32_t reps;
    int32_t n_inst;
    int32_t cyc_k;             // cycle offset of this launch inside a captured graph
};

struct AptArgs {
    const QuadDesc *desc;
    const InstDev *inst;
    const uint4 *rec_col;
    const uint4 *rec_j;
    const uint4 *rowA;
    const uint4 *rowB;
    const uint4 *rowC;
    uint8_t *spins;            // physical replica buffers, bytes 0/1 (1 = spin up)
    const int32_t *perm;       // logical slot -> physical buffer (per instance)
    const uint32_t *lut;       // heat-bath thresholds, NI per table
    const int32_t *slot_lut;   // logical slot -> table index
    const uint8_t *icm_on;     // per (instance, beta index): ICM applies
    int32_t *E;                // energies per logical slot
    int64_t *mom;              // per logical slot {sum E, sum E^2} (adaptive stage)
    int32_t *icm_info;         // per (instance, beta, pair) {m, seed, size, branch}
    uint32_t *ctr;             // device counters {sweeps, icm calls, swaps, cycles}
    uint32_t key0, key1;
    uint32_t tag;              // sweep purpose (APT or adaptive)
    int32_t n_sweeps;
    int32_t do_icm;
    int32_t do_energy;         // 0: leave E, 1: E += change in this launch, 2: recompute E
    int32_t mom_from;          // accumulate moments after sweep index >= mom_from (-1: never)
    int32_t reps;              // ICM labels per temperature
    int32_t icm_pairs;         // 4 labels: pairs moved per temperature per ICM call (2 or 1)
    int32_t imax;              // LUT covers fields -imax..imax
    int32_t ni;                // 2 * imax + 1
    int32_t n_blocks;
    int32_t nb4;               // slots per instance padded to a multiple of 4 (= slot stride)
    int32_t cyc_k;             // cycle offset of this launch inside a captured graph: the
                               // kernel uses sweep counter ctr[0] + cyc_k * n_sweeps and ICM
                               // call ctr[1] + cyc_k + 1; counters advance only between graphs
    int32_t waves;             // kernel variant: at least 8 or 7 (also for 0) waves per SIMD
    int32_t boff;              // 1: rec_col holds neighbour byte offsets (kernel variant)
    int32_t fused_swap;        // 1: first perform the replica exchange described by sw (the
                               //    previous cycle's attempt) for this work-group's slots,
                               //    reading sw.perm_in / sw.E_in and writing sw.perm and E
    SwapArgs sw;
};

// DT-SQA: spins of replica (inst, r) are n+1 pairs of 32-bit words
// {even slices, odd slices}; slice k = 2h + p sits at bit h of word p.
struct SqaArgs {
    const InstDev *inst;
    const uint4 *rec;          // phase-sorted records (p in bit 31 of x)
    const uint4 *rec_j;        // site-ordered records
    uint32_t *spins;           // [inst][R][npad + 1][2]
    const uint32_t *lut;       // [step][NL]: index (s + smax) * 3 + (number of up Trotter neighbours)
    int32_t *slice_E;          // [inst][R][M]
    int32_t R;
    int32_t M;
    int32_t H;                 // M / 2
    int32_t smax;
    int32_t nl;
    int32_t t0;                // global index of the first step
    int32_t n_steps;
    int32_t lut_step0;         // row of lut used for the first step
    int32_t do_energy;
    int32_t no_field;          // 1: every field is zero (bit-sliced energy readout)
    uint64_t *best_key;        // [inst] or null: atomic minimum of (E + 2^30) << 32 | (r M + k)
                               // over the slices of the energy pass (ties: lowest r M + k)
    uint32_t key0, key1;
};

constexpr int kSqaPlanes = 10;   // bits of the readout's per-thread unsatisfied-bond counters

// Adaptive-ladder stage with the chains bit-packed: word w of a site holds chains
// 32 w .. 32 w + 31 of its instance (bit b = chain 32 w + b; 1 = up), all at the
// instance's current beta.  Fields must be zero (energies count unsatisfied bonds).
constexpr int kAdaptThreads = 512;
constexpr int kAdaptPlanes = 10;   // bits of the per-thread unsatisfied-bond counters
constexpr int kAdaptTabWords = 256 + 16 + 64;            // static tables of adapt_kernel
constexpr int kAdaptRedWords = kAdaptThreads / 64 * 32 + 1;   // its reduction scratch
struct AdaptArgs {
    const InstDev *inst;
    const uint4 *rec_col;      // colour-sorted site records
    const uint4 *rec_j;        // site-ordered site records
    uint32_t *words;           // [inst][nw][wstride]: the chains' spin words
    const uint32_t *lut;       // [inst][ni]: heat-bath thresholds at the instance's beta
    int64_t *mom;              // [inst][n_chains][2]: sum of E, sum of E^2 over the tail
    int64_t wstride;           // words per (instance, word) block, >= npad + 1
    uint32_t t0;               // sweep counter of the launch's first sweep
    int32_t n_inst, n_chains, nw, n_sweeps, mom_from, imax, ni, planes;
    uint32_t key0, key1;
};

// Host-callable launch wrappers (defined in sg_kernels.hip).
hipError_t launch_apt_init(const InstDev *inst_d, const QuadDesc *desc, int n_blocks,
                           uint8_t *spins, const int32_t *perm, uint32_t key0, uint32_t key1,
                           uint32_t tag, hipStream_t s);
hipError_t launch_apt_quad(const AptArgs &a, size_t lds_bytes, hipStream_t s);
hipError_t launch_apt_swap(const SwapArgs &a, hipStream_t s);
hipError_t launch_sqa_init(const SqaArgs &a, int n_inst, hipStream_t s);
// DT-SQA kernel with a work-group of `threads` (a multiple of 64 in 128..1024).
bool sqa_config_valid(int threads);
hipError_t launch_sqa(const SqaArgs &a, int n_inst, size_t lds_bytes, int threads, hipStream_t s);
// The slice chosen by best_key[i] of every instance as +1/-1 bytes, out[i][n_max].
hipError_t launch_sqa_best_state(const SqaArgs &a, int n_inst, int n_max, int8_t *out,
                                 hipStream_t s);
// agree[inst][r][k]: sites where slice k of replica r agrees with its slice 0.
hipError_t launch_widen_rows(const int32_t *src, int src_stride, int64_t *dst, int rows, int cols,
                             hipStream_t s);
hipError_t launch_apt_spins_out(const uint8_t *spins, const int32_t *perm, const InstDev *inst,
                                int n_inst, int nb4, int n_slots, int n_max, int8_t *out, hipStream_t s);
hipError_t launch_sqa_spins_out(const uint32_t *words, const InstDev *inst, int n_inst, int R, int M,
                                int n_max, int8_t *out, hipStream_t s);
hipError_t launch_best_key_energy(const uint64_t *key, int n, int64_t *out, hipStream_t s);
hipError_t launch_sqa_corr(const SqaArgs &a, int n_inst, int32_t *agree, hipStream_t s);
hipError_t launch_adapt_init(const AdaptArgs &a, int n_inst, hipStream_t s);
hipError_t launch_adapt(const AdaptArgs &a, int n_inst, size_t lds_bytes, hipStream_t s);
hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// ctr[i] += d[i] for the four counters (one thread; ordered by the stream).
hipError_t launch_advance(uint32_t *ctr, uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3,
                          hipStream_t s);

// MLP kernels (sg_mlp.hip).  Parameters: 6625 floats, then mean[4], std[4].
hipError_t launch_mlp_pass(const float *P, const float *x, const float *y, const int *idx,
                           int batch, int nblk, float *grad_acc, float *loss_acc, float *out,
                           float *grad, hipStream_t s);
hipError_t launch_mlp_adam2(float *P, const float *g, float *m, float *v, float lr, float b1,
                            float b2, float eps, int step, hipStream_t s);
// Allocation-free prediction: at most kPredictMax instances per call; the staging area
// (raw features [kPredictMax][4], then outputs [kPredictMax][33]) is a static device array
// of the library, one per GPU.  mlp_scratch gives its address on the current device
// (resolved once per device, then cached).
constexpr int kPredictMax = 4096;
constexpr int kPredictScratchFloats = kPredictMax * (4 + 33);
constexpr int kMaxDevices = 64;
hipError_t mlp_scratch(float **p);
// Message returned by sg_last_error(NULL) (calls without a context).
void set_global_error(const char *msg);

}  // namespace sg
