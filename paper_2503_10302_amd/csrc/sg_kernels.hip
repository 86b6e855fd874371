// sg_kernels.hip -- gfx950 kernels of libsg.
//
// APT replica kernel: one work-group owns four consecutive logical replica
// slots of one instance.  Their lattices are gathered from the physical
// replica buffers into LDS, interleaved one byte per slot in a 32-bit word per
// site, so that one LDS read returns a neighbour's spin in all four slots and
// the aligned-bond count of Eq. (5) is a byte-wise sum.  One Philox4x32-10
// block per site and sweep gives the four uniform words of Eq. (6).  Colour
// classes are separated by work-group barriers (Methods, "Graph Coloring").
//
// DT-SQA kernel: one work-group owns one replica of the (d+1)-dimensional
// lattice of Supplementary Eq. S.3.  Up to 64 Trotter slices are bit-packed
// per site, even and odd slices in separate words; the six spatial
// neighbours are summed bit-sliced over all slices of a parity at once.
#include <algorithm>
#include "sg_internal.h"

namespace sg {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds, two 32x32->64 products.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = n0;
        x2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(x0, x1, x2, x3);
}

// a ^ b ^ k as one vector operation; k must be wave-uniform (it is read from a scalar
// register).  On gfx950 a two-operand XOR that reads a scalar register issues at half
// rate, so the pair of XORs of a Philox round costs three full-rate slots and this
// three-input form two.
__device__ __forceinline__ uint32_t xor3_vvs(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "s"(k));
    return d;
}

// Round R of Philox4x32-10 for a counter whose words 1..3 are wave-uniform and word 0
// varies between lanes: words that are still uniform after round R - 1 (all of x1..x3
// before round 0; x0, x1 and x3 before round 1; x3 before round 2) are left to plain
// code, which keeps them on the scalar unit; from round 2 (x0 side) and round 3 (x2
// side) on, both operands of each XOR pair vary and the pair is one three-input
// operation with the round key.  The result is Philox4x32-10 whatever the counter.
template <int R>
__device__ __forceinline__ void philox_round_v(uint32_t x[4], uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * x[2];
    const uint32_t n0 = R >= 2 ? xor3_vvs((uint32_t)(p1 >> 32), x[1], k[0])
                               : (uint32_t)(p1 >> 32) ^ x[1] ^ k[0];
    const uint32_t n2 = R >= 3 ? xor3_vvs((uint32_t)(p0 >> 32), x[3], k[1])
                               : (uint32_t)(p0 >> 32) ^ x[3] ^ k[1];
    x[1] = (uint32_t)p1;
    x[3] = (uint32_t)p0;
    x[0] = n0;
    x[2] = n2;
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
}

// Rounds [R0, R1) of Philox4x32-10 on the state x with the key k of round R0 (the key
// is advanced): the block split in two so that other work can sit between the halves.
// For counters laid out as philox_round_v expects.
template <int R0, int R1>
__device__ __forceinline__ void philox_rounds(uint32_t x[4], uint32_t k[2])
{
    if constexpr (R0 < R1) {
        philox_round_v<R0>(x, k);
        philox_rounds<R0 + 1, R1>(x, k);
    }
}

__device__ __forceinline__ uint32_t lds_word(const uint32_t *base, uint32_t byte_off)
{
    return *(const uint32_t *)((const uint8_t *)base + byte_off);
}

// acc = 2 acc + (u < T): the borrow of u - T shifted into acc (two VOP2 operations).
__device__ __forceinline__ uint32_t shift_in_lt(uint32_t acc, uint32_t u, uint32_t T)
{
    uint32_t d;
    asm("v_sub_co_u32_e32 %1, vcc, %2, %3\n\t"
        "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc"
        : "+v"(acc), "=&v"(d)
        : "v"(u), "v"(T)
        : "vcc");
    return acc;
}

__device__ __forceinline__ uint32_t bytemask(uint32_t bit) { return bit * 0x01010101u; }

// 4 x 4 byte transpose: out[m] byte i = byte m of in[i] (eight byte permutes; v_perm_b32
// picks each result byte from {S0, S1}, selectors 0-3 the bytes of S1 and 4-7 those of S0).
__device__ __forceinline__ void transpose_bytes(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                                uint32_t out[4])
{
    const uint32_t ab_lo = __builtin_amdgcn_perm(b, a, 0x05010400u);   // a0 b0 a1 b1
    const uint32_t ab_hi = __builtin_amdgcn_perm(b, a, 0x07030602u);   // a2 b2 a3 b3
    const uint32_t cd_lo = __builtin_amdgcn_perm(d, c, 0x05010400u);
    const uint32_t cd_hi = __builtin_amdgcn_perm(d, c, 0x07030602u);
    out[0] = __builtin_amdgcn_perm(cd_lo, ab_lo, 0x05040100u);         // a0 b0 c0 d0
    out[1] = __builtin_amdgcn_perm(cd_lo, ab_lo, 0x07060302u);
    out[2] = __builtin_amdgcn_perm(cd_hi, ab_hi, 0x05040100u);
    out[3] = __builtin_amdgcn_perm(cd_hi, ab_hi, 0x07060302u);
}

// Per byte (slot): number of present bonds whose J * s_neighbour = +1.
__device__ __forceinline__ uint32_t aligned_count(const uint32_t *sp, const uint4 r)
{
    const uint32_t jn = r.x >> 19;
    uint32_t k = sp[r.y & 0xFFFFu] ^ bytemask(jn & 1u);
    k += sp[r.y >> 16] ^ bytemask((jn >> 1) & 1u);
    k += sp[r.z & 0xFFFFu] ^ bytemask((jn >> 2) & 1u);
    k += sp[r.z >> 16] ^ bytemask((jn >> 3) & 1u);
    k += sp[r.w & 0xFFFFu] ^ bytemask((jn >> 4) & 1u);
    k += sp[r.w >> 16] ^ bytemask((jn >> 5) & 1u);
    return k;
}

// Sum over the 64 lanes of a wave (all lanes active): DPP exchanges inside each row of 16
// lanes (pairs, quads, half rows, rows: no LDS round trips), then the four row sums read
// from lanes 0, 16, 32 and 48.  The result is wave-uniform.
__device__ __forceinline__ int32_t wave_sum(int32_t v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);   // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);   // row_mirror
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

__device__ __forceinline__ int32_t wave_min(int32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sum of four values (blockDim = 256).  red: >= 16 ints of LDS.
__device__ __forceinline__ void block_sum4(int32_t v[4], int32_t *red)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
        for (int i = 0; i < 4; ++i) red[wv * 4 + i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = red[i] + red[4 + i] + red[8 + i] + red[12 + i];
    __syncthreads();
}

// block_sum4 for the work-group's last use of red: the totals are read by threads 0..3
// only (into v), and there is no trailing barrier.
__device__ __forceinline__ void block_sum4_last(int32_t v[4], int32_t *red)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
        for (int i = 0; i < 4; ++i) red[wv * 4 + i] = v[i];
    __syncthreads();
    if (threadIdx.x < 4)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = red[i] + red[4 + i] + red[8 + i] + red[12 + i];
}

// Exclusive prefix of v over the block in thread order; returns it and the total.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *red, int32_t *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) red[wv] = incl;
    __syncthreads();
    int32_t base = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wv) base += red[w];
        tot += red[w];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

// Energies (Eq. 8) of the four slots held in sp: E = -1/2 sum_j s_j (I_j + h_j).
__device__ void quad_energy(const uint32_t *sp, const uint4 *recj, int n, int32_t *red, int32_t e[4])
{
    int32_t acc[4] = {0, 0, 0, 0};
    uint4 rnext = ((int)threadIdx.x < n) ? recj[threadIdx.x] : make_uint4(0u, 0u, 0u, 0u);
    for (int j = threadIdx.x; j < n; j += kQuadThreads) {
        const uint4 r = rnext;
        if (j + kQuadThreads < n) rnext = recj[j + kQuadThreads];   // prefetch
        const uint32_t k = aligned_count(sp, r);
        const int32_t d = (int32_t)((r.x >> 16) & 7u);
        const int32_t hh = (int32_t)((r.x >> 25) & 63u) - 32;
        const uint32_t w = sp[j];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int32_t v = 2 * (int32_t)((k >> (8 * i)) & 0xFFu) - d + 2 * hh;
            acc[i] += ((w >> (8 * i)) & 1u) ? v : -v;
        }
    }
    block_sum4(acc, red);
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = -acc[i] / 2;
}

// Houdayer move on the replica pair held in bytes ba, bb of sp (Algorithm S2,
// ICMop).  LDS work space: queue[n] (uint16), vis[(n + 31) / 32], red[>= 24].
__device__ void icm_pair(uint32_t *sp, const uint4 *recj, int n, int ba, int bb, uint32_t w0,
                         uint32_t w1, uint16_t *queue, uint32_t *vis, int32_t *red, int32_t *info)
{
    const int tid = threadIdx.x;
    const uint32_t mA = 1u << (8 * ba), mB = 1u << (8 * bb);
    const int chunk = (n + kQuadThreads - 1) / kQuadThreads;
    const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
    int32_t cnt = 0;
    for (int j = lo; j < hi; ++j) {
        const uint32_t w = sp[j];
        cnt += ((w & mA) != 0) != ((w & mB) != 0);
    }
    const int nvis = (n + 31) >> 5;
    for (int i = tid; i < nvis; i += kQuadThreads) vis[i] = 0u;
    int32_t m;
    const int32_t prefix = block_exclusive_scan(cnt, red, &m);
    if (m == 0) {
        if (tid == 0 && info) { info[0] = 0; info[1] = -1; info[2] = 0; info[3] = 0; }
        __syncthreads();
        return;
    }
    const int32_t k = (int32_t)(((uint64_t)w0 * (uint64_t)(uint32_t)m) >> 32);
    if (prefix <= k && k < prefix + cnt) {
        int32_t c = prefix;
        for (int j = lo; j < hi; ++j) {
            const uint32_t w = sp[j];
            if (((w & mA) != 0) != ((w & mB) != 0)) {
                if (c == k) {
                    red[16] = j;
                    queue[0] = (uint16_t)j;
                    vis[j >> 5] = 1u << (j & 31);
                    break;
                }
                ++c;
            }
        }
    }
    if (tid == 0) red[17] = 1;   // queue tail
    __syncthreads();
    const int32_t seed = red[16];
    // Level-synchronous breadth-first search over bonds with J != 0 inside q = -1.
    int32_t head = 0, tail = 1;
    while (head < tail) {
        for (int i = head + tid; i < tail; i += kQuadThreads) {
            const int j = queue[i];
            const uint4 r = recj[j];
            const uint32_t nb[6] = {r.y & 0xFFFFu, r.y >> 16, r.z & 0xFFFFu, r.z >> 16,
                                    r.w & 0xFFFFu, r.w >> 16};
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                const uint32_t v = nb[a];
                if ((int)v == n) continue;
                const uint32_t w = sp[v];
                if (((w & mA) != 0) == ((w & mB) != 0)) continue;
                const uint32_t bit = 1u << (v & 31u);
                const uint32_t old = atomicOr(&vis[v >> 5], bit);
                if (old & bit) continue;
                const int pos = atomicAdd(&red[17], 1);
                queue[pos] = (uint16_t)v;
            }
        }
        __syncthreads();
        head = tail;
        tail = red[17];
        __syncthreads();
    }
    const int32_t size = tail;
    int32_t branch;
    if (2 * size > n) {
        const uint32_t X = ((w1 >> 31) == 0u) ? mA : mB;
        branch = ((w1 >> 31) == 0u) ? 1 : 2;
        for (int j = tid; j < n; j += kQuadThreads) sp[j] ^= X;
    } else {
        branch = 0;
        for (int i = tid; i < size; i += kQuadThreads) sp[queue[i]] ^= (mA | mB);
    }
    if (tid == 0 && info) { info[0] = m; info[1] = seed; info[2] = size; info[3] = branch; }
    __syncthreads();
}

// Closure along x without iterating site by site.  A site y can take the cluster from y - 1
// when y and y - 1 are both in Q and joined by a bond (mr bit y - 1); the runs of such
// receivers (eu) are filled from the seeds by one addition, whose carry runs through a run of
// ones and stops at its end.  The same on the bit-reversed row fills towards lower x (edr),
// and a second pass continues a run through the wrap bond (bit lx - 1 to bit 0) from its other
// end.  low: bit 0 of each row in the word (one row, or two rows of at most 16 sites packed at
// bits 0 and 16).
struct XMasks {
    uint32_t eu;    // sites that can take the cluster from x - 1
    uint32_t edr;   // bit-reversed: sites that can take it from x + 1
    uint32_t w0;    // bit 0 of a row, reachable from bit lx - 1 through the wrap bond
    uint32_t whi;   // bit lx - 1, reachable from bit 0
};

__device__ __forceinline__ XMasks x_masks(uint32_t Q, uint32_t mr, uint32_t hi, uint32_t low)
{
    XMasks m;
    m.eu = Q & (Q << 1) & (mr << 1) & ~low;
    m.edr = __builtin_bitreverse32(Q & (Q >> 1) & mr & ~(low << hi));
    const uint32_t wb = (mr >> hi) & low;   // the wrap bond of each row, at its bit 0
    m.w0 = wb & Q;
    m.whi = (wb << hi) & Q;
    return m;
}

__device__ __forceinline__ uint32_t xfill_linear(uint32_t V, const XMasks &m)
{
    const uint32_t bu = (V << 1) & m.eu;
    const uint32_t fu = (((m.eu + bu) ^ m.eu) | bu) & m.eu;
    const uint32_t bd = (__builtin_bitreverse32(V) << 1) & m.edr;
    const uint32_t fd = (((m.edr + bd) ^ m.edr) | bd) & m.edr;
    return V | fu | __builtin_bitreverse32(fd);
}

// V (seeds, a subset of Q) grown to its connected part along x.
__device__ __forceinline__ uint32_t xfill(uint32_t V, const XMasks &m, uint32_t hi)
{
    const uint32_t U = xfill_linear(V, m);
    const uint32_t W = U | ((U >> hi) & m.w0) | ((U << hi) & m.whi);
    return W != U ? xfill_linear(W, m) : U;
}

// A lattice row's words (lx <= 32 sites; byte i = slot i, 0/1) folded four sites at a time:
// byte i of c[g] holds slot i at sites 4g..4g+3 in bits 0..3, then byte i of C[h] holds sites
// 8h..8h+7, so that one byte permute per 16 sites gathers a slot's row bits.
struct RowFold {
    uint32_t C[4];
};

__device__ __forceinline__ RowFold fold_row(const uint32_t *row, int lx)
{
    uint32_t c[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        c[g] = 0u;
        if (4 * g < lx) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (4 * g + t < lx) c[g] |= row[4 * g + t] << t;
        }
    }
    RowFold f;
#pragma unroll
    for (int h = 0; h < 4; ++h) f.C[h] = c[2 * h] | (c[2 * h + 1] << 4);
    return f;
}

// Bit x: the spin (1 = up) of the slot at site x of the folded row.
__device__ __forceinline__ uint32_t slot_row(const RowFold &f, uint32_t slot)
{
    const uint32_t sel = slot | ((slot + 4u) << 8) | 0x0C0C0000u;   // 0x0C: zero byte
    return __builtin_amdgcn_perm(f.C[1], f.C[0], sel) |
           (__builtin_amdgcn_perm(f.C[3], f.C[2], sel) << 16);
}

// Flip bytes X0 at the sites of row bits F0 and bytes X1 at those of F1 (the two pairs of a
// tile use different bytes); every word of the row is read before any is written.
__device__ __forceinline__ void flip_row(uint32_t *row, int lx, uint32_t F0, uint32_t X0,
                                         uint32_t F1, uint32_t X1)
{
#pragma unroll
    for (int x0 = 0; x0 < 32; x0 += 8) {
        if (x0 >= lx) break;
        uint32_t w[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (x0 + t < lx) w[t] = row[x0 + t];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (x0 + t < lx) {
                const uint32_t f0 = 0u - ((F0 >> (x0 + t)) & 1u);
                const uint32_t f1 = 0u - ((F1 >> (x0 + t)) & 1u);
                row[x0 + t] = w[t] ^ (f0 & X0) ^ (f1 & X1);
            }
        }
    }
}

// One propagation step of a row: the Q sites next to the cluster in the +-y, +-z rows join,
// then the row is closed along x.
__device__ __forceinline__ uint32_t row_step(const uint32_t *Vp, int r, uint32_t hi, const uint4 a,
                                             const uint4 b, uint32_t Q)
{
    const uint32_t V = Vp[r];
    const uint32_t N = (Vp[b.z & 0xFFFFu] & a.z) | (Vp[b.z >> 16] & a.w) |
                       (Vp[b.w & 0xFFFFu] & b.x) | (Vp[b.w >> 16] & b.y);
    return xfill(V | (N & Q), x_masks(Q, a.x, hi, 1u), hi);
}

// Houdayer moves on up to two replica pairs at once, on rows of lx <= 32 sites (Algorithm S2,
// ICMop).  The overlap set Q and the cluster V of each pair are bit rows; one propagation step
// adds every Q site next to V through a bond with J != 0 along y or z and then closes the row
// along x, until no row of either pair changes.  This reaches the same connected component as
// a breadth-first search from the seed.  Each thread owns consecutive rows; the bond masks of
// its first row stay in registers.  LDS: Qr[2][n_rows], Vr[2][n_rows], red[>= 24].  Pair p uses
// bytes (pa >> 8p) & 3 and (pb >> 8p) & 3 of the site words.
__device__ void icm_pairs_rows(uint32_t *sp, const uint4 *rowA, const uint4 *rowB,
                               const uint4 *rowC, int n, int lx, int nrows, int np, uint32_t pa,
                               uint32_t pb, uint4 w01, uint32_t *Qr, uint32_t *Vr, int32_t *red,
                               int32_t *info0, int32_t *info1, int32_t *dE01)
{
    uint32_t *Sr = Vr + 2 * nrows;   // spins of each pair's first replica (bit = up)
    const int tid = threadIdx.x;
    const int rpt = (nrows + kQuadThreads - 1) / kQuadThreads;
    const int r0 = min(nrows, tid * rpt), r1 = min(nrows, r0 + rpt);
    const uint32_t mA0 = 1u << (8 * (pa & 3u)), mB0 = 1u << (8 * (pb & 3u));
    const uint32_t mA1 = 1u << (8 * ((pa >> 8) & 3u)), mB1 = 1u << (8 * ((pb >> 8) & 3u));
    int32_t c0 = 0, c1 = 0;
    for (int r = r0; r < r1; ++r) {
        const RowFold f = fold_row(sp + r * lx, lx);
        const uint32_t s0 = slot_row(f, pa & 3u), q0 = s0 ^ slot_row(f, pb & 3u);
        const uint32_t s1 = slot_row(f, (pa >> 8) & 3u), q1 = s1 ^ slot_row(f, (pb >> 8) & 3u);
        Qr[r] = q0;
        Vr[r] = 0u;
        Sr[r] = s0;
        c0 += __popc(q0);
        if (np > 1) {
            Qr[nrows + r] = q1;
            Vr[nrows + r] = 0u;
            Sr[nrows + r] = s1;
            c1 += __popc(q1);
        }
    }
    int32_t m0, m1 = 0;
    for (int p = 0; p < np; ++p) {
        const int32_t cnt = p ? c1 : c0;
        int32_t m;
        const int32_t prefix = block_exclusive_scan(cnt, red, &m);
        if (p) m1 = m; else m0 = m;
        if (m == 0) continue;
        const uint32_t w = p ? w01.z : w01.x;
        const int32_t k = (int32_t)(((uint64_t)w * (uint64_t)(uint32_t)m) >> 32);
        if (prefix <= k && k < prefix + cnt) {
            int32_t c = prefix;
            for (int r = r0; r < r1; ++r) {
                uint32_t qq = Qr[p * nrows + r];
                const int32_t pc = __popc(qq);
                if (k < c + pc) {
                    for (int32_t i = 0; i < k - c; ++i) qq &= qq - 1u;
                    const int x = __builtin_ctz(qq);
                    Vr[p * nrows + r] = 1u << x;
                    red[16 + p] = r * lx + x;
                    break;
                }
                c += pc;
            }
        }
    }
    __syncthreads();
    const int32_t seed0 = m0 > 0 ? red[16] : -1;
    const int32_t seed1 = (np > 1 && m1 > 0) ? red[17] : -1;
    const uint32_t hi = (uint32_t)(lx - 1);
    const bool act0 = m0 > 0, act1 = np > 1 && m1 > 0;
    uint4 a0 = make_uint4(0u, 0u, 0u, 0u), b0 = a0;
    if (r0 < r1) {
        a0 = rowA[r0];
        b0 = rowB[r0];
    }
    while (true) {
        int changed = 0;
        for (int r = r0; r < r1; ++r) {
            const uint4 a = (r == r0) ? a0 : rowA[r];
            const uint4 b = (r == r0) ? b0 : rowB[r];
            if (act0) {
                const uint32_t Vn = row_step(Vr, r, hi, a, b, Qr[r]);
                if (Vn != Vr[r]) { Vr[r] = Vn; changed = 1; }
            }
            if (act1) {
                const uint32_t Vn = row_step(Vr + nrows, r, hi, a, b, Qr[nrows + r]);
                if (Vn != Vr[nrows + r]) { Vr[nrows + r] = Vn; changed = 1; }
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
    // cluster sizes and, for each pair, the sum of J s_i s_j of the first replica over
    // bonds that cross the cluster boundary (counted once, along +x, +y, +z)
    int32_t tot[4] = {0, 0, 0, 0};
    for (int r = r0; r < r1; ++r) {
        const uint4 a = rowA[r], b = rowB[r], cc = rowC[r];
        for (int p = 0; p < np; ++p) {
            const uint32_t *Vp = Vr + p * nrows, *Sp = Sr + p * nrows;
            const uint32_t V = Vp[r], S = Sp[r];
            tot[p] += __popc(V);
            const uint32_t Vx = (V >> 1) | (V << hi), Sx = (S >> 1) | (S << hi);
            const uint32_t X0 = (V ^ Vx) & a.x, N0 = S ^ Sx ^ cc.x;
            const uint32_t X1 = (V ^ Vp[b.z & 0xFFFFu]) & a.z, N1 = S ^ Sp[b.z & 0xFFFFu] ^ cc.y;
            const uint32_t X2 = (V ^ Vp[b.w & 0xFFFFu]) & b.x, N2 = S ^ Sp[b.w & 0xFFFFu] ^ cc.z;
            tot[2 + p] += __popc(X0 & ~N0) - __popc(X0 & N0) + __popc(X1 & ~N1) - __popc(X1 & N1) +
                          __popc(X2 & ~N2) - __popc(X2 & N2);
        }
    }
    block_sum4(tot, red);
    // cluster flip of the first replica: crossing bonds change sign -> dE = 2 * sum
    dE01[0] = (m0 > 0 && 2 * tot[0] <= n) ? 2 * tot[2] : 0;
    dE01[1] = (np > 1 && m1 > 0 && 2 * tot[1] <= n) ? 2 * tot[3] : 0;
    // both pairs' moves in one pass over the thread's rows (as in icm_pairs_planes): pair p
    // flips bytes Xf[p] at its cluster, or, for a cluster of more than half the lattice, the
    // whole lattice of one replica
    bool whole[2] = {false, false};
    uint32_t Xf[2] = {0u, 0u};
    const uint32_t all = lx >= 32 ? 0xFFFFFFFFu : (1u << lx) - 1u;
    for (int p = 0; p < np; ++p) {
        const int32_t m = p ? m1 : m0, size = tot[p];
        const uint32_t mA = p ? mA1 : mA0, mB = p ? mB1 : mB0;
        const uint32_t w1 = p ? w01.w : w01.y;
        int32_t branch = 0;
        if (m > 0) {
            if (2 * size > n) {
                Xf[p] = ((w1 >> 31) == 0u) ? mA : mB;
                branch = ((w1 >> 31) == 0u) ? 1 : 2;
                whole[p] = true;
            } else {
                Xf[p] = mA | mB;
            }
        }
        int32_t *o = p ? info1 : info0;
        if (tid == 0 && o) {
            if (m == 0) { o[0] = 0; o[1] = -1; o[2] = 0; o[3] = 0; }
            else { o[0] = m; o[1] = p ? seed1 : seed0; o[2] = size; o[3] = branch; }
        }
    }
    for (int r = r0; r < r1; ++r) {
        const uint32_t F0 = Xf[0] == 0u ? 0u : (whole[0] ? all : Vr[r]);
        const uint32_t F1 = Xf[1] == 0u ? 0u : (whole[1] ? all : Vr[nrows + r]);
        if (F0 | F1) flip_row(sp + r * lx, lx, F0, Xf[0], F1, Xf[1]);
    }
    __syncthreads();
}

// The same moves as icm_pairs_rows, for lattices whose x-rows fit one per lane with whole
// y-z planes in each wave (wave w holds planes [w ppw, (w + 1) ppw), ppw = 64 / ly).  The
// breadth-first search becomes a flood fill: inside a wave, rows grow along x in registers
// and along y and z by lane shuffles until nothing changes; then waves exchange the rows of
// their boundary planes through LDS at a work-group barrier, until no wave gains a site.
// The fill reaches the same connected component, so the cluster (and every result) is the
// same as the search's.

// The flood fill of icm_pairs_planes for both pairs (V0, V1: this lane's row of each
// pair's cluster, seeds on entry).  PACK (rows of at most 16 sites): both pairs in one
// word, so one fill along x, four lane shuffles and one exchanged word per row serve
// both.  On return Vr holds the final rows: packed (Vr[row]) or Vr[p * nrows + row].
template <bool PACK>
__device__ __forceinline__ void plane_fill(uint32_t &V0, uint32_t &V1, uint32_t Q0, uint32_t Q1,
                                           const uint4 a, const uint32_t mk[4], const int src[4],
                                           const int nbr[4], bool own, int r, int nrows,
                                           int lane, uint32_t hi, uint32_t *Vr)
{
    if (PACK) {
        uint32_t W = V0 | (V1 << 16);
        const uint32_t Qw = Q0 | (Q1 << 16);
        const XMasks xm = x_masks(Qw, a.x | (a.x << 16), hi, 0x00010001u);
        uint32_t mkw[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) mkw[d] = mk[d] | (mk[d] << 16);
        uint32_t X[2] = {0u, 0u};   // +z / -z rows from other waves
        while (true) {
            while (true) {   // closure inside the wave
                W = xfill(W, xm, hi);
                uint32_t N = 0u;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int sl = src[d] >= 0 ? src[d] : lane;
                    const uint32_t u = __shfl(W, sl, 64);
                    const uint32_t e = src[d] >= 0 ? u : (d == 2 ? X[0] : (d == 3 ? X[1] : 0u));
                    N |= e & mkw[d];
                }
                const uint32_t n = W | (N & Qw);
                const int grew = n != W;
                W = n;
                if (!__any(grew)) break;
            }
            // exchange boundary planes between waves
            if (own) Vr[r] = W;
            __syncthreads();
            int changed = 0;
            if (own) {
#pragma unroll
                for (int d = 2; d < 4; ++d) {
                    if (src[d] >= 0) continue;
                    X[d - 2] = Vr[nbr[d]];
                    if (X[d - 2] & mkw[d] & Qw & ~W) changed = 1;
                }
            }
            if (!__syncthreads_or(changed)) break;
        }
        V0 = W & 0xFFFFu;
        V1 = W >> 16;
    } else {
        uint32_t X0[2] = {0u, 0u}, X1[2] = {0u, 0u};   // +z / -z rows from other waves
        const XMasks xm0 = x_masks(Q0, a.x, hi, 1u), xm1 = x_masks(Q1, a.x, hi, 1u);
        while (true) {
            // closure inside the wave
            while (true) {
                V0 = xfill(V0, xm0, hi);
                V1 = xfill(V1, xm1, hi);
                uint32_t N0 = 0u, N1 = 0u;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int sl = src[d] >= 0 ? src[d] : lane;
                    const uint32_t u0 = __shfl(V0, sl, 64), u1 = __shfl(V1, sl, 64);
                    const uint32_t e0 = src[d] >= 0 ? u0 : (d == 2 ? X0[0] : (d == 3 ? X0[1] : 0u));
                    const uint32_t e1 = src[d] >= 0 ? u1 : (d == 2 ? X1[0] : (d == 3 ? X1[1] : 0u));
                    N0 |= e0 & mk[d];
                    N1 |= e1 & mk[d];
                }
                const uint32_t n0 = V0 | (N0 & Q0), n1 = V1 | (N1 & Q1);
                const int grew = (n0 != V0) || (n1 != V1);
                V0 = n0;
                V1 = n1;
                if (!__any(grew)) break;
            }
            // exchange boundary planes between waves
            if (own) {
                Vr[r] = V0;
                Vr[nrows + r] = V1;
            }
            __syncthreads();
            int changed = 0;
            if (own) {
#pragma unroll
                for (int d = 2; d < 4; ++d) {
                    if (src[d] >= 0) continue;
                    X0[d - 2] = Vr[nbr[d]];
                    X1[d - 2] = Vr[nrows + nbr[d]];
                    if ((X0[d - 2] & mk[d] & Q0 & ~V0) | (X1[d - 2] & mk[d] & Q1 & ~V1)) changed = 1;
                }
            }
            if (!__syncthreads_or(changed)) break;
        }
    }
}

__device__ void icm_pairs_planes(uint32_t *sp, const uint4 *rowA, const uint4 *rowB,
                                 const uint4 *rowC, int n, int lx, int ly, int lz, int np,
                                 uint32_t pa, uint32_t pb, uint4 w01, uint32_t *Qr, uint32_t *Vr,
                                 int32_t *red, int32_t *info0, int32_t *info1, int32_t *dE01)
{
    const int nrows = ly * lz;
    uint32_t *Sr = Vr + 2 * nrows;   // spins of each pair's first replica (bit = up)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ppw = 64 / ly;
    const int pl = lane / ly;
    const int z = wv * ppw + pl, y = lane - pl * ly;
    const bool own = pl < ppw && z < lz;
    const int r = own ? z * ly + y : 0;
    const uint32_t mA0 = 1u << (8 * (pa & 3u)), mB0 = 1u << (8 * (pb & 3u));
    const uint32_t mA1 = 1u << (8 * ((pa >> 8) & 3u)), mB1 = 1u << (8 * ((pb >> 8) & 3u));
    // this lane's bond masks and neighbour rows, loaded first so that the row bitsets, the
    // seed scan and its barriers cover their latency
    uint4 a = make_uint4(0u, 0u, 0u, 0u), b = a, cc = a;
    if (own) {
        a = rowA[r];
        b = rowB[r];
        cc = rowC[r];
    }
    uint32_t q0 = 0u, q1 = 0u, s0 = 0u, s1 = 0u;
    if (own) {
        const RowFold f = fold_row(sp + r * lx, lx);
        s0 = slot_row(f, pa & 3u);
        q0 = s0 ^ slot_row(f, pb & 3u);
        s1 = slot_row(f, (pa >> 8) & 3u);
        q1 = s1 ^ slot_row(f, (pb >> 8) & 3u);
        Sr[r] = s0;
        if (np > 1) Sr[nrows + r] = s1;
        else q1 = 0u;
    }
    // seeds: the k-th site with q = -1 in ascending site order; threads hold rows in
    // ascending row order (lanes past the last plane of a wave hold none)
    // (both pairs in one scan: counts of pair 1 in the upper 16 bits; n < 2^16 here)
    uint32_t V0 = 0u, V1 = 0u;
    int32_t mm;
    const int32_t pre01 = block_exclusive_scan(__popc(q0) | (__popc(q1) << 16), red, &mm);
    const int32_t m0 = mm & 0xFFFF, m1 = (int32_t)((uint32_t)mm >> 16);
    for (int p = 0; p < np; ++p) {
        const uint32_t qq0 = p ? q1 : q0;
        const int32_t cnt = __popc(qq0);
        const int32_t m = p ? m1 : m0;
        const int32_t prefix = p ? (int32_t)((uint32_t)pre01 >> 16) : (pre01 & 0xFFFF);
        if (m == 0) continue;
        const uint32_t w = p ? w01.z : w01.x;
        const int32_t k = (int32_t)(((uint64_t)w * (uint64_t)(uint32_t)m) >> 32);
        if (own && prefix <= k && k < prefix + cnt) {
            uint32_t qq = qq0;
            for (int32_t i = 0; i < k - prefix; ++i) qq &= qq - 1u;
            const int x = __builtin_ctz(qq);
            if (p) V1 = 1u << x; else V0 = 1u << x;
            red[16 + p] = r * lx + x;
        }
    }
    __syncthreads();
    const int32_t seed0 = m0 > 0 ? red[16] : -1;
    const int32_t seed1 = (np > 1 && m1 > 0) ? red[17] : -1;
    const uint32_t hi = (uint32_t)(lx - 1);
    // source lanes of the +y, -y, +z, -z neighbour rows inside this wave, -1 outside
    const int nbr[4] = {(int)(b.z & 0xFFFFu), (int)(b.z >> 16), (int)(b.w & 0xFFFFu),
                        (int)(b.w >> 16)};
    int src[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int zr = nbr[d] / ly, yr = nbr[d] - (nbr[d] / ly) * ly;
        src[d] = (own && zr / ppw == wv) ? (zr - wv * ppw) * ly + yr : -1;
    }
    const uint32_t mk[4] = {a.z, a.w, b.x, b.y};
    const uint32_t Q0 = (m0 > 0) ? q0 : 0u, Q1 = (m1 > 0) ? q1 : 0u;
    const bool pack = lx <= 16;
    if (pack)
        plane_fill<true>(V0, V1, Q0, Q1, a, mk, src, nbr, own, r, nrows, lane, hi, Vr);
    else
        plane_fill<false>(V0, V1, Q0, Q1, a, mk, src, nbr, own, r, nrows, lane, hi, Vr);
    // cluster sizes and, for each pair, the sum of J s_i s_j of the first replica over
    // bonds that cross the cluster boundary (counted once, along +x, +y, +z)
    int32_t tot[4] = {0, 0, 0, 0};
    if (own) {
        for (int p = 0; p < np; ++p) {
            const uint32_t *Sp = Sr + p * nrows;
            // final cluster row idx of pair p (packed rows: half p of Vr[idx])
            auto vrow = [&](uint32_t idx) {
                return pack ? (Vr[idx] >> (16 * p)) & 0xFFFFu : Vr[p * nrows + idx];
            };
            const uint32_t V = p ? V1 : V0, S = p ? s1 : s0;
            tot[p] += __popc(V);
            const uint32_t Vx = (V >> 1) | (V << hi), Sx = (S >> 1) | (S << hi);
            const uint32_t X0b = (V ^ Vx) & a.x, N0b = S ^ Sx ^ cc.x;
            const uint32_t X1b = (V ^ vrow(b.z & 0xFFFFu)) & a.z, N1b = S ^ Sp[b.z & 0xFFFFu] ^ cc.y;
            const uint32_t X2b = (V ^ vrow(b.w & 0xFFFFu)) & b.x, N2b = S ^ Sp[b.w & 0xFFFFu] ^ cc.z;
            tot[2 + p] += __popc(X0b & ~N0b) - __popc(X0b & N0b) + __popc(X1b & ~N1b) -
                          __popc(X1b & N1b) + __popc(X2b & ~N2b) - __popc(X2b & N2b);
        }
    }
    block_sum4(tot, red);
    // cluster flip of the first replica: crossing bonds change sign -> dE = 2 * sum
    dE01[0] = (m0 > 0 && 2 * tot[0] <= n) ? 2 * tot[2] : 0;
    dE01[1] = (np > 1 && m1 > 0 && 2 * tot[1] <= n) ? 2 * tot[3] : 0;
    // The moves of both pairs touch different bytes of the site words, so they are made in
    // one pass over this lane's row: pair p flips bytes Xf[p] at the sites of row bits F[p],
    // the cluster in both replicas, or (a cluster of more than half the lattice) the whole
    // lattice of one replica, which leaves the same pair of states up to a global flip.
    uint32_t F[2] = {0u, 0u}, Xf[2] = {0u, 0u};
    const uint32_t all = lx >= 32 ? 0xFFFFFFFFu : (1u << lx) - 1u;
    for (int p = 0; p < np; ++p) {
        const int32_t m = p ? m1 : m0, size = tot[p];
        const uint32_t mA = p ? mA1 : mA0, mB = p ? mB1 : mB0;
        const uint32_t w1 = p ? w01.w : w01.y;
        int32_t branch = 0;
        if (m > 0) {
            if (2 * size > n) {
                Xf[p] = ((w1 >> 31) == 0u) ? mA : mB;
                branch = ((w1 >> 31) == 0u) ? 1 : 2;
                F[p] = all;
            } else {
                Xf[p] = mA | mB;
                F[p] = p ? V1 : V0;
            }
        }
        int32_t *o = p ? info1 : info0;
        if (tid == 0 && o) {
            if (m == 0) { o[0] = 0; o[1] = -1; o[2] = 0; o[3] = 0; }
            else { o[0] = m; o[1] = p ? seed1 : seed0; o[2] = size; o[3] = branch; }
        }
    }
    if (own && (F[0] | F[1])) flip_row(sp + r * lx, lx, F[0], Xf[0], F[1], Xf[1]);
    __syncthreads();
}

// Replica exchange (Eq. 4): the decision for temperature pair (b, b + 1), label l, at
// attempt a.  A non-negative Delta-beta * Delta-E is always accepted; otherwise the
// precomputed threshold for |Delta E| is compared with the pair's random word.
__device__ __forceinline__ int swap_decision(const SwapArgs &A, int inst, const InstDev &I, int b,
                                             int l, int32_t e0, int32_t e1, uint32_t a)
{
    const int32_t dE = e1 - e0;
    if (dE >= 0) return 1;
    const int pair = I.swap_off + b;
    const int32_t d = -dE;
    if (d >= A.tab_len[pair]) return 0;
    const uint32_t u = philox10((uint32_t)(b * A.reps + l), a, 0u, ((uint32_t)inst << 4) | TAG_SWAP,
                                A.key0, A.key1).x;
    return u < A.tab[A.tab_off[pair] + d] ? 1 : 0;
}

// Running minimum of the instance's energies after an attempt and its trace entry.
__device__ __forceinline__ void record_best(const SwapArgs &A, int inst, int32_t m)
{
    const uint32_t cyc = A.ctr[3] + (uint32_t)A.cyc_k + 1u;
    int64_t best = A.best[inst];
    if ((int64_t)m < best) best = m;
    A.best[inst] = best;
    if (A.trace && A.record_every > 0 && (cyc % (uint32_t)A.record_every) == 0u) {
        const int64_t ti = (int64_t)(cyc / (uint32_t)A.record_every) - 1;
        if (ti < A.trace_cap) A.trace[(int64_t)inst * A.trace_cap + ti] = best;
    }
}

// Replica exchange for one instance, run by one work-group.  An accepted exchange
// swaps the logical->physical mapping of the two slots and their energies; the random
// word is keyed by the logical pair, so this is the same chain as exchanging the
// states.  Reads perm_in / E_in and writes perm / E (in place when they are the same).
__device__ void swap_instance(const SwapArgs &A, int inst, int32_t *red)
{
    const InstDev &I = A.inst[inst];
    const int R = A.reps, nb = A.n_beta;
    const int npt = (nb - 1) * R;
    const uint32_t a = A.ctr[2] + (uint32_t)A.cyc_k + 1u;
    const int32_t *pin = A.perm_in + I.slot_off, *ein = A.E_in + I.slot_off;
    int32_t *perm = A.perm + I.slot_off;
    int32_t *E = A.E + I.slot_off;
    const int nt = blockDim.x;
    if (pin != perm) {
        // separate buffers: carry every slot (padding included) over first
        const int nb4 = (I.n_slots + 3) & ~3;
        for (int i = threadIdx.x; i < nb4; i += nt) {
            perm[i] = pin[i];
            E[i] = ein[i];
        }
        __syncthreads();
    }
    if (A.acc_out)
        for (int i = threadIdx.x; i < npt; i += nt) A.acc_out[(int64_t)inst * npt + i] = -1;
    const int first = (a & 1u) ? 0 : 1;
    const int npairs = (nb - 1 - first + 1) / 2;
    for (int idx = threadIdx.x; idx < npairs * R; idx += nt) {
        const int b = first + 2 * (idx / R), l = idx - (idx / R) * R;
        const int s0 = b * R + l, s1 = s0 + R;
        const int32_t e0 = ein[s0], e1 = ein[s1];
        const int32_t p0 = pin[s0], p1 = pin[s1];
        const int acc = swap_decision(A, inst, I, b, l, e0, e1, a);
        if (acc) {
            perm[s0] = p1;
            perm[s1] = p0;
            E[s0] = e1;
            E[s1] = e0;
        }
        if (A.acc_out) A.acc_out[(int64_t)inst * npt + s0] = acc;
        A.acc_count[(int64_t)inst * npt + s0] += acc;
    }
    __syncthreads();
    int32_t m = 0x7FFFFFFF;
    for (int s = threadIdx.x; s < nb * R; s += nt) m = min(m, E[s]);
    m = wave_min(m);
    if ((threadIdx.x & 63) == 0) red[20 + (threadIdx.x >> 6)] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (nt + 63) / 64; ++w) m = min(m, red[20 + w]);
        record_best(A, inst, m);
    }
    __syncthreads();
}

// The exchange of the previous cycle done at the start of an APT work-group instead of
// in a launch of its own: the same decisions as swap_instance for the work-group's four
// logical slots (the work-group of a pair's lower slot counts it), and on quad 0 the
// running minimum.  The new mapping and energies of the four slots go to lperm / lE
// (LDS) and the mapping to A.perm.
__device__ void fused_swap_quad(const SwapArgs &A, int slot_off, int inst, int q, int32_t *lperm,
                                int32_t *lE)
{
    // the instance's slot range and swap tables follow from its index alone, so these
    // reads need not wait for its descriptor
    const int n_slots = A.n_beta * A.reps, swap_off = inst * (A.n_beta - 1);
    const int tid = threadIdx.x;
    const uint32_t a = A.ctr[2] + (uint32_t)A.cyc_k + 1u;
    const int32_t *pin = A.perm_in + slot_off, *ein = A.E_in + slot_off;
    if (tid < 4) {
        // every load of the decision is issued before any of it is used: the slot's and
        // its partner's mapping and energy, the pair's table bounds, and the random word
        const int s = 4 * q + tid;
        const int R = A.reps, nb = A.n_beta;
        const int b = s / R, l = s - b * R;
        const int first = (a & 1u) ? 0 : 1;
        int lo = -1;
        if (s < n_slots) {
            if (b >= first && ((b - first) & 1) == 0 && b + 1 < nb) lo = b;
            else if (b - 1 >= first && ((b - 1 - first) & 1) == 0) lo = b - 1;
        }
        const int s0 = lo >= 0 ? lo * R + l : s;
        const int pt = lo < 0 ? s : (s == s0 ? s0 + R : s0);
        int32_t pv = pin[s], ev = ein[s];
        const int32_t pp = pin[pt], ep = ein[pt];
        int32_t len = 0, off = 0;
        if (lo >= 0) {
            len = A.tab_len[swap_off + lo];
            off = A.tab_off[swap_off + lo];
        }
        const uint32_t u = philox10((uint32_t)s0, a, 0u, ((uint32_t)inst << 4) | TAG_SWAP, A.key0,
                                    A.key1).x;
        if (lo >= 0) {
            // Delta E of the pair (b, b + 1) = E(b + 1) - E(b)
            const int32_t dE = (s == s0) ? ep - ev : ev - ep;
            const int acc = dE >= 0 ? 1 : (-dE < len && u < A.tab[off - dE]) ? 1 : 0;
            if (acc) {
                pv = pp;
                ev = ep;
            }
            if (s == s0) A.acc_count[(int64_t)inst * (nb - 1) * R + s0] += acc;
        }
        A.perm[slot_off + s] = pv;
        lperm[tid] = pv;
        lE[tid] = ev;
    }
    if (q == 0 && tid < 64) {
        // running minimum of the energies after the exchange (the same set as before it)
        int32_t m = 0x7FFFFFFF;
        for (int i = tid; i < n_slots; i += 64) m = min(m, ein[i]);
        m = wave_min(m);
        if (tid == 0) record_best(A, inst, m);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Random initial spins (Algorithm S2: random states), slot s = 4q + i uses
// word i of the block at counter (j, 0, q, inst << 4 | tag).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kQuadThreads) void apt_init_kernel(const InstDev *insts,
                                                                const QuadDesc *desc,
                                                                uint8_t *spins, const int32_t *perm,
                                                                uint32_t key0, uint32_t key1,
                                                                uint32_t tag)
{
    const QuadDesc D = desc[blockIdx.x];
    if (D.inst < 0) return;
    const InstDev I = insts[D.inst];
    const uint32_t c3 = ((uint32_t)D.inst << 4) | tag;
    uint8_t *base = spins + I.spin_off;
    const int32_t *pp = perm + I.slot_off + 4 * D.quad;
    for (int j = threadIdx.x; j < I.npad; j += kQuadThreads) {
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if (j < I.n) w = philox10((uint32_t)j, 0u, (uint32_t)D.quad, c3, key0, key1);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            base[(int64_t)pp[i] * I.npad + j] = (j < I.n && ws[i] < 0x80000000u) ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// APT replica kernel: n_sweeps sweeps, optional ICM, optional energies.
// ---------------------------------------------------------------------------
// SCALED: rows of at most 16 thresholds (no fields), so the four table offsets of a site
// are bytes of one word.  At most 72 VGPRs, seven waves per SIMD (measured faster than six
// with more registers and than eight with spills).
// defined with the DT-SQA kernel
__device__ __forceinline__ uint4 sqa_group_words(uint32_t t, uint32_t x2, uint32_t k0, uint32_t k1);

// One site of a colour class in all four slots of the tile (Eq. 5, Eq. 6): the aligned-bond
// count per slot byte, one Philox4x32-10 block (site j, sweep, quad, instance) for the four
// uniform words, the heat-bath compare against each slot's threshold row, and the packed
// energy-change sums (Eq. 8).  Record r: x = j | d << 16 | jneg << 19 | (h + 32) << 25 and y, z, w
// the six neighbours in 16-bit fields as site indices; or with BOFF x = j | jneg << 16 |
// (h - d + imax) << 24 and the neighbours as byte offsets into the tile (4 x index), which
// saves the scaling of each neighbour address and the assembly of the table index base.
template <bool SCALED, bool BOFF>
__device__ __forceinline__ void apt_site(const AptArgs &A, uint32_t *sp, const uint32_t *lut,
                                         const uint4 r, const uint4 uq, const uint32_t c3,
                                         const uint32_t soff4, const uint32_t rev4, uint32_t &V02,
                                         uint32_t &V13, uint32_t &C4)
{
    const int ni = A.ni;
    const uint32_t j = r.x & 0xFFFFu;
    // The first half of the site's Philox block covers the latency of the neighbour reads,
    // the second half that of the threshold reads.
    const uint32_t jn = BOFF ? r.x >> 16 : r.x >> 19;
    uint32_t nb0, nb1, nb2, nb3, nb4, nb5;
    if (BOFF) {
        nb0 = lds_word(sp, r.y & 0xFFFFu);
        nb1 = lds_word(sp, r.y >> 16);
        nb2 = lds_word(sp, r.z & 0xFFFFu);
        nb3 = lds_word(sp, r.z >> 16);
        nb4 = lds_word(sp, r.w & 0xFFFFu);
        nb5 = lds_word(sp, r.w >> 16);
    } else {
        nb0 = sp[r.y & 0xFFFFu];
        nb1 = sp[r.y >> 16];
        nb2 = sp[r.z & 0xFFFFu];
        nb3 = sp[r.z >> 16];
        nb4 = sp[r.w & 0xFFFFu];
        nb5 = sp[r.w >> 16];
    }
    const uint32_t old = sp[j];
    __builtin_amdgcn_sched_barrier(0);
    // Philox block (j, t, q, instance): rounds 0-1 split into the site's part and the
    // work-group's per-sweep words (uq, as in sqa_slices), then round 2 and rounds 3-4
    const uint64_t pj = (uint64_t)0xD2511F53u * j;
    const uint32_t B = (uint32_t)(pj >> 32) ^ c3 ^ A.key1;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * B;
    const uint32_t x0r = (uint32_t)(pb >> 32) ^ uq.x, x2r = (uint32_t)pj ^ uq.y;
    const uint64_t p0r = (uint64_t)0xD2511F53u * x0r;
    const uint64_t p1r = (uint64_t)0xCD9E8D57u * x2r;
    uint32_t x[4] = {xor3_vvs((uint32_t)(p1r >> 32), (uint32_t)pb, A.key0 + 2u * 0x9E3779B9u),
                     (uint32_t)p1r, (uint32_t)(p0r >> 32) ^ uq.z, (uint32_t)p0r};
    // The round keys are derived afresh for every site (scalar additions), not held across
    // the sweep: kept live, they crowd the scalar registers of the whole kernel.
    uint32_t k0 = A.key0, k1 = A.key1;
    asm volatile("" : "+s"(k0), "+s"(k1));
    uint32_t key[2] = {k0 + 3u * 0x9E3779B9u, k1 + 3u * 0xBB67AE85u};
    philox_rounds<3, 5>(x, key);
    __builtin_amdgcn_sched_barrier(0);
    // per byte (slot): number of present bonds whose J * s_neighbour = +1
    const uint32_t k4 = (nb0 ^ bytemask(jn & 1u)) + (nb1 ^ bytemask((jn >> 1) & 1u)) +
                        (nb2 ^ bytemask((jn >> 2) & 1u)) + (nb3 ^ bytemask((jn >> 3) & 1u)) +
                        (nb4 ^ bytemask((jn >> 4) & 1u)) + (nb5 ^ bytemask((jn >> 5) & 1u));
    // table index per slot byte: 2 k + h - d + imax (>= 0, <= 2 imax)
    const uint32_t base =
        BOFF ? r.x >> 24 : ((r.x >> 25) & 63u) + (uint32_t)(A.imax - 32) - ((r.x >> 16) & 7u);
    const uint32_t idx4 = (k4 << 1) + __builtin_amdgcn_perm(0u, base, 0u);   // base in every byte
    uint32_t o0, o1, o2, o3;
    if (SCALED) {
        const uint32_t off4 = (idx4 + soff4) << 2;
        o0 = off4 & 0xFFu;
        o1 = (off4 >> 8) & 0xFFu;
        o2 = (off4 >> 16) & 0xFFu;
        o3 = off4 >> 24;
    } else {
        o0 = (idx4 & 0xFFu) << 2;
        o1 = (((idx4 >> 8) & 0xFFu) + (uint32_t)ni) << 2;
        o2 = (((idx4 >> 16) & 0xFFu) + 2u * (uint32_t)ni) << 2;
        o3 = ((idx4 >> 24) + 3u * (uint32_t)ni) << 2;
    }
    const uint32_t T3 = lds_word(lut, o3), T2 = lds_word(lut, o2);
    const uint32_t T1 = lds_word(lut, o1), T0 = lds_word(lut, o0);
    __builtin_amdgcn_sched_barrier(0);
    philox_rounds<5, 10>(x, key);
    uint32_t acc = 0u;   // bit b: new state of slot b (Eq. 6)
    acc = shift_in_lt(acc, x[3], T3);
    acc = shift_in_lt(acc, x[2], T2);
    acc = shift_in_lt(acc, x[1], T1);
    acc = shift_in_lt(acc, x[0], T0);
    const uint32_t nw = __umul24(acc, 0x00204081u) & 0x01010101u;   // bit b -> byte b
    // Eq. (8): the update changes E by -(s_new - s_old) I_j = 2 (o - n) I_j, with o, n the
    // old and new states (0/1) and I_j = index - imax
    const uint32_t fl = old ^ nw;                    // flipped slots, bytes 0/1
    // byte 1 -> 0xFF, 0 -> 0x00 (two full-rate operations, no carries)
    const uint32_t mo = (old + 0x7F7F7F7Fu) ^ 0x7F7F7F7Fu;   // where o = 1
    const uint32_t mf = (fl + 0x7F7F7F7Fu) ^ 0x7F7F7F7Fu;    // where flipped
    const uint32_t v4 = (((idx4 ^ (rev4 - idx4)) & mo) ^ (rev4 - idx4)) & mf;
    V02 += v4 & 0x00FF00FFu;
    V13 += (v4 >> 8) & 0x00FF00FFu;
    C4 += fl;
    sp[j] = nw;
}

// W: at least W waves per SIMD (the register budget: 64 VGPRs for W = 8, 72 for W = 7), a
// launch-configuration choice of the autotuner; results do not depend on it.  BOFF: the
// colour-sorted records carry byte offsets (every instance of at most 16383 sites).
template <bool SCALED, int W, bool BOFF>
__global__ __launch_bounds__(kQuadThreads) __attribute__((amdgpu_waves_per_eu(W, 8)))
void apt_quad_kernel(AptArgs A)
{
    // SCALED (at most 16 threshold entries per slot): the four tables sit in static LDS at
    // a constant address, so that a threshold read needs no base register.
    __shared__ uint32_t lut_static[SCALED ? 64 : 1];
    extern __shared__ uint32_t lds[];
    const QuadDesc D = A.desc[blockIdx.x];
    if (D.inst >= 0) {
        const InstDev I = A.inst[D.inst];
        const int tid = threadIdx.x;
        const int n = I.n, npad = I.npad, ni = A.ni;
        uint32_t *sp = lds;                              // npad + 4 words
        uint32_t *lut = SCALED ? lut_static : sp + npad + 4;   // 4 * ni
        int32_t *red = (int32_t *)(sp + npad + 4 + 4 * ni);    // 32
        uint32_t *Qr = (uint32_t *)(red + 32);           // 2 * n_rows
        uint32_t *Vr = Qr + 2 * I.n_rows;                // 2 * n_rows, then S rows 2 * n_rows
        // queue search only (no row tables: rows longer than 32 sites, or too many rows): in
        // place of the row scratch, allocated when some instance needs it
        uint32_t *vis = I.row_off >= 0 ? Vr + 4 * I.n_rows : Qr;   // (npad + 31) / 32 + 1
        uint16_t *queue = (uint16_t *)(vis + ((npad + 31) >> 5) + 1);   // npad
        const int q = D.quad;
        const int slot_off = D.inst * A.nb4;   // == I.slot_off, without waiting for I
        // The threshold rows are loaded by waves 1..3 while wave 0 makes the exchange, so that
        // the two chains of dependent loads overlap (the exchange ends with a barrier; without
        // it the gather's barrier orders the rows before the sweep).
        for (int e = tid - 64; e >= 0 && e < 4 * ni; e += kQuadThreads - 64) {
            const int i = e / ni;
            lut[e] = A.lut[(int64_t)A.slot_lut[slot_off + 4 * q + i] * ni + (e - i * ni)];
        }
        int32_t e_in = 0;   // fused exchange: this slot's energy after it (threads 0..3)
        int32_t pq[4];
        if (A.fused_swap) {
            fused_swap_quad(A.sw, slot_off, D.inst, q, red + 24, red + 28);
            for (int i = 0; i < 4; ++i) pq[i] = red[24 + i];
            if (tid < 4) e_in = red[28 + tid];
        } else {
            for (int i = 0; i < 4; ++i) pq[i] = A.perm[slot_off + 4 * q + i];
        }
        const int64_t b0 = (int64_t)pq[0] * npad, b1 = (int64_t)pq[1] * npad;
        const int64_t b2 = (int64_t)pq[2] * npad, b3 = (int64_t)pq[3] * npad;
        const uint8_t *gs = A.spins + I.spin_off;
        // gather + transpose: word j holds byte i = spin of slot 4q+i at site j; two groups of
        // four sites per thread and pass, all eight loads issued before either is transposed
        const int ng4 = npad >> 2;
        for (int g0 = tid; g0 < ng4; g0 += 2 * kQuadThreads) {
            const int g1 = g0 + kQuadThreads;
            const bool two = g1 < ng4;
            uint32_t v[2][4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int g = h ? (two ? g1 : g0) : g0;
                v[h][0] = *(const uint32_t *)(gs + b0 + 4 * g);
                v[h][1] = *(const uint32_t *)(gs + b1 + 4 * g);
                v[h][2] = *(const uint32_t *)(gs + b2 + 4 * g);
                v[h][3] = *(const uint32_t *)(gs + b3 + 4 * g);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h && !two) break;
                const int g = h ? g1 : g0;
                uint32_t o[4];
                transpose_bytes(v[h][0], v[h][1], v[h][2], v[h][3], o);
#pragma unroll
                for (int m = 0; m < 4; ++m) sp[4 * g + m] = o[m];
            }
        }
        if (tid < 4) sp[npad + tid] = 0u;
        __syncthreads();

        const uint32_t t0 = A.ctr[0] + (uint32_t)(A.cyc_k * A.n_sweeps);
        const uint32_t c3 = ((uint32_t)D.inst << 4) | A.tag;
        // this thread's share of each slot's energy change in this launch
        int32_t dE[4] = {0, 0, 0, 0};
        // Within a sweep the changes are summed in packed form: every flip of slot b adds
        // v = idx_b (a 1 -> 0 flip) or 2 imax - idx_b (0 -> 1) to 16-bit lane b of V02 (b = 0, 2)
        // or V13 (b = 1, 3), and 1 to byte b of C4; the slot's energy change is then
        // 2 (sum v - imax * flips) (Eq. 8 with I_j = idx_b - imax).  A thread updates at most
        // about 131 sites per sweep, so lanes and bytes do not overflow before the flush.
        uint32_t V02 = 0u, V13 = 0u, C4 = 0u;
        const uint32_t rev4 = 2u * (uint32_t)A.imax * 0x01010101u;
        bool full_energy = A.do_energy == 2;
        // threshold offsets: table of slot b at b * ni; with ni <= 16 the four byte offsets
        // of one site fit one word (index bytes + table starts, times 4)
        const uint32_t soff4 = (uint32_t)ni * 0x03020100u;
        for (int sw = 0; sw < A.n_sweeps; ++sw) {
            const uint32_t t = t0 + (uint32_t)sw;
            // the work-group's words of Philox rounds 0-1 for this sweep, held in vector
            // registers so that the XORs with a site's words are two-operand vector ones
            uint4 uq = sqa_group_words(t, (uint32_t)q, A.key0, A.key1);
            asm volatile("" : "+v"(uq.x), "+v"(uq.y), "+v"(uq.z));
            for (int c = 0; c < I.n_colours; ++c) {
                const uint4 *rc = A.rec_col + I.rec_off + A.inst[D.inst].col_off[c];
                const int cnt = A.inst[D.inst].col_cnt[c];
                // two sites per pass, each with its own record register, so that the record
                // of the next site loads while this one is updated
                uint4 ra = (tid < cnt) ? rc[tid] : make_uint4(0u, 0u, 0u, 0u);
                for (int i = tid; i < cnt; i += 2 * kQuadThreads) {
                    const bool has_b = i + kQuadThreads < cnt;
                    uint4 rb = make_uint4(0u, 0u, 0u, 0u);
                    if (has_b) rb = rc[i + kQuadThreads];
                    apt_site<SCALED, BOFF>(A, sp, lut, ra, uq, c3, soff4, rev4, V02, V13, C4);
                    if (!has_b) break;
                    if (i + 2 * kQuadThreads < cnt) ra = rc[i + 2 * kQuadThreads];
                    apt_site<SCALED, BOFF>(A, sp, lut, rb, uq, c3, soff4, rev4, V02, V13, C4);
                }
                __syncthreads();
            }
            dE[0] += 2 * ((int32_t)(V02 & 0xFFFFu) - A.imax * (int32_t)(C4 & 0xFFu));
            dE[1] += 2 * ((int32_t)(V13 & 0xFFFFu) - A.imax * (int32_t)((C4 >> 8) & 0xFFu));
            dE[2] += 2 * ((int32_t)(V02 >> 16) - A.imax * (int32_t)((C4 >> 16) & 0xFFu));
            dE[3] += 2 * ((int32_t)(V13 >> 16) - A.imax * (int32_t)(C4 >> 24));
            V02 = V13 = C4 = 0u;
            if (A.mom_from >= 0 && sw >= A.mom_from) {
                int32_t e[4] = {dE[0], dE[1], dE[2], dE[3]};
                block_sum4(e, red);
                if (tid < 4) {
                    const int s = 4 * q + tid;
                    if (s < I.n_slots) {
                        const int32_t e0 = A.fused_swap ? e_in : A.E[I.slot_off + s];
                        const int64_t ec = (int64_t)e0 + e[tid];
                        int64_t *mm = A.mom + 2 * (int64_t)(I.slot_off + s);
                        mm[0] += ec;
                        mm[1] += ec * ec;
                    }
                }
            }
        }

        if (A.do_icm && A.reps >= 2) {
            const uint32_t a = A.ctr[1] + (uint32_t)A.cyc_k + 1u;
            const int n_beta = I.n_slots / A.reps;
            const int npair = A.reps / 2;
            const uint4 *recj = A.rec_j + I.recj_off;
            // up to two pairs in this tile: bytes (pa, pb) and their record / random-word indices
            uint32_t pa = 0u, pb = 0u;
            int np = 0, pidx0 = 0, pidx1 = 0;
            if (A.reps == 2) {
                for (int half = 0; half < 2; ++half) {
                    const int b = 2 * q + half;
                    if (b >= n_beta || !A.icm_on[D.inst * n_beta + b]) continue;
                    pa |= (uint32_t)(2 * half) << (8 * np);
                    pb |= (uint32_t)(2 * half + 1) << (8 * np);
                    if (np) pidx1 = b; else pidx0 = b;
                    ++np;
                }
            } else if (A.reps == 4) {
                const int b = q;
                if (b < n_beta && A.icm_on[D.inst * n_beta + b]) {
                    const uint4 wp = philox10((uint32_t)b, a, 0u,
                                              ((uint32_t)D.inst << 4) | TAG_ICM_PAIR, A.key0, A.key1);
                    const uint32_t pairing = (uint32_t)(((uint64_t)wp.x * 3u) >> 32);
                    // matchings {01,23}, {02,13}, {03,12}: partner of label 0, then the other two
                    const uint32_t p1 = pairing + 1u;
                    pa = 0u | ((p1 == 1u ? 2u : 1u) << 8);
                    pb = p1 | ((p1 == 3u ? 2u : 3u) << 8);
                    pidx0 = b * npair;
                    pidx1 = b * npair + 1;
                    np = 2;
                    if (A.icm_pairs == 1) {
                        // one move per call: the pair named by the top bit of the block's word 1
                        if (wp.y >> 31) {
                            pa >>= 8;
                            pb >>= 8;
                            pidx0 = pidx1;
                        }
                        pa &= 0xFFu;
                        pb &= 0xFFu;
                        np = 1;
                    }
                }
            }
            if (np > 0) {
                const uint32_t c3p = ((uint32_t)D.inst << 4) | TAG_ICM_PICK;
                const uint4 u0 = philox10((uint32_t)pidx0, a, 0u, c3p, A.key0, A.key1);
                const uint4 u1 = philox10((uint32_t)pidx1, a, 0u, c3p, A.key0, A.key1);
                int32_t *info0 = A.icm_info + ((int64_t)I.info_off + pidx0) * 4;
                int32_t *info1 = A.icm_info + ((int64_t)I.info_off + pidx1) * 4;
                if (I.row_off >= 0) {
                    int32_t d01[2];
                    if (I.planes)
                        icm_pairs_planes(sp, A.rowA + I.row_off, A.rowB + I.row_off,
                                         A.rowC + I.row_off, n, I.lx, I.ly, I.lz, np, pa, pb,
                                         make_uint4(u0.x, u0.y, u1.x, u1.y), Qr, Vr, red, info0,
                                         info1, d01);
                    else
                        icm_pairs_rows(sp, A.rowA + I.row_off, A.rowB + I.row_off,
                                       A.rowC + I.row_off, n, I.lx, I.n_rows, np, pa, pb,
                                       make_uint4(u0.x, u0.y, u1.x, u1.y), Qr, Vr, red, info0,
                                       info1, d01);
                    if (tid == 0) {
                        // isoenergetic move: the partner's energy changes by the opposite amount
                        dE[pa & 3u] += d01[0];
                        dE[pb & 3u] -= d01[0];
                        if (np > 1) {
                            dE[(pa >> 8) & 3u] += d01[1];
                            dE[(pb >> 8) & 3u] -= d01[1];
                        }
                    }
                } else {
                    full_energy = true;
                    icm_pair(sp, recj, n, (int)(pa & 3u), (int)(pb & 3u), u0.x, u0.y, queue, vis,
                             red, info0);
                    if (np > 1)
                        icm_pair(sp, recj, n, (int)((pa >> 8) & 3u), (int)((pb >> 8) & 3u), u1.x,
                                 u1.y, queue, vis, red, info1);
                }
            }
        }

        if (A.do_energy && full_energy) {
            int32_t e[4];
            quad_energy(sp, A.rec_j + I.recj_off, n, red, e);
            if (tid < 4) {
                const int s = 4 * q + tid;
                if (s < I.n_slots) A.E[I.slot_off + s] = e[tid];
            }
        } else if (A.do_energy) {
            block_sum4_last(dE, red);
            if (tid < 4) {
                const int s = 4 * q + tid;
                if (s < I.n_slots) {
                    if (A.fused_swap) A.E[I.slot_off + s] = e_in + dE[tid];
                    else A.E[I.slot_off + s] += dE[tid];
                }
            }
        } else if (A.fused_swap && tid < 4 && 4 * q + tid < I.n_slots) {
            A.E[I.slot_off + 4 * q + tid] = e_in;
        }

        if (A.n_sweeps > 0 || A.do_icm) {
            uint8_t *gw = A.spins + I.spin_off;
            for (int g = tid; g < (npad >> 2); g += kQuadThreads) {
                uint32_t o[4];
                transpose_bytes(sp[4 * g], sp[4 * g + 1], sp[4 * g + 2], sp[4 * g + 3], o);
                *(uint32_t *)(gw + b0 + 4 * g) = o[0];
                *(uint32_t *)(gw + b1 + 4 * g) = o[1];
                *(uint32_t *)(gw + b2 + 4 * g) = o[2];
                *(uint32_t *)(gw + b3 + 4 * g) = o[3];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Replica exchange (Eq. 4) as its own launch, one 64-lane work-group per instance.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void apt_swap_kernel(SwapArgs A)
{
    __shared__ int32_t red[32];
    swap_instance(A, blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// DT-SQA
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSqaThreads) void sqa_init_kernel(SqaArgs A)
{
    const int inst = blockIdx.x / A.R, r = blockIdx.x - inst * A.R;
    const InstDev I = A.inst[inst];
    uint32_t *g = A.spins + I.spin_off + (int64_t)r * I.npad * 2;
    const uint32_t c3 = ((uint32_t)inst << 4) | TAG_SQA_INIT;
    const int ngrp = (A.H + 3) >> 2;
    for (int j = threadIdx.x; j < I.npad; j += kSqaThreads) {
        uint32_t wd[2] = {0u, 0u};
        if (j < I.n) {
            for (int p = 0; p < 2; ++p)
                for (int gq = 0; gq < ngrp; ++gq) {
                    const uint4 u = philox10(((uint32_t)j << 1) | (uint32_t)p, 0u,
                                             ((uint32_t)r << 16) | (uint32_t)gq, c3, A.key0, A.key1);
                    const uint32_t us[4] = {u.x, u.y, u.z, u.w};
                    for (int i = 0; i < 4; ++i) {
                        const int h = 4 * gq + i;
                        // word 0 holds slices 0, 2, ..., word 1 slices 1, 3, ... (M / 2 of them)
                        if (h < (p == 0 ? A.H : A.M / 2) && us[i] < 0x80000000u) wd[p] |= 1u << h;
                    }
                }
        }
        g[2 * j] = wd[0];
        g[2 * j + 1] = wd[1];
    }
}

__device__ __forceinline__ uint32_t rotl_h(uint32_t x, int H, uint32_t mask)
{
    return ((x << 1) | (x >> (H - 1))) & mask;
}

__device__ __forceinline__ uint32_t rotr_h(uint32_t x, int H, uint32_t mask)
{
    return ((x >> 1) | (x << (H - 1))) & mask;
}

// Byte offset of the 4-bit slice group g of a bit plane into a 16-entry
// 32-bit table: ((x >> 4g) & 15) * 4.
__device__ __forceinline__ uint32_t nib_off(uint32_t x, int g)
{
    return g == 0 ? ((x << 2) & 0x3Cu) : ((x >> (4 * g - 2)) & 0x3Cu);
}

// Two bit planes a, b interleaved by 4-bit slice group: byte m of the even word holds
// group 2m of a (low nibble) and of b (high nibble), byte m of the odd word group 2m + 1.
__device__ __forceinline__ void pair_planes(uint32_t a, uint32_t b, uint32_t &ev, uint32_t &od)
{
    ev = (a & 0x0F0F0F0Fu) | ((b << 4) & 0xF0F0F0F0u);
    od = ((a >> 4) & 0x0F0F0F0Fu) | (b & 0xF0F0F0F0u);
}

// Byte offset of group g of a pair of planes into a 256-entry 32-bit table.
__device__ __forceinline__ uint32_t pair_off(uint32_t ev, uint32_t od, int g)
{
    return (((g & 1) ? od : ev) >> (8 * (g >> 1)) & 0xFFu) << 2;
}

// New states of the H slices of one parity at one site (Supplementary Eq. S.3 with
// the heat-bath rule of Eq. 6).  Slice h = 4 g + i takes word i of the Philox block
// of group g; its threshold index is a byte of idx4 (relative to lut, the row already
// moved by the site's field and degree), the sum of the contributions of the bit
// planes of the aligned-neighbour count (c0, c1, c2) and of the number of up Trotter
// neighbours (t0, t1), read from two pair tables (planes c0, c1 and c2, t0, indexed by
// a byte of pair_planes) and one 16-entry table (t1).  Groups run from the
// highest to the lowest so that the borrow chain leaves slice h at bit h.  The block
// counter is (2 j + p, step, r << 16 | g, instance): the groups of a site differ only in
// word 2, so the first two rounds split into a part of the site (D, C, E: the products
// of 2 j + p and of round 0's second output word, see sqa_site) and a part of the group
// and step, U = {U1, U2, U3} from ug[g] (sqa_group_words), after which the state of round 2
// is (D ^ U1, E, C ^ U2, .) and round 2's second XOR pair takes U3.  SCALED: table indices
// are stored pre-multiplied by 4 (byte offsets), possible when the table has <= 64 rows.
// NG > 0: NG groups, unrolled; NG == 0: ngrp groups, not unrolled.
template <int NG, bool SCALED>
__device__ __forceinline__ uint32_t sqa_slices(const uint32_t *lut, const uint32_t *tab01,
                                               const uint32_t *tab2t, const uint32_t *tab1,
                                               uint32_t e01, uint32_t o01, uint32_t e2t,
                                               uint32_t o2t, uint32_t t1b, uint32_t D,
                                               uint32_t C, uint32_t E, const uint4 *ug,
                                               uint32_t k0, uint32_t k1, int ngrp)
{
    uint32_t res = 0u;
    const int ng = NG > 0 ? NG : ngrp;
    // Software pipeline: the spread-table reads of group g - 1 and the threshold reads
    // of group g are issued before group g's Philox block, whose arithmetic covers
    // their LDS latency.
    uint32_t s0 = lds_word(tab01, pair_off(e01, o01, ng - 1));
    uint32_t s1 = lds_word(tab2t, pair_off(e2t, o2t, ng - 1));
    uint32_t s2 = lds_word(tab1, nib_off(t1b, ng - 1));
    uint4 U = ug[ng - 1];
#pragma unroll
    for (int g = ng - 1; g >= 0; --g) {
        const uint32_t idx4 = s0 + s1 + s2;
        uint32_t o0, o1, o2, o3;
        if (SCALED) {
            o0 = idx4 & 0xFFu;
            o1 = (idx4 >> 8) & 0xFFu;
            o2 = (idx4 >> 16) & 0xFFu;
            o3 = idx4 >> 24;
        } else {
            o0 = (idx4 << 2) & 0x3FCu;
            o1 = (idx4 >> 6) & 0x3FCu;
            o2 = (idx4 >> 14) & 0x3FCu;
            o3 = (idx4 >> 22) & 0x3FCu;
        }
        const uint32_t T3 = lds_word(lut, o3), T2 = lds_word(lut, o2);
        const uint32_t T1 = lds_word(lut, o1), T0 = lds_word(lut, o0);
        const uint4 Ug = U;
        if (g > 0) {
            s0 = lds_word(tab01, pair_off(e01, o01, g - 1));
            s1 = lds_word(tab2t, pair_off(e2t, o2t, g - 1));
            s2 = lds_word(tab1, nib_off(t1b, g - 1));
            U = ug[g - 1];
        }
        __builtin_amdgcn_sched_barrier(0);
        // round 2 (key k + 2 W) on the state after round 1, then rounds 3..9
        const uint32_t x0 = D ^ Ug.x, x2 = C ^ Ug.y;
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t x[4] = {xor3_vvs((uint32_t)(p1 >> 32), E, k0 + 2u * 0x9E3779B9u), (uint32_t)p1,
                         (uint32_t)(p0 >> 32) ^ Ug.z, (uint32_t)p0};
        uint32_t key[2] = {k0 + 3u * 0x9E3779B9u, k1 + 3u * 0xBB67AE85u};
        philox_rounds<3, 10>(x, key);
        res = shift_in_lt(res, x[3], T3);
        res = shift_in_lt(res, x[2], T2);
        res = shift_in_lt(res, x[1], T1);
        res = shift_in_lt(res, x[0], T0);
    }
    return res;
}

// The group-and-step part of the first two Philox rounds of sqa_slices for counter
// (., t, r << 16 | g, c3) under (k0, k1): U1 = lo(M1 x2) ^ (k0 + W0), and with
// A = hi(M1 x2) ^ t ^ k0 (round 0's first output word), U2 = hi(M0 A) ^ (k1 + W1) and
// U3 = lo(M0 A) ^ (k1 + 2 W1).
__device__ __forceinline__ uint4 sqa_group_words(uint32_t t, uint32_t x2, uint32_t k0, uint32_t k1)
{
    const uint64_t q = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t A = (uint32_t)(q >> 32) ^ t ^ k0;
    const uint64_t pa = (uint64_t)0xD2511F53u * A;
    return make_uint4((uint32_t)q ^ (k0 + 0x9E3779B9u), (uint32_t)(pa >> 32) ^ (k1 + 0xBB67AE85u),
                      (uint32_t)pa ^ (k1 + 2u * 0xBB67AE85u), 0u);
}

// Heat-bath update of the slices of parity P (slice 2 h + P at bit h) at the site of record
// rr (Supplementary Eq. S.3): the aligned-neighbour count of every slice, bit-sliced over the
// six spatial neighbours, the number of up Trotter neighbours from the other parity's word,
// then sqa_slices.  ODD (an odd number M of slices, H = (M + 1) / 2): word 0 holds H slices and
// word 1 H - 1; the ring closes between slice M - 1 (bit H - 1 of word 0) and slice 0 (bit 0),
// so word 0's Trotter neighbours come partly from word 0 itself, and only the bits in umask
// are written (the rest keep their values: they belong to other phases).
template <int NG, bool SCALED, int P, bool ODD = false>
__device__ __forceinline__ void sqa_site(const SqaArgs &A, const uint4 rr, uint32_t *sp,
                                         const uint32_t *lrow, const uint32_t *tab01,
                                         const uint32_t *tab2t, const uint32_t *tab1,
                                         uint32_t mask, int H, const uint4 *ug, uint32_t c3,
                                         int ngrp, uint32_t umask = 0u)
{
    const uint32_t j = rr.x & 0xFFFFu;
    const uint32_t jn = rr.x >> 19;
    // aligned words: bit h = 1 when J * s_neighbour = +1 in slice 2h + P
    // (the record holds the neighbours' word offsets 2 nb + P)
    const uint32_t a0 = sp[rr.y & 0xFFFFu] ^ (0u - (jn & 1u));
    const uint32_t a1 = sp[rr.y >> 16] ^ (0u - ((jn >> 1) & 1u));
    const uint32_t a2 = sp[rr.z & 0xFFFFu] ^ (0u - ((jn >> 2) & 1u));
    const uint32_t a3 = sp[rr.z >> 16] ^ (0u - ((jn >> 3) & 1u));
    const uint32_t a4 = sp[rr.w & 0xFFFFu] ^ (0u - ((jn >> 4) & 1u));
    const uint32_t a5 = sp[rr.w >> 16] ^ (0u - ((jn >> 5) & 1u));
    // bit-sliced 6-input count: k = c0 + 2 c1 + 4 c2 per slice
    const uint32_t s1 = a0 ^ a1 ^ a2, k1 = (a0 & a1) | (a2 & (a0 ^ a1));
    const uint32_t s2 = a3 ^ a4 ^ a5, k2 = (a3 & a4) | (a5 & (a3 ^ a4));
    const uint32_t cy = s1 & s2;
    const uint32_t c0 = (s1 ^ s2) & mask;
    const uint32_t c1 = (k1 ^ k2 ^ cy) & mask;
    const uint32_t c2 = ((k1 & k2) | (cy & (k1 ^ k2))) & mask;
    // Trotter neighbours 2h + P - 1 and 2h + P + 1 from the other parity's word
    uint32_t up, dn;
    if constexpr (ODD) {
        const uint32_t mask1 = mask >> 1;   // word 1's H - 1 slices
        const uint32_t ev = sp[2 * j];
        if (P) {
            up = ev & mask1;                 // slice 2h
            dn = (ev >> 1) & mask1;          // slice 2h + 2 (bit H - 1: slice M - 1)
        } else {
            const uint32_t od = sp[2 * j + 1] & mask1;
            up = od | ((ev & 1u) << (H - 1));                    // 2h + 1; for M - 1: slice 0
            dn = ((od << 1) & mask) | ((ev >> (H - 1)) & 1u);    // 2h - 1; for 0: slice M - 1
        }
    } else if (P) {
        const uint32_t ev = sp[2 * j];
        up = ev;
        dn = rotr_h(ev, H, mask);
    } else {
        const uint32_t od = sp[2 * j + 1];
        up = rotl_h(od, H, mask);
        dn = od;
    }
    const uint32_t t0b = up ^ dn, t1b = up & dn;
    // the site's part of the threshold index, 3 (h - d + smax), moves the row
    const uint32_t *lsite = lrow + 3 * ((int32_t)((rr.x >> 25) & 63u) - 32 -
                                        (int32_t)((rr.x >> 16) & 7u) + A.smax);
    uint32_t e01, o01, e2t, o2t;
    pair_planes(c0, c1, e01, o01);
    pair_planes(c2, t0b, e2t, o2t);
    // the site's part of Philox rounds 0 and 1 (word 0 of the counter is 2 j + P)
    const uint64_t pj = (uint64_t)0xD2511F53u * ((j << 1) | (uint32_t)P);
    const uint32_t B = (uint32_t)(pj >> 32) ^ c3 ^ A.key1;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * B;
    const uint32_t res = sqa_slices<NG, SCALED>(lsite, tab01, tab2t, tab1, e01, o01, e2t, o2t,
                                                t1b, (uint32_t)(pb >> 32), (uint32_t)pj,
                                                (uint32_t)pb, ug, A.key0, A.key1, ngrp);
    if constexpr (ODD)
        sp[2 * j + P] = (sp[2 * j + P] & ~umask) | (res & umask);
    else
        sp[2 * j + P] = res & mask;
}

// v += c for P-bit vertical counters (plane q = bit q of every bit position's count).
template <int P>
__device__ __forceinline__ void vadd(uint32_t v[P], uint32_t c)
{
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const uint32_t d = v[q] & c;
        v[q] ^= c;
        c = d;
    }
}

// Per-slice totals over a wave of the vertical counters v0 (slices 2h, bit h) and v1 (slices
// 2h + 1): plane q of slice bit h across the 64 lanes is one ballot.  Returns, in lane
// k = 2h + p, the wave's count for slice k (0 in lanes >= 2H).
template <int P>
__device__ __forceinline__ int32_t ballot_slice_counts(const uint32_t v0[P], const uint32_t v1[P], int H)
{
    const int lane = threadIdx.x & 63;
    int32_t mine = 0;
#pragma unroll
    for (int h = 0; h < 32; ++h) {
        if (h >= H) break;
        int32_t u0 = 0, u1 = 0;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            u0 += (int32_t)__popcll(__ballot((v0[q] >> h) & 1u)) << q;
            u1 += (int32_t)__popcll(__ballot((v1[q] >> h) & 1u)) << q;
        }
        mine = lane == 2 * h ? u0 : mine;
        mine = lane == 2 * h + 1 ? u1 : mine;
    }
    return mine;
}

// Unsatisfied bonds of every slice of one replica (no fields): the calling thread folds the
// forward bonds of its sites (j = tid, tid + threads, ...), 32 slices per parity word, into
// P-bit vertical counters; ballot_slice_counts turns them into the wave's per-slice counts.
template <int P>
__device__ __forceinline__ int32_t sqa_unsat_counts(const uint4 *recj, const uint32_t *sp, int n,
                                                    int threads, uint32_t mask, int H)
{
    uint32_t v0[P], v1[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v0[q] = v1[q] = 0u;
    for (int j = threadIdx.x; j < n; j += threads) {
        const uint4 rr = recj[j];
        const uint32_t jn = rr.x >> 19, w0 = sp[2 * j], w1 = sp[2 * j + 1];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint32_t nb = a == 0 ? (rr.y & 0xFFFFu) : (a == 1 ? (rr.z & 0xFFFFu) : (rr.w & 0xFFFFu));
            // no bond (dummy neighbour): nothing to count
            const uint32_t live = nb == (uint32_t)n ? 0u : mask;
            const uint32_t neg = 0u - ((jn >> (2 * a)) & 1u);
            vadd<P>(v0, (w0 ^ sp[2 * nb] ^ neg) & live);
            vadd<P>(v1, (w1 ^ sp[2 * nb + 1] ^ neg) & live);
        }
    }
    return ballot_slice_counts<P>(v0, v1, H);
}

// Sites where slice k disagrees with slice 0 (word 0, bit 0), for every slice of one replica
// held in global memory (pairs of words per site, as in SqaArgs::spins).
template <int P>
__device__ __forceinline__ int32_t sqa_disagree_counts(const uint32_t *g, int n, uint32_t mask, int H)
{
    uint32_t v0[P], v1[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v0[q] = v1[q] = 0u;
    for (int j = threadIdx.x; j < n; j += 256) {
        const uint2 w = *(const uint2 *)(g + 2 * j);
        const uint32_t b = 0u - (w.x & 1u);
        vadd<P>(v0, (w.x ^ b) & mask);
        vadd<P>(v1, (w.y ^ b) & mask);
    }
    return ballot_slice_counts<P>(v0, v1, H);
}

// The work-group size is a launch-time choice (a multiple of 64, at most 1024);
// waves are limited to 64 VGPRs (8 waves per SIMD).
template <int NG, bool SCALED>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8)))
void sqa_kernel(SqaArgs A)
{
    const int THREADS = blockDim.x;
    // Tables at fixed (static) LDS addresses, so that table offsets need no base
    // register: thresholds (<= 256 entries), spread tables, reduction scratch.  The
    // replica lives in dynamic LDS.
    __shared__ __align__(16) uint32_t tabs[kSqaTabWords];
    extern __shared__ uint32_t lds[];
    const int inst = blockIdx.x / A.R, r = blockIdx.x - inst * A.R;
    const InstDev I = A.inst[inst];
    const int tid = threadIdx.x;
    const int n = I.n, npad = I.npad, H = A.H;
    const uint32_t mask = (H >= 32) ? 0xFFFFFFFFu : ((1u << H) - 1u);
    uint32_t *lut = tabs;                       // 2 * 128 (double-buffered rows)
    // Spread tables: for 4-bit slice groups of bit planes, the planes' contribution
    // to the four threshold indices, one byte per slice.  Index weights: 6, 12, 24
    // for the aligned-neighbour count bits, 1, 2 for the number of up Trotter
    // neighbours (table index = 6 k + t + 3 (h - d + smax)), times 4 when SCALED.
    // Planes c0 and c1 share one 256-entry table, c2 and t0 another.
    uint32_t *tab01 = tabs + 256;               // 256
    uint32_t *tab2t = tabs + 512;               // 256
    uint32_t *tab1 = tabs + 768;                // 16
    int32_t *red = (int32_t *)(tabs + 784);     // 2 * 64
    uint4 *ugrp = (uint4 *)(tabs + 912);        // [2][8] group words of the Philox rounds
                                                // 0-1 (sqa_group_words), by step parity
    uint32_t *sp = lds;                         // 2 * (npad + 1)
    uint32_t *g = A.spins + I.spin_off + (int64_t)r * npad * 2;
    for (int i = tid; i < 2 * npad; i += THREADS) sp[i] = g[i];
    if (tid < 2) sp[2 * npad + tid] = 0u;
    for (int e = tid; e < 528; e += THREADS) {
        // bit i of a nibble -> byte i
        auto spread = [](uint32_t nib) {
            return (nib & 1u) | ((nib & 2u) << 7) | ((nib & 4u) << 14) | ((nib & 8u) << 21);
        };
        const uint32_t lo = (uint32_t)e & 15u, hi = ((uint32_t)e >> 4) & 15u;
        const uint32_t v = e < 256   ? 6u * spread(lo) + 12u * spread(hi)
                           : e < 512 ? 24u * spread(lo) + spread(hi)
                                     : 2u * spread(lo);
        tabs[256 + e] = (SCALED ? 4u : 1u) * v;
    }
    const uint32_t c3 = ((uint32_t)inst << 4) | TAG_SQA_SWEEP;
    const int ngrp = (H + 3) >> 2;
    if (A.n_steps > 0 && tid < ngrp)
        ugrp[tid] = sqa_group_words((uint32_t)A.t0, ((uint32_t)r << 16) | (uint32_t)tid, A.key0,
                                    A.key1);
    // Threshold rows: a table of <= 128 entries is double-buffered, the next step's
    // row written during the current step's first phase (no extra barrier); a larger
    // table is reloaded between steps.
    // An energy-only launch (n_steps == 0) has no threshold table (A.lut may be null).
    const bool dbuf = A.nl <= 128;
    if (dbuf && A.n_steps > 0)
        for (int i = tid; i < A.nl; i += THREADS) lut[i] = A.lut[(int64_t)A.lut_step0 * A.nl + i];
    __syncthreads();
    for (int st = 0; st < A.n_steps; ++st) {
        const uint32_t t = (uint32_t)(A.t0 + st);
        const uint32_t *lrow = lut + (dbuf ? 128 * (st & 1) : 0);
        const uint4 *ug = ugrp + 8 * (st & 1);
        if (!dbuf) {
            for (int i = tid; i < A.nl; i += THREADS)
                lut[i] = A.lut[(int64_t)(A.lut_step0 + st) * A.nl + i];
            __syncthreads();
        }
        // every phase ends with a barrier, so the previous step's readers of this
        // step's double buffer (and of a reloaded table) are done
        for (int c = 0; c < I.n_colours; ++c) {
            if (dbuf && c == 0 && st + 1 < A.n_steps)
                for (int i = tid; i < A.nl; i += THREADS)
                    lut[128 * ((st + 1) & 1) + i] = A.lut[(int64_t)(A.lut_step0 + st + 1) * A.nl + i];
            if (c == 0 && st + 1 < A.n_steps && tid < ngrp)
                ugrp[8 * ((st + 1) & 1) + tid] = sqa_group_words(
                    t + 1u, ((uint32_t)r << 16) | (uint32_t)tid, A.key0, A.key1);
            const uint4 *rc = A.rec + I.rec_off + A.inst[inst].col_off[c];
            const int cnt = A.inst[inst].col_cnt[c];
            // parity 0 sites first, then parity 1 (each thread continues its stride across
            // the boundary, so only the wave that straddles it runs both bodies)
            const int n0 = A.inst[inst].col_p1[c];
            int i = tid;
            if constexpr (NG == 0) {
                if (A.M & 1) {
                    // odd M: word 0 but its last slice, word 1, then the last slice alone
                    const int n2 = A.inst[inst].col_p2[c];
                    const uint32_t last = 1u << (H - 1);
                    for (; i < n0; i += THREADS)
                        sqa_site<0, SCALED, 0, true>(A, rc[i], sp, lrow, tab01, tab2t, tab1, mask,
                                                     H, ug, c3, ngrp, mask & ~last);
                    for (; i < n2; i += THREADS)
                        sqa_site<0, SCALED, 1, true>(A, rc[i], sp, lrow, tab01, tab2t, tab1, mask,
                                                     H, ug, c3, ngrp, mask >> 1);
                    for (; i < cnt; i += THREADS)
                        sqa_site<0, SCALED, 0, true>(A, rc[i], sp, lrow, tab01, tab2t, tab1, mask,
                                                     H, ug, c3, ngrp, last);
                    __syncthreads();
                    continue;
                }
            }
            for (; i < n0; i += THREADS)
                sqa_site<NG, SCALED, 0>(A, rc[i], sp, lrow, tab01, tab2t, tab1, mask, H, ug, c3,
                                        ngrp);
            for (; i < cnt; i += THREADS)
                sqa_site<NG, SCALED, 1>(A, rc[i], sp, lrow, tab01, tab2t, tab1, mask, H, ug, c3,
                                        ngrp);
            __syncthreads();
        }
    }
    __syncthreads();
    for (int i = tid; i < 2 * npad; i += THREADS) g[i] = sp[i];
    if (A.do_energy && A.no_field) {
        // Energy (Eq. 8, original couplings, no fields) of every slice k = 2h + p:
        // E_k = 2 U_k - bonds with U_k the number of unsatisfied bonds, counted bit-sliced
        // per wave (sqa_unsat_counts) and summed over the waves in red[k].
        const int M = A.M;
        for (int k = tid; k < M; k += THREADS) red[k] = 0;
        const int per = 3 * ((n + THREADS - 1) / THREADS);
        const int lane = tid & 63;
        const uint4 *recj = A.rec_j + I.recj_off;
        const int32_t mine = per < 32 ? sqa_unsat_counts<5>(recj, sp, n, THREADS, mask, H)
                                      : sqa_unsat_counts<kSqaPlanes>(recj, sp, n, THREADS, mask, H);
        __syncthreads();
        if (lane < M) atomicAdd(&red[lane], mine);
        __syncthreads();
        for (int k = tid; k < M; k += THREADS) {
            const int32_t e = 2 * red[k] - I.n_bonds;
            A.slice_E[((int64_t)inst * A.R + r) * M + k] = e;
            red[64 + k] = e;
        }
    } else if (A.do_energy) {
        // Energy (Eq. 8, original couplings) of every slice k, threads split over (k, sites).
        const int M = A.M;
        for (int k = tid; k < 2 * M; k += THREADS) red[k] = 0;
        __syncthreads();
        const uint4 *recj = A.rec_j + I.recj_off;
        const int parts = THREADS / M > 1 ? THREADS / M : 1;
        for (int task = tid; task < M * parts; task += THREADS) {
            const int k = task % M, part = task / M;
            const int p = k & 1, h = k >> 1;
            int32_t acc = 0;
            for (int j = part; j < n; j += parts) {
                const uint4 rr = recj[j];
                const uint32_t jn = rr.x >> 19;
                const uint32_t nbs[6] = {rr.y & 0xFFFFu, rr.y >> 16, rr.z & 0xFFFFu, rr.z >> 16,
                                         rr.w & 0xFFFFu, rr.w >> 16};
                int32_t kk = 0;
#pragma unroll
                for (int a = 0; a < 6; ++a)
                    kk += (int32_t)(((sp[2 * nbs[a] + p] >> h) & 1u) ^ ((jn >> a) & 1u));
                const int32_t d = (int32_t)((rr.x >> 16) & 7u);
                const int32_t hh = (int32_t)((rr.x >> 25) & 63u) - 32;
                const int32_t v = 2 * kk - d + 2 * hh;
                acc += ((sp[2 * j + p] >> h) & 1u) ? v : -v;
            }
            atomicAdd(&red[k], acc);
        }
        __syncthreads();
        for (int k = tid; k < M; k += THREADS) {
            const int32_t e = -red[k] / 2;
            A.slice_E[((int64_t)inst * A.R + r) * M + k] = e;
            red[64 + k] = e;
        }
    }
    if (A.do_energy && A.best_key) {
        // this replica's lowest slice energy (ties: lowest slice), then the instance minimum
        __syncthreads();
        if (tid < 64) {
            uint64_t key = ~0ull;
            if (tid < A.M)
                key = ((uint64_t)(uint32_t)(red[64 + tid] + 0x40000000) << 32) |
                      (uint32_t)(r * A.M + tid);
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                const uint64_t o = __shfl_xor(key, d, 64);
                key = o < key ? o : key;
            }
            if (tid == 0) atomicMin((unsigned long long *)&A.best_key[inst], (unsigned long long)key);
        }
    }
}

// Correlation along the Trotter direction (C_k = (1/n) sum_i s_{i,0} s_{i,k}), exactly: the
// number of sites where slice k agrees with slice 0, agree[inst][r][k], one work-group of 256
// threads per replica.
__global__ __launch_bounds__(256) void sqa_corr_kernel(SqaArgs A, int32_t *agree)
{
    __shared__ int32_t red[64];
    const int inst = blockIdx.x / A.R, r = blockIdx.x - inst * A.R;
    const InstDev I = A.inst[inst];
    const uint32_t *g = A.spins + I.spin_off + (int64_t)r * I.npad * 2;
    const int H = A.H, n = I.n, M = A.M;
    const uint32_t mask = (H >= 32) ? 0xFFFFFFFFu : ((1u << H) - 1u);
    if (threadIdx.x < 64) red[threadIdx.x] = 0;
    const int per = (n + 255) / 256;
    const int32_t mine = per < 32 ? sqa_disagree_counts<5>(g, n, mask, H)
                                  : sqa_disagree_counts<kSqaPlanes>(g, n, mask, H);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    if (lane < M) atomicAdd(&red[lane], mine);
    __syncthreads();
    if (threadIdx.x < M) agree[((int64_t)inst * A.R + r) * M + threadIdx.x] = n - red[threadIdx.x];
}

// Spins of the slice that best_key[i] names (replica r, slice k = 2h + p: bit h of word p),
// as +1/-1, one work-group per instance.
__global__ __launch_bounds__(256) void sqa_best_state_kernel(SqaArgs A, int n_max, int8_t *out)
{
    const int inst = blockIdx.x;
    const InstDev I = A.inst[inst];
    const uint32_t q = (uint32_t)A.best_key[inst];
    const int r = (int)(q / (uint32_t)A.M), k = (int)(q % (uint32_t)A.M);
    const uint32_t *g = A.spins + I.spin_off + (int64_t)r * I.npad * 2;
    int8_t *o = out + (int64_t)inst * n_max;
    for (int j = threadIdx.x; j < n_max; j += 256)
        o[j] = j < I.n ? (((g[2 * j + (k & 1)] >> (k >> 1)) & 1u) ? 1 : -1) : 0;
}

__global__ void advance_kernel(uint32_t *ctr, uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr[0] += d0;
        ctr[1] += d1;
        ctr[2] += d2;
        ctr[3] += d3;
    }
}

__global__ void fill_i64_kernel(int64_t *p, int64_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Results written to the caller's device memory (the device-output calls).
// ---------------------------------------------------------------------------
// The first `cols` entries of every row of src (row stride src_stride), widened to int64, rows
// packed one after another.
__global__ void widen_rows_kernel(const int32_t *src, int src_stride, int64_t *dst, int rows, int cols)
{
    const int64_t total = (int64_t)rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols;
        dst[i] = src[r * src_stride + (i - r * cols)];
    }
}

// APT spins as +1/-1, [n_inst][n_slots][n_max] (0 past an instance's n): logical slot s of
// instance i is physical buffer perm[i][s].  Grid (n_slots, n_inst).
__global__ void apt_spins_out_kernel(const uint8_t *spins, const int32_t *perm, const InstDev *inst,
                                     int nb4, int n_slots, int n_max, int8_t *out)
{
    const int s = blockIdx.x, i = blockIdx.y;
    const InstDev I = inst[i];
    const uint8_t *src = spins + I.spin_off + (int64_t)perm[(int64_t)i * nb4 + s] * I.npad;
    int8_t *dst = out + ((int64_t)i * n_slots + s) * n_max;
    for (int j = threadIdx.x; j < n_max; j += blockDim.x)
        dst[j] = j < I.n ? (src[j] ? 1 : -1) : 0;
}

// DT-SQA spins as +1/-1, [n_inst][R][M][n_max]: slice k = 2 h + p is bit h of word p.
// Grid (R * M, n_inst).
__global__ void sqa_spins_out_kernel(const uint32_t *words, const InstDev *inst, int R, int M,
                                     int n_max, int8_t *out)
{
    const int rk = blockIdx.x, i = blockIdx.y;
    const int r = rk / M, k = rk - r * M;
    const InstDev I = inst[i];
    const uint32_t *w = words + I.spin_off + (int64_t)r * I.npad * 2;
    int8_t *dst = out + (((int64_t)i * R + r) * M + k) * n_max;
    for (int j = threadIdx.x; j < n_max; j += blockDim.x)
        dst[j] = j < I.n ? (((w[2 * j + (k & 1)] >> (k >> 1)) & 1u) ? 1 : -1) : 0;
}

// The lowest slice energy of every instance from its key ((E + 2^30) << 32 | (r M + k)).
__global__ void best_key_energy_kernel(const uint64_t *key, int n, int64_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int64_t)(uint32_t)(key[i] >> 32) - 0x40000000;
}

// ---------------------------------------------------------------------------
// Adaptive-ladder stage (Methods, APT details): all chains of an instance run at the
// instance's current beta, so 32 of them share one word per site and one threshold
// row, and the aligned-neighbour count is summed bit-sliced as in the DT-SQA kernel.
// One work-group per (instance, word of 32 chains); the words stay in LDS for all
// sweeps of a launch.  Chain c = 32 w + 4 g + i takes word i of the Philox block
// (site, sweep, 8 w + g, instance) -- the counter of slot c in the APT sweep.
// ---------------------------------------------------------------------------
// New states of the chains of one word at one site (heat-bath rule of Eq. 6 at the
// instance's beta): chain 4 g + i takes word i of the Philox block (j, t, 8 w + g,
// instance) of group g (rounds 0-1 split as in sqa_slices: D, C, E of the site, ug[g] of the
// group and sweep); its threshold index is a byte of the sum of a pair-table read
// (planes c0, c1) and a 16-entry table read (plane c2), relative to lsite, the row moved
// by the site's field and degree.  Groups run from the highest to the lowest so that the
// borrow chain leaves chain b at bit b; the table reads of group g - 1 and the threshold
// reads of group g are issued before group g's Philox block.  NG > 0: NG groups,
// unrolled; NG == 0: ngrp groups, not unrolled.
template <int NG>
__device__ __forceinline__ uint32_t adapt_groups(const uint32_t *lsite, const uint32_t *tab01,
                                                 const uint32_t *tab2, uint32_t e01, uint32_t o01,
                                                 uint32_t c2, uint32_t D, uint32_t C, uint32_t E,
                                                 const uint4 *ug, uint32_t k0, uint32_t k1,
                                                 int ngrp)
{
    const int ng = NG > 0 ? NG : ngrp;
    uint32_t res = 0u;
    uint32_t s0v = lds_word(tab01, pair_off(e01, o01, ng - 1));
    uint32_t s1v = lds_word(tab2, nib_off(c2, ng - 1));
    uint4 U = ug[ng - 1];
#pragma unroll
    for (int g = ng - 1; g >= 0; --g) {
        const uint32_t idx4 = s0v + s1v;
        const uint32_t T3 = lds_word(lsite, idx4 >> 24);
        const uint32_t T2 = lds_word(lsite, (idx4 >> 16) & 0xFFu);
        const uint32_t T1 = lds_word(lsite, (idx4 >> 8) & 0xFFu);
        const uint32_t T0 = lds_word(lsite, idx4 & 0xFFu);
        const uint4 Ug = U;
        if (g > 0) {
            s0v = lds_word(tab01, pair_off(e01, o01, g - 1));
            s1v = lds_word(tab2, nib_off(c2, g - 1));
            U = ug[g - 1];
        }
        __builtin_amdgcn_sched_barrier(0);
        // round 2 (key k + 2 W) on the state after round 1, then rounds 3..9
        const uint32_t x0 = D ^ Ug.x, x2 = C ^ Ug.y;
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t x[4] = {xor3_vvs((uint32_t)(p1 >> 32), E, k0 + 2u * 0x9E3779B9u), (uint32_t)p1,
                         (uint32_t)(p0 >> 32) ^ Ug.z, (uint32_t)p0};
        uint32_t key[2] = {k0 + 3u * 0x9E3779B9u, k1 + 3u * 0xBB67AE85u};
        philox_rounds<3, 10>(x, key);
        res = shift_in_lt(res, x[3], T3);
        res = shift_in_lt(res, x[2], T2);
        res = shift_in_lt(res, x[1], T1);
        res = shift_in_lt(res, x[0], T0);
    }
    return res;
}

// One colour phase of the adaptive stage's sweep: the sites of the phase are split over
// the work-group's threads; each updates all chains of the word at its sites.
template <int NG>
__device__ __forceinline__ void adapt_phase(const AdaptArgs &A, const uint4 *rc, int cnt,
                                            uint32_t *sp, const uint32_t *tab01,
                                            const uint32_t *tab2, const uint32_t *lut,
                                            const uint4 *ug, uint32_t c3, int ng, uint32_t vmask)
{
    for (int i = threadIdx.x; i < cnt; i += kAdaptThreads) {
        const uint4 r = rc[i];
        const uint32_t j = r.x & 0xFFFFu, jn = r.x >> 19;
        // aligned words: bit b = 1 when J s_neighbour = +1 for chain b
        const uint32_t a0 = sp[r.y & 0xFFFFu] ^ (0u - (jn & 1u));
        const uint32_t a1 = sp[r.y >> 16] ^ (0u - ((jn >> 1) & 1u));
        const uint32_t a2 = sp[r.z & 0xFFFFu] ^ (0u - ((jn >> 2) & 1u));
        const uint32_t a3 = sp[r.z >> 16] ^ (0u - ((jn >> 3) & 1u));
        const uint32_t a4 = sp[r.w & 0xFFFFu] ^ (0u - ((jn >> 4) & 1u));
        const uint32_t a5 = sp[r.w >> 16] ^ (0u - ((jn >> 5) & 1u));
        const uint32_t s1 = a0 ^ a1 ^ a2, k1 = (a0 & a1) | (a2 & (a0 ^ a1));
        const uint32_t s2 = a3 ^ a4 ^ a5, k2 = (a3 & a4) | (a5 & (a3 ^ a4));
        const uint32_t cy = s1 & s2;
        const uint32_t c0 = s1 ^ s2, c1 = k1 ^ k2 ^ cy, c2 = (k1 & k2) | (cy & (k1 ^ k2));
        // the site's part of the table index, h - d + imax, moves the row
        const uint32_t *lsite = lut + ((int32_t)((r.x >> 25) & 63u) - 32 -
                                       (int32_t)((r.x >> 16) & 7u) + A.imax);
        uint32_t e01, o01;
        pair_planes(c0, c1, e01, o01);
        // the site's part of Philox rounds 0 and 1 (word 0 of the counter is j)
        const uint64_t pj = (uint64_t)0xD2511F53u * j;
        const uint32_t B = (uint32_t)(pj >> 32) ^ c3 ^ A.key1;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * B;
        const uint32_t res = adapt_groups<NG>(lsite, tab01, tab2, e01, o01, c2,
                                              (uint32_t)(pb >> 32), (uint32_t)pj, (uint32_t)pb, ug,
                                              A.key0, A.key1, ng);
        sp[j] = res & vmask;
    }
}

// Work-group -> (instance, chain word).  When the last word of each instance holds fewer
// than 32 chains (one to seven Philox groups against eight), the full words come first
// and the short ones last: work-groups are handed to the eight XCDs in turn, so with the
// natural order (instance-major) every short word of a four-word instance would land on
// two of the eight XCDs and the full ones on the other six.
__device__ __forceinline__ void adapt_block(const AdaptArgs &A, int b, int &inst, int &w)
{
    const int nf = A.nw - 1;
    if ((A.n_chains & 31) == 0 || nf == 0) {
        inst = b / A.nw;
        w = b - inst * A.nw;
    } else if (b < A.n_inst * nf) {
        inst = b / nf;
        w = b - inst * nf;
    } else {
        inst = b - A.n_inst * nf;
        w = nf;
    }
}

__global__ __launch_bounds__(kAdaptThreads) void adapt_init_kernel(AdaptArgs A)
{
    int inst, w;
    adapt_block(A, blockIdx.x, inst, w);
    const InstDev I = A.inst[inst];
    const int nch = min(32, A.n_chains - 32 * w), ng = (nch + 3) >> 2;
    const uint32_t c3 = ((uint32_t)inst << 4) | TAG_ADAPT_INIT;
    uint32_t *g = A.words + ((int64_t)inst * A.nw + w) * A.wstride;
    for (int j = threadIdx.x; j < (int)A.wstride; j += kAdaptThreads) {
        uint32_t wd = 0u;
        if (j < I.n)
            for (int gq = 0; gq < ng; ++gq) {
                const uint4 u = philox10((uint32_t)j, 0u, (uint32_t)(8 * w + gq), c3, A.key0, A.key1);
                const uint32_t us[4] = {u.x, u.y, u.z, u.w};
                for (int i = 0; i < 4; ++i)
                    if (4 * gq + i < nch && us[i] < 0x80000000u) wd |= 1u << (4 * gq + i);
            }
        g[j] = wd;
    }
}

__global__ __launch_bounds__(kAdaptThreads) void adapt_kernel(AdaptArgs A)
{
    // Static LDS: pair spread table of planes c0, c1 (256), spread table of c2 (16),
    // threshold row (<= 64), per-thread counters for the energies, reduction scratch.
    __shared__ uint32_t tabs[kAdaptTabWords];
    __shared__ uint32_t vc[kAdaptPlanes * kAdaptThreads];
    constexpr int kWaves = kAdaptThreads / 64;
    __shared__ int32_t red[kAdaptRedWords];
    // group words of Philox rounds 0-1 (sqa_group_words) by sweep parity and group
    __shared__ __align__(16) uint4 ugrp[2 * 8];
    extern __shared__ uint32_t sp[];   // npad + 1 words, the last one the zero dummy
    int inst, w;
    adapt_block(A, blockIdx.x, inst, w);
    const InstDev I = A.inst[inst];
    const int tid = threadIdx.x, n = I.n, npad = I.npad;
    const int nch = min(32, A.n_chains - 32 * w), ng = (nch + 3) >> 2;
    const uint32_t vmask = nch >= 32 ? 0xFFFFFFFFu : ((1u << nch) - 1u);
    uint32_t *gw = A.words + ((int64_t)inst * A.nw + w) * A.wstride;
    for (int i = tid; i <= npad; i += kAdaptThreads) sp[i] = i < npad ? gw[i] : 0u;
    uint32_t *tab01 = tabs, *tab2 = tabs + 256, *lut = tabs + 272;
    for (int e = tid; e < 272; e += kAdaptThreads) {
        // bit i of a nibble -> byte i; table index = I + imax = 2 k + (h - d + imax), k =
        // c0 + 2 c1 + 4 c2, stored times 4 (byte offsets into the threshold row)
        auto spread = [](uint32_t nib) {
            return (nib & 1u) | ((nib & 2u) << 7) | ((nib & 4u) << 14) | ((nib & 8u) << 21);
        };
        const uint32_t lo = (uint32_t)e & 15u, hi = ((uint32_t)e >> 4) & 15u;
        tabs[e] = e < 256 ? 8u * spread(lo) + 16u * spread(hi) : 32u * spread(lo);
    }
    for (int i = tid; i < A.ni; i += kAdaptThreads) lut[i] = A.lut[(int64_t)inst * A.ni + i];
    // bonds along +x, +y, +z present (J != 0): E = 2 (unsatisfied) - bonds
    if (tid == 0) red[kWaves * 32] = 0;
    __syncthreads();
    int32_t nbc = 0;
    for (int j = tid; j < n; j += kAdaptThreads) {
        const uint4 r = A.rec_j[I.recj_off + j];
        nbc += ((r.y & 0xFFFFu) != (uint32_t)n) + ((r.z & 0xFFFFu) != (uint32_t)n) +
               ((r.w & 0xFFFFu) != (uint32_t)n);
    }
    if (A.n_sweeps > 0 && tid < ng)
        ugrp[tid] = sqa_group_words(A.t0, 8u * (uint32_t)w + (uint32_t)tid, A.key0, A.key1);
    atomicAdd(&red[kWaves * 32], nbc);
    __syncthreads();
    const int32_t bonds = red[kWaves * 32];
    const uint32_t c3 = ((uint32_t)inst << 4) | TAG_ADAPT_SWEEP;
    int64_t S1 = 0, S2 = 0;   // moments of chain 32 w + tid (threads < nch)
    for (int sw = 0; sw < A.n_sweeps; ++sw) {
        const uint32_t t = A.t0 + (uint32_t)sw;
        const uint4 *ug = ugrp + 8 * (sw & 1);
        for (int c = 0; c < I.n_colours; ++c) {
            // the next sweep's group words into the other buffer (its readers, the previous
            // sweep's phases, are past a barrier)
            if (c == 0 && sw + 1 < A.n_sweeps && tid < ng)
                ugrp[8 * ((sw + 1) & 1) + tid] =
                    sqa_group_words(t + 1u, 8u * (uint32_t)w + (uint32_t)tid, A.key0, A.key1);
            const uint4 *rc = A.rec_col + I.rec_off + A.inst[inst].col_off[c];
            const int cnt = A.inst[inst].col_cnt[c];
            if (ng == 8)
                adapt_phase<8>(A, rc, cnt, sp, tab01, tab2, lut, ug, c3, ng, vmask);
            else
                adapt_phase<0>(A, rc, cnt, sp, tab01, tab2, lut, ug, c3, ng, vmask);
            __syncthreads();
        }
        if (sw >= A.mom_from) {
            // unsatisfied bonds per chain: each thread adds the +x, +y, +z bonds of its
            // sites into a vertical counter (plane p = bit p of every chain's count)
            uint32_t v[kAdaptPlanes];
#pragma unroll
            for (int p = 0; p < kAdaptPlanes; ++p) v[p] = 0u;
            for (int j = tid; j < n; j += kAdaptThreads) {
                const uint4 r = A.rec_j[I.recj_off + j];
                const uint32_t jn = r.x >> 19, wj = sp[j];
                const uint32_t nbf[3] = {r.y & 0xFFFFu, r.z & 0xFFFFu, r.w & 0xFFFFu};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (nbf[a] == (uint32_t)n) continue;
                    uint32_t carry = wj ^ sp[nbf[a]] ^ (0u - ((jn >> (2 * a)) & 1u));
#pragma unroll
                    for (int p = 0; p < kAdaptPlanes; ++p) {
                        if (p >= A.planes) break;
                        const uint32_t cp = v[p] & carry;
                        v[p] ^= carry;
                        carry = cp;
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < kAdaptPlanes; ++p)
                if (p < A.planes) vc[p * kAdaptThreads + tid] = v[p];
            __syncthreads();
            // chain cc, sources part * 32 .. part * 32 + 31
            const int cc = tid & 31, part = tid >> 5;
            int32_t cntu = 0;
            for (int src = part * 32; src < part * 32 + 32; ++src)
#pragma unroll
                for (int p = 0; p < kAdaptPlanes; ++p)
                    if (p < A.planes) cntu += (int32_t)(((vc[p * kAdaptThreads + src] >> cc) & 1u) << p);
            cntu += __shfl_xor(cntu, 32, 64);
            if ((tid & 63) < 32) red[(tid >> 6) * 32 + cc] = cntu;
            __syncthreads();
            if (tid < nch) {
                int32_t u = 0;
#pragma unroll
                for (int q = 0; q < kWaves; ++q) u += red[q * 32 + tid];
                const int64_t e = 2 * (int64_t)u - bonds;
                S1 += e;
                S2 += e * e;
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < npad; i += kAdaptThreads) gw[i] = sp[i];
    if (tid < nch) {
        int64_t *m = A.mom + ((int64_t)inst * A.n_chains + 32 * w + tid) * 2;
        m[0] = S1;
        m[1] = S2;
    }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_apt_init(const InstDev *inst_d, const QuadDesc *desc, int n_blocks,
                           uint8_t *spins, const int32_t *perm, uint32_t key0, uint32_t key1,
                           uint32_t tag, hipStream_t s)
{
    hipLaunchKernelGGL(apt_init_kernel, dim3(n_blocks), dim3(kQuadThreads), 0, s, inst_d, desc,
                       spins, perm, key0, key1, tag);
    return hipGetLastError();
}

static hipError_t allow_lds(const void *fn, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <bool SCALED, int W, bool BOFF>
hipError_t launch_apt_quad_t(const AptArgs &a, size_t lds_bytes, hipStream_t s)
{
    hipError_t e = allow_lds((const void *)apt_quad_kernel<SCALED, W, BOFF>, lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((apt_quad_kernel<SCALED, W, BOFF>), dim3(a.n_blocks), dim3(kQuadThreads),
                       lds_bytes, s, a);
    return hipGetLastError();
}

template <bool SCALED, bool BOFF>
hipError_t launch_apt_quad_w(const AptArgs &a, size_t lds_bytes, hipStream_t s)
{
    if (a.waves == 8) return launch_apt_quad_t<SCALED, 8, BOFF>(a, lds_bytes, s);
    return launch_apt_quad_t<SCALED, 7, BOFF>(a, lds_bytes, s);
}

hipError_t launch_apt_quad(const AptArgs &a, size_t lds_bytes, hipStream_t s)
{
    if (a.boff)
        return a.ni <= 16 ? launch_apt_quad_w<true, true>(a, lds_bytes, s)
                          : launch_apt_quad_w<false, true>(a, lds_bytes, s);
    return a.ni <= 16 ? launch_apt_quad_w<true, false>(a, lds_bytes, s)
                      : launch_apt_quad_w<false, false>(a, lds_bytes, s);
}

hipError_t launch_apt_swap(const SwapArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(apt_swap_kernel, dim3(a.n_inst), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sqa_init(const SqaArgs &a, int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL(sqa_init_kernel, dim3(n_inst * a.R), dim3(kSqaThreads), 0, s, a);
    return hipGetLastError();
}

template <int NG, bool SCALED>
hipError_t launch_sqa_t(const SqaArgs &a, int n_inst, size_t lds_bytes, int threads, hipStream_t s)
{
    const void *k = (const void *)sqa_kernel<NG, SCALED>;
    hipError_t e = allow_lds(k, lds_bytes);   // the dynamic part (the tables are static)
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((sqa_kernel<NG, SCALED>), dim3(n_inst * a.R), dim3(threads), lds_bytes, s, a);
    return hipGetLastError();
}

bool sqa_config_valid(int threads) { return threads >= 128 && threads <= 1024 && threads % 64 == 0; }

hipError_t launch_sqa(const SqaArgs &a, int n_inst, size_t lds_bytes, int threads, hipStream_t s)
{
    if (!sqa_config_valid(threads)) return hipErrorInvalidValue;
    const bool scaled = a.nl <= 64;
    const int ngrp = (a.H + 3) >> 2;
    if (a.M & 1)   // odd M: the general kernel, which holds the three-part phases
        return scaled ? launch_sqa_t<0, true>(a, n_inst, lds_bytes, threads, s)
                      : launch_sqa_t<0, false>(a, n_inst, lds_bytes, threads, s);
    if (ngrp == 8)
        return scaled ? launch_sqa_t<8, true>(a, n_inst, lds_bytes, threads, s)
                      : launch_sqa_t<8, false>(a, n_inst, lds_bytes, threads, s);
    // M = 32 and M = 16 with pre-scaled tables also run unrolled
    if (ngrp == 4 && scaled) return launch_sqa_t<4, true>(a, n_inst, lds_bytes, threads, s);
    if (ngrp == 2 && scaled) return launch_sqa_t<2, true>(a, n_inst, lds_bytes, threads, s);
    return scaled ? launch_sqa_t<0, true>(a, n_inst, lds_bytes, threads, s)
                  : launch_sqa_t<0, false>(a, n_inst, lds_bytes, threads, s);
}

hipError_t launch_widen_rows(const int32_t *src, int src_stride, int64_t *dst, int rows, int cols,
                             hipStream_t s)
{
    const int64_t total = (int64_t)rows * cols;
    const int blocks = (int)std::min<int64_t>(4096, (total + 255) / 256);
    hipLaunchKernelGGL(widen_rows_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, s, src, src_stride,
                       dst, rows, cols);
    return hipGetLastError();
}

hipError_t launch_apt_spins_out(const uint8_t *spins, const int32_t *perm, const InstDev *inst,
                                int n_inst, int nb4, int n_slots, int n_max, int8_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(apt_spins_out_kernel, dim3(n_slots, n_inst), dim3(256), 0, s, spins, perm, inst,
                       nb4, n_slots, n_max, out);
    return hipGetLastError();
}

hipError_t launch_sqa_spins_out(const uint32_t *words, const InstDev *inst, int n_inst, int R, int M,
                                int n_max, int8_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(sqa_spins_out_kernel, dim3(R * M, n_inst), dim3(256), 0, s, words, inst, R, M,
                       n_max, out);
    return hipGetLastError();
}

hipError_t launch_best_key_energy(const uint64_t *key, int n, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(best_key_energy_kernel, dim3((n + 255) / 256), dim3(256), 0, s, key, n, out);
    return hipGetLastError();
}

hipError_t launch_sqa_best_state(const SqaArgs &a, int n_inst, int n_max, int8_t *out,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(sqa_best_state_kernel, dim3(n_inst), dim3(256), 0, s, a, n_max, out);
    return hipGetLastError();
}

hipError_t launch_sqa_corr(const SqaArgs &a, int n_inst, int32_t *agree, hipStream_t s)
{
    hipLaunchKernelGGL(sqa_corr_kernel, dim3(n_inst * a.R), dim3(256), 0, s, a, agree);
    return hipGetLastError();
}

hipError_t launch_adapt_init(const AdaptArgs &a, int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL(adapt_init_kernel, dim3(n_inst * a.nw), dim3(kAdaptThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adapt(const AdaptArgs &a, int n_inst, size_t lds_bytes, hipStream_t s)
{
    hipError_t e = allow_lds((const void *)adapt_kernel, lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adapt_kernel, dim3(n_inst * a.nw), dim3(kAdaptThreads), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_advance(uint32_t *ctr, uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3,
                          hipStream_t s)
{
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, ctr, d0, d1, d2, d3);
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(fill_i64_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace sg
