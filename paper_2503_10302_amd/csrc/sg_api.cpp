// sg_api.cpp -- host side of libsg: validation, colour classes, FP64
// acceptance tables, device memory, launches and the C ABI of include/sg.h.
//
// Threshold tables are built in FP64 and rounded to 32-bit integers here, on
// the host, so that every spin decision on the device is an exact integer
// comparison.  This file must be compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <system_error>
#include <thread>
#include <tuple>
#include <vector>

#include "sg.h"
#include "sg_internal.h"
#include "sg_host.h"

using namespace sg;

namespace {

// ------------------------------------------------------------------ errors
struct Failure {
    sg_status code;
    std::string msg;
};

[[noreturn]] void fail(sg_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Failure{code, buf};
}

void hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return;
    // The failed call also left the thread's last error set; clear it, or the next kernel
    // launch, checked with hipGetLastError, would report this failure again.
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory) fail(SG_ENOMEM, "%s: out of device memory", what);
    fail(SG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count, const char *what)
    {
        release();
        if (count == 0) count = 1;
        hip_check(hipMalloc((void **)&p, count * sizeof(T)), what);
        n = count;
    }
    void upload(const T *h, size_t count, hipStream_t s, const char *what)
    {
        if (count > n) alloc(count, what);
        hip_check(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s), what);
    }
    void upload(const std::vector<T> &v, hipStream_t s, const char *what)
    {
        alloc(v.size(), what);
        if (!v.empty())
            hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s),
                      what);
    }
    void download(T *h, size_t count, hipStream_t s, const char *what) const
    {
        hip_check(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s), what);
    }
};

// ------------------------------------------------------------------ geometry
struct Lat {
    int Lx, Ly, Lz;
    uint32_t periodic;
    int n;
    std::vector<int8_t> J;        // [n][3]
    std::vector<int8_t> h;        // [n]
    std::vector<int8_t> cmap;     // [n] given colour map, or empty: the closed form
    int cmap_colours = 0;
    int len(int a) const { return a == 0 ? Lx : (a == 1 ? Ly : Lz); }
    int coord(int j, int a) const
    {
        if (a == 0) return j % Lx;
        if (a == 1) return (j / Lx) % Ly;
        return j / (Lx * Ly);
    }
    int stride(int a) const { return a == 0 ? 1 : (a == 1 ? Lx : Lx * Ly); }
    // neighbours: nbt[6 j + 2 a + s], along axis a in direction +1 (s = 0) or -1 (s = 1),
    // -1 where there is none (an open end, or an axis of one site)
    std::vector<int32_t> nbt;
    void build_neighbours()
    {
        nbt.assign((size_t)6 * n, -1);
        for (int z = 0; z < Lz; ++z)
            for (int y = 0; y < Ly; ++y)
                for (int x = 0; x < Lx; ++x) {
                    const int j = (z * Ly + y) * Lx + x;
                    const int c[3] = {x, y, z};
                    for (int a = 0; a < 3; ++a) {
                        const int L = len(a), st = stride(a);
                        if (L < 2) continue;
                        const bool per = (periodic >> a) & 1u;
                        int32_t *o = &nbt[(size_t)6 * j + 2 * a];
                        if (c[a] + 1 < L) o[0] = j + st;
                        else if (per) o[0] = j - (L - 1) * st;
                        if (c[a] > 0) o[1] = j - st;
                        else if (per) o[1] = j + (L - 1) * st;
                    }
                }
    }
    // neighbour of j along axis a (dir = +1/-1) or -1
    int nbr(int j, int a, int dir) const { return nbt[(size_t)6 * j + 2 * a + (dir < 0)]; }
    int coupling(int j, int a, int dir) const
    {
        const int nb = nbr(j, a, dir);
        if (nb < 0) return 0;
        return dir > 0 ? J[3 * j + a] : J[3 * nb + a];
    }
    bool odd_ring(int a) const
    {
        const int L = len(a);
        return ((periodic >> a) & 1u) && L >= 3 && (L & 1);
    }
    // Per-axis colour label: i mod 2, or 2 at the last site of an odd periodic axis
    // (when three colours are in use).  Neighbours differ in exactly one label.
    int label_sum(int j, bool three) const
    {
        int s = 0;
        for (int a = 0; a < 3; ++a) {
            const int c = coord(j, a);
            s += (three && odd_ring(a) && c == len(a) - 1) ? 2 : (c & 1);
        }
        return s;
    }
    bool any_odd_ring() const { return odd_ring(0) || odd_ring(1) || odd_ring(2); }
    // Spatial colouring (Methods, "Graph Coloring"): the given map, else the closed form
    // (label sum mod 2, or mod 3 with an odd periodic axis).
    int n_colours() const
    {
        if (!cmap.empty()) return std::max(cmap_colours, 1);
        return any_odd_ring() ? 3 : 2;
    }
    int colour(int j) const
    {
        if (!cmap.empty()) return cmap[j];
        const bool three = any_odd_ring();
        return label_sum(j, three) % (three ? 3 : 2);
    }
    int hmax() const
    {
        int m = 0;
        for (int8_t v : h) m = std::max(m, std::abs((int)v));
        return m;
    }
    bool has_field() const
    {
        for (int8_t v : h)
            if (v) return true;
        return false;
    }
    int bonds() const
    {
        int b = 0;
        for (int j = 0; j < n; ++j)
            for (int a = 0; a < 3; ++a) b += coupling(j, a, +1) != 0;
        return b;
    }
    int64_t max_energy_gap() const
    {
        int64_t s = 0;
        for (int j = 0; j < n; ++j) {
            for (int a = 0; a < 3; ++a) s += std::abs(coupling(j, a, +1));
            s += std::abs((int)h[j]);
        }
        return 2 * s;
    }
};

Lat copy_lattice(const sg_lattice &L, int idx)
{
    if (L.Lx < 1 || L.Ly < 1 || L.Lz < 1) fail(SG_EINVAL, "instance %d: lattice size < 1", idx);
    const int64_t n = (int64_t)L.Lx * L.Ly * L.Lz;
    if (n > kMaxN) fail(SG_EINVAL, "instance %d: %lld sites exceed %d", idx, (long long)n, kMaxN);
    if (L.periodic > 7u) fail(SG_EINVAL, "instance %d: periodic mask must be 0..7", idx);
    if (!L.J) fail(SG_EINVAL, "instance %d: J is NULL", idx);
    Lat t;
    t.Lx = L.Lx; t.Ly = L.Ly; t.Lz = L.Lz;
    t.periodic = L.periodic;
    t.n = (int)n;
    t.J.assign(L.J, L.J + 3 * n);
    t.h.assign(n, 0);
    if (L.h) t.h.assign(L.h, L.h + n);
    for (int64_t i = 0; i < 3 * n; ++i)
        if (t.J[i] < -1 || t.J[i] > 1) fail(SG_EINVAL, "instance %d: J must be -1, 0 or +1", idx);
    for (int8_t v : t.h)
        if (v < -kMaxH || v > kMaxH) fail(SG_EINVAL, "instance %d: |h| must be <= %d", idx, kMaxH);
    t.build_neighbours();
    // values stored across open boundaries are not bonds
    for (int j = 0; j < t.n; ++j)
        for (int a = 0; a < 3; ++a)
            if (t.nbr(j, a, +1) < 0) t.J[3 * j + a] = 0;
    return t;
}

// Site record, see sg_internal.h.
uint4 make_record(const Lat &L, int j, uint32_t parity)
{
    uint32_t nb[6];
    uint32_t jneg = 0, d = 0;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s) {
            const int dir = s ? -1 : +1;
            const int v = L.nbr(j, a, dir);
            const int c = v < 0 ? 0 : L.J[3 * (s ? v : j) + a];   // L.coupling(j, a, dir)
            const int slot = 2 * a + s;
            if (v < 0 || c == 0) {
                nb[slot] = (uint32_t)L.n;
            } else {
                nb[slot] = (uint32_t)v;
                ++d;
                if (c < 0) jneg |= 1u << slot;
            }
        }
    uint4 r;
    r.x = (uint32_t)j | (d << 16) | (jneg << 19) | ((uint32_t)(L.h[j] + 32) << 25) | (parity << 31);
    r.y = nb[0] | (nb[1] << 16);
    r.z = nb[2] | (nb[3] << 16);
    r.w = nb[4] | (nb[5] << 16);
    return r;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// ------------------------------------------------------------------ thresholds (FP64)
uint32_t to_threshold(double p)
{
    if (p >= 1.0) return 0xFFFFFFFFu;
    return (uint32_t)(p * 4294967296.0);
}

// Eq. (6): P(s = +1 | I) = (1 + tanh(beta I)) / 2.
uint32_t heat_bath_threshold(double beta, int I)
{
    const double x = beta * (double)I;
    const double p = 0.5 * (1.0 + std::tanh(x));
    return to_threshold(p);
}

// Supplementary Eq. S.3 with M slices: argument (beta/M) s + K tau,
// K = beta J_perp = -(1/2) ln tanh(beta Gamma / M).
uint32_t trotter_threshold(double beta, int M, double K, int s, int tau)
{
    const double x = (beta / (double)M) * (double)s + K * (double)tau;
    const double p = 0.5 * (1.0 + std::tanh(x));
    return to_threshold(p);
}

double trotter_K(double beta, int M, double gamma)
{
    return -0.5 * std::log(std::tanh(beta * gamma / (double)M));
}

// Eq. (4) for dE = -d < 0: accept iff u < floor(exp(dbeta * dE) * 2^32).
uint32_t swap_threshold(double beta_lo, double beta_hi, int64_t d)
{
    const double x = (beta_hi - beta_lo) * (double)(-d);
    const double e = std::exp(x) * 4294967296.0;
    return (uint32_t)e;
}

// ------------------------------------------------------------------ timers
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

// ====================================================================== context
struct sg_ctx {
    int mode = 0;
    int n_inst = 0;
    uint64_t seed = 0;
    uint32_t key0 = 0, key1 = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::vector<Lat> lat;
    std::vector<InstDev> idev;
    int n_max = 0;
    int hmax = 0;
    DevBuf<InstDev> d_inst;
    DevBuf<uint4> d_rec, d_recj;
    DevBuf<uint4> d_recb;      // APT: d_rec with byte offsets (empty when a lattice is too large)
    DevBuf<uint32_t> d_ctr;      // {sweeps/steps, icm calls, swap attempts, cycles, done}
    Timer timer;
    // events around every main kernel launch (DT-SQA kernel, APT cycle graph)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> kev;
    size_t kev_used = 0;
    bool ktime = false;

    // APT
    int n_beta = 0, reps = 0, n_slots = 0, n_quads = 0, imax = 0, ni = 0;
    std::vector<double> beta;    // [n_inst][n_beta]
    DevBuf<uint8_t> d_spins;
    DevBuf<int32_t> d_perm, d_E, d_slot_lut, d_tab_off, d_tab_len, d_icm_info;
    DevBuf<int32_t> d_perm2, d_E2;   // second mapping / energy buffers of the cycle graph
    DevBuf<uint32_t> d_lut, d_tab;
    DevBuf<uint8_t> d_icm_on;
    DevBuf<int64_t> d_best, d_acc_count, d_mom, d_trace;
    DevBuf<int32_t> d_acc_out;
    DevBuf<QuadDesc> d_desc;
    DevBuf<uint4> d_rowA, d_rowB, d_rowC;
    int n_blocks = 0;
    size_t quad_lds = 0;
    // two launch groups (a launch configuration): the graph's replica kernels of group 1 run
    // on stream2, forked from and joined back into the context's stream
    bool apt_split = false;
    DevBuf<QuadDesc> d_desc_g[2];
    int n_blocks_g[2] = {0, 0};
    size_t lds_g[2] = {0, 0};
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int apt_config = 0;        // launch configuration asked for: 0 = the autotuner's on the next run
    int apt_config_used = 1;   // configuration of d_desc / apt_waves (1: order 0, 7 waves)
    int apt_waves = 7;
    std::vector<double> icm_cutoff_loaded;   // per instance, as last uploaded into d_icm_on
    // graph cache for APT cycles
    hipGraphExec_t gexec = nullptr;
    int g_sweeps = -1, g_icm = -1, g_record = -1, g_cycles = 0, g_pairs = -1;
    int64_t *g_trace = nullptr;
    int g_trace_cap = 0;

    int device = 0;   // the HIP device the context's memory lives on

    // DT-SQA
    int M = 0, R = 0, H = 0, smax = 0, nl = 0;
    double sqa_beta = 0.0;
    DevBuf<uint32_t> d_sqa, d_sqa_lut;
    DevBuf<int32_t> d_slice_E;
    DevBuf<int64_t> d_best_key;   // per instance: (E + 2^30) << 32 | (r M + k) of the lowest slice
    DevBuf<int8_t> d_best_state;  // per instance: that slice, +1/-1 [n_max]
    size_t sqa_lds = 0;
    uint32_t sqa_steps = 0;
    int sqa_threads = 0;   // work-group size; 0: chosen by the autotuner on the next anneal

    ~sg_ctx()
    {
        for (auto &e : kev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (timer.a) (void)hipEventDestroy(timer.a);
        if (timer.b) (void)hipEventDestroy(timer.b);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        if (stream2) (void)hipStreamDestroy(stream2);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
    }
};

namespace {

void set_key(sg_ctx *c, uint64_t seed)
{
    c->seed = seed;
    c->key0 = (uint32_t)seed;
    c->key1 = (uint32_t)(seed >> 32);
}

void init_stream(sg_ctx *c, void *s)
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        fail(SG_EHIP, "no HIP device");
    }
    hip_check(hipGetDevice(&c->device), "hipGetDevice");
    if (s) {
        c->stream = (hipStream_t)s;
    } else {
        hip_check(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
        c->own_stream = true;
    }
}

// LDS of one APT work-group (see apt_quad_kernel): tile, four threshold tables,
// reduction scratch, cluster-search row bitmaps, and for the queue search (rows longer
// than 32 sites) the visited bits and the queue.
size_t apt_lds_bytes(int npad, int n_rows, int ni, bool queue)
{
    // tile, threshold rows, reduction scratch; then the row scratch of the row-bitset cluster
    // search, or in its place the visited bits and the queue of the breadth-first search
    size_t words = (size_t)(npad + 4 + 4 * ni + 32) + (queue ? 0 : (size_t)6 * n_rows);
    size_t bytes = 16;
    if (queue) {
        words += (size_t)((npad + 31) / 32 + 1);
        bytes += sizeof(uint16_t) * (size_t)npad;
    }
    return sizeof(uint32_t) * words + bytes;
}

// Colour classes of the spatial lattice (Methods, "Graph Coloring").
void apt_records(const Lat &L, std::vector<uint4> &rec, std::vector<uint4> &recj, InstDev &I)
{
    const int C = L.n_colours();
    I.n_colours = C;
    I.rec_off = (int64_t)rec.size();
    I.recj_off = (int64_t)recj.size();
    // the records in site order, then the colour classes in ascending site order (one stable
    // bucket pass over the site colours)
    std::vector<uint8_t> col(L.n);
    int cnt[kMaxColours] = {};
    for (int j = 0; j < L.n; ++j) {
        recj.push_back(make_record(L, j, 0u));
        col[j] = (uint8_t)L.colour(j);
        ++cnt[col[j]];
    }
    int off = 0;
    int64_t pos[kMaxColours];
    for (int c = 0; c < kMaxColours; ++c) {
        I.col_off[c] = off;
        I.col_cnt[c] = c < C ? cnt[c] : 0;
        pos[c] = I.rec_off + off;
        off += I.col_cnt[c];
    }
    rec.resize(rec.size() + (size_t)L.n);
    for (int j = 0; j < L.n; ++j) rec[(size_t)pos[col[j]]++] = recj[(size_t)I.recj_off + j];
}

// Phases of the (d+1)-dimensional lattice with an even periodic Trotter ring:
// colour(j, k) = (spatial colour + k) mod C, C = max(spatial colours, 2), so in phase c
// site j updates the slices of parity p = (c - spatial colour) mod C when p is 0 or 1.
// DT-SQA phases (Methods, "Graph Coloring", with the Trotter direction as a fourth axis):
// slice k of site j takes colour (c(j) + t(k)) mod C with t(k) = k mod 2, except t(M - 1) = 2
// when M is odd (an odd Trotter ring); c is the given map, else the closed form, which takes
// three colours when any ring, spatial or Trotter, is odd.  C = max(spatial colours, 2, and 3
// for odd M).  A site is listed in each phase with the part of its slices that phase updates:
// part 0, word 0 (even slices; with odd M all but the last), part 1, word 1 (odd slices), and
// with odd M part 2, the last slice M - 1 alone.
void sqa_records(const Lat &L, int M, std::vector<uint4> &rec, std::vector<uint4> &recj, InstDev &I)
{
    if (2 * L.n + 1 > 0xFFFF) fail(SG_EUNSUPPORTED, "DT-SQA lattice of %d sites is too large", L.n);
    const bool odd_m = (M & 1) != 0;
    int C;
    std::vector<int> cs(L.n);
    if (!L.cmap.empty()) {
        C = std::max(L.n_colours(), odd_m ? 3 : 2);
        for (int j = 0; j < L.n; ++j) cs[j] = L.cmap[j];
    } else {
        const bool three = L.any_odd_ring() || odd_m;
        C = three ? 3 : 2;
        for (int j = 0; j < L.n; ++j) cs[j] = L.label_sum(j, three) % C;
    }
    if (C > kMaxColours) fail(SG_EUNSUPPORTED, "more than %d DT-SQA phases", kMaxColours);
    I.n_colours = C;
    I.rec_off = (int64_t)rec.size();
    I.recj_off = (int64_t)recj.size();
    const int parts = odd_m ? 3 : 2;
    int off = 0;
    for (int c = 0; c < kMaxColours; ++c) {
        I.col_off[c] = off;
        I.col_cnt[c] = 0;
        I.col_p1[c] = 0;
        I.col_p2[c] = 0;
        if (c >= C) continue;
        // the phase's records by part, so that the kernel sweeps each part with the word fixed
        for (int q = 0; q < parts; ++q) {
            if (q == 1) I.col_p1[c] = I.col_cnt[c];
            if (q == 2) I.col_p2[c] = I.col_cnt[c];
            const uint32_t p = q == 1 ? 1u : 0u;
            for (int j = 0; j < L.n; ++j) {
                if ((cs[j] + q) % C != c) continue;
                uint4 rr = make_record(L, j, p);
                // neighbour fields -> word offsets 2 nb + p into the replica's spin words
                auto wo = [p](uint32_t f) {
                    return (2u * (f & 0xFFFFu) + p) | ((2u * (f >> 16) + p) << 16);
                };
                rr.y = wo(rr.y);
                rr.z = wo(rr.z);
                rr.w = wo(rr.w);
                rec.push_back(rr);
                ++I.col_cnt[c];
            }
        }
        if (!odd_m) I.col_p2[c] = I.col_cnt[c];
        off += I.col_cnt[c];
    }
    for (int j = 0; j < L.n; ++j) recj.push_back(make_record(L, j, 0u));
}

// Row tables for the cluster search (see sg_internal.h); rows of lx <= 32.
void apt_rows(const Lat &L, std::vector<uint4> &rowA, std::vector<uint4> &rowB,
              std::vector<uint4> &rowC, InstDev &I)
{
    I.lx = L.Lx;
    I.ly = L.Ly;
    I.lz = L.Lz;
    I.n_rows = L.Ly * L.Lz;
    I.planes = 0;
    if (L.Lx > 32 || I.n_rows > kQuadThreads * 4) {   // rows of one word, <= 4 rows per thread
        I.row_off = -1;
        return;
    }
    if (L.Ly <= 64) {
        const int ppw = 64 / L.Ly;
        I.planes = (L.Lz + ppw - 1) / ppw <= kQuadThreads / 64 ? 1 : 0;
    }
    I.row_off = (int32_t)rowA.size();
    for (int r = 0; r < I.n_rows; ++r) {
        uint32_t m[6] = {0, 0, 0, 0, 0, 0};
        uint32_t nbrow[4] = {(uint32_t)r, (uint32_t)r, (uint32_t)r, (uint32_t)r};
        for (int x = 0; x < L.Lx; ++x) {
            const int j = r * L.Lx + x;
            for (int a = 0; a < 3; ++a)
                for (int s = 0; s < 2; ++s) {
                    const int dir = s ? -1 : +1;
                    const int v = L.nbr(j, a, dir);
                    if (v < 0 || L.J[3 * (s ? v : j) + a] == 0) continue;   // L.coupling
                    m[2 * a + s] |= 1u << x;
                    if (a > 0) nbrow[2 * (a - 1) + s] = (uint32_t)(v / L.Lx);
                }
        }
        uint32_t neg[3] = {0, 0, 0};
        for (int x = 0; x < L.Lx; ++x)
            for (int a = 0; a < 3; ++a)
                if (L.coupling(r * L.Lx + x, a, +1) < 0) neg[a] |= 1u << x;
        rowA.push_back(make_uint4(m[0], m[1], m[2], m[3]));
        rowB.push_back(make_uint4(m[4], m[5], nbrow[0] | (nbrow[1] << 16), nbrow[2] | (nbrow[3] << 16)));
        rowC.push_back(make_uint4(neg[0], neg[1], neg[2], 0u));
    }
}

// Work-group order of the APT replica kernel (a launch-configuration choice: every order
// gives the same results).  Orders 0-3: instances spread over the eight XCDs by size (an
// instance's quads share one XCD's L2 for its site records); within an XCD, quads sorted by
// estimated cost, largest first: sites, times w = 3, 1, 2 or 4 for quads holding a
// temperature >= 1 (where the cluster moves usually run).  Order 4: one global cost sort
// (w = 3), handed to the XCDs in turn.  Order 5: instance-major, quads ascending.
// sel: the instances to include (all when null).
constexpr int kAptOrders = 6;
// Two-group configurations (order 0, 7 waves): the largest instances, up to this share of
// all sites, in one launch and the rest in a second launch on a second stream; the two run
// side by side, each with the LDS size of its own largest instance.
constexpr double kAptSplitShare[3] = {0.65, 0.75, 0.85};
constexpr int kAptConfigs = 2 * kAptOrders + 3;   // x {7, 8} waves per SIMD, then the splits

std::vector<QuadDesc> make_quad_descs(const std::vector<Lat> &lat, int n_quads,
                                      const std::vector<double> &beta, int n_beta, int reps,
                                      int order, const std::vector<char> *sel = nullptr)
{
    std::vector<int> idx;
    for (int i = 0; i < (int)lat.size(); ++i)
        if (!sel || (*sel)[(size_t)i]) idx.push_back(i);
    const int ni = (int)idx.size();
    std::vector<QuadDesc> out;
    if (order == 5) {
        for (int i : idx)
            for (int q = 0; q < n_quads; ++q) out.push_back({i, q});
        return out;
    }
    static const int kWeight[5] = {3, 1, 2, 4, 3};
    const int w = kWeight[order];
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return lat[a].n > lat[b].n; });
    auto cost = [&](const QuadDesc &d) {
        bool icm = false;
        for (int k = 0; k < 4 && reps >= 2; ++k) {
            const int b = std::min(4 * d.quad + k, n_beta * reps - 1) / reps;
            icm |= beta[(size_t)d.inst * n_beta + b] >= 1.0;
        }
        return (int64_t)lat[d.inst].n * (icm ? w : 1);
    };
    auto by_cost = [&](std::vector<QuadDesc> &v) {
        std::stable_sort(v.begin(), v.end(),
                         [&](const QuadDesc &a, const QuadDesc &b) { return cost(a) > cost(b); });
    };
    // within an instance the last quads hold the largest betas: start them first
    if (ni < 8 || order == 4) {
        for (int i : idx)
            for (int q = n_quads - 1; q >= 0; --q) out.push_back({i, q});
        by_cost(out);
        return out;
    }
    const int X = 8;
    std::vector<std::vector<QuadDesc>> qs(X);
    std::vector<int64_t> load(X, 0);
    for (int i : idx) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += (int64_t)lat[i].n;
        for (int q = n_quads - 1; q >= 0; --q) qs[x].push_back({i, q});
    }
    for (auto &v : qs) by_cost(v);
    size_t len = 0;
    for (auto &v : qs) len = std::max(len, v.size());
    out.assign(len * X, QuadDesc{-1, 0});
    for (int x = 0; x < X; ++x)
        for (size_t m = 0; m < qs[x].size(); ++m) out[m * X + x] = qs[x][m];
    return out;
}

// A given colour map: values 0..kMaxColours-1, and no two sites joined by a bond (J != 0)
// share a colour, so that every colour class can be updated in parallel.
void set_colour_map(Lat &L, const int8_t *map, int idx)
{
    int C = 1;
    for (int j = 0; j < L.n; ++j) {
        if (map[j] < 0 || map[j] >= kMaxColours)
            fail(SG_EINVAL, "instance %d: colour of site %d must be in 0..%d", idx, j, kMaxColours - 1);
        C = std::max(C, (int)map[j] + 1);
    }
    for (int j = 0; j < L.n; ++j)
        for (int a = 0; a < 3; ++a) {
            const int nb = L.nbr(j, a, +1);
            if (nb >= 0 && nb != j && L.coupling(j, a, +1) != 0 && map[nb] == map[j])
                fail(SG_EINVAL, "instance %d: bonded sites %d and %d share colour %d", idx, j, nb,
                     (int)map[j]);
        }
    L.cmap.assign(map, map + L.n);
    L.cmap_colours = C;
}

// The neighbour tables are needed only while the context's tables are built (24 bytes per
// site): released before the first device call.
void release_neighbours(sg_ctx *c)
{
    for (Lat &L : c->lat) std::vector<int32_t>().swap(L.nbt);
}

void build_common(sg_ctx *c, const sg_config *cfg, const int8_t *const *colour = nullptr)
{
    if (cfg->n_inst < 1) fail(SG_EINVAL, "n_inst must be >= 1");
    if (!cfg->inst) fail(SG_EINVAL, "inst is NULL");
    c->lat.resize((size_t)cfg->n_inst);
    parallel_for(cfg->n_inst, [&](int i) {
        c->lat[i] = copy_lattice(cfg->inst[i], i);
        if (colour && colour[i]) set_colour_map(c->lat[i], colour[i], i);
    });
    c->n_inst = cfg->n_inst;
    for (auto &L : c->lat) {
        c->n_max = std::max(c->n_max, L.n);
        c->hmax = std::max(c->hmax, L.hmax());
    }
    set_key(c, cfg->seed);
}

// --------------------------------------------------------------------- APT
void create_apt(sg_ctx *c, const sg_config *cfg, const int8_t *const *colour = nullptr)
{
    if (cfg->n_beta < 2) fail(SG_EINVAL, "n_beta must be >= 2");
    if (!cfg->beta) fail(SG_EINVAL, "beta is NULL");
    if (cfg->reps_per_beta != 1 && cfg->reps_per_beta != 2 && cfg->reps_per_beta != 4)
        fail(SG_EINVAL, "reps_per_beta must be 1, 2 or 4");
    if ((int64_t)cfg->n_inst * cfg->n_beta * cfg->reps_per_beta > (1 << 26))
        fail(SG_ENOMEM, "too many replicas");
    c->n_beta = cfg->n_beta;
    c->reps = cfg->reps_per_beta;
    c->n_slots = c->n_beta * c->reps;
    c->n_quads = (c->n_slots + 3) / 4;
    c->beta.assign(cfg->beta, cfg->beta + (size_t)cfg->n_inst * cfg->n_beta);
    for (int i = 0; i < cfg->n_inst; ++i)
        for (int b = 0; b < c->n_beta; ++b) {
            const double v = c->beta[(size_t)i * c->n_beta + b];
            if (!std::isfinite(v) || v < 0.0) fail(SG_EINVAL, "beta must be finite and >= 0");
            if (b > 0 && !(v > c->beta[(size_t)i * c->n_beta + b - 1]))
                fail(SG_EINVAL, "beta must be strictly ascending");
        }
    build_common(c, cfg, colour);
    const int nb4 = 4 * c->n_quads;   // physical buffers per instance (slots padded to a quad)

    c->imax = 6 + c->hmax;
    c->ni = 2 * c->imax + 1;
    // Each instance's tables (site records, bond rows, heat-bath rows, swap tables) depend on
    // that instance alone: they are built on several host threads, with offsets relative to
    // the instance's own tables, then joined in instance order.
    struct Tables {
        InstDev I{};
        std::vector<uint4> rec, recj, rowA, rowB, rowC;
        std::vector<uint32_t> lut, tab;
        std::vector<int32_t> tab_off, tab_len;
    };
    std::vector<Tables> per((size_t)c->n_inst);
    parallel_for(c->n_inst, [&](int i) {
        const Lat &L = c->lat[i];
        Tables &T = per[i];
        InstDev &I = T.I;
        I.n = L.n;
        I.npad = round_up(L.n, 16);
        I.n_slots = c->n_slots;
        apt_records(L, T.rec, T.recj, I);
        I.n_bonds = L.bonds();
        apt_rows(L, T.rowA, T.rowB, T.rowC, I);
        const double *bt = &c->beta[(size_t)i * c->n_beta];
        for (int b = 0; b < c->n_beta; ++b)
            for (int I2 = -c->imax; I2 <= c->imax; ++I2) T.lut.push_back(heat_bath_threshold(bt[b], I2));
        const int64_t gap = L.max_energy_gap();
        for (int b = 0; b + 1 < c->n_beta; ++b) {
            T.tab_off.push_back((int32_t)T.tab.size());
            T.tab.push_back(0xFFFFFFFFu);   // d = 0 is always accepted and never looked up
            int64_t d = 1;
            for (; d <= gap; ++d) {
                const uint32_t Tv = swap_threshold(bt[b], bt[b + 1], d);
                if (Tv == 0u) break;
                T.tab.push_back(Tv);
            }
            T.tab_len.push_back((int32_t)d);
            if (T.tab.size() > (size_t)1 << 30) fail(SG_ENOMEM, "swap tables too large");
        }
    });
    std::vector<uint4> rec, recj, rowA, rowB, rowC;
    std::vector<int32_t> perm, slot_lut, tab_off, tab_len;
    std::vector<uint32_t> lut, tab;
    int64_t spin_bytes = 0;
    for (int i = 0; i < c->n_inst; ++i) {
        Tables &T = per[i];
        InstDev I = T.I;
        I.rec_off += (int64_t)rec.size();
        I.recj_off += (int64_t)recj.size();
        if (I.row_off >= 0) I.row_off += (int32_t)rowA.size();
        rec.insert(rec.end(), T.rec.begin(), T.rec.end());
        recj.insert(recj.end(), T.recj.begin(), T.recj.end());
        rowA.insert(rowA.end(), T.rowA.begin(), T.rowA.end());
        rowB.insert(rowB.end(), T.rowB.begin(), T.rowB.end());
        rowC.insert(rowC.end(), T.rowC.begin(), T.rowC.end());
        I.spin_off = spin_bytes;
        spin_bytes += (int64_t)nb4 * I.npad;
        I.slot_off = i * nb4;
        I.swap_off = i * (c->n_beta - 1);
        I.info_off = i * c->n_beta * std::max(1, c->reps / 2);
        for (int s2 = 0; s2 < nb4; ++s2) {
            perm.push_back(s2);
            slot_lut.push_back(i * c->n_beta + std::min(s2, c->n_slots - 1) / c->reps);
        }
        lut.insert(lut.end(), T.lut.begin(), T.lut.end());
        for (int32_t o : T.tab_off) tab_off.push_back((int32_t)tab.size() + o);
        tab_len.insert(tab_len.end(), T.tab_len.begin(), T.tab_len.end());
        tab.insert(tab.end(), T.tab.begin(), T.tab.end());
        if (tab.size() > (size_t)1 << 30) fail(SG_ENOMEM, "swap tables too large");
        c->idev.push_back(I);
        T = Tables{};   // release this instance's copies
    }
    // every host-side table is built before the first device call
    release_neighbours(c);
    init_stream(c, cfg->hip_stream);
    hipStream_t s = c->stream;
    c->d_inst.upload(c->idev, s, "instances");
    c->d_rec.upload(rec, s, "records");
    // The sweep's copy of the colour-sorted records: neighbour fields as byte offsets into the
    // tile (4 x site index, at most 4 x 16383 in 16 bits), and x = j | jneg << 16 | base << 24
    // with base = h - d + imax, the table index of a site with no aligned bond (0..2 imax, at
    // most 74).  Kept until the stream is synchronised.
    std::vector<uint4> recb;
    if (c->n_max <= kMaxByteOffsetSites) {
        recb = rec;
        for (uint4 &r : recb) {
            const uint32_t j = r.x & 0xFFFFu, d = (r.x >> 16) & 7u, jneg = (r.x >> 19) & 63u;
            const int h = (int)((r.x >> 25) & 63u) - 32;
            const uint32_t base = (uint32_t)(h - (int)d + c->imax);
            r.x = j | (jneg << 16) | (base << 24);
            r.y <<= 2;
            r.z <<= 2;
            r.w <<= 2;
        }
        c->d_recb.upload(recb, s, "records");
    }
    c->d_recj.upload(recj, s, "records");
    c->d_rowA.upload(rowA, s, "row tables");
    c->d_rowB.upload(rowB, s, "row tables");
    c->d_rowC.upload(rowC, s, "row tables");
    c->d_perm.upload(perm, s, "perm");
    c->d_slot_lut.upload(slot_lut, s, "slot tables");
    c->d_lut.upload(lut, s, "thresholds");
    c->d_tab.upload(tab, s, "swap thresholds");
    c->d_tab_off.upload(tab_off, s, "swap offsets");
    c->d_tab_len.upload(tab_len, s, "swap lengths");
    c->d_spins.alloc((size_t)spin_bytes, "spins");
    c->d_E.alloc((size_t)c->n_inst * nb4, "energies");
    c->d_perm2.alloc((size_t)c->n_inst * nb4, "perm");
    c->d_E2.alloc((size_t)c->n_inst * nb4, "energies");
    c->d_mom.alloc((size_t)c->n_inst * nb4 * 2, "moments");
    c->d_best.alloc((size_t)c->n_inst, "best");
    c->d_acc_count.alloc((size_t)c->n_inst * (c->n_beta - 1) * c->reps, "swap counts");
    c->d_acc_out.alloc((size_t)c->n_inst * (c->n_beta - 1) * c->reps, "swap flags");
    c->d_icm_info.alloc((size_t)c->n_inst * c->n_beta * std::max(1, c->reps / 2) * 4, "icm info");
    c->d_icm_on.alloc((size_t)c->n_inst * c->n_beta, "icm flags");
    c->d_ctr.alloc(8, "counters");
    std::vector<QuadDesc> desc = make_quad_descs(c->lat, c->n_quads, c->beta, c->n_beta, c->reps, 0);
    c->n_blocks = (int)desc.size();
    c->d_desc.upload(desc, s, "tasks");
    c->quad_lds = 0;
    for (auto &I : c->idev) {
        const size_t need = apt_lds_bytes(I.npad, I.n_rows, c->ni, I.row_off < 0);
        c->quad_lds = std::max(c->quad_lds, need);
    }
    if (c->quad_lds + 64 * sizeof(uint32_t) > kMaxLds)   // + the kernel's static threshold tables
        fail(SG_EUNSUPPORTED, "instance too large for one work-group's LDS (%zu bytes)", c->quad_lds);
    hip_check(launch_fill_u32(c->d_ctr.p, 0u, 8, s), "init");
    hip_check(launch_fill_i64(c->d_best.p, std::numeric_limits<int64_t>::max(), c->n_inst, s), "init");
    hip_check(launch_fill_i64(c->d_acc_count.p, 0, (int64_t)c->d_acc_count.n, s), "init");
    hip_check(launch_fill_i64(c->d_mom.p, 0, (int64_t)c->d_mom.n, s), "init");
    hip_check(launch_fill_u32((uint32_t *)c->d_spins.p, 0u, (int64_t)(spin_bytes / 4), s), "init");
    hip_check(launch_apt_init(c->d_inst.p, c->d_desc.p, c->n_blocks, c->d_spins.p, c->d_perm.p,
                              c->key0, c->key1, TAG_APT_INIT, s),
              "apt init");
    // energies of the initial state (no sweep, no counter change)
    AptArgs a{};
    a.desc = c->d_desc.p; a.inst = c->d_inst.p; a.rec_col = c->d_rec.p; a.rec_j = c->d_recj.p;
    a.spins = c->d_spins.p; a.perm = c->d_perm.p; a.lut = c->d_lut.p; a.slot_lut = c->d_slot_lut.p;
    a.icm_on = c->d_icm_on.p; a.E = c->d_E.p; a.mom = c->d_mom.p; a.icm_info = c->d_icm_info.p;
    a.rowA = c->d_rowA.p; a.rowB = c->d_rowB.p; a.rowC = c->d_rowC.p;
    a.ctr = c->d_ctr.p; a.key0 = c->key0; a.key1 = c->key1; a.tag = TAG_APT_SWEEP;
    a.do_energy = 2; a.mom_from = -1; a.reps = c->reps; a.imax = c->imax; a.ni = c->ni;
    a.n_blocks = c->n_blocks;
    a.nb4 = 4 * c->n_quads;
    hip_check(launch_apt_quad(a, c->quad_lds, s), "initial energies");
}

// ICM applies at (instance i, temperature b) when beta[i][b] >= cutoff[i].
void upload_icm_flags(sg_ctx *c, const std::vector<double> &cutoff)
{
    if (c->icm_cutoff_loaded == cutoff) return;
    std::vector<uint8_t> on((size_t)c->n_inst * c->n_beta);
    for (size_t i = 0; i < on.size(); ++i) on[i] = c->beta[i] >= cutoff[i / c->n_beta] ? 1 : 0;
    c->d_icm_on.upload(on.data(), on.size(), c->stream, "icm flags");
    hip_check(hipStreamSynchronize(c->stream), "icm flags");
    c->icm_cutoff_loaded = cutoff;
}

AptArgs apt_args(sg_ctx *c, int n_sweeps, int do_icm)
{
    AptArgs a{};
    a.desc = c->d_desc.p;
    a.inst = c->d_inst.p;
    a.boff = c->d_recb.p != nullptr;
    a.rec_col = a.boff ? c->d_recb.p : c->d_rec.p;
    a.rec_j = c->d_recj.p;
    a.spins = c->d_spins.p;
    a.perm = c->d_perm.p;
    a.lut = c->d_lut.p;
    a.slot_lut = c->d_slot_lut.p;
    a.icm_on = c->d_icm_on.p;
    a.E = c->d_E.p;
    a.mom = c->d_mom.p;
    a.icm_info = c->d_icm_info.p;
    a.rowA = c->d_rowA.p;
    a.rowB = c->d_rowB.p;
    a.rowC = c->d_rowC.p;
    a.ctr = c->d_ctr.p;
    a.key0 = c->key0;
    a.key1 = c->key1;
    a.tag = TAG_APT_SWEEP;
    a.n_sweeps = n_sweeps;
    a.do_icm = do_icm;
    a.do_energy = 1;
    a.mom_from = -1;
    a.reps = c->reps;
    a.icm_pairs = 2;
    a.imax = c->imax;
    a.ni = c->ni;
    a.cyc_k = 0;
    a.n_blocks = c->n_blocks;
    a.nb4 = 4 * c->n_quads;
    a.fused_swap = 0;
    a.waves = c->apt_waves;
    return a;
}

SwapArgs swap_args(sg_ctx *c, int32_t *acc_out, int64_t *trace, int trace_cap, int record_every)
{
    SwapArgs a{};
    a.inst = c->d_inst.p;
    a.perm_in = c->d_perm.p;
    a.E_in = c->d_E.p;
    a.perm = c->d_perm.p;
    a.E = c->d_E.p;
    a.tab = c->d_tab.p;
    a.tab_off = c->d_tab_off.p;
    a.tab_len = c->d_tab_len.p;
    a.best = c->d_best.p;
    a.trace = trace;
    a.trace_cap = trace_cap;
    a.record_every = record_every;
    a.acc_count = c->d_acc_count.p;
    a.acc_out = acc_out;
    a.ctr = c->d_ctr.p;
    a.key0 = c->key0;
    a.key1 = c->key1;
    a.n_beta = c->n_beta;
    a.reps = c->reps;
    a.n_inst = c->n_inst;
    a.cyc_k = 0;
    return a;
}

void require(sg_ctx *c, int mode)
{
    if (!c) fail(SG_EINVAL, "context is NULL");
    if (c->mode != mode) fail(SG_ESTATE, "call does not match the context mode");
}

// ICM would move some pair: two or more labels and a temperature >= its instance's cutoff.
bool icm_applies(const sg_ctx *c, const std::vector<double> &cutoff)
{
    if (c->reps < 2) return false;
    for (size_t i = 0; i < c->beta.size(); ++i)
        if (c->beta[i] >= cutoff[i / c->n_beta]) return true;
    return false;
}

// Per-instance ICM cutoffs from one value or an array (validated: no NaN).
std::vector<double> cutoffs_of(const sg_ctx *c, double all, const double *per_inst)
{
    std::vector<double> v((size_t)c->n_inst, all);
    if (per_inst) v.assign(per_inst, per_inst + c->n_inst);
    for (double x : v)
        if (std::isnan(x)) fail(SG_EINVAL, "ICM cutoff is NaN");
    return v;
}

bool any_field(const sg_ctx *c)
{
    for (auto &L : c->lat)
        if (L.has_field()) return true;
    return false;
}

// --------------------------------------------------------------------- DT-SQA
void create_sqa(sg_ctx *c, const sg_config *cfg, const int8_t *const *colour = nullptr)
{
    if (cfg->M < 2 || cfg->M > 64) fail(SG_EINVAL, "M must be in 2..64");
    if (cfg->R < 1 || cfg->R > 65535) fail(SG_EINVAL, "R must be in 1..65535");
    if (!(cfg->sqa_beta > 0.0) || !std::isfinite(cfg->sqa_beta)) fail(SG_EINVAL, "sqa_beta must be > 0");
    if ((int64_t)cfg->n_inst * cfg->R > (1 << 28)) fail(SG_ENOMEM, "too many replicas");
    build_common(c, cfg, colour);
    c->M = cfg->M;
    c->R = cfg->R;
    c->H = (cfg->M + 1) / 2;   // slices per word 0 (word 1 holds M / 2)
    c->sqa_beta = cfg->sqa_beta;
    c->smax = 6 + c->hmax;
    c->nl = (2 * c->smax + 1) * 3;
    std::vector<uint4> rec, recj;
    int64_t words = 0;
    int npad_max = 0;
    for (int i = 0; i < c->n_inst; ++i) {
        const Lat &L = c->lat[i];
        InstDev I{};
        I.n = L.n;
        I.npad = round_up(L.n, 16);
        I.n_slots = c->M;
        sqa_records(L, c->M, rec, recj, I);
        I.n_bonds = L.bonds();
        I.spin_off = words;
        words += (int64_t)c->R * I.npad * 2;
        npad_max = std::max(npad_max, I.npad);
        c->idev.push_back(I);
    }
    // every host-side table is built before the first device call
    release_neighbours(c);
    init_stream(c, cfg->hip_stream);
    hipStream_t s = c->stream;
    c->d_inst.upload(c->idev, s, "instances");
    c->d_rec.upload(rec, s, "records");
    c->d_recj.upload(recj, s, "records");
    c->d_sqa.alloc((size_t)words, "spins");
    c->d_slice_E.alloc((size_t)c->n_inst * c->R * c->M, "slice energies");
    c->d_best_key.alloc((size_t)c->n_inst, "best slices");
    c->d_best_state.alloc((size_t)c->n_inst * c->n_max, "best slices");
    c->d_ctr.alloc(8, "counters");
    hip_check(launch_fill_u32(c->d_ctr.p, 0u, 8, s), "init");
    if (c->nl > 256) fail(SG_EUNSUPPORTED, "field range too large for the threshold table");
    c->sqa_lds = sizeof(uint32_t) * (size_t)(2 * (npad_max + 1)) + 16;
    if (c->sqa_lds + sizeof(uint32_t) * kSqaTabWords > kMaxLds)
        fail(SG_EUNSUPPORTED, "instance too large for one work-group's LDS (%zu bytes)", c->sqa_lds);
    SqaArgs a{};
    a.inst = c->d_inst.p;
    a.spins = c->d_sqa.p;
    a.R = c->R;
    a.M = c->M;
    a.H = c->H;
    a.key0 = c->key0;
    a.key1 = c->key1;
    hip_check(launch_sqa_init(a, c->n_inst, s), "sqa init");
}

SqaArgs sqa_args(sg_ctx *c)
{
    SqaArgs a{};
    a.inst = c->d_inst.p;
    a.rec = c->d_rec.p;
    a.rec_j = c->d_recj.p;
    a.spins = c->d_sqa.p;
    a.lut = c->d_sqa_lut.p;
    a.slice_E = c->d_slice_E.p;
    a.R = c->R;
    a.M = c->M;
    a.H = c->H;
    a.smax = c->smax;
    a.nl = c->nl;
    a.no_field = c->hmax == 0 ? 1 : 0;
    a.key0 = c->key0;
    a.key1 = c->key1;
    return a;
}

// ---- on-disk autotuner cache: one "key value" line per workload shape, the key a hash of
// the device, the library build and the shape; file $SG_TUNE_CACHE or ~/.cache/libsg_tune.txt
// (best effort: an unreadable or unwritable file only disables the cache)
std::string tune_cache_path()
{
    if (const char *e = std::getenv("SG_TUNE_CACHE")) return e;
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/libsg_tune.txt";
    return "";
}

std::string tune_disk_key(const std::string &shape)
{
    int dev = 0;
    hipDeviceProp_t p{};
    std::string arch = "?";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
        arch = p.gcnArchName;
    else
        (void)hipGetLastError();
    const std::string all = arch + "|" __DATE__ " " __TIME__ "|" + shape;
    uint64_t h = 1469598103934665603ull;   // FNV-1a
    for (unsigned char ch : all) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    char buf[24];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    return buf;
}

bool tune_disk_lookup(const std::string &shape, int *value)
{
    const std::string path = tune_cache_path();
    if (path.empty()) return false;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    const std::string key = tune_disk_key(shape);
    char k[64];
    int v = 0;
    bool found = false;
    while (std::fscanf(f, "%63s %d", k, &v) == 2)
        if (key == k) {
            *value = v;
            found = true;
        }
    std::fclose(f);
    return found;
}

void tune_disk_store(const std::string &shape, int value)
{
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", tune_disk_key(shape).c_str(), value);
    std::fclose(f);
}

// ---- DT-SQA launch-configuration autotuner
// Candidates: work-groups of 4, 8, 12 and 16 waves (a whole number of waves per
// SIMD; other sizes leave the four SIMDs of a CU unevenly loaded and measured 10-25 %
// slower).  Each is timed over 2..32 steps on a scratch copy of the replicas (the
// context's state, counters and results are untouched: every size computes the same
// bits), twice, and the fastest minimum wins.  The size sets the number of record
// passes per colour phase (its ragged last pass) and, with the LDS per replica, the
// work-groups and waves resident per CU.  The choice is cached per workload shape for
// the life of the process.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

std::string sqa_tune_key(const sg_ctx *c)
{
    std::string k = "sqa/" + std::to_string(c->n_inst) + "/" + std::to_string(c->R) + "/" +
                    std::to_string(c->M) + "/" + std::to_string(c->nl);
    for (const InstDev &I : c->idev)
        k += ":" + std::to_string(I.npad) + "," + std::to_string(I.col_cnt[0]) + "," +
             std::to_string(I.col_cnt[1]) + "," + std::to_string(I.col_cnt[2]);
    return k;
}

void sqa_autotune(sg_ctx *c, const SqaArgs &base, int ns)
{
    const std::string key = sqa_tune_key(c);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            c->sqa_threads = it->second;
            return;
        }
    }
    int cached = 0;
    if (tune_disk_lookup(key, &cached) && sqa_config_valid(cached)) {
        c->sqa_threads = cached;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = cached;
        return;
    }
    constexpr int kCand = 4;   // 256, 512, 768, 1024 threads
    DevBuf<uint32_t> scratch;
    scratch.alloc(c->d_sqa.n, "autotune scratch");
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "autotune");
    hip_check(hipEventCreate(&e1), "autotune");
    float best_ms[kCand];
    for (int q = 0; q < kCand; ++q) best_ms[q] = std::numeric_limits<float>::infinity();
    SqaArgs a = base;
    a.spins = scratch.p;
    // about 1.5e10 spin updates per timed launch (a few ms), 2..32 steps
    double per_step = 0.0;
    for (const InstDev &I : c->idev) per_step += (double)I.n * c->M * c->R;
    const int want = (int)std::min(32.0, std::max(2.0, 1.5e10 / std::max(per_step, 1.0)));
    a.n_steps = std::min(ns, want);
    a.do_energy = 0;
    hipError_t err = hipSuccess;
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep)
        for (int q = 0; q < kCand && err == hipSuccess; ++q) {
            const int threads = 256 * (q + 1);
            err = hipMemcpyAsync(scratch.p, c->d_sqa.p, c->d_sqa.n * sizeof(uint32_t),
                                 hipMemcpyDeviceToDevice, c->stream);
            if (err == hipSuccess) err = hipEventRecord(e0, c->stream);
            if (err == hipSuccess) err = launch_sqa(a, c->n_inst, c->sqa_lds, threads, c->stream);
            if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess) best_ms[q] = std::min(best_ms[q], ms);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hip_check(err, "autotune");
    int pick = 0;
    for (int q = 1; q < kCand; ++q)
        if (best_ms[q] < best_ms[pick]) pick = q;
    c->sqa_threads = 256 * (pick + 1);
    tune_disk_store(key, c->sqa_threads);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = c->sqa_threads;
}

int sqa_threads_or_default(const sg_ctx *c) { return c->sqa_threads ? c->sqa_threads : 512; }

// ---- APT launch configuration: code 1 + order + kAptOrders * (8 waves ? 1 : 0), order as in
// make_quad_descs.  Every configuration computes the same bits (counter-based random numbers,
// each work-group's work fixed by its quad).
void apply_apt_config(sg_ctx *c, int code)
{
    if (code == c->apt_config_used) return;
    const bool split_code = code > 2 * kAptOrders;
    const int order = split_code ? 0 : (code - 1) % kAptOrders;
    std::vector<QuadDesc> d = make_quad_descs(c->lat, c->n_quads, c->beta, c->n_beta, c->reps, order);
    std::vector<char> in0((size_t)c->n_inst, 0);
    int n0 = 0;
    if (split_code) {
        std::vector<int> idx((size_t)c->n_inst);
        for (int i = 0; i < c->n_inst; ++i) idx[(size_t)i] = i;
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int a, int b) { return c->lat[(size_t)a].n > c->lat[(size_t)b].n; });
        int64_t total = 0, cum = 0;
        for (const Lat &L : c->lat) total += L.n;
        const double share = kAptSplitShare[code - 2 * kAptOrders - 1];
        for (int i : idx) {
            if (n0 > 0 && (double)(cum + c->lat[(size_t)i].n) > share * (double)total) break;
            in0[(size_t)i] = 1;
            cum += c->lat[(size_t)i].n;
            ++n0;
        }
    }
    // one group when the share leaves the second empty
    const bool split = split_code && n0 < c->n_inst;
    // launches in flight still read the old task lists
    hip_check(hipStreamSynchronize(c->stream), "launch config");
    if (c->stream2) hip_check(hipStreamSynchronize(c->stream2), "launch config");
    // the cached cycle graph holds the old lists' addresses
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    // one group until every list of the new configuration is in place (a failure below leaves
    // a consistent single-group context)
    c->apt_split = false;
    c->d_desc.upload(d, c->stream, "tasks");
    c->n_blocks = (int)d.size();
    if (split) {
        if (!c->stream2) {
            hip_check(hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking), "hipStreamCreate");
            hip_check(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "event");
            hip_check(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "event");
        }
        for (int g = 0; g < 2; ++g) {
            std::vector<char> sel((size_t)c->n_inst);
            for (size_t i = 0; i < sel.size(); ++i) sel[i] = (char)(in0[i] == (g == 0 ? 1 : 0));
            const std::vector<QuadDesc> dg =
                make_quad_descs(c->lat, c->n_quads, c->beta, c->n_beta, c->reps, 0, &sel);
            c->d_desc_g[g].upload(dg, c->stream, "tasks");
            c->n_blocks_g[g] = (int)dg.size();
            c->lds_g[g] = 0;
            for (int i = 0; i < c->n_inst; ++i) {
                if (!sel[(size_t)i]) continue;
                const InstDev &I = c->idev[(size_t)i];
                c->lds_g[g] = std::max(c->lds_g[g], apt_lds_bytes(I.npad, I.n_rows, c->ni, I.row_off < 0));
            }
        }
    }
    // the task lists are copied from host vectors that end with this call
    hip_check(hipStreamSynchronize(c->stream), "launch config");
    c->apt_split = split;
    c->apt_waves = !split_code && (code - 1) / kAptOrders ? 8 : 7;
    c->apt_config_used = code;
}

// body(stream, task list, work-groups, LDS bytes) launches replica kernels over one launch
// group.  With two groups, group 1 goes to the second stream, forked from the context's
// stream before and joined into it after, so that work queued after the call waits for both
// (in a graph capture the groups become parallel branches).
template <class F>
hipError_t apt_on_groups(sg_ctx *c, F body)
{
    if (!c->apt_split) return body(c->stream, (const QuadDesc *)c->d_desc.p, c->n_blocks, c->quad_lds);
    hipError_t e = hipEventRecord(c->ev_fork, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->stream2, c->ev_fork, 0);
    if (e != hipSuccess) return e;
    hipError_t eb = body(c->stream, (const QuadDesc *)c->d_desc_g[0].p, c->n_blocks_g[0], c->lds_g[0]);
    if (eb == hipSuccess)
        eb = body(c->stream2, (const QuadDesc *)c->d_desc_g[1].p, c->n_blocks_g[1], c->lds_g[1]);
    hipError_t ej = hipEventRecord(c->ev_join, c->stream2);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(c->stream, c->ev_join, 0);
    return eb != hipSuccess ? eb : ej;
}

std::string apt_tune_key(const sg_ctx *c, int S, bool icm, int pairs)
{
    std::string k = "apt2/" + std::to_string(c->n_inst) + "/" + std::to_string(c->n_beta) + "/" +
                    std::to_string(c->reps) + "/" + std::to_string(c->imax) + "/" + std::to_string(S) +
                    "/" + std::to_string((int)icm) + "/" + std::to_string(pairs);
    for (const InstDev &I : c->idev)
        k += ":" + std::to_string(I.n) + "," + std::to_string(I.n_colours) + "," +
             std::to_string(I.row_off >= 0) + std::to_string(I.planes);
    k += "/";   // temperatures with cluster moves (their share of the cost)
    for (const double &cut : c->icm_cutoff_loaded) k += std::to_string(cut) + ",";
    return k;
}

std::map<std::string, int> g_apt_tune_cache;   // guarded by g_tune_mu

// Candidates: the six work-group orders x {7, 8} waves per SIMD and the three two-group
// splits, each timed over 32 replica-kernel launches of the run's shape (sweeps, cluster
// moves), best of five; the state is saved before and restored after, so the context is
// unchanged.  The pick is cached per workload shape for the process and on disk.
void apt_autotune(sg_ctx *c, int S, bool icm, int pairs)
{
    const std::string key = apt_tune_key(c, S, icm, pairs);
    int pick = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_apt_tune_cache.find(key);
        if (it != g_apt_tune_cache.end()) pick = it->second;
    }
    if (pick == 0 && tune_disk_lookup(key, &pick) && (pick < 1 || pick > kAptConfigs)) pick = 0;
    if (pick == 0) {
        hipStream_t st = c->stream;
        DevBuf<uint8_t> s_spins;
        DevBuf<int32_t> s_perm, s_E, s_info;
        DevBuf<int64_t> s_best, s_acc, s_mom;
        DevBuf<uint32_t> s_ctr;
        auto save = [&](auto &dst, auto &src) {
            dst.alloc(src.n, "autotune snapshot");
            hip_check(hipMemcpyAsync(dst.p, src.p, src.n * sizeof(*src.p), hipMemcpyDeviceToDevice, st),
                      "autotune snapshot");
        };
        auto restore = [&](auto &dst, auto &src) {
            hip_check(hipMemcpyAsync(dst.p, src.p, src.n * sizeof(*src.p), hipMemcpyDeviceToDevice, st),
                      "autotune restore");
        };
        save(s_spins, c->d_spins);
        save(s_perm, c->d_perm);
        save(s_E, c->d_E);
        save(s_info, c->d_icm_info);
        save(s_best, c->d_best);
        save(s_acc, c->d_acc_count);
        save(s_mom, c->d_mom);
        save(s_ctr, c->d_ctr);
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "autotune");
        hip_check(hipEventCreate(&e1), "autotune");
        std::vector<float> best_ms(kAptConfigs + 1, std::numeric_limits<float>::infinity());
        hipError_t err = hipSuccess;
        try {
            for (int rep = 0; rep < 5 && err == hipSuccess; ++rep)
                for (int code = 1; code <= kAptConfigs && err == hipSuccess; ++code) {
                    apply_apt_config(c, code);
                    AptArgs a = apt_args(c, S, icm ? 1 : 0);
                    a.icm_pairs = pairs;
                    err = hipEventRecord(e0, st);
                    if (err == hipSuccess)
                        err = apt_on_groups(c, [&](hipStream_t gs, const QuadDesc *desc, int nb, size_t lds) {
                            AptArgs b = a;
                            b.desc = desc;
                            b.n_blocks = nb;
                            hipError_t r = hipSuccess;
                            for (int k = 0; k < 32 && r == hipSuccess; ++k) r = launch_apt_quad(b, lds, gs);
                            return r;
                        });
                    if (err == hipSuccess) err = hipEventRecord(e1, st);
                    if (err == hipSuccess) err = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                    if (err == hipSuccess) best_ms[code] = std::min(best_ms[code], ms);
                }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        hip_check(err, "autotune");
        restore(c->d_spins, s_spins);
        restore(c->d_perm, s_perm);
        restore(c->d_E, s_E);
        restore(c->d_icm_info, s_info);
        restore(c->d_best, s_best);
        restore(c->d_acc_count, s_acc);
        restore(c->d_mom, s_mom);
        restore(c->d_ctr, s_ctr);
        hip_check(hipStreamSynchronize(st), "autotune restore");
        pick = 1;
        for (int code = 2; code <= kAptConfigs; ++code)
            if (best_ms[code] < best_ms[pick]) pick = code;
        tune_disk_store(key, pick);
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_apt_tune_cache[key] = pick;
    }
    c->apt_config = pick;
    apply_apt_config(c, pick);
}

// Event pair bracketing one main-kernel launch when kernel timing is on.
hipEvent_t kernel_event(sg_ctx *c, bool start)
{
    if (!c->ktime) return nullptr;
    if (start) {
        if (c->kev_used == c->kev.size()) {
            hipEvent_t a, b;
            hip_check(hipEventCreate(&a), "event");
            hip_check(hipEventCreate(&b), "event");
            c->kev.push_back({a, b});
        }
        hipEvent_t e = c->kev[c->kev_used].first;
        hip_check(hipEventRecord(e, c->stream), "event");
        return e;
    }
    hipEvent_t e = c->kev[c->kev_used++].second;
    hip_check(hipEventRecord(e, c->stream), "event");
    return e;
}

template <class F>
sg_status guarded(sg_ctx *c, F &&f)
{
    try {
        f();
        if (c) c->err.clear();
        return SG_OK;
    } catch (const Failure &e) {
        if (c) c->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        return SG_ENOMEM;
    }
}

thread_local std::string g_create_error;

}  // namespace

void sg::set_global_error(const char *msg) { g_create_error = msg ? msg : ""; }

// ====================================================================== C ABI
extern "C" {

sg_status sg_create(const sg_config *cfg, sg_ctx **out) { return sg_create_ex(cfg, nullptr, out); }

sg_status sg_create_ex(const sg_config *cfg, const int8_t *const *colour, sg_ctx **out)
{
    if (!out) return SG_EINVAL;
    *out = nullptr;
    sg_ctx *c = nullptr;
    try {
        if (!cfg) fail(SG_EINVAL, "config is NULL");
        c = new sg_ctx();
        c->mode = cfg->mode;
        if (cfg->mode == SG_APT) create_apt(c, cfg, colour);
        else if (cfg->mode == SG_SQA) create_sqa(c, cfg, colour);
        else fail(SG_EINVAL, "mode must be SG_APT or SG_SQA");
        hip_check(hipStreamSynchronize(c->stream), "create");
    } catch (const Failure &e) {
        g_create_error = e.msg;
        delete c;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_create_error = "host allocation failed";
        delete c;
        return SG_ENOMEM;
    }
    g_create_error.clear();
    *out = c;
    return SG_OK;
}

sg_status sg_dsatur_colouring(const sg_lattice *inst, int8_t *colour_out, int32_t *n_colours)
{
    try {
        if (!inst || !colour_out || !n_colours) fail(SG_EINVAL, "NULL argument");
        const Lat L = copy_lattice(*inst, 0);
        // interaction graph: sites joined by a bond with J != 0
        std::vector<std::array<int, 6>> adj((size_t)L.n);
        std::vector<int> deg((size_t)L.n, 0);
        for (int j = 0; j < L.n; ++j)
            for (int a = 0; a < 3; ++a)
                for (int dir = -1; dir <= 1; dir += 2) {
                    const int nb = L.nbr(j, a, dir);
                    if (nb < 0 || nb == j || L.coupling(j, a, dir) == 0) continue;
                    bool seen = false;   // an axis of length 2 reaches one neighbour twice
                    for (int k = 0; k < deg[j]; ++k) seen |= adj[j][k] == nb;
                    if (!seen) adj[j][deg[j]++] = nb;
                }
        // Brelaz's DSATUR: repeatedly colour the uncoloured site with the most distinct
        // neighbour colours (ties: most uncoloured neighbours, then lowest index) with the
        // smallest colour none of its neighbours has.
        std::vector<int> col((size_t)L.n, -1), udeg(deg), sat((size_t)L.n, 0);
        std::vector<uint32_t> seen((size_t)L.n, 0u);   // bit c: a neighbour has colour c
        std::set<std::tuple<int, int, int>> open;       // (-sat, -udeg, site)
        for (int j = 0; j < L.n; ++j) open.insert({0, -udeg[j], j});
        int C = 1;
        while (!open.empty()) {
            const int v = std::get<2>(*open.begin());
            open.erase(open.begin());
            int cv = 0;
            while ((seen[v] >> cv) & 1u) ++cv;
            col[v] = cv;
            C = std::max(C, cv + 1);
            for (int k = 0; k < deg[v]; ++k) {
                const int u = adj[v][k];
                if (col[u] >= 0) continue;
                open.erase({-sat[u], -udeg[u], u});
                --udeg[u];
                if (!((seen[u] >> cv) & 1u)) {
                    seen[u] |= 1u << cv;
                    ++sat[u];
                }
                open.insert({-sat[u], -udeg[u], u});
            }
        }
        if (C > kMaxColours) fail(SG_EUNSUPPORTED, "the colouring needs %d > %d colours", C, kMaxColours);
        for (int j = 0; j < L.n; ++j) colour_out[j] = (int8_t)col[j];
        *n_colours = C;
    } catch (const Failure &e) {
        g_create_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_create_error = "host allocation failed";
        return SG_ENOMEM;
    }
    return SG_OK;
}

void sg_destroy(sg_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->stream2) (void)hipStreamSynchronize(c->stream2);
    delete c;
}

const char *sg_last_error(const sg_ctx *c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

sg_status sg_sweep(sg_ctx *c, int32_t n_sweeps)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        if (n_sweeps < 0) fail(SG_EINVAL, "n_sweeps must be >= 0");
        if (n_sweeps == 0) return;
        AptArgs a = apt_args(c, n_sweeps, 0);
        hip_check(launch_apt_quad(a, c->quad_lds, c->stream), "sweep");
        hip_check(launch_advance(c->d_ctr.p, (uint32_t)n_sweeps, 0u, 0u, 0u, c->stream), "sweep");
    });
}

}  // extern "C"

namespace {

void icm_call(sg_ctx *c, const std::vector<double> &cut, int icm_pairs, int32_t *info_host)
{
    if (icm_pairs != 1 && icm_pairs != 2) fail(SG_EINVAL, "icm_pairs must be 1 or 2");
    if (icm_applies(c, cut) && any_field(c))
        fail(SG_EUNSUPPORTED, "ICM with non-zero fields is not supported");
    upload_icm_flags(c, cut);
    hip_check(launch_fill_u32((uint32_t *)c->d_icm_info.p, 0xFFFFFFFFu, (int64_t)c->d_icm_info.n,
                              c->stream),
              "icm");
    AptArgs a = apt_args(c, 0, 1);
    a.icm_pairs = icm_pairs;
    hip_check(launch_apt_quad(a, c->quad_lds, c->stream), "icm");
    hip_check(launch_advance(c->d_ctr.p, 0u, 1u, 0u, 0u, c->stream), "icm");
    if (info_host) {
        c->d_icm_info.download(info_host, c->d_icm_info.n, c->stream, "icm info");
        hip_check(hipStreamSynchronize(c->stream), "icm");
        if (c->reps == 1)
            for (size_t i = 0; i < c->d_icm_info.n; ++i) info_host[i] = -1;
    }
}

}  // namespace

extern "C" {

sg_status sg_icm(sg_ctx *c, double cutoff, int32_t *info_host)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        icm_call(c, cutoffs_of(c, cutoff, nullptr), 2, info_host);
    });
}

sg_status sg_icm_ex(sg_ctx *c, const sg_apt_options *opt, int32_t *info_host)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        if (!opt) fail(SG_EINVAL, "options are NULL");
        icm_call(c, cutoffs_of(c, opt->icm_cutoff, opt->icm_cutoff_per_inst), opt->icm_pairs,
                 info_host);
    });
}

sg_status sg_energy(sg_ctx *c, int64_t *E_host)
{
    return guarded(c, [&] {
        if (!c) fail(SG_EINVAL, "context is NULL");
        if (!E_host) fail(SG_EINVAL, "E_host is NULL");
        if (c->mode == SG_APT) {
            const int nb4 = 4 * c->n_quads;
            std::vector<int32_t> e((size_t)c->n_inst * nb4);
            c->d_E.download(e.data(), e.size(), c->stream, "energy");
            hip_check(hipStreamSynchronize(c->stream), "energy");
            for (int i = 0; i < c->n_inst; ++i)
                for (int s = 0; s < c->n_slots; ++s)
                    E_host[(size_t)i * c->n_slots + s] = e[(size_t)i * nb4 + s];
        } else {
            SqaArgs a = sqa_args(c);
            a.n_steps = 0;
            a.do_energy = 1;
            a.lut = nullptr;
            hip_check(launch_sqa(a, c->n_inst, c->sqa_lds, sqa_threads_or_default(c), c->stream),
                      "energy");
            std::vector<int32_t> e((size_t)c->n_inst * c->R * c->M);
            c->d_slice_E.download(e.data(), e.size(), c->stream, "energy");
            hip_check(hipStreamSynchronize(c->stream), "energy");
            for (size_t i = 0; i < e.size(); ++i) E_host[i] = e[i];
        }
    });
}

sg_status sg_swap(sg_ctx *c, int32_t *accepted_host)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        SwapArgs a = swap_args(c, accepted_host ? c->d_acc_out.p : nullptr, nullptr, 0, 0);
        hip_check(launch_apt_swap(a, c->stream), "swap");
        hip_check(launch_advance(c->d_ctr.p, 0u, 0u, 1u, 0u, c->stream), "swap");
        if (accepted_host) {
            c->d_acc_out.download(accepted_host, (size_t)c->n_inst * (c->n_beta - 1) * c->reps,
                                  c->stream, "swap");
            hip_check(hipStreamSynchronize(c->stream), "swap");
        }
    });
}

}  // extern "C"

namespace {

void run_apt(sg_ctx *c, int64_t n_cycles, int32_t sweeps_per_swap, const std::vector<double> &cut,
             int32_t icm_pairs, int32_t record_every, int64_t *best_trace)
{
    {
        if (n_cycles < 0 || sweeps_per_swap < 1) fail(SG_EINVAL, "bad cycle or sweep count");
        if (icm_pairs != 1 && icm_pairs != 2) fail(SG_EINVAL, "icm_pairs must be 1 or 2");
        if (record_every < 0 || (best_trace && record_every == 0))
            fail(SG_EINVAL, "record_every must be > 0 with a trace");
        const bool icm = icm_applies(c, cut);
        if (icm && any_field(c)) fail(SG_EUNSUPPORTED, "ICM with non-zero fields is not supported");
        if (n_cycles == 0) return;
        upload_icm_flags(c, icm ? cut : std::vector<double>((size_t)c->n_inst,
                                                              std::numeric_limits<double>::infinity()));
        if (c->apt_config == 0) apt_autotune(c, sweeps_per_swap, icm, icm_pairs);
        else apply_apt_config(c, c->apt_config);
        const int cap = best_trace ? (int)(n_cycles / record_every) : 0;
        if (best_trace) {
            if ((size_t)c->n_inst * cap > c->d_trace.n) c->d_trace.alloc((size_t)c->n_inst * cap, "trace");
        }
        int64_t *trace = best_trace ? c->d_trace.p : nullptr;
        const int rec = best_trace ? record_every : 0;
        hip_check(launch_fill_u32(c->d_ctr.p + 3, 0u, 1, c->stream), "cycle counter");
        AptArgs qa = apt_args(c, sweeps_per_swap, icm ? 1 : 0);
        qa.icm_pairs = icm_pairs;
        SwapArgs sa = swap_args(c, nullptr, trace, cap, rec);
        const uint32_t S = (uint32_t)sweeps_per_swap;
        // Replay a captured graph of K cycles.  Inside the graph cycle k reads
        // its step numbers as (counters + k * per-cycle increments); one
        // one-thread kernel at the end advances the counters by K cycles, so
        // the same graph is valid on every replay.  The exchange of cycle k - 1
        // runs at the start of cycle k's replica kernel, which reads the mapping
        // and energies from one buffer pair and writes them to the other; a last
        // exchange launch after cycle K - 1 brings them back to the first pair.
        const int K = 32;
        if (!c->gexec || c->g_sweeps != sweeps_per_swap || c->g_icm != (int)icm || c->g_record != rec ||
            c->g_trace != trace || c->g_trace_cap != cap || c->g_pairs != icm_pairs) {
            if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
            hipGraph_t g = nullptr;
            hip_check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "capture");
            hipError_t e = hipSuccess;
            int32_t *pa = c->d_perm.p, *pb = c->d_perm2.p, *ea = c->d_E.p, *eb = c->d_E2.p;
            e = apt_on_groups(c, [&](hipStream_t gs, const QuadDesc *desc, int nb, size_t lds) {
                hipError_t r = hipSuccess;
                for (int k = 0; k < K && r == hipSuccess; ++k) {
                    AptArgs fa = qa;
                    fa.desc = desc;
                    fa.n_blocks = nb;
                    fa.cyc_k = k;
                    if (k > 0) {
                        const bool odd = (k & 1) != 0;
                        fa.fused_swap = 1;
                        fa.sw = sa;
                        fa.sw.cyc_k = k - 1;
                        fa.sw.perm_in = odd ? pa : pb;
                        fa.sw.E_in = odd ? ea : eb;
                        fa.sw.perm = odd ? pb : pa;
                        fa.sw.E = fa.E = odd ? eb : ea;
                        fa.perm = fa.sw.perm;
                    }
                    r = launch_apt_quad(fa, lds, gs);
                }
                return r;
            });
            static_assert(K % 2 == 0, "the last replica kernel must write the second buffers");
            SwapArgs last = sa;
            last.cyc_k = K - 1;
            last.perm_in = pb;
            last.E_in = eb;
            if (e == hipSuccess) e = launch_apt_swap(last, c->stream);
            if (e == hipSuccess) e = launch_advance(c->d_ctr.p, K * S, K, K, K, c->stream);
            hipError_t e2 = hipStreamEndCapture(c->stream, &g);
            hip_check(e, "capture launch");
            hip_check(e2, "end capture");
            hipError_t e3 = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            hip_check(e3, "graph instantiate");
            c->g_sweeps = sweeps_per_swap;
            c->g_icm = (int)icm;
            c->g_record = rec;
            c->g_trace = trace;
            c->g_trace_cap = cap;
            c->g_pairs = icm_pairs;
        }
        int64_t done = 0;
        for (; done + K <= n_cycles; done += K) {
            kernel_event(c, true);
            hip_check(hipGraphLaunch(c->gexec, c->stream), "graph launch");
            kernel_event(c, false);
        }
        qa.cyc_k = 0;
        sa.cyc_k = 0;
        for (; done < n_cycles; ++done) {
            hip_check(launch_apt_quad(qa, c->quad_lds, c->stream), "cycle");
            hip_check(launch_apt_swap(sa, c->stream), "cycle");
            hip_check(launch_advance(c->d_ctr.p, S, 1u, 1u, 1u, c->stream), "cycle");
        }
        if (best_trace) {
            std::vector<int64_t> t((size_t)c->n_inst * cap);
            c->d_trace.download(t.data(), t.size(), c->stream, "trace");
            hip_check(hipStreamSynchronize(c->stream), "trace");
            std::memcpy(best_trace, t.data(), t.size() * sizeof(int64_t));
        }
    }
}

}  // namespace

extern "C" {

sg_status sg_run_apt(sg_ctx *c, int64_t n_cycles, int32_t sweeps_per_swap, double icm_cutoff,
                     int32_t record_every, int64_t *best_trace)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        run_apt(c, n_cycles, sweeps_per_swap, cutoffs_of(c, icm_cutoff, nullptr), 2, record_every,
                best_trace);
    });
}

sg_status sg_run_apt_ex(sg_ctx *c, int64_t n_cycles, const sg_apt_options *opt, int64_t *best_trace)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        if (!opt) fail(SG_EINVAL, "options are NULL");
        run_apt(c, n_cycles, opt->sweeps_per_swap,
                cutoffs_of(c, opt->icm_cutoff, opt->icm_cutoff_per_inst), opt->icm_pairs,
                opt->record_every, best_trace);
    });
}

sg_status sg_threshold_heat_bath(double beta, int32_t I, uint32_t *T)
{
    if (!T || !std::isfinite(beta)) {
        sg::set_global_error("sg_threshold_heat_bath: NULL output or non-finite beta");
        return SG_EINVAL;
    }
    *T = heat_bath_threshold(beta, I);
    return SG_OK;
}

sg_status sg_threshold_sqa(double beta, int32_t M, double gamma, int32_t s, int32_t tau, uint32_t *T)
{
    if (!T || !(beta > 0.0) || !std::isfinite(beta) || M < 1 || !(gamma > 0.0) ||
        !std::isfinite(gamma)) {
        sg::set_global_error("sg_threshold_sqa: NULL output, beta or gamma not > 0, or M < 1");
        return SG_EINVAL;
    }
    *T = trotter_threshold(beta, M, trotter_K(beta, M, gamma), s, tau);
    return SG_OK;
}

sg_status sg_threshold_swap(double beta_lo, double beta_hi, int64_t d, uint32_t *T)
{
    if (!T || d < 1 || !std::isfinite(beta_lo) || !std::isfinite(beta_hi)) {
        sg::set_global_error("sg_threshold_swap: NULL output, d < 1 or non-finite beta");
        return SG_EINVAL;
    }
    *T = swap_threshold(beta_lo, beta_hi, d);
    return SG_OK;
}

sg_status sg_best(sg_ctx *c, int64_t *best_host)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        if (!best_host) fail(SG_EINVAL, "best_host is NULL");
        c->d_best.download(best_host, (size_t)c->n_inst, c->stream, "best");
        hip_check(hipStreamSynchronize(c->stream), "best");
    });
}

sg_status sg_swap_counts(sg_ctx *c, int64_t *counts)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        if (!counts) fail(SG_EINVAL, "counts is NULL");
        c->d_acc_count.download(counts, (size_t)c->n_inst * (c->n_beta - 1) * c->reps, c->stream,
                                "swap counts");
        hip_check(hipStreamSynchronize(c->stream), "swap counts");
    });
}

sg_status sg_get_launch_config(sg_ctx *c, int32_t *config)
{
    return guarded(c, [&] {
        if (!c) fail(SG_EINVAL, "context is NULL");
        if (!config) fail(SG_EINVAL, "config is NULL");
        *config = c->mode == SG_SQA ? c->sqa_threads : c->apt_config;
    });
}

sg_status sg_set_launch_config(sg_ctx *c, int32_t config)
{
    return guarded(c, [&] {
        if (!c) fail(SG_EINVAL, "context is NULL");
        if (c->mode == SG_SQA) {
            if (config != 0 && !sqa_config_valid(config))
                fail(SG_EINVAL, "work-group size must be a multiple of 64 in 128..1024");
            c->sqa_threads = config;
        } else {
            if (config < 0 || config > kAptConfigs)
                fail(SG_EINVAL, "APT launch configuration must be 0..%d", kAptConfigs);
            c->apt_config = config;
            if (config) apply_apt_config(c, config);
        }
    });
}

}  // extern "C"

namespace {

// Algorithm S1 over the schedule gamma[0 .. n_steps) and the energy pass, leaving the lowest
// slice of every instance in d_best_key (also for n_steps = 0: the energies of the present
// state).
void run_sqa_anneal(sg_ctx *c, const double *gamma, int32_t n_steps)
{
    if (n_steps < 0 || (n_steps > 0 && !gamma)) fail(SG_EINVAL, "bad schedule");
    for (int t = 0; t < n_steps; ++t)
        if (!(gamma[t] > 0.0) || !std::isfinite(gamma[t])) fail(SG_EINVAL, "gamma must be > 0");
    // thresholds for every step, FP64 -> uint32 (Supplementary Eq. S.3)
    const int chunk = 256;
    int done = 0;
    std::vector<uint32_t> lut;
    while (done < n_steps) {
        const int ns = std::min(chunk, n_steps - done);
        lut.assign((size_t)ns * c->nl, 0u);
        for (int t = 0; t < ns; ++t) {
            const double K = trotter_K(c->sqa_beta, c->M, gamma[done + t]);
            for (int s = -c->smax; s <= c->smax; ++s)
                for (int tt = 0; tt < 3; ++tt)
                    lut[(size_t)t * c->nl + (s + c->smax) * 3 + tt] =
                        trotter_threshold(c->sqa_beta, c->M, K, s, 2 * tt - 2);
        }
        // the previous chunk's kernel may still read the table: wait before replacing it
        hip_check(hipStreamSynchronize(c->stream), "anneal");
        c->d_sqa_lut.upload(lut.data(), lut.size(), c->stream, "sqa thresholds");
        SqaArgs a = sqa_args(c);
        a.t0 = (int32_t)c->sqa_steps;
        a.n_steps = ns;
        a.lut_step0 = 0;
        a.do_energy = (done + ns == n_steps) ? 1 : 0;
        if (c->sqa_threads == 0) sqa_autotune(c, a, ns);
        if (a.do_energy) {
            hip_check(launch_fill_i64(c->d_best_key.p, -1, c->n_inst, c->stream), "anneal");
            a.best_key = (uint64_t *)c->d_best_key.p;
        }
        kernel_event(c, true);
        hip_check(launch_sqa(a, c->n_inst, c->sqa_lds, c->sqa_threads, c->stream),
                  "anneal");
        kernel_event(c, false);
        c->sqa_steps += (uint32_t)ns;
        done += ns;
    }
    if (n_steps == 0) {
        hip_check(launch_fill_i64(c->d_best_key.p, -1, c->n_inst, c->stream), "anneal");
        SqaArgs a = sqa_args(c);
        a.n_steps = 0;
        a.do_energy = 1;
        a.best_key = (uint64_t *)c->d_best_key.p;
        hip_check(launch_sqa(a, c->n_inst, c->sqa_lds, sqa_threads_or_default(c), c->stream),
                  "anneal");
    }
}

// A device pointer for a device-output call: memory of the context's device (SG_EINVAL
// otherwise, so that a host pointer is refused instead of being written by a kernel).
void check_device_ptr(const sg_ctx *c, const void *p, const char *what)
{
    if (!p) fail(SG_EINVAL, "%s is NULL", what);
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        fail(SG_EINVAL, "%s is not device memory", what);
    }
    if ((at.type != hipMemoryTypeDevice && !at.isManaged) || at.device != c->device)
        fail(SG_EINVAL, "%s is not device memory of the context's device %d", what, c->device);
}

}  // namespace

extern "C" {

sg_status sg_sqa_anneal(sg_ctx *c, const double *gamma, int32_t n_steps, int64_t *best_E,
                        int8_t *best_state)
{
    return guarded(c, [&] {
        require(c, SG_SQA);
        run_sqa_anneal(c, gamma, n_steps);
        // Alg. S1, last lines: the lowest slice energy of every instance and its state, both
        // reduced on the device (the energy pass keeps an atomic minimum per instance)
        if (best_E || best_state) {
            if (best_state) {
                SqaArgs a = sqa_args(c);
                a.best_key = (uint64_t *)c->d_best_key.p;
                hip_check(launch_sqa_best_state(a, c->n_inst, c->n_max, c->d_best_state.p, c->stream),
                          "best state");
                c->d_best_state.download(best_state, (size_t)c->n_inst * c->n_max, c->stream,
                                         "best state");
            }
            std::vector<int64_t> key((size_t)c->n_inst);
            c->d_best_key.download(key.data(), key.size(), c->stream, "anneal");
            hip_check(hipStreamSynchronize(c->stream), "anneal");
            if (best_E)
                for (int i = 0; i < c->n_inst; ++i)
                    best_E[i] = (int64_t)(uint32_t)((uint64_t)key[i] >> 32) - 0x40000000;
        }
    });
}

sg_status sg_sqa_anneal_dev(sg_ctx *c, const double *gamma, int32_t n_steps, int64_t *best_E_dev,
                            int8_t *best_state_dev)
{
    return guarded(c, [&] {
        require(c, SG_SQA);
        if (best_E_dev) check_device_ptr(c, best_E_dev, "best_E_dev");
        if (best_state_dev) check_device_ptr(c, best_state_dev, "best_state_dev");
        run_sqa_anneal(c, gamma, n_steps);
        if (best_state_dev) {
            SqaArgs a = sqa_args(c);
            a.best_key = (uint64_t *)c->d_best_key.p;
            hip_check(launch_sqa_best_state(a, c->n_inst, c->n_max, best_state_dev, c->stream),
                      "best state");
        }
        if (best_E_dev)
            hip_check(launch_best_key_energy((const uint64_t *)c->d_best_key.p, c->n_inst, best_E_dev,
                                             c->stream),
                      "best energy");
    });
}

sg_status sg_energy_dev(sg_ctx *c, int64_t *E_dev)
{
    return guarded(c, [&] {
        if (!c) fail(SG_EINVAL, "context is NULL");
        check_device_ptr(c, E_dev, "E_dev");
        if (c->mode == SG_APT) {
            hip_check(launch_widen_rows(c->d_E.p, 4 * c->n_quads, E_dev, c->n_inst, c->n_slots,
                                        c->stream),
                      "energy");
        } else {
            SqaArgs a = sqa_args(c);
            a.n_steps = 0;
            a.do_energy = 1;
            a.lut = nullptr;
            hip_check(launch_sqa(a, c->n_inst, c->sqa_lds, sqa_threads_or_default(c), c->stream),
                      "energy");
            hip_check(launch_widen_rows(c->d_slice_E.p, c->R * c->M, E_dev, c->n_inst, c->R * c->M,
                                        c->stream),
                      "energy");
        }
    });
}

sg_status sg_best_dev(sg_ctx *c, int64_t *best_dev)
{
    return guarded(c, [&] {
        require(c, SG_APT);
        check_device_ptr(c, best_dev, "best_dev");
        hip_check(hipMemcpyAsync(best_dev, c->d_best.p, sizeof(int64_t) * (size_t)c->n_inst,
                                 hipMemcpyDeviceToDevice, c->stream),
                  "best");
    });
}

sg_status sg_get_spins_dev(sg_ctx *c, int8_t *spins_dev)
{
    return guarded(c, [&] {
        if (!c) fail(SG_EINVAL, "context is NULL");
        check_device_ptr(c, spins_dev, "spins_dev");
        if (c->mode == SG_APT)
            hip_check(launch_apt_spins_out(c->d_spins.p, c->d_perm.p, c->d_inst.p, c->n_inst,
                                           4 * c->n_quads, c->n_slots, c->n_max, spins_dev, c->stream),
                      "spins");
        else
            hip_check(launch_sqa_spins_out(c->d_sqa.p, c->d_inst.p, c->n_inst, c->R, c->M, c->n_max,
                                           spins_dev, c->stream),
                      "spins");
    });
}

sg_status sg_sqa_trotter_agreement(sg_ctx *c, int32_t *agree_host)
{
    return guarded(c, [&] {
        require(c, SG_SQA);
        if (!agree_host) fail(SG_EINVAL, "agree_host is NULL");
        DevBuf<int32_t> d;
        d.alloc((size_t)c->n_inst * c->R * c->M, "correlation");
        SqaArgs a = sqa_args(c);
        hip_check(launch_sqa_corr(a, c->n_inst, d.p, c->stream), "correlation");
        d.download(agree_host, d.n, c->stream, "correlation");
        hip_check(hipStreamSynchronize(c->stream), "correlation");
    });
}

sg_status sg_get_spins(sg_ctx *c, int8_t *out)
{
    return guarded(c, [&] {
        if (!c || !out) fail(SG_EINVAL, "NULL argument");
        if (c->mode == SG_APT) {
            const int nb4 = 4 * c->n_quads;
            std::vector<uint8_t> raw(c->d_spins.n);
            std::vector<int32_t> perm((size_t)c->n_inst * nb4);
            c->d_spins.download(raw.data(), raw.size(), c->stream, "spins");
            c->d_perm.download(perm.data(), perm.size(), c->stream, "spins");
            hip_check(hipStreamSynchronize(c->stream), "spins");
            for (int i = 0; i < c->n_inst; ++i) {
                const InstDev &I = c->idev[i];
                for (int s = 0; s < c->n_slots; ++s) {
                    const uint8_t *src = raw.data() + I.spin_off + (int64_t)perm[(size_t)i * nb4 + s] * I.npad;
                    int8_t *dst = out + ((size_t)i * c->n_slots + s) * c->n_max;
                    std::memset(dst, 0, (size_t)c->n_max);
                    for (int j = 0; j < I.n; ++j) dst[j] = src[j] ? 1 : -1;
                }
            }
        } else {
            std::vector<uint32_t> raw(c->d_sqa.n);
            c->d_sqa.download(raw.data(), raw.size(), c->stream, "spins");
            hip_check(hipStreamSynchronize(c->stream), "spins");
            for (int i = 0; i < c->n_inst; ++i) {
                const InstDev &I = c->idev[i];
                for (int r = 0; r < c->R; ++r)
                    for (int k = 0; k < c->M; ++k) {
                        const uint32_t *w = raw.data() + I.spin_off + (int64_t)r * I.npad * 2;
                        int8_t *dst = out + (((size_t)i * c->R + r) * c->M + k) * c->n_max;
                        std::memset(dst, 0, (size_t)c->n_max);
                        for (int j = 0; j < I.n; ++j)
                            dst[j] = ((w[2 * j + (k & 1)] >> (k >> 1)) & 1u) ? 1 : -1;
                    }
            }
        }
    });
}

sg_status sg_get_spins_range(sg_ctx *c, int32_t inst, int32_t first, int32_t count, int8_t *out)
{
    return guarded(c, [&] {
        if (!c || !out) fail(SG_EINVAL, "NULL argument");
        if (inst < 0 || inst >= c->n_inst) fail(SG_EINVAL, "instance out of range");
        const int total = c->mode == SG_APT ? c->n_slots : c->R;
        if (first < 0 || count < 0 || (int64_t)first + count > total)
            fail(SG_EINVAL, "range outside the instance's %s", c->mode == SG_APT ? "slots" : "replicas");
        const InstDev &I = c->idev[inst];
        if (count == 0) return;
        if (c->mode == SG_APT) {
            const int nb4 = 4 * c->n_quads;
            std::vector<int32_t> perm((size_t)nb4);
            hip_check(hipMemcpyAsync(perm.data(), c->d_perm.p + (size_t)inst * nb4, perm.size() * 4,
                                     hipMemcpyDeviceToHost, c->stream),
                      "spins");
            hip_check(hipStreamSynchronize(c->stream), "spins");
            std::vector<uint8_t> buf((size_t)I.npad);
            for (int s = 0; s < count; ++s) {
                hip_check(hipMemcpyAsync(buf.data(),
                                         c->d_spins.p + I.spin_off + (int64_t)perm[first + s] * I.npad,
                                         buf.size(), hipMemcpyDeviceToHost, c->stream),
                          "spins");
                hip_check(hipStreamSynchronize(c->stream), "spins");
                for (int j = 0; j < I.n; ++j) out[(size_t)s * I.n + j] = buf[j] ? 1 : -1;
            }
        } else {
            std::vector<uint32_t> w((size_t)count * I.npad * 2);
            hip_check(hipMemcpyAsync(w.data(), c->d_sqa.p + I.spin_off + (int64_t)first * I.npad * 2,
                                     w.size() * 4, hipMemcpyDeviceToHost, c->stream),
                      "spins");
            hip_check(hipStreamSynchronize(c->stream), "spins");
            for (int r = 0; r < count; ++r)
                for (int k = 0; k < c->M; ++k)
                    for (int j = 0; j < I.n; ++j)
                        out[((size_t)r * c->M + k) * I.n + j] =
                            ((w[(size_t)r * I.npad * 2 + 2 * j + (k & 1)] >> (k >> 1)) & 1u) ? 1 : -1;
        }
    });
}

sg_status sg_set_spins(sg_ctx *c, const int8_t *in)
{
    return guarded(c, [&] {
        if (!c || !in) fail(SG_EINVAL, "NULL argument");
        if (c->mode == SG_APT) {
            const int nb4 = 4 * c->n_quads;
            for (int i = 0; i < c->n_inst; ++i)
                for (int s = 0; s < c->n_slots; ++s)
                    for (int j = 0; j < c->idev[i].n; ++j) {
                        const int8_t v = in[((size_t)i * c->n_slots + s) * c->n_max + j];
                        if (v != 1 && v != -1) fail(SG_EINVAL, "spins must be +1 or -1");
                    }
            std::vector<uint8_t> raw(c->d_spins.n, 0);
            std::vector<int32_t> perm((size_t)c->n_inst * nb4);
            for (int i = 0; i < c->n_inst; ++i) {
                const InstDev &I = c->idev[i];
                for (int s = 0; s < nb4; ++s) {
                    perm[(size_t)i * nb4 + s] = s;
                    if (s >= c->n_slots) continue;
                    uint8_t *dst = raw.data() + I.spin_off + (int64_t)s * I.npad;
                    const int8_t *src = in + ((size_t)i * c->n_slots + s) * c->n_max;
                    for (int j = 0; j < I.n; ++j) dst[j] = src[j] > 0 ? 1 : 0;
                }
            }
            c->d_spins.upload(raw.data(), raw.size(), c->stream, "spins");
            c->d_perm.upload(perm.data(), perm.size(), c->stream, "perm");
            // energies of the new state
            AptArgs a = apt_args(c, 0, 0);
            a.do_energy = 2;
            hip_check(launch_apt_quad(a, c->quad_lds, c->stream), "energy");
            hip_check(hipStreamSynchronize(c->stream), "spins");
        } else {
            std::vector<uint32_t> raw(c->d_sqa.n, 0u);
            for (int i = 0; i < c->n_inst; ++i) {
                const InstDev &I = c->idev[i];
                for (int r = 0; r < c->R; ++r)
                    for (int k = 0; k < c->M; ++k) {
                        const int8_t *src = in + (((size_t)i * c->R + r) * c->M + k) * c->n_max;
                        uint32_t *w = raw.data() + I.spin_off + (int64_t)r * I.npad * 2;
                        for (int j = 0; j < I.n; ++j) {
                            if (src[j] != 1 && src[j] != -1) fail(SG_EINVAL, "spins must be +1 or -1");
                            if (src[j] > 0) w[2 * j + (k & 1)] |= 1u << (k >> 1);
                        }
                    }
            }
            c->d_sqa.upload(raw.data(), raw.size(), c->stream, "spins");
            hip_check(hipStreamSynchronize(c->stream), "spins");
        }
    });
}

sg_status sg_get_counters(sg_ctx *c, uint32_t *out3)
{
    return guarded(c, [&] {
        if (!c || !out3) fail(SG_EINVAL, "NULL argument");
        uint32_t v[8];
        c->d_ctr.download(v, 8, c->stream, "counters");
        hip_check(hipStreamSynchronize(c->stream), "counters");
        if (c->mode == SG_SQA) v[0] = c->sqa_steps;
        out3[0] = v[0];
        out3[1] = v[1];
        out3[2] = v[2];
    });
}

// blob: magic, mode, n_inst, sizes, counters[3], best[n_inst], spins (logical, int8)
static size_t state_size(const sg_ctx *c)
{
    const size_t spins = c->mode == SG_APT ? (size_t)c->n_inst * c->n_slots * c->n_max
                                           : (size_t)c->n_inst * c->R * c->M * c->n_max;
    return 64 + 8 * (size_t)c->n_inst + spins + (c->mode == SG_APT ? 8 * (size_t)c->n_inst * (c->n_beta - 1) * c->reps : 0);
}

sg_status sg_get_state(sg_ctx *c, void *blob, size_t *len)
{
    return guarded(c, [&] {
        if (!c || !len) fail(SG_EINVAL, "NULL argument");
        const size_t need = state_size(c);
        if (!blob) { *len = need; return; }
        if (*len < need) fail(SG_EINVAL, "blob too small (%zu < %zu)", *len, need);
        uint8_t *b = (uint8_t *)blob;
        std::memset(b, 0, 64);
        const uint32_t hdr[6] = {0x53474331u, (uint32_t)c->mode, (uint32_t)c->n_inst,
                                 (uint32_t)c->n_max, (uint32_t)c->n_slots, (uint32_t)(c->R * c->M)};
        std::memcpy(b, hdr, sizeof hdr);
        uint32_t ctr[3];
        if (sg_get_counters(c, ctr) != SG_OK) fail(SG_EHIP, "%s", c->err.c_str());
        std::memcpy(b + 24, ctr, sizeof ctr);
        size_t off = 64;
        if (c->mode == SG_APT) {
            c->d_best.download((int64_t *)(b + off), (size_t)c->n_inst, c->stream, "state");
            off += 8 * (size_t)c->n_inst;
            const size_t na = (size_t)c->n_inst * (c->n_beta - 1) * c->reps;
            c->d_acc_count.download((int64_t *)(b + off), na, c->stream, "state");
            off += 8 * na;
            hip_check(hipStreamSynchronize(c->stream), "state");
        } else {
            off += 8 * (size_t)c->n_inst;
        }
        if (sg_get_spins(c, (int8_t *)(b + off)) != SG_OK) fail(SG_EHIP, "%s", c->err.c_str());
        *len = need;
    });
}

sg_status sg_set_state(sg_ctx *c, const void *blob, size_t len)
{
    return guarded(c, [&] {
        if (!c || !blob) fail(SG_EINVAL, "NULL argument");
        if (len != state_size(c)) fail(SG_EINVAL, "blob size does not match the context");
        const uint8_t *b = (const uint8_t *)blob;
        uint32_t hdr[6];
        std::memcpy(hdr, b, sizeof hdr);
        if (hdr[0] != 0x53474331u || hdr[1] != (uint32_t)c->mode || hdr[2] != (uint32_t)c->n_inst ||
            hdr[3] != (uint32_t)c->n_max || hdr[4] != (uint32_t)c->n_slots ||
            hdr[5] != (uint32_t)(c->R * c->M))
            fail(SG_EINVAL, "blob belongs to a different context shape");
        uint32_t ctr[3];
        std::memcpy(ctr, b + 24, sizeof ctr);
        size_t off = 64;
        if (c->mode == SG_APT) {
            c->d_best.upload((const int64_t *)(b + off), (size_t)c->n_inst, c->stream, "state");
            off += 8 * (size_t)c->n_inst;
            const size_t na = (size_t)c->n_inst * (c->n_beta - 1) * c->reps;
            c->d_acc_count.upload((const int64_t *)(b + off), na, c->stream, "state");
            off += 8 * na;
        } else {
            off += 8 * (size_t)c->n_inst;
        }
        if (sg_set_spins(c, (const int8_t *)(b + off)) != SG_OK) fail(SG_EINVAL, "%s", c->err.c_str());
        uint32_t v[8] = {ctr[0], ctr[1], ctr[2], 0u, 0u, 0u, 0u, 0u};
        c->d_ctr.upload(v, 8, c->stream, "state");
        if (c->mode == SG_SQA) c->sqa_steps = ctr[0];
        hip_check(hipStreamSynchronize(c->stream), "state");
    });
}

sg_status sg_timer_start(sg_ctx *c)
{
    return guarded(c, [&] {
        if (!c) fail(SG_EINVAL, "context is NULL");
        if (!c->timer.a) hip_check(hipEventCreate(&c->timer.a), "event");
        if (!c->timer.b) hip_check(hipEventCreate(&c->timer.b), "event");
        hip_check(hipEventRecord(c->timer.a, c->stream), "event");
    });
}

sg_status sg_timer_stop(sg_ctx *c, float *ms)
{
    return guarded(c, [&] {
        if (!c || !ms) fail(SG_EINVAL, "NULL argument");
        if (!c->timer.a) fail(SG_ESTATE, "timer not started");
        hip_check(hipEventRecord(c->timer.b, c->stream), "event");
        hip_check(hipEventSynchronize(c->timer.b), "event");
        hip_check(hipEventElapsedTime(ms, c->timer.a, c->timer.b), "event");
    });
}

sg_status sg_kernel_timing(sg_ctx *c, int32_t enable)
{
    return guarded(c, [&] {
        if (!c) fail(SG_EINVAL, "context is NULL");
        c->ktime = enable != 0;
        c->kev_used = 0;
    });
}

sg_status sg_kernel_time(sg_ctx *c, float *ms, int32_t *launches)
{
    return guarded(c, [&] {
        if (!c || !ms || !launches) fail(SG_EINVAL, "NULL argument");
        hip_check(hipStreamSynchronize(c->stream), "kernel time");
        double tot = 0.0;
        for (size_t i = 0; i < c->kev_used; ++i) {
            float m = 0.f;
            hip_check(hipEventElapsedTime(&m, c->kev[i].first, c->kev[i].second), "kernel time");
            tot += m;
        }
        *ms = (float)tot;
        *launches = (int32_t)c->kev_used;
        c->kev_used = 0;
    });
}

sg_status sg_synchronize(sg_ctx *c)
{
    return guarded(c, [&] {
        if (!c) fail(SG_EINVAL, "context is NULL");
        hip_check(hipStreamSynchronize(c->stream), "synchronize");
    });
}

}  // extern "C"

// ====================================================================== adaptive ladder
namespace {

double sigma_of_moments(int64_t S1, int64_t S2, int64_t N)
{
    const int64_t num = N * S2 - S1 * S1;
    const double var = (double)num / ((double)N * (double)(N - 1));
    return std::sqrt(var);
}

}  // namespace

// The adaptive stage with 32 chains per word (adapt_kernel), for instances without
// fields.  Returns false, having done nothing, when it does not apply; the caller then
// runs the chains as APT slots.
bool adaptive_packed(sg_ctx *c, const sg_adaptive_params *p, double *beta_out,
                     double *sigma_out, int32_t *len_out)
{
    if (any_field(c) || c->ni > 64) return false;
    int max_npad = 0, max_n = 0;
    for (const InstDev &I : c->idev) {
        max_npad = std::max(max_npad, I.npad);
        max_n = std::max(max_n, I.n);
    }
    const int per_thread = 3 * ((max_n + kAdaptThreads - 1) / kAdaptThreads);
    int planes = 1;
    while ((1 << planes) <= per_thread) ++planes;
    const size_t lds = sizeof(uint32_t) * (size_t)(max_npad + 1);
    // + the kernel's static LDS: tables, energy counters, reduction scratch
    const size_t lds_static =
        sizeof(uint32_t) * (kAdaptTabWords + kAdaptPlanes * kAdaptThreads + kAdaptRedWords + 64);
    if (planes > kAdaptPlanes || lds + lds_static > kMaxLds) return false;
    const int n_inst = c->n_inst, nc = p->n_chains, nw = (nc + 31) / 32;
    // one work-group per (instance, chain word): with fewer work-groups than CUs the
    // chains spread wider as APT slots (four per work-group)
    int dev = 0, cus = 0;
    hip_check(hipGetDevice(&dev), "device");
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device");
    if ((int64_t)n_inst * nw < cus) return false;
    hipStream_t s = c->stream;
    AdaptArgs a{};
    a.inst = c->d_inst.p;
    a.rec_col = c->d_rec.p;
    a.rec_j = c->d_recj.p;
    a.wstride = max_npad + 1;
    DevBuf<uint32_t> words;
    words.alloc((size_t)n_inst * nw * (size_t)a.wstride, "adaptive chains");
    DevBuf<int64_t> mom;
    mom.alloc((size_t)n_inst * nc * 2, "moments");
    a.words = words.p;
    a.lut = c->d_lut.p;
    a.mom = mom.p;
    a.n_inst = n_inst;
    a.n_chains = nc;
    a.nw = nw;
    a.imax = c->imax;
    a.ni = c->ni;
    a.planes = planes;
    a.key0 = c->key0;
    a.key1 = c->key1;
    hip_check(launch_adapt_init(a, n_inst, s), "adaptive init");
    std::vector<double> bt(n_inst, p->beta0);
    std::vector<int> len(n_inst, 0);
    std::vector<char> active(n_inst, 1);
    std::vector<uint32_t> lut((size_t)n_inst * c->ni);
    std::vector<int64_t> m((size_t)n_inst * nc * 2);
    uint32_t tglob = 0;
    for (int step = 0; step < p->max_steps; ++step) {
        bool any = false;
        for (int i = 0; i < n_inst; ++i) any |= active[i] != 0;
        if (!any) break;
        for (int i = 0; i < n_inst; ++i)
            for (int I2 = -c->imax; I2 <= c->imax; ++I2)
                lut[(size_t)i * c->ni + (I2 + c->imax)] = heat_bath_threshold(bt[i], I2);
        hip_check(hipStreamSynchronize(s), "adaptive");
        c->d_lut.upload(lut.data(), lut.size(), s, "adaptive tables");
        a.t0 = tglob;
        a.n_sweeps = p->sweeps;
        a.mom_from = p->sweeps - p->tail;
        hip_check(launch_adapt(a, n_inst, lds, s), "adaptive sweeps");
        tglob += (uint32_t)p->sweeps;
        mom.download(m.data(), m.size(), s, "moments");
        hip_check(hipStreamSynchronize(s), "adaptive");
        for (int i = 0; i < n_inst; ++i) {
            if (!active[i]) continue;
            double sum = 0.0;
            for (int k = 0; k < nc; ++k) {
                const int64_t *mk = &m[((size_t)i * nc + k) * 2];
                sum += sigma_of_moments(mk[0], mk[1], p->tail);
            }
            const double sigma = sum / (double)nc;
            beta_out[(size_t)i * p->max_steps + step] = bt[i];
            if (sigma_out) sigma_out[(size_t)i * p->max_steps + step] = sigma;
            len[i] = step + 1;
            if (sigma < p->tol) active[i] = 0;
            else bt[i] = bt[i] + p->alpha / sigma;
        }
    }
    for (int i = 0; i < n_inst; ++i) len_out[i] = len[i];
    return true;
}

extern "C" sg_status sg_adaptive_ladder(const sg_lattice *inst, int32_t n_inst,
                                        const sg_adaptive_params *p, uint64_t seed,
                                        void *hip_stream, double *beta_out, double *sigma_out,
                                        int32_t *len_out)
{
    sg_ctx *c = nullptr;
    try {
        if (!inst || n_inst < 1 || !p || !beta_out || !len_out) fail(SG_EINVAL, "bad arguments");
        if (p->n_chains < 1 || p->sweeps < 1 || p->tail < 2 || p->tail > p->sweeps || p->max_steps < 1)
            fail(SG_EINVAL, "bad adaptive parameters");
        if (!(p->alpha > 0.0) || !std::isfinite(p->beta0) || p->beta0 < 0.0)
            fail(SG_EINVAL, "bad adaptive parameters");
        // Chains are the slots of an APT context with one temperature per instance.
        c = new sg_ctx();
        c->mode = SG_APT;
        // slots = chains: n_beta * reps must equal n_chains -> reps = 1, n_beta = chains
        std::vector<double> ladder((size_t)n_inst * p->n_chains);
        for (int i = 0; i < n_inst; ++i)
            for (int k = 0; k < p->n_chains; ++k) ladder[(size_t)i * p->n_chains + k] = p->beta0 + k;
        sg_config cfg{};
        cfg.mode = SG_APT;
        cfg.n_inst = n_inst;
        cfg.inst = inst;
        cfg.n_beta = std::max(2, p->n_chains);
        if (p->n_chains < 2) {
            ladder.assign((size_t)n_inst * 2, 0.0);
            for (int i = 0; i < n_inst; ++i) { ladder[2 * i] = p->beta0; ladder[2 * i + 1] = p->beta0 + 1.0; }
        }
        cfg.beta = ladder.data();
        cfg.reps_per_beta = 1;
        cfg.seed = seed;
        cfg.hip_stream = hip_stream;
        create_apt(c, &cfg);
        if (adaptive_packed(c, p, beta_out, sigma_out, len_out)) {
            delete c;
            return SG_OK;
        }
        hipStream_t s = c->stream;
        const int nb4 = 4 * c->n_quads;
        // re-initialise with the adaptive-stage purpose tag
        hip_check(launch_apt_init(c->d_inst.p, c->d_desc.p, c->n_blocks, c->d_spins.p, c->d_perm.p,
                                  c->key0, c->key1, TAG_ADAPT_INIT, s),
                  "adaptive init");
        {   // energies of the re-initialised chains
            AptArgs a = apt_args(c, 0, 0);
            a.do_energy = 2;
            hip_check(launch_apt_quad(a, c->quad_lds, s), "adaptive energies");
        }
        // every slot of instance i uses table i (the current beta_t of instance i)
        std::vector<int32_t> slot_lut((size_t)n_inst * nb4);
        for (int i = 0; i < n_inst; ++i)
            for (int k = 0; k < nb4; ++k) slot_lut[(size_t)i * nb4 + k] = i;
        c->d_slot_lut.upload(slot_lut, s, "adaptive tables");
        std::vector<double> bt(n_inst, p->beta0);
        std::vector<int> len(n_inst, 0);
        std::vector<char> active(n_inst, 1);
        std::vector<uint32_t> lut((size_t)n_inst * c->ni);
        std::vector<int64_t> mom((size_t)n_inst * nb4 * 2);
        for (int step = 0; step < p->max_steps; ++step) {
            bool any = false;
            for (int i = 0; i < n_inst; ++i) any |= active[i] != 0;
            if (!any) break;
            for (int i = 0; i < n_inst; ++i)
                for (int I2 = -c->imax; I2 <= c->imax; ++I2)
                    lut[(size_t)i * c->ni + (I2 + c->imax)] = heat_bath_threshold(bt[i], I2);
            hip_check(hipStreamSynchronize(s), "adaptive");
            c->d_lut.upload(lut.data(), lut.size(), s, "adaptive tables");
            hip_check(launch_fill_i64(c->d_mom.p, 0, (int64_t)c->d_mom.n, s), "adaptive");
            AptArgs a = apt_args(c, p->sweeps, 0);
            a.tag = TAG_ADAPT_SWEEP;
            a.mom_from = p->sweeps - p->tail;
            a.do_energy = 1;
            hip_check(launch_apt_quad(a, c->quad_lds, s), "adaptive sweeps");
            hip_check(launch_advance(c->d_ctr.p, (uint32_t)p->sweeps, 0u, 0u, 0u, s), "adaptive");
            c->d_mom.download(mom.data(), mom.size(), s, "moments");
            hip_check(hipStreamSynchronize(s), "adaptive");
            for (int i = 0; i < n_inst; ++i) {
                if (!active[i]) continue;
                double sum = 0.0;
                for (int k = 0; k < p->n_chains; ++k) {
                    const int64_t *m = &mom[((size_t)i * nb4 + k) * 2];
                    sum += sigma_of_moments(m[0], m[1], p->tail);
                }
                const double sigma = sum / (double)p->n_chains;
                beta_out[(size_t)i * p->max_steps + step] = bt[i];
                if (sigma_out) sigma_out[(size_t)i * p->max_steps + step] = sigma;
                len[i] = step + 1;
                if (sigma < p->tol) active[i] = 0;
                else bt[i] = bt[i] + p->alpha / sigma;
            }
        }
        for (int i = 0; i < n_inst; ++i) len_out[i] = len[i];
    } catch (const Failure &e) {
        g_create_error = e.msg;
        delete c;
        return e.code;
    } catch (const std::bad_alloc &) {
        delete c;
        return SG_ENOMEM;
    }
    delete c;
    return SG_OK;
}
