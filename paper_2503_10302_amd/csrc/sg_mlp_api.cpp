// sg_mlp_api.cpp -- host side of the ladder-predictor network (C ABI in sg.h).
// The network is a project component that replaces the adaptive stage of
// Algorithm S2 with a prediction from instance statistics; the adaptive stage
// remains the fallback and the source of training targets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "sg.h"
#include "sg_internal.h"
#include "sg_host.h"

using namespace sg;

namespace {
constexpr int NP = SG_MLP_NPARAM;
constexpr int NPX = NP + 8;   // + feature mean[4], std[4]
constexpr int NBLK = 64;

struct Err {
    sg_status code;
};

void chk(hipError_t e)
{
    if (e == hipSuccess) return;
    (void)hipGetLastError();   // clear the thread's last error (see hip_check in sg_api.cpp)
    if (e == hipErrorOutOfMemory) throw Err{SG_ENOMEM};
    throw Err{SG_EHIP};
}

template <class T>
T *dalloc(size_t n)
{
    T *p = nullptr;
    chk(hipMalloc((void **)&p, std::max<size_t>(n, 1) * sizeof(T)));
    return p;
}

// Same geometry conventions as the spin-glass contexts: j = x + Lx*(y + Ly*z).
struct Geo {
    const sg_lattice &L;
    int n;
    explicit Geo(const sg_lattice &l) : L(l), n(l.Lx * l.Ly * l.Lz) {}
    int len(int a) const { return a == 0 ? L.Lx : (a == 1 ? L.Ly : L.Lz); }
    int coord(int j, int a) const
    {
        return a == 0 ? j % L.Lx : (a == 1 ? (j / L.Lx) % L.Ly : j / (L.Lx * L.Ly));
    }
    int stride(int a) const { return a == 0 ? 1 : (a == 1 ? L.Lx : L.Lx * L.Ly); }
    int nbr(int j, int a, int dir) const
    {
        const int Ln = len(a);
        if (Ln < 2) return -1;
        int c = coord(j, a), c2 = c + dir;
        if (c2 < 0 || c2 >= Ln) {
            if (!((L.periodic >> a) & 1u)) return -1;
            c2 = (c2 + Ln) % Ln;
        }
        return j + (c2 - c) * stride(a);
    }
    int bond(int j, int a, int dir) const
    {
        const int nb = nbr(j, a, dir);
        if (nb < 0) return 0;
        return dir > 0 ? L.J[3 * j + a] : L.J[3 * nb + a];
    }
};

// Features: cube root of n; mean and variance over sites of |sum of the site's
// couplings|; fraction of elementary plaquettes (all four bonds present) whose
// coupling product is negative (frustrated).
void features_of(const sg_lattice &L, double *f)
{
    Geo g(L);
    double s1 = 0.0, s2 = 0.0;
    for (int j = 0; j < g.n; ++j) {
        int c = 0;
        for (int a = 0; a < 3; ++a) c += g.bond(j, a, +1) + g.bond(j, a, -1);
        const double v = std::fabs((double)c);
        s1 += v;
        s2 += v * v;
    }
    const double mean = s1 / (double)g.n;
    int64_t plaq = 0, frus = 0;
    for (int j = 0; j < g.n; ++j)
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b) {
                const int ja = g.nbr(j, a, +1), jb = g.nbr(j, b, +1);
                if (ja < 0 || jb < 0) continue;
                const int p = g.bond(j, a, +1) * g.bond(ja, b, +1) * g.bond(jb, a, +1) * g.bond(j, b, +1);
                if (p == 0) continue;
                ++plaq;
                frus += p < 0;
            }
    f[0] = std::cbrt((double)g.n);
    f[1] = mean;
    f[2] = s2 / (double)g.n - mean * mean;
    f[3] = plaq ? (double)frus / (double)plaq : 0.0;
}

}  // namespace

struct sg_mlp {
    hipStream_t stream = nullptr;
    bool own = false;
    float *P = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *gacc = nullptr, *loss = nullptr;
    int step = 0;
    uint64_t seed = 0;
    float *scratch = nullptr;   // the library's static staging area on this network's GPU
    ~sg_mlp()
    {
        for (float *p : {P, m, v, grad, gacc, loss})
            if (p) (void)hipFree(p);
        if (own && stream) (void)hipStreamDestroy(stream);
    }
};

extern "C" {

sg_status sg_instance_features(const sg_lattice *inst, int32_t n_inst, double *features)
{
    if (!inst || n_inst < 1 || !features) return SG_EINVAL;
    for (int i = 0; i < n_inst; ++i) {
        const sg_lattice &L = inst[i];
        if (L.Lx < 1 || L.Ly < 1 || L.Lz < 1 || !L.J || (int64_t)L.Lx * L.Ly * L.Lz > kMaxN)
            return SG_EINVAL;
    }
    // one instance per host thread at a time: each instance's sums keep their site order
    try {
        parallel_for(n_inst, [&](int i) { features_of(inst[i], features + 4 * (size_t)i); });
    } catch (const std::bad_alloc &) {
        return SG_ENOMEM;
    }
    return SG_OK;
}

sg_status sg_mlp_create(const float *params, uint64_t seed, void *hip_stream, sg_mlp **out)
{
    if (!out) return SG_EINVAL;
    *out = nullptr;
    sg_mlp *m = new (std::nothrow) sg_mlp();
    if (!m) return SG_ENOMEM;
    try {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) throw Err{SG_EHIP};
        if (hip_stream) {
            m->stream = (hipStream_t)hip_stream;
        } else {
            chk(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
            m->own = true;
        }
        m->seed = seed;
        // address of the allocation-free entry point's staging area on this GPU (once per
        // device, with the device current)
        chk(mlp_scratch(&m->scratch));
        std::vector<float> h(NPX, 0.f);
        if (params) {
            std::memcpy(h.data(), params, sizeof(float) * NPX);
        } else {
            std::mt19937_64 rng(seed);
            auto fill = [&](int off, int rows, int fan_in) {
                std::uniform_real_distribution<float> U(-1.f / std::sqrt((float)fan_in),
                                                        1.f / std::sqrt((float)fan_in));
                for (int i = 0; i < rows * fan_in; ++i) h[off + i] = U(rng);
            };
            fill(0, 64, 4);
            fill(64 * 4 + 64, 64, 64);
            fill(64 * 4 + 64 + 64 * 64 + 64, 33, 64);
            for (int k = 0; k < 4; ++k) { h[NP + k] = 0.f; h[NP + 4 + k] = 1.f; }
        }
        for (int k = 0; k < 4; ++k)
            if (!(h[NP + 4 + k] > 0.f)) throw Err{SG_EINVAL};
        m->P = dalloc<float>(NPX);
        m->m = dalloc<float>(NP);
        m->v = dalloc<float>(NP);
        m->grad = dalloc<float>(NP);
        m->gacc = dalloc<float>((size_t)NBLK * NP);
        m->loss = dalloc<float>(NBLK);
        chk(hipMemcpyAsync(m->P, h.data(), sizeof(float) * NPX, hipMemcpyHostToDevice, m->stream));
        chk(hipMemsetAsync(m->m, 0, sizeof(float) * NP, m->stream));
        chk(hipMemsetAsync(m->v, 0, sizeof(float) * NP, m->stream));
        chk(hipStreamSynchronize(m->stream));
    } catch (const Err &e) {
        delete m;
        return e.code;
    }
    *out = m;
    return SG_OK;
}

void sg_mlp_destroy(sg_mlp *m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    delete m;
}

sg_status sg_mlp_set_standardisation(sg_mlp *m, const float *mean4, const float *std4)
{
    if (!m || !mean4 || !std4) return SG_EINVAL;
    for (int k = 0; k < 4; ++k)
        if (!(std4[k] > 0.f)) return SG_EINVAL;
    float h[8];
    std::memcpy(h, mean4, 16);
    std::memcpy(h + 4, std4, 16);
    try {
        chk(hipMemcpyAsync(m->P + NP, h, sizeof h, hipMemcpyHostToDevice, m->stream));
        chk(hipStreamSynchronize(m->stream));
    } catch (const Err &e) {
        return e.code;
    }
    return SG_OK;
}

sg_status sg_mlp_get_params(sg_mlp *m, float *params)
{
    if (!m || !params) return SG_EINVAL;
    try {
        chk(hipMemcpyAsync(params, m->P, sizeof(float) * NPX, hipMemcpyDeviceToHost, m->stream));
        chk(hipStreamSynchronize(m->stream));
    } catch (const Err &e) {
        return e.code;
    }
    return SG_OK;
}

sg_status sg_mlp_loss_grad(sg_mlp *m, const float *x, const float *y, int32_t batch, float *loss,
                           float *grad)
{
    if (!m || !x || !y || batch < 1 || !loss) return SG_EINVAL;
    float *dx = nullptr, *dy = nullptr;
    try {
        dx = dalloc<float>((size_t)batch * 4);
        dy = dalloc<float>((size_t)batch * 33);
        chk(hipMemcpyAsync(dx, x, sizeof(float) * 4 * batch, hipMemcpyHostToDevice, m->stream));
        chk(hipMemcpyAsync(dy, y, sizeof(float) * 33 * batch, hipMemcpyHostToDevice, m->stream));
        const int nblk = std::min(NBLK, (int)batch);
        chk(launch_mlp_pass(m->P, dx, dy, nullptr, batch, nblk, m->gacc, m->loss, nullptr, m->grad,
                            m->stream));
        std::vector<float> l(nblk);
        chk(hipMemcpyAsync(l.data(), m->loss, sizeof(float) * nblk, hipMemcpyDeviceToHost, m->stream));
        if (grad) chk(hipMemcpyAsync(grad, m->grad, sizeof(float) * NP, hipMemcpyDeviceToHost, m->stream));
        chk(hipStreamSynchronize(m->stream));
        double s = 0.0;
        for (float v : l) s += v;
        *loss = (float)(s / ((double)batch * 33.0));
    } catch (const Err &e) {
        (void)hipFree(dx);
        (void)hipFree(dy);
        return e.code;
    }
    (void)hipFree(dx);
    (void)hipFree(dy);
    return SG_OK;
}

sg_status sg_mlp_train(sg_mlp *m, const float *x, const float *y, int32_t n, int32_t batch,
                       int32_t epochs, float lr, float *loss_per_epoch)
{
    if (!m || !x || !y || n < 1 || batch < 1 || epochs < 0 || !(lr > 0.f)) return SG_EINVAL;
    float *dx = nullptr, *dy = nullptr;
    int *didx = nullptr;
    try {
        dx = dalloc<float>((size_t)n * 4);
        dy = dalloc<float>((size_t)n * 33);
        didx = dalloc<int>((size_t)n);
        chk(hipMemcpyAsync(dx, x, sizeof(float) * 4 * (size_t)n, hipMemcpyHostToDevice, m->stream));
        chk(hipMemcpyAsync(dy, y, sizeof(float) * 33 * (size_t)n, hipMemcpyHostToDevice, m->stream));
        std::vector<int> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::mt19937_64 rng(m->seed ^ 0x9E3779B97F4A7C15ull);
        std::vector<float> l(NBLK);
        for (int ep = 0; ep < epochs; ++ep) {
            std::shuffle(order.begin(), order.end(), rng);
            chk(hipStreamSynchronize(m->stream));
            chk(hipMemcpyAsync(didx, order.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice,
                               m->stream));
            double lsum = 0.0;
            for (int s0 = 0; s0 < n; s0 += batch) {
                const int b = std::min(batch, n - s0);
                const int nblk = std::min(NBLK, b);
                chk(launch_mlp_pass(m->P, dx, dy, didx + s0, b, nblk, m->gacc, m->loss, nullptr,
                                    m->grad, m->stream));
                chk(launch_mlp_adam2(m->P, m->grad, m->m, m->v, lr, 0.9f, 0.999f, 1e-8f, ++m->step,
                                     m->stream));
                chk(hipMemcpyAsync(l.data(), m->loss, sizeof(float) * nblk, hipMemcpyDeviceToHost,
                                   m->stream));
                chk(hipStreamSynchronize(m->stream));
                for (int k = 0; k < nblk; ++k) lsum += l[k];
            }
            if (loss_per_epoch) loss_per_epoch[ep] = (float)(lsum / ((double)n * 33.0));
        }
    } catch (const Err &e) {
        (void)hipFree(dx); (void)hipFree(dy); (void)hipFree(didx);
        return e.code;
    }
    (void)hipFree(dx); (void)hipFree(dy); (void)hipFree(didx);
    return SG_OK;
}

sg_status sg_ladder_predict(sg_mlp *m, const sg_lattice *inst, int32_t n_inst, double *beta_out,
                            double *cutoff_out)
{
    if (!m || !inst || n_inst < 1 || !beta_out) return SG_EINVAL;
    std::vector<double> f((size_t)n_inst * 4);
    sg_status st = sg_instance_features(inst, n_inst, f.data());
    if (st != SG_OK) return st;
    std::vector<float> xf(f.begin(), f.end()), out((size_t)n_inst * 33);
    float *dx = nullptr, *dout = nullptr;
    try {
        dx = dalloc<float>((size_t)n_inst * 4);
        dout = dalloc<float>((size_t)n_inst * 33);
        chk(hipMemcpyAsync(dx, xf.data(), sizeof(float) * xf.size(), hipMemcpyHostToDevice, m->stream));
        chk(launch_mlp_pass(m->P, dx, nullptr, nullptr, n_inst, std::min(NBLK, (int)n_inst), nullptr,
                            nullptr, dout, nullptr, m->stream));
        chk(hipMemcpyAsync(out.data(), dout, sizeof(float) * out.size(), hipMemcpyDeviceToHost, m->stream));
        chk(hipStreamSynchronize(m->stream));
    } catch (const Err &e) {
        (void)hipFree(dx); (void)hipFree(dout);
        return e.code;
    }
    (void)hipFree(dx); (void)hipFree(dout);
    for (int i = 0; i < n_inst; ++i) {
        for (int k = 0; k < 32; ++k) beta_out[(size_t)i * 32 + k] = std::exp((double)out[(size_t)i * 33 + k]);
        if (cutoff_out) cutoff_out[i] = std::exp((double)out[(size_t)i * 33 + 32]);
    }
    return SG_OK;
}

}  // extern "C"

namespace {

// Monotone linear interpolation of a ladder of len rungs onto k rungs at evenly spaced points
// of the normalised rung index (the end points kept exactly).
void resample_ladder(const double *b, int len, int k, double *out)
{
    if (len == 1) {
        for (int i = 0; i < k; ++i) out[i] = b[0];
        return;
    }
    const double step = (double)(len - 1) / (double)(k - 1);
    for (int i = 0; i < k; ++i) {
        const double u = i == k - 1 ? (double)(len - 1) : (double)i * step;
        int j = (int)u;
        if (j >= len - 1) {
            out[i] = b[len - 1];
            continue;
        }
        const double slope = b[j + 1] - b[j];
        out[i] = slope * (u - (double)j) + b[j];
    }
}

// Inverse of the complementary error function on (0, 1]: Newton's method on erfc(x) = y,
// kept inside a bracket [lo, hi] of the root (erfc falls from 1 at 0 to below 1e-300 at 27)
// and bisecting whenever a step would leave it.
double erfc_inv(double y)
{
    constexpr double kPi = 3.14159265358979323846;
    double lo = 0.0, hi = 27.0, x = 1.0;
    for (int it = 0; it < 200; ++it) {
        const double f = std::erfc(x) - y;   // decreasing in x
        if (f > 0.0)
            lo = x;
        else
            hi = x;
        const double d = -2.0 / std::sqrt(kPi) * std::exp(-x * x);
        double xn = d != 0.0 ? x - f / d : 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 1e-15 * std::max(1.0, x)) return xn;
        x = xn;
    }
    return x;
}

constexpr int kRungs = 32, kPairs = kRungs - 1, kPilotReps = 2;
constexpr int kPilotLaunchConfig = 1;   // APT launch configuration of the pilots
// Pilot acceptances are clamped to [kAccEps, 1 - kAccEps] before they are turned into lengths.
constexpr double kAccEps = 1e-3;

// Swap acceptance of every adjacent pair of each instance over a pilot APT+ICM run: two labels,
// one sweep per attempt, each instance at its own ICM cutoff.  Pair b is attempted on every other
// attempt (odd attempts try the even pairs), once per label.
sg_status pilot_acceptance(const sg_lattice *inst, int n, const double *beta, const double *cutoff,
                           int cycles, uint64_t seed, double *acc)
{
    sg_config cfg{};
    cfg.mode = SG_APT;
    cfg.n_inst = n;
    cfg.inst = inst;
    cfg.n_beta = kRungs;
    cfg.beta = beta;
    cfg.reps_per_beta = kPilotReps;
    cfg.seed = seed;
    cfg.hip_stream = nullptr;
    sg_ctx *c = nullptr;
    sg_status st = sg_create(&cfg, &c);
    if (st != SG_OK) return st;
    // A fixed launch configuration (work-groups ordered by cost within each XCD, at least
    // seven waves per SIMD): a pilot is short, and every configuration gives the same results,
    // so timing the candidates on its fresh shape would cost more than it could save.
    st = sg_set_launch_config(c, kPilotLaunchConfig);
    if (st != SG_OK) {
        set_global_error(sg_last_error(c));
        sg_destroy(c);
        return st;
    }
    sg_apt_options opt{};
    opt.sweeps_per_swap = 1;
    opt.icm_pairs = 2;
    opt.icm_cutoff = 0.0;
    opt.icm_cutoff_per_inst = cutoff;
    opt.record_every = 0;
    std::vector<int64_t> counts((size_t)n * kPairs * kPilotReps);
    st = sg_run_apt_ex(c, cycles, &opt, nullptr);
    if (st == SG_OK) st = sg_swap_counts(c, counts.data());
    if (st != SG_OK) {
        set_global_error(sg_last_error(c));
        sg_destroy(c);
        return st;
    }
    sg_destroy(c);
    for (int i = 0; i < n; ++i)
        for (int b = 0; b < kPairs; ++b) {
            const int64_t attempts = (cycles + (1 - b % 2)) / 2;
            int64_t a = 0;
            for (int l = 0; l < kPilotReps; ++l) a += counts[((size_t)i * kPairs + b) * kPilotReps + l];
            acc[(size_t)i * kPairs + b] = (double)a / (double)(kPilotReps * attempts);
        }
    return SG_OK;
}

bool in_band(const double *acc, const double *lo, const double *hi)
{
    for (int b = 0; b < kPairs; ++b)
        if (!(acc[b] >= lo[b] && acc[b] <= hi[b])) return false;
    return true;
}

}  // namespace

extern "C" {

sg_status sg_ladder_repair(const double *beta, const double *acc, const double *band_lo,
                           const double *band_hi, int32_t n_beta, double damping, double *beta_out)
{
    if (!beta || !acc || !band_lo || !band_hi || !beta_out || n_beta < 2 ||
        !(damping > 0.0 && damping <= 1.0)) {
        set_global_error("sg_ladder_repair: NULL argument, n_beta < 2 or damping outside (0, 1]");
        return SG_EINVAL;
    }
    const int NP = n_beta - 1;
    for (int k = 0; k < n_beta; ++k)
        if (!(beta[k] > 0.0) || !std::isfinite(beta[k]) || (k > 0 && !(beta[k] > beta[k - 1]))) {
            set_global_error("sg_ladder_repair: betas must be finite, positive and strictly ascending");
            return SG_EINVAL;
        }
    for (int b = 0; b < NP; ++b)
        if (!(acc[b] >= 0.0 && acc[b] <= 1.0) || !(band_lo[b] <= band_hi[b]) ||
            !std::isfinite(band_lo[b]) || !std::isfinite(band_hi[b])) {
            set_global_error("sg_ladder_repair: acceptance outside [0, 1] or an empty band");
            return SG_EINVAL;
        }
    // Length of each pair under the Gaussian-energy acceptance erfc(dbeta sigma / 2): measured
    // (S, from the pilot) and wanted (T, from the band's midpoint), accumulated over the rungs.
    auto length = [](double a) { return 2.0 * erfc_inv(std::min(std::max(a, kAccEps), 1.0 - kAccEps)); };
    std::vector<double> S(n_beta, 0.0), T(n_beta, 0.0), out(n_beta);
    for (int b = 0; b < NP; ++b) {
        S[b + 1] = S[b] + length(acc[b]);
        T[b + 1] = T[b] + length(0.5 * (band_lo[b] + band_hi[b]));
    }
    // Rung k moves to where the instance's measured length reaches the share T[k] / T[NP] of
    // its total, interpolated linearly in log beta between the old rungs; the end rungs stay.
    int j = 0;
    for (int k = 0; k < n_beta; ++k) {
        double lb;
        if (k == 0) {
            lb = std::log(beta[0]);
        } else if (k == NP) {
            lb = std::log(beta[NP]);
        } else {
            const double P = S[NP] * T[k] / T[NP];
            while (j < NP - 1 && S[j + 1] < P) ++j;
            const double u = (P - S[j]) / (S[j + 1] - S[j]);
            lb = std::log(beta[j]) + u * (std::log(beta[j + 1]) - std::log(beta[j]));
        }
        out[k] = std::exp((1.0 - damping) * std::log(beta[k]) + damping * lb);
    }
    out[0] = beta[0];
    out[NP] = beta[NP];
    std::copy(out.begin(), out.end(), beta_out);
    return SG_OK;
}

sg_status sg_judge_ladders(const sg_lattice *inst, int32_t n_inst, const double *band_lo,
                           const double *band_hi, const sg_adaptive_params *fallback,
                           int32_t pilot_cycles, int32_t repair_rounds, uint64_t seed,
                           double *beta_io, double *cutoff_io, int32_t *status, double *acc_out)
{
    if (!inst || n_inst < 1 || !band_lo || !band_hi || !fallback || pilot_cycles < 2 ||
        repair_rounds < 0 || !beta_io || !cutoff_io || !status) {
        set_global_error("sg_judge_ladders: bad arguments");
        return SG_EINVAL;
    }
    const size_t n = (size_t)n_inst;
    std::vector<double> acc(n * kPairs);
    // 1. pilot on the candidate ladders, band check of every pair
    sg_status st = pilot_acceptance(inst, n_inst, beta_io, cutoff_io, pilot_cycles, seed, acc.data());
    if (st != SG_OK) return st;
    std::vector<int> bad;
    for (size_t i = 0; i < n; ++i) {
        const bool ok = in_band(&acc[i * kPairs], &band_lo[i * kPairs], &band_hi[i * kPairs]);
        status[i] = ok ? 0 : 1;
        if (!ok) bad.push_back((int)i);
    }
    // 2. repair rounds on the failing instances: re-space the rungs from the last pilot's
    //    acceptance (the full step first, half steps after), pilot again, keep what passes
    for (int r = 0; r < repair_rounds && !bad.empty(); ++r) {
        const size_t m = bad.size();
        std::vector<sg_lattice> sub(m);
        std::vector<double> lad(m * kRungs), cut(m), acc2(m * kPairs);
        for (size_t q = 0; q < m; ++q) {
            const size_t i = (size_t)bad[q];
            sub[q] = inst[i];
            cut[q] = cutoff_io[i];
            st = sg_ladder_repair(&beta_io[i * kRungs], &acc[i * kPairs], &band_lo[i * kPairs],
                                  &band_hi[i * kPairs], kRungs, r == 0 ? 1.0 : 0.5, &lad[q * kRungs]);
            if (st != SG_OK) return st;
        }
        st = pilot_acceptance(sub.data(), (int)m, lad.data(), cut.data(), pilot_cycles, seed + 2 + r,
                              acc2.data());
        if (st != SG_OK) return st;
        std::vector<int> still;
        for (size_t q = 0; q < m; ++q) {
            const size_t i = (size_t)bad[q];
            std::copy(&lad[q * kRungs], &lad[q * kRungs] + kRungs, &beta_io[i * kRungs]);
            std::copy(&acc2[q * kPairs], &acc2[q * kPairs] + kPairs, &acc[i * kPairs]);
            if (in_band(&acc[i * kPairs], &band_lo[i * kPairs], &band_hi[i * kPairs]))
                status[i] = 2;
            else
                still.push_back((int)i);
        }
        bad.swap(still);
    }
    if (acc_out) std::copy(acc.begin(), acc.end(), acc_out);
    if (bad.empty()) return SG_OK;
    // 3. the adaptive stage for every instance still outside the band, resampled to 32 rungs;
    //    its cutoff is the first rung at or above 1
    std::vector<sg_lattice> sub;
    for (int i : bad) sub.push_back(inst[i]);
    const int ms = fallback->max_steps;
    std::vector<double> lad((size_t)sub.size() * ms);
    std::vector<int32_t> len(sub.size());
    st = sg_adaptive_ladder(sub.data(), (int32_t)sub.size(), fallback, seed + 1, nullptr, lad.data(),
                            nullptr, len.data());
    if (st != SG_OK) return st;
    for (size_t q = 0; q < bad.size(); ++q) {
        double *o = beta_io + (size_t)bad[q] * kRungs;
        resample_ladder(&lad[q * ms], len[q], kRungs, o);
        int r = 0;
        while (r < kRungs - 1 && o[r] < 1.0) ++r;
        cutoff_io[bad[q]] = o[r];
        status[bad[q]] = 1;
    }
    return SG_OK;
}

sg_status sg_learned_ladders(sg_mlp *m, const sg_lattice *inst, int32_t n_inst, const double *band_lo,
                             const double *band_hi, const sg_adaptive_params *fallback,
                             int32_t pilot_cycles, int32_t repair_rounds, uint64_t seed,
                             double *beta_out, double *cutoff_out, int32_t *status, double *acc_out)
{
    if (!m || !inst || n_inst < 1 || !band_lo || !band_hi || !fallback || pilot_cycles < 2 ||
        repair_rounds < 0 || !beta_out || !cutoff_out || !status) {
        set_global_error("sg_learned_ladders: bad arguments");
        return SG_EINVAL;
    }
    // the network's ladders and cutoffs, then the judge
    const sg_status st = sg_ladder_predict(m, inst, n_inst, beta_out, cutoff_out);
    if (st != SG_OK) return st;
    return sg_judge_ladders(inst, n_inst, band_lo, band_hi, fallback, pilot_cycles, repair_rounds,
                            seed, beta_out, cutoff_out, status, acc_out);
}

sg_status sg_ladder_predict_noalloc(sg_mlp *m, const sg_lattice *inst, int32_t n_inst,
                                    double *beta_out, double *cutoff_out)
{
    if (!m || !inst || n_inst < 1 || !beta_out) {
        set_global_error("sg_ladder_predict_noalloc: NULL argument or n_inst < 1");
        return SG_EINVAL;
    }
    if (n_inst > kPredictMax) {
        char msg[128];
        std::snprintf(msg, sizeof msg, "sg_ladder_predict_noalloc: n_inst = %d exceeds the limit of %d",
                      (int)n_inst, kPredictMax);
        set_global_error(msg);
        return SG_EINVAL;
    }
    for (int i = 0; i < n_inst; ++i) {
        const sg_lattice &L = inst[i];
        if (L.Lx < 1 || L.Ly < 1 || L.Lz < 1 || !L.J || (int64_t)L.Lx * L.Ly * L.Lz > kMaxN) {
            set_global_error("sg_ladder_predict_noalloc: invalid lattice");
            return SG_EINVAL;
        }
    }
    if (!m->scratch) {
        set_global_error("sg_ladder_predict_noalloc: no staging area on this device");
        return SG_EHIP;
    }
    // Host staging lives in beta_out itself (256 bytes per instance): the float features
    // in its first 16 n bytes, the 33 float outputs in its last 132 n bytes.  Expanding
    // instance i's outputs to doubles writes bytes [256 i, 256 i + 256), which lie below
    // the outputs of every later instance (124 n + 132 (i + 1) >= 256 (i + 1) for i < n).
    const size_t n = (size_t)n_inst;
    float *hx = reinterpret_cast<float *>(beta_out);
    float *hout = reinterpret_cast<float *>(beta_out) + 31 * n;
    for (size_t i = 0; i < n; ++i) {
        double f[4];
        features_of(inst[i], f);
        for (int k = 0; k < 4; ++k) hx[4 * i + k] = (float)f[k];
    }
    float *dx = m->scratch, *dout = m->scratch + (size_t)kPredictMax * 4;
    try {
        chk(hipMemcpyAsync(dx, hx, sizeof(float) * 4 * n, hipMemcpyHostToDevice, m->stream));
        chk(launch_mlp_pass(m->P, dx, nullptr, nullptr, n_inst, std::min(NBLK, (int)n_inst), nullptr,
                            nullptr, dout, nullptr, m->stream));
        chk(hipMemcpyAsync(hout, dout, sizeof(float) * 33 * n, hipMemcpyDeviceToHost, m->stream));
        chk(hipStreamSynchronize(m->stream));
    } catch (const Err &e) {
        set_global_error("sg_ladder_predict_noalloc: HIP error");
        return e.code;
    }
    for (size_t i = 0; i < n; ++i) {
        float o[33];
        std::memcpy(o, hout + 33 * i, sizeof o);
        for (int k = 0; k < 32; ++k) beta_out[i * 32 + k] = std::exp((double)o[k]);
        if (cutoff_out) cutoff_out[i] = std::exp((double)o[32]);
    }
    set_global_error("");
    return SG_OK;
}

}  // extern "C"
