"""Learned inverse-temperature ladders for APT (a project component, not in the paper).

The adaptive stage of Algorithm S2 (Methods, "APT details") builds a β ladder per
instance from energy fluctuations of chains run at each rung.  Here a small MLP
predicts a 32-rung ladder and the ICM cutoff from four instance statistics; it is
trained on ladders that the adaptive stage itself produced on generated instances.
The adaptive stage stays the judge: a predicted ladder is used only if every
adjacent pair's swap acceptance in a short pilot run lies in the band
[0.5, 1.5] * erfc(alpha / 2); otherwise the adaptive stage runs for that instance.

All Monte Carlo work and the network's forward/backward/Adam steps run in libsg's
HIP kernels; this module only arranges data and calls the C ABI.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import sg

N_RUNGS = 32
ALPHA = 1.25
# Default band (every adjacent pair): [0.5, 1.5] x erfc(alpha / 2), the acceptance of Gaussian
# energies on a ladder with beta steps alpha / sigma_E.  The shipped network carries per-size,
# per-pair bands calibrated on the adaptive stage's own ladders (band_tables), which replace
# it: the paper reports roughly constant acceptance except for the last few replicas.
BAND = (0.5 * math.erfc(ALPHA / 2), 1.5 * math.erfc(ALPHA / 2))   # ~ (0.19, 0.57)


def resample(betas, k=N_RUNGS):
    """Monotone linear interpolation of a ladder to k rungs in normalised rung index."""
    b = np.asarray(betas, np.float64)
    if b.size == 1:
        return np.full(k, b[0])
    u = np.linspace(0.0, b.size - 1.0, k)
    return np.interp(u, np.arange(b.size), b)


def cutoff_label(ladder, beta_star=1.0):
    """ICM cutoff target: the first rung at or above beta_star (the last rung if none)."""
    ladder = np.asarray(ladder)
    idx = np.searchsorted(ladder, beta_star)
    return float(ladder[min(idx, ladder.size - 1)])


def features(instances):
    lib = sg.load()
    arr, keep = sg._lattices(instances)
    f = np.zeros((len(instances), 4), np.float64)
    rc = lib.sg_instance_features(arr, len(instances), f.ctypes.data_as(C.c_void_p))
    if rc != sg.SG_OK:
        raise sg.SGError(rc, "sg_instance_features")
    return f


def adaptive_ladders(instances, seed, **params):
    """Adaptive stage on the GPU, one batch per lattice size (instances of one size finish
    after a similar number of rungs)."""
    sizes = [int(np.prod(np.asarray(J).shape[:3])) for J, *_ in instances]
    out = [None] * len(instances)
    for n in sorted(set(sizes)):
        idx = [i for i, s in enumerate(sizes) if s == n]
        res = sg.adaptive_ladder([instances[i] for i in idx], seed, **params)
        for i, r in zip(idx, res):
            out[i] = r
    return out


def targets(ladder):
    """Network target: log of the 32-rung ladder and log of the cutoff."""
    l32 = resample(ladder)
    return np.concatenate([np.log(l32), [math.log(cutoff_label(l32))]])


class Predictor:
    """The ladder MLP; parameters live on the GPU (libsg sg_mlp)."""

    def __init__(self, params=None, seed=1):
        self.lib = sg.load()
        h = C.c_void_p()
        p = None if params is None else np.ascontiguousarray(params, np.float32)
        rc = self.lib.sg_mlp_create(None if p is None else p.ctypes.data_as(C.c_void_p), int(seed),
                                    None, C.byref(h))
        if rc != sg.SG_OK:
            raise sg.SGError(rc, "sg_mlp_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.sg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_standardisation(self, mean, std):
        m = np.ascontiguousarray(mean, np.float32)
        s = np.ascontiguousarray(std, np.float32)
        rc = self.lib.sg_mlp_set_standardisation(self.h, m.ctypes.data_as(C.c_void_p),
                                                 s.ctypes.data_as(C.c_void_p))
        if rc != sg.SG_OK:
            raise sg.SGError(rc, "sg_mlp_set_standardisation")

    def train(self, X, Y, epochs=300, batch=64, lr=1e-3):
        x = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(Y, np.float32)
        losses = np.zeros(epochs, np.float32)
        rc = self.lib.sg_mlp_train(self.h, x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p),
                                   x.shape[0], batch, epochs, C.c_float(lr),
                                   losses.ctypes.data_as(C.c_void_p))
        if rc != sg.SG_OK:
            raise sg.SGError(rc, "sg_mlp_train")
        return losses

    def loss(self, X, Y):
        """Mean squared error over the batch and the 33 outputs (network kernels)."""
        x = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(Y, np.float32)
        out = C.c_float()
        rc = self.lib.sg_mlp_loss_grad(self.h, x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p),
                                       x.shape[0], C.byref(out), None)
        if rc != sg.SG_OK:
            raise sg.SGError(rc, "sg_mlp_loss_grad")
        return out.value

    def params(self):
        p = np.zeros(sg.MLP_NPARAM + 8, np.float32)
        rc = self.lib.sg_mlp_get_params(self.h, p.ctypes.data_as(C.c_void_p))
        if rc != sg.SG_OK:
            raise sg.SGError(rc, "sg_mlp_get_params")
        return p

    def predict(self, instances):
        arr, keep = sg._lattices(instances)
        b = np.zeros((len(instances), N_RUNGS), np.float64)
        c = np.zeros(len(instances), np.float64)
        rc = self.lib.sg_ladder_predict(self.h, arr, len(instances), b.ctypes.data_as(C.c_void_p),
                                        c.ctypes.data_as(C.c_void_p))
        if rc != sg.SG_OK:
            raise sg.SGError(rc, "sg_ladder_predict")
        return b, c

    def predict_noalloc(self, instances):
        """The same prediction through the allocation-free entry point (at most
        sg.PREDICT_NOALLOC_MAX instances per call)."""
        arr, keep = sg._lattices(instances)
        b = np.zeros((len(instances), N_RUNGS), np.float64)
        c = np.zeros(len(instances), np.float64)
        rc = self.lib.sg_ladder_predict_noalloc(self.h, arr, len(instances),
                                                b.ctypes.data_as(C.c_void_p),
                                                c.ctypes.data_as(C.c_void_p))
        if rc != sg.SG_OK:
            raise sg.SGError(rc, self.lib.sg_last_error(None).decode())
        return b, c


OFF_B3 = sg.MLP_NPARAM - (N_RUNGS + 1)
OFF_W3 = OFF_B3 - (N_RUNGS + 1) * 64


def initial_params(Y, mean, std, seed=1, w3_scale=0.1):
    """Random network whose output layer starts at the mean target: bias b3 maps to the
    mean log beta_0, the inverse softplus of the mean log increments and the mean log
    cutoff; W3 is scaled down so the first predictions sit near the mean ladder."""
    m = Predictor(seed=seed)
    p = m.params()
    m.close()
    ym = np.asarray(Y, np.float64).mean(axis=0)
    inc = np.maximum(np.diff(ym[:N_RUNGS]), 1e-4)
    b3 = np.concatenate([[ym[0]], inc + np.log(-np.expm1(-inc)), [ym[N_RUNGS]]])
    p[OFF_W3:OFF_B3] *= w3_scale
    p[OFF_B3:sg.MLP_NPARAM] = b3
    p[sg.MLP_NPARAM:sg.MLP_NPARAM + 4] = mean
    p[sg.MLP_NPARAM + 4:sg.MLP_NPARAM + 8] = std
    return p


def fit(X, Y, epochs=400, batch=64, lrs=(1e-3, 3e-4, 1e-4), seed=1):
    """Train a Predictor on features X [N][4] and targets Y [N][33]; the epochs are split
    evenly over the learning rates in `lrs`."""
    mean, std = X.mean(axis=0), X.std(axis=0)
    std = np.where(std > 1e-9, std, 1.0)
    m = Predictor(initial_params(Y, mean, std, seed))
    losses = [m.train(X, Y, epochs=max(1, epochs // len(lrs)), batch=batch, lr=lr) for lr in lrs]
    return m, np.concatenate(losses)


def acceptance(counts, cycles, n_beta, reps=2):
    """Per-pair swap acceptance from a context's accepted-swap counters after `cycles`
    swap attempts counted from the context's creation.  Attempt a = 1, 2, ... tries pairs
    (0,1), (2,3), ... when a is odd and (1,2), (3,4), ... when a is even.  A pair with no
    attempt yet gets NaN."""
    c = np.asarray(counts).reshape(-1, n_beta - 1, reps).sum(axis=2)
    attempts = np.array([(cycles + (1 - b % 2)) // 2 for b in range(n_beta - 1)], np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(attempts > 0, c / (reps * attempts), np.nan)


def pilot_acceptance(instances, ladders, seed, cycles=1000, cutoff=1.0, reps=2):
    """Swap acceptance of every adjacent pair over a pilot APT+ICM run (per instance; cutoff a
    value or one per instance)."""
    lad = np.ascontiguousarray(ladders, np.float64)
    ctx = sg.apt(instances, lad, seed, reps_per_beta=reps)
    ctx.run_apt_ex(cycles, 1, cutoff, 2)
    acc = acceptance(ctx.swap_counts(), cycles, lad.shape[1], reps)
    ctx.close()
    return acc


def in_band(acc, lo=BAND[0], hi=BAND[1]):
    """Band check over every adjacent pair; lo and hi scalars or per-pair arrays [..][31]."""
    a = np.asarray(acc)
    return np.all((a >= lo) & (a <= hi), axis=1)


_PARAMS = __import__("os").path.join(__import__("os").path.dirname(__file__), "ladder_mlp.npz")


def default_params():
    """The shipped network (ladder_mlp.npz): trained on adaptive-stage ladders of generated
    +-1 cubic instances, L in {8, 10, 12, 15}, a random fraction of bonds in [0, 0.3) removed,
    the stage at the Methods settings."""
    return np.load(_PARAMS)["params"]


def default_tables():
    """Per-size tables shipped with the network: 'sizes' [k]; 'band_lo', 'band_hi' [k][31] the
    per-pair acceptance bands; 'size_mean' [k][33] the mean target (log betas, log cutoff) of
    the training instances of each size -- the lookup-table baseline."""
    d = np.load(_PARAMS)
    if "sizes" not in d:
        return None
    return {k: d[k] for k in ("sizes", "band_lo", "band_hi", "size_mean")}


def _size_index(instances, sizes):
    L = np.array([round(np.prod(np.asarray(J).shape[:3]) ** (1 / 3)) for J, *_ in instances])
    return np.abs(L[:, None] - np.asarray(sizes)[None, :]).argmin(axis=1)


def bands_for(instances, tables=None):
    """Per-instance, per-pair bands [n][31] from the table of the nearest size (the default
    band for every pair without tables)."""
    n = len(instances)
    if tables is None:
        return np.full((n, N_RUNGS - 1), BAND[0]), np.full((n, N_RUNGS - 1), BAND[1])
    k = _size_index(instances, tables["sizes"])
    return tables["band_lo"][k].astype(np.float64), tables["band_hi"][k].astype(np.float64)


def table_ladders(instances, tables):
    """The lookup-table baseline: the mean training ladder (and cutoff) of the nearest size."""
    k = _size_index(instances, tables["sizes"])
    y = tables["size_mean"][k]
    return np.exp(y[:, :N_RUNGS]), np.exp(y[:, N_RUNGS])


# Repair rounds of the judge before the adaptive fallback (sg_judge_ladders).
REPAIR_ROUNDS = 3
# Status codes of a judged ladder.
KEPT, ADAPTIVE_FALLBACK, REPAIRED = 0, 1, 2


def repair(beta, acc, lo, hi, damping=1.0):
    """sg_ladder_repair: one re-spacing of a ladder from a pilot's per-pair acceptance towards
    the middle of the band (end rungs fixed).  Host arithmetic, no GPU."""
    lib = sg.load()
    b = np.ascontiguousarray(beta, np.float64)
    a = np.ascontiguousarray(acc, np.float64)
    lo = np.ascontiguousarray(np.broadcast_to(lo, a.shape), np.float64)
    hi = np.ascontiguousarray(np.broadcast_to(hi, a.shape), np.float64)
    out = np.zeros_like(b)
    rc = lib.sg_ladder_repair(b.ctypes.data_as(C.c_void_p), a.ctypes.data_as(C.c_void_p),
                              lo.ctypes.data_as(C.c_void_p), hi.ctypes.data_as(C.c_void_p), b.size,
                              float(damping), out.ctypes.data_as(C.c_void_p))
    if rc != sg.SG_OK:
        raise sg.SGError(rc, lib.sg_last_error(None).decode())
    return out


def _judge_args(instances, tables):
    lo, hi = bands_for(instances, tables)
    p = sg._Adaptive(*(ADAPTIVE[k] for k in ("beta0", "alpha", "tol", "n_chains", "sweeps", "tail",
                                             "max_steps")))
    return np.ascontiguousarray(lo), np.ascontiguousarray(hi), p


def judge_ladders(instances, ladders, cutoffs, seed, pilot=1000, tables="default",
                  repair_rounds=REPAIR_ROUNDS):
    """sg_judge_ladders on given candidate ladders (e.g. the lookup table's): pilot, per-pair
    band check, repair rounds, adaptive fallback.  Returns (ladders [n][32], cutoffs [n],
    status [n] (KEPT, REPAIRED or ADAPTIVE_FALLBACK), acceptance of the last pilot [n][31])."""
    if isinstance(tables, str):
        tables = default_tables()
    lo, hi, p = _judge_args(instances, tables)
    arr, keep = sg._lattices(instances)
    n = len(instances)
    lad = np.ascontiguousarray(ladders, np.float64).copy()
    cut = np.ascontiguousarray(np.broadcast_to(cutoffs, (n,)), np.float64).copy()
    st = np.zeros(n, np.int32)
    acc = np.zeros((n, N_RUNGS - 1), np.float64)
    lib = sg.load()
    rc = lib.sg_judge_ladders(arr, n, lo.ctypes.data_as(C.c_void_p), hi.ctypes.data_as(C.c_void_p),
                              C.byref(p), int(pilot), int(repair_rounds), int(seed),
                              lad.ctypes.data_as(C.c_void_p), cut.ctypes.data_as(C.c_void_p),
                              st.ctypes.data_as(C.c_void_p), acc.ctypes.data_as(C.c_void_p))
    if rc != sg.SG_OK:
        raise sg.SGError(rc, lib.sg_last_error(None).decode())
    return lad, cut, st, acc


def learned_ladders(instances, seed, params=None, pilot=1000, tables="default",
                    repair_rounds=REPAIR_ROUNDS):
    """The learned-ladder flow (libsg sg_learned_ladders): predicted ladders and per-instance
    cutoffs put through the judge (pilot APT+ICM run, band check of every adjacent pair, repair
    rounds, the adaptive stage for every instance still outside the band).

    Returns (ladders [n][32], cutoffs [n], status [n] (KEPT, REPAIRED or ADAPTIVE_FALLBACK),
    acceptance of the last pilot [n][31])."""
    if isinstance(tables, str):
        tables = default_tables() if params is None else None
    lo, hi, p = _judge_args(instances, tables)
    m = Predictor(default_params() if params is None else params)
    arr, keep = sg._lattices(instances)
    n = len(instances)
    lad = np.zeros((n, N_RUNGS), np.float64)
    cut = np.zeros(n, np.float64)
    st = np.zeros(n, np.int32)
    acc = np.zeros((n, N_RUNGS - 1), np.float64)
    rc = m.lib.sg_learned_ladders(m.h, arr, n, lo.ctypes.data_as(C.c_void_p),
                                  hi.ctypes.data_as(C.c_void_p), C.byref(p), int(pilot),
                                  int(repair_rounds), int(seed), lad.ctypes.data_as(C.c_void_p),
                                  cut.ctypes.data_as(C.c_void_p), st.ctypes.data_as(C.c_void_p),
                                  acc.ctypes.data_as(C.c_void_p))
    m.close()
    if rc != sg.SG_OK:
        raise sg.SGError(rc, m.lib.sg_last_error(None).decode())
    return lad, cut, st, acc


# ----------------------------------------------------------------------------------------
# Study driver: training data from the adaptive stage, training, held-out evaluation.
# ----------------------------------------------------------------------------------------
# The adaptive stage at the settings of the Methods section (APT details): beta0 = 0.5,
# alpha = 1.25, 100 chains, variance over the last 1000 of 10000 sweeps, stop once the
# mean standard deviation falls below min|J| / 2.
ADAPTIVE = dict(beta0=0.5, alpha=ALPHA, tol=0.5, n_chains=100, sweeps=10000, tail=1000, max_steps=64)
ICM_CUTOFF = 1.0


def dilution_of(i, seed0, p_max):
    """Fraction of absent bonds of instance seed0 + i: uniform in [0, p_max), drawn from a
    generator seeded by the instance (0 when p_max = 0)."""
    if p_max <= 0:
        return 0.0
    return float(np.random.default_rng([0xD1A, seed0 + i]).random() * p_max)


def _instances(idx, sizes, seed0, p_max=0.0):
    """Periodic +-J instances seed0 + i of size sizes[i mod len(sizes)], with a random fraction
    (dilution_of) of their bonds removed when p_max > 0."""
    from .inputs import diluted_couplings, ej_couplings
    out = []
    for i in idx:
        L = sizes[i % len(sizes)]
        p = dilution_of(i, seed0, p_max)
        J = diluted_couplings(L, 7, seed0 + i, p) if p > 0 else ej_couplings(L, 7, seed=seed0 + i)[0]
        out.append((J, 7, None))
    return out


def _log(**kw):
    import json
    print(json.dumps(kw), flush=True)


def make_dataset(n, path, sizes=(8, 10, 12, 15), seed0=30000, seed=4242, chunk=250, params=None,
                 p_max=0.0):
    """Adaptive ladders for instances seed0 .. seed0+n-1 (size sizes[i mod 4], dilution up to
    p_max), one batch of up to `chunk` same-size instances per call, a progress line per batch."""
    import time
    prm = dict(ADAPTIVE if params is None else params)
    X = np.zeros((n, 4))
    Y = np.zeros((n, N_RUNGS + 1))
    lad = np.zeros((n, prm["max_steps"]))
    sig = np.zeros((n, prm["max_steps"]))
    lens = np.zeros(n, np.int32)
    total = 0.0
    for L in sizes:
        idx = [i for i in range(n) if sizes[i % len(sizes)] == L]
        for k in range(0, len(idx), chunk):
            part = idx[k:k + chunk]
            inst = _instances(part, sizes, seed0, p_max)
            t0 = time.perf_counter()
            res = sg.adaptive_ladder(inst, seed + part[0], **prm)
            dt = time.perf_counter() - t0
            total += dt
            X[part] = features(inst)
            for j, (b, s) in zip(part, res):
                lens[j] = len(b)
                lad[j, :len(b)] = b
                sig[j, :len(s)] = s
                Y[j] = targets(b)
            flips = sum(L ** 3 * prm["n_chains"] * prm["sweeps"] * int(lens[j]) for j in part)
            _log(L=L, done=k + len(part), of=len(idx), seconds=round(dt, 2),
                 flips_per_ns=round(flips / dt / 1e9, 1),
                 rungs=[int(lens[part].min()), int(lens[part].max())])
    np.savez(path, X=X, Y=Y, ladders=lad, sigmas=sig, lens=lens, seconds=total,
             sizes=np.array(sizes), seed0=seed0, p_max=p_max,
             params=np.array([prm[k] for k in sorted(prm)]))
    return total, lens


def calibrate_bands(data, per_size=128, pilot=1000, seed=555, factor=(0.5, 1.5), q=(0.005, 0.995),
                    widen=(0.9, 1.1)):
    """Per-size, per-pair acceptance bands from the adaptive stage's own ladders (training data
    sets, the Algorithm S2 settings): per_size instances of each size, split over the data
    sets, run a pilot on their adaptive ladders (resampled to 32 rungs, each at its own cutoff
    label); per pair the band is [min(0.5 c, 0.9 q_0.5%), max(1.5 c, 1.1 q_99.5%)] with c the
    mean acceptance, so that the stage's own ladders pass it and a predicted ladder is checked
    on every pair."""
    sizes = tuple(int(x) for x in data[0]["sizes"])
    out = {"sizes": np.array(sizes), "band_lo": [], "band_hi": [], "pass": [], "mean": []}
    for L in sizes:
        inst, lad = [], []
        for d in data:
            p_max = float(d["p_max"]) if "p_max" in d else 0.0
            idx = [i for i in range(d["lens"].size) if sizes[i % len(sizes)] == L][:per_size // len(data)]
            inst += _instances(idx, sizes, int(d["seed0"]), p_max)
            lad += [resample(d["ladders"][i, :d["lens"][i]]) for i in idx]
        lad = np.stack(lad)
        cut = np.array([cutoff_label(x) for x in lad])
        acc = pilot_acceptance(inst, lad, seed, pilot, cut)
        c = acc.mean(axis=0)
        lo = np.minimum(factor[0] * c, widen[0] * np.quantile(acc, q[0], axis=0))
        hi = np.maximum(factor[1] * c, widen[1] * np.quantile(acc, q[1], axis=0))
        out["band_lo"].append(lo)
        out["band_hi"].append(hi)
        out["pass"].append(float(in_band(acc, lo, hi).mean()))
        out["mean"].append(c)
    for k in ("band_lo", "band_hi", "mean"):
        out[k] = np.stack(out[k])
    return out


def _first_hit(tr, target):
    hit = tr <= target[:, None]
    return np.where(hit.any(axis=1), hit.argmax(axis=1) + 1, -1)


def mean_rho_cycles(tr, E0, nspins, rho0):
    """First cycle (1-based) at which the residual energy per spin averaged over the instances
    (Eq. 2: the mean over instances of (E_best(t) - E0) / n) is at most rho0, or -1.  tr is the
    per-cycle running best energy [n_inst][cycles]."""
    rho = ((np.asarray(tr, np.float64) - np.asarray(E0, np.float64)[:, None])
           / np.asarray(nspins, np.float64).reshape(-1, 1)).mean(axis=0)
    hit = np.flatnonzero(rho <= rho0)
    return int(hit[0]) + 1 if hit.size else -1


def _batched(inst, lad, cut, seed, cycles):
    """One batched APT+ICM run with per-cycle best-energy traces: (trace, ms per cycle, pair
    acceptance)."""
    c = sg.apt(inst, lad, seed, 2)
    c.synchronize()
    c.timer_start()
    tr = c.run_apt_ex(cycles, 1, cut, 2, record_every=1)
    ms = c.timer_stop()
    acc = acceptance(c.swap_counts(), cycles, N_RUNGS, 2)
    c.close()
    return tr, ms / cycles, acc


def evaluate(params, tables, n=256, seed0=90000, L=15, p_max=0.0, cycles=20000, pilot=1000, seed=777,
             rho0=0.007, e0_cycles=20000, plain_sample=16, repair_rounds=REPAIR_ROUNDS):
    """Plain, batched-adaptive, batched-learned and batched-lookup-table APT+ICM on held-out
    instances (size L, dilution up to p_max).  Each form's time to target counts its ladder
    construction: the adaptive stage on all instances at once; the learned flow (inference,
    pilot, band check, repair rounds, adaptive fallback); the table lookup alone (nothing to
    time) and the table lookup through the same judge as the learned flow.  Every form runs
    each instance at its own ICM cutoff.  Plain: one instance at a time, its own adaptive stage
    and APT run, on the first plain_sample instances, scaled to n.  Also the ladders' rms
    distance in log beta from the adaptive stage's.  Two targets: the residual energy per spin
    averaged over the instances reaching rho0 (Eq. 2, the paper's criterion: cycles_mean_rho,
    total_s_mean_rho), and every instance within rho0 n of its E0 (cycles_all, total_s)."""
    import time
    inst = _instances(range(n), (L,), seed0, p_max)
    nsp = L ** 3
    t0 = time.perf_counter()
    res = adaptive_ladders(inst, seed, **ADAPTIVE)
    t_adapt = time.perf_counter() - t0
    lad_a = np.stack([resample(r[0]) for r in res])
    cut_a = np.array([cutoff_label(x) for x in lad_a])
    t0 = time.perf_counter()
    lad_l, cut_l, st_l, acc_pilot = learned_ladders(inst, seed + 9, params, pilot, tables, repair_rounds)
    t_learn = time.perf_counter() - t0
    lad_t, cut_t = table_ladders(inst, tables) if tables is not None else (None, None)
    forms = {"adaptive": (lad_a, cut_a, t_adapt), "learned": (lad_l, cut_l, t_learn)}
    st_t = None
    if lad_t is not None:
        forms["table"] = (lad_t, cut_t, 0.0)
        # the lookup ladders through the same judge: pilot, per-pair band, repair, fallback
        t0 = time.perf_counter()
        lad_tj, cut_tj, st_t, _ = judge_ladders(inst, lad_t, cut_t, seed + 9, pilot, tables,
                                                repair_rounds)
        forms["table_judged"] = (lad_tj, cut_tj, time.perf_counter() - t0)
    E0 = np.full(n, np.iinfo(np.int64).max)
    for sd in (11, 12):
        c = sg.apt(inst, lad_a, sd, 2)
        c.run_apt_ex(e0_cycles, 1, cut_a, 2)
        E0 = np.minimum(E0, c.best())
        c.close()
    runs = {}
    for name, (lad, cut, _) in forms.items():
        runs[name] = _batched(inst, lad, cut, seed + 3, cycles)
        E0 = np.minimum(E0, runs[name][0][:, -1])
    plain = []
    for i in range(min(plain_sample, n)):
        t0 = time.perf_counter()
        r = sg.adaptive_ladder([inst[i]], seed + 5 + i, **ADAPTIVE)
        t_ad = time.perf_counter() - t0
        l32 = resample(r[0][0])
        ci = sg.apt([inst[i]], l32[None, :], seed + 1000 + i, 2)
        target = E0[i] + rho0 * nsp
        done, hit = 0, -1
        ci.synchronize()
        ci.timer_start()
        while done < cycles:
            tr_i = ci.run_apt_ex(250, 1, cutoff_label(l32), 2, record_every=1)[0]
            done += 250
            if tr_i[-1] <= target:
                hit = done - 250 + int(np.argmax(tr_i <= target)) + 1
                break
        ms = ci.timer_stop()
        ci.close()
        # charged for the cycles up to the target at the measured cost per cycle
        per = ms / 1e3 / done
        plain.append((t_ad, per * (hit if hit > 0 else done), per))
    target = E0 + rho0 * nsp
    out = {"n": n, "L": L, "p_max": p_max, "rho0": rho0, "pilot_cycles": pilot, "cycles_max": cycles,
           "adaptive_params": ADAPTIVE, "repair_rounds": repair_rounds,
           "learned_fallbacks": int((st_l == ADAPTIVE_FALLBACK).sum()),
           "learned_repaired": int((st_l == REPAIRED).sum()),
           "table_judged_fallbacks": None if st_t is None else int((st_t == ADAPTIVE_FALLBACK).sum()),
           "table_judged_repaired": None if st_t is None else int((st_t == REPAIRED).sum()),
           "e0": f"min over two {e0_cycles}-cycle runs on the adaptive ladders and every run here"}
    for name, (lad, cut, t_build) in forms.items():
        tr, mspc, acc = runs[name]
        first = _first_hit(tr, target)
        reached = int((first > 0).sum())
        apt_s = first.max() * mspc / 1e3 if reached == n else None
        cm = mean_rho_cycles(tr, E0, nsp, rho0)
        out[name] = {"ladder_s": round(t_build, 3),
                     "cycles_mean_rho": cm if cm > 0 else None,
                     "total_s_mean_rho": round(t_build + cm * mspc / 1e3, 3) if cm > 0 else None,
                     "reached": reached,
                     "cycles_all": int(first.max()) if reached == n else None,
                     "apt_s": None if apt_s is None else round(apt_s, 3),
                     "total_s": None if apt_s is None else round(t_build + apt_s, 3),
                     "cycles_median": float(np.median(first[first > 0])) if reached else None,
                     "acc_mean": round(float(acc.mean()), 4),
                     "acc_spread": round(float(acc.std(axis=1).mean()), 4),
                     "rms_log_beta_vs_adaptive": round(float(np.sqrt(np.mean((np.log(lad) - np.log(lad_a)) ** 2))), 4)}
    pl = np.array(plain)
    if pl.size:
        out["plain_sample"] = {"instances": len(plain),
                               "ladder_s_mean": round(float(pl[:, 0].mean()), 3),
                               "apt_s_mean": round(float(pl[:, 1].mean()), 4),
                               "total_s_scaled_to_n": round(float(pl[:, :2].sum(axis=1).mean() * n), 2)}
        cm = out["adaptive"]["cycles_mean_rho"]
        if cm is not None:
            # every instance alone for as many cycles as the batched adaptive form needed
            out["plain_sample"]["total_s_mean_rho_scaled_to_n"] = round(
                float((pl[:, 0] + cm * pl[:, 2]).mean() * n), 2)
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned-ladder study")
    ap.add_argument("stage", choices=["data", "train", "eval"])
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--data", nargs="+", default=[])
    ap.add_argument("--out", default=None)
    ap.add_argument("--params", default=None)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lrs", type=float, nargs="+", default=[3e-4],
                    help="learning rates, the epochs split evenly over them")
    ap.add_argument("--seed0", type=int, default=None,
                    help="first instance seed (default 30000 for data, 90000 for eval)")
    ap.add_argument("--cycles", type=int, default=20000)
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--p-max", type=float, default=0.0,
                    help="largest fraction of absent bonds of the generated instances")
    ap.add_argument("--budget", choices=["paper", "small"], default="paper",
                    help="adaptive-stage budget: the paper's, or 8 chains x 500 sweeps (tests)")
    a = ap.parse_args()
    if a.budget == "small":
        ADAPTIVE.update(n_chains=8, sweeps=500, tail=250)
    if a.stage == "data":
        dt, lens = make_dataset(a.n, a.out, seed0=30000 if a.seed0 is None else a.seed0, p_max=a.p_max)
        _log(seconds=round(dt, 2), n=a.n, rungs_min=int(lens.min()), rungs_max=int(lens.max()),
             rungs_mean=float(lens.mean()))
    elif a.stage == "train":
        data = [np.load(f) for f in a.data]
        X = np.concatenate([d["X"] for d in data])
        Y = np.concatenate([d["Y"] for d in data])
        d = data[0]
        perm = np.random.default_rng(0).permutation(X.shape[0])
        nval = max(1, X.shape[0] // 10)
        va, trn = perm[:nval], perm[nval:]
        import time
        t0 = time.perf_counter()
        m, losses = fit(X[trn], Y[trn], epochs=a.epochs, lrs=tuple(a.lrs))
        t_train = time.perf_counter() - t0
        sizes = tuple(int(x) for x in d["sizes"])
        size_of = np.concatenate([[sizes[i % len(sizes)] for i in range(dd["X"].shape[0])] for dd in data])
        size_mean = np.stack([Y[trn][size_of[trn] == L].mean(axis=0) for L in sizes])
        per = size_mean[np.searchsorted(np.array(sizes), size_of[va])]
        cal = calibrate_bands(data)
        np.savez(a.out, params=m.params(), sizes=np.array(sizes), band_lo=cal["band_lo"],
                 band_hi=cal["band_hi"], size_mean=size_mean)
        _log(train_seconds=round(t_train, 2), train_loss_first=float(losses[0]),
             train_loss_last=float(losses[-1]), val_loss=float(m.loss(X[va], Y[va])),
             val_loss_size_mean=float(np.mean((Y[va] - per) ** 2)),
             val_loss_global_mean=float(np.mean((Y[va] - Y[trn].mean(axis=0)) ** 2)),
             n_train=int(trn.size), n_val=int(va.size), band_pass_by_size=cal["pass"],
             band_lo_coldest=np.round(cal["band_lo"][:, -3:], 3).tolist(),
             band_hi_coldest=np.round(cal["band_hi"][:, -3:], 3).tolist(),
             acc_mean_by_size=np.round(cal["mean"], 3).tolist())
    else:
        p = np.load(a.params)
        tables = {k: p[k] for k in ("sizes", "band_lo", "band_hi", "size_mean")} if "sizes" in p else None
        print(json.dumps(evaluate(p["params"], tables, n=a.n, cycles=a.cycles, e0_cycles=a.cycles,
                                  plain_sample=a.plain_sample, p_max=a.p_max,
                                  seed0=90000 if a.seed0 is None else a.seed0)), flush=True)
