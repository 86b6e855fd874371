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
# The coldest two adjacent pairs are left out of the band check: the paper reports roughly
# constant acceptance except for the last few replicas, and with two pairs exempt every
# ladder of the adaptive stage itself passed (100 of 100 held-apart L=15 instances; with
# none exempt, 16 of 100).
TAIL_EXEMPT = 2
ALPHA = 1.25
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
    """Swap acceptance of every adjacent pair over a pilot APT+ICM run (per instance)."""
    lad = np.ascontiguousarray(ladders, np.float64)
    ctx = sg.apt(instances, lad, seed, reps_per_beta=reps)
    ctx.run_apt(cycles, 1, float(cutoff))
    acc = acceptance(ctx.swap_counts(), cycles, lad.shape[1], reps)
    ctx.close()
    return acc


def in_band(acc, band=BAND, skip_last=None):
    """Band check: every adjacent pair except the last `skip_last` (coldest) ones."""
    k = TAIL_EXEMPT if skip_last is None else int(skip_last)
    a = np.asarray(acc)
    a = a[:, :a.shape[1] - k] if k > 0 else a
    return np.all((a >= band[0]) & (a <= band[1]), axis=1)


_PARAMS = __import__("os").path.join(__import__("os").path.dirname(__file__), "ladder_mlp.npz")


def default_params():
    """The shipped network: trained on adaptive-stage ladders of 10^4 generated +-1 cubic
    instances (L in {8, 10, 12, 15}, the stage at the Methods settings), 400 epochs."""
    return np.load(_PARAMS)["params"]


def learned_ladders(instances, seed, params=None, pilot=1000, cutoff=None):
    """The learned-ladder flow: predicted ladders, a pilot APT+ICM run, the band check, and the
    adaptive stage for every instance whose ladder fails it.

    Returns (ladders [n][32], fell_back [n] bool, pilot acceptance [n][31])."""
    m = Predictor(default_params() if params is None else params)
    lad, cut = m.predict(instances)
    m.close()
    cut_run = float(np.median(cut)) if cutoff is None else float(cutoff)
    acc = pilot_acceptance(instances, lad, seed, pilot, cut_run)
    ok = in_band(acc)
    bad = np.flatnonzero(~ok)
    if bad.size:
        fb = adaptive_ladders([instances[i] for i in bad], seed + 1, **ADAPTIVE)
        for i, r in zip(bad, fb):
            lad[i] = resample(r[0])
    return lad, ~ok, acc


# ----------------------------------------------------------------------------------------
# Study driver: training data from the adaptive stage, training, held-out evaluation.
# ----------------------------------------------------------------------------------------
# The adaptive stage at the settings of the Methods section (APT details): beta0 = 0.5,
# alpha = 1.25, 100 chains, variance over the last 1000 of 10000 sweeps, stop once the
# mean standard deviation falls below min|J| / 2.
ADAPTIVE = dict(beta0=0.5, alpha=ALPHA, tol=0.5, n_chains=100, sweeps=10000, tail=1000, max_steps=64)
ICM_CUTOFF = 1.0


def _instances(idx, sizes, seed0):
    from .inputs import ej_couplings
    return [(ej_couplings(sizes[i % len(sizes)], 7, seed=seed0 + i)[0], 7, None) for i in idx]


def _log(**kw):
    import json
    print(json.dumps(kw), flush=True)


def make_dataset(n, path, sizes=(8, 10, 12, 15), seed0=30000, seed=4242, chunk=250, params=None):
    """Adaptive ladders for instances seed0 .. seed0+n-1 (size sizes[i mod 4]), one batch of
    up to `chunk` same-size instances per call, a progress line per batch."""
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
            inst = _instances(part, sizes, seed0)
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
             sizes=np.array(sizes), seed0=seed0, params=np.array([prm[k] for k in sorted(prm)]))
    return total, lens


def band_calibration(data_path, L=15, n=256, pilot=1000, seed=555):
    """Pilot acceptance of the adaptive stage's own ladders on training instances: how
    many of them pass the band with the last k pairs exempt, for k = 0..8."""
    d = np.load(data_path)
    sizes = tuple(int(x) for x in d["sizes"])
    idx = [i for i in range(d["lens"].size) if sizes[i % len(sizes)] == L][:n]
    inst = _instances(idx, sizes, int(d["seed0"]))
    lad = np.stack([resample(d["ladders"][i, :d["lens"][i]]) for i in idx])
    acc = pilot_acceptance(inst, lad, seed, pilot, ICM_CUTOFF)
    return {"pass_by_k": {k: int(in_band(acc, skip_last=k).sum()) for k in range(9)},
            "n": len(idx), "acc_mean_by_pair": np.round(acc.mean(axis=0), 3).tolist(),
            "acc_p05_by_pair": np.round(np.quantile(acc, 0.05, axis=0), 3).tolist(),
            "acc_p95_by_pair": np.round(np.quantile(acc, 0.95, axis=0), 3).tolist()}


def _first_hit(tr, target):
    hit = tr <= target[:, None]
    return np.where(hit.any(axis=1), hit.argmax(axis=1) + 1, -1)


def evaluate(params, n=256, seed0=90000, L=15, cycles=20000, pilot=1000, seed=777, rho0=0.007,
             e0_cycles=20000, plain_sample=16):
    """Plain, batched-adaptive and batched-learned APT+ICM on held-out instances.

    Each form's time to target counts its ladder construction.  Adaptive: the adaptive
    stage on all instances at once.  Learned: inference, then the production run whose
    first `pilot` cycles are the pilot; instances outside the band get the adaptive stage
    and a production run of their own.  Plain: one instance at a time, its own adaptive
    stage and APT run, on the first `plain_sample` instances (scaled to n).
    """
    import time
    inst = _instances(range(n), (L,), seed0)
    nsp = L ** 3
    reps = 2
    # ---- adaptive form: ladder construction
    t0 = time.perf_counter()
    res = adaptive_ladders(inst, seed, **ADAPTIVE)
    t_adapt = time.perf_counter() - t0
    lens_a = np.array([len(r[0]) for r in res])
    lad_a = np.stack([resample(r[0]) for r in res])
    # ---- learned form: inference
    m = Predictor(params)
    t0 = time.perf_counter()
    lad_l, cut_l = m.predict(inst)
    t_pred = time.perf_counter() - t0
    m.close()
    cut_learned = float(np.median(cut_l))
    # ---- E0: long runs on the adaptive ladders (putative ground energies)
    E0 = np.full(n, np.iinfo(np.int64).max)
    for sd in (11, 12):
        c = sg.apt(inst, lad_a, sd, reps)
        c.run_apt(e0_cycles, 1, ICM_CUTOFF)
        E0 = np.minimum(E0, c.best())
        c.close()
    # ---- batched runs with per-cycle traces
    c = sg.apt(inst, lad_a, seed + 3, reps)
    c.synchronize()
    c.timer_start()
    tr_a = c.run_apt(cycles, 1, ICM_CUTOFF, record_every=1)
    ms_a = c.timer_stop()
    acc_a = acceptance(c.swap_counts(), cycles, N_RUNGS, reps)
    c.close()
    c = sg.apt(inst, lad_l, seed + 3, reps)
    c.synchronize()
    c.timer_start()
    tr_l1 = c.run_apt(pilot, 1, cut_learned, record_every=1)
    ms_l1 = c.timer_stop()
    acc_l = acceptance(c.swap_counts(), pilot, N_RUNGS, reps)
    ok = in_band(acc_l)
    c.timer_start()
    tr_l2 = c.run_apt(cycles - pilot, 1, cut_learned, record_every=1)
    ms_l2 = c.timer_stop()
    acc_l_full = acceptance(c.swap_counts(), cycles, N_RUNGS, reps)
    c.close()
    tr_l = np.concatenate([tr_l1, tr_l2], axis=1)
    bad = np.flatnonzero(~ok)
    t_fb, ms_fb, tr_fb = 0.0, 0.0, None
    if bad.size:
        sub = [inst[i] for i in bad]
        t0 = time.perf_counter()
        fb = adaptive_ladders(sub, seed + 2, **ADAPTIVE)
        t_fb = time.perf_counter() - t0
        lad_fb = np.stack([resample(r[0]) for r in fb])
        c = sg.apt(sub, lad_fb, seed + 4, reps)
        c.synchronize()
        c.timer_start()
        tr_fb = c.run_apt(cycles, 1, ICM_CUTOFF, record_every=1)
        ms_fb = c.timer_stop()
        c.close()
    E0 = np.minimum(E0, np.minimum(tr_a[:, -1], tr_l[:, -1]))
    if bad.size:
        E0[bad] = np.minimum(E0[bad], tr_fb[:, -1])
    # ---- plain form on a sample, after E0 is fixed
    plain = []
    for i in range(min(plain_sample, n)):
        t0 = time.perf_counter()
        r = sg.adaptive_ladder([inst[i]], seed + 5 + i, **ADAPTIVE)
        t_ad = time.perf_counter() - t0
        ci = sg.apt([inst[i]], resample(r[0][0])[None, :], seed + 1000 + i, reps)
        target = E0[i] + rho0 * nsp
        done, hit = 0, -1
        ci.synchronize()
        ci.timer_start()
        while done < cycles:
            ci.run_apt(250, 1, ICM_CUTOFF)
            done += 250
            if int(ci.best()[0]) <= target:
                hit = done
                break
        ms = ci.timer_stop()
        ci.close()
        plain.append((t_ad, ms / 1e3, hit))
    target = E0 + rho0 * nsp
    first_a = _first_hit(tr_a, target)
    first_l = _first_hit(tr_l, target)
    mspc_a = ms_a / cycles
    mspc_l = (ms_l1 + ms_l2) / cycles
    out = {"n": n, "L": L, "rho0": rho0, "pilot_cycles": pilot, "cycles_max": cycles,
           "band": [round(BAND[0], 4), round(BAND[1], 4)], "tail_exempt": TAIL_EXEMPT,
           "adaptive_params": ADAPTIVE, "adaptive_rungs": [int(lens_a.min()), int(lens_a.max())]}
    reached_a = int((first_a > 0).sum())
    apt_a = first_a.max() * mspc_a / 1e3 if reached_a == n else None
    out["adaptive"] = {
        "ladder_s": round(t_adapt, 3), "reached": reached_a,
        "cycles_all": int(first_a.max()) if reached_a == n else None,
        "apt_s": None if apt_a is None else round(apt_a, 3),
        "total_s": None if apt_a is None else round(t_adapt + apt_a, 3),
        "cycles_median": float(np.median(first_a[first_a > 0])) if reached_a else None,
        "acc_mean": round(float(acc_a.mean()), 4),
        "acc_spread": round(float(acc_a[:, :N_RUNGS - 1 - TAIL_EXEMPT].std(axis=1).mean()), 4),
        "acc_mean_by_pair": np.round(acc_a.mean(axis=0), 3).tolist(),
        "in_band": int(in_band(acc_a).sum())}
    # learned: accepted instances need max(pilot, their cycles); the rest their fallback
    acc_ok = ok.copy()
    fl = np.where(acc_ok, first_l, -1)
    reached_ok = int((fl > 0).sum())
    need_a = int(max(pilot, fl[acc_ok].max())) if acc_ok.any() and reached_ok == acc_ok.sum() else None
    if bad.size:
        first_fb = _first_hit(tr_fb, target[bad])
        fb_ok = bool((first_fb > 0).all())
        t_fb_apt = first_fb.max() * ms_fb / cycles / 1e3 if fb_ok else None
    else:
        first_fb, fb_ok, t_fb_apt = np.zeros(0, int), True, 0.0
    total_l = None
    if (need_a is not None or not acc_ok.any()) and fb_ok:
        t_ctx = (need_a or pilot) * mspc_l / 1e3
        total_l = t_pred + t_ctx + t_fb + t_fb_apt
    out["learned"] = {
        "inference_s": round(t_pred, 4), "accepted": int(acc_ok.sum()), "fallbacks": int(bad.size),
        "fallback_ladder_s": round(t_fb, 3), "cutoff": round(cut_learned, 4),
        "reached": reached_ok + int((first_fb > 0).sum()),
        "cycles_all_accepted": need_a,
        "total_s": None if total_l is None else round(total_l, 3),
        "cycles_median": float(np.median(first_l[first_l > 0])) if (first_l > 0).any() else None,
        "acc_mean": round(float(acc_l_full.mean()), 4),
        "acc_spread": round(float(acc_l_full[:, :N_RUNGS - 1 - TAIL_EXEMPT].std(axis=1).mean()), 4),
        "acc_mean_by_pair": np.round(acc_l_full.mean(axis=0), 3).tolist(),
        "pilot_pass_by_k": {k: int(in_band(acc_l, skip_last=k).sum()) for k in range(9)},
        "ladder_rms_log_diff": round(float(np.sqrt(np.mean((np.log(lad_l) - np.log(lad_a)) ** 2))), 4)}
    pl = np.array(plain)
    if pl.size:
        reached_p = int((pl[:, 2] > 0).sum())
        out["plain_sample"] = {
            "instances": len(plain), "reached": reached_p,
            "ladder_s_mean": round(float(pl[:, 0].mean()), 3),
            "apt_s_mean": round(float(pl[:, 1].mean()), 4),
            "total_s_scaled_to_n": round(float((pl[:, 0] + pl[:, 1]).mean() * n), 2)}
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned-ladder study")
    ap.add_argument("stage", choices=["data", "calibrate", "train", "eval"])
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--data", nargs="+", default=[])
    ap.add_argument("--out", default=None)
    ap.add_argument("--params", default=None)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--seed0", type=int, default=30000)
    ap.add_argument("--cycles", type=int, default=20000)
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--budget", choices=["paper", "small"], default="paper",
                    help="adaptive-stage budget: the paper's, or 8 chains x 500 sweeps (tests)")
    a = ap.parse_args()
    if a.budget == "small":
        ADAPTIVE.update(n_chains=8, sweeps=500, tail=250)
    if a.stage == "data":
        dt, lens = make_dataset(a.n, a.out, seed0=a.seed0)
        _log(seconds=round(dt, 2), n=a.n, rungs_min=int(lens.min()), rungs_max=int(lens.max()),
             rungs_mean=float(lens.mean()))
    elif a.stage == "calibrate":
        print(json.dumps(band_calibration(a.data[0])), flush=True)
    elif a.stage == "train":
        X = np.concatenate([np.load(p)["X"] for p in a.data])
        Y = np.concatenate([np.load(p)["Y"] for p in a.data])
        perm = np.random.default_rng(0).permutation(X.shape[0])
        nval = max(1, X.shape[0] // 10)
        va, trn = perm[:nval], perm[nval:]
        import time
        t0 = time.perf_counter()
        m, losses = fit(X[trn], Y[trn], epochs=a.epochs)
        t_train = time.perf_counter() - t0
        np.savez(a.out, params=m.params())
        # baselines: the global mean ladder, and the mean ladder of the instance's size
        glob = np.mean((Y[va] - Y[trn].mean(axis=0)) ** 2)
        size_of = np.round(X[:, 0]).astype(int)   # feature 0 is the cube root of n
        per = np.zeros_like(Y[va])
        for k, i in enumerate(va):
            same = trn[size_of[trn] == size_of[i]]
            per[k] = Y[same].mean(axis=0)
        _log(train_seconds=round(t_train, 2), train_loss_first=float(losses[0]),
             train_loss_last=float(losses[-1]), val_loss=float(m.loss(X[va], Y[va])),
             val_loss_global_mean=float(glob), val_loss_size_mean=float(np.mean((Y[va] - per) ** 2)),
             n_train=int(trn.size), n_val=int(va.size))
    else:
        p = np.load(a.params)["params"]
        print(json.dumps(evaluate(p, n=a.n, cycles=a.cycles, e0_cycles=a.cycles,
                                  plain_sample=a.plain_sample)), flush=True)
