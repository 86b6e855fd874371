"""ctypes binding of libsg (include/sg.h): argument marshalling only.

Every step of the Monte Carlo path runs in the HIP kernels of libsg.so; this
module converts numpy arrays to pointers and status codes to exceptions.  It
raises if the library is not built or cannot initialise a GPU -- there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_PKG, "libsg.so")

SG_OK, SG_EINVAL, SG_ENOMEM, SG_EHIP, SG_ESTATE, SG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SG_APT, SG_SQA = 1, 2
MLP_NPARAM = 6625
PREDICT_NOALLOC_MAX = 4096
_NAMES = {SG_EINVAL: "SG_EINVAL", SG_ENOMEM: "SG_ENOMEM", SG_EHIP: "SG_EHIP",
          SG_ESTATE: "SG_ESTATE", SG_EUNSUPPORTED: "SG_EUNSUPPORTED"}


class SGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Lattice(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("Lz", C.c_int32),
                ("periodic", C.c_uint32), ("J", C.c_void_p), ("h", C.c_void_p)]


class _Config(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_inst", C.c_int32), ("inst", C.POINTER(_Lattice)),
                ("n_beta", C.c_int32), ("beta", C.c_void_p), ("reps_per_beta", C.c_int32),
                ("M", C.c_int32), ("R", C.c_int32), ("sqa_beta", C.c_double),
                ("seed", C.c_uint64), ("hip_stream", C.c_void_p)]


class _AptOptions(C.Structure):
    _fields_ = [("sweeps_per_swap", C.c_int32), ("icm_pairs", C.c_int32), ("icm_cutoff", C.c_double),
                ("icm_cutoff_per_inst", C.c_void_p), ("record_every", C.c_int32)]


class _Adaptive(C.Structure):
    _fields_ = [("beta0", C.c_double), ("alpha", C.c_double), ("tol", C.c_double),
                ("n_chains", C.c_int32), ("sweeps", C.c_int32), ("tail", C.c_int32),
                ("max_steps", C.c_int32)]


EXPORTS = [
    "sg_create", "sg_create_ex", "sg_dsatur_colouring", "sg_destroy", "sg_last_error", "sg_sweep", "sg_icm", "sg_energy", "sg_swap",
    "sg_run_apt", "sg_run_apt_ex", "sg_icm_ex", "sg_best", "sg_swap_counts", "sg_sqa_anneal", "sg_sqa_trotter_agreement", "sg_get_launch_config",
    "sg_set_launch_config", "sg_get_spins", "sg_get_spins_range", "sg_set_spins",
    "sg_get_counters", "sg_get_state", "sg_set_state", "sg_timer_start", "sg_timer_stop",
    "sg_synchronize", "sg_kernel_timing", "sg_kernel_time", "sg_adaptive_ladder", "sg_mlp_create", "sg_mlp_destroy",
    "sg_instance_features", "sg_mlp_set_standardisation", "sg_mlp_loss_grad", "sg_mlp_train",
    "sg_mlp_get_params", "sg_ladder_predict", "sg_learned_ladders", "sg_ladder_predict_noalloc",
    "sg_ladder_repair", "sg_judge_ladders", "sg_energy_dev", "sg_get_spins_dev", "sg_best_dev",
    "sg_sqa_anneal_dev", "sg_threshold_heat_bath", "sg_threshold_sqa", "sg_threshold_swap",
]

_lib = None


def load():
    """Load libsg.so (built by __graft_entry__.build() or paper_2503_10302_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise RuntimeError(f"{SO_PATH} is missing: build the HIP library first")
    L = C.CDLL(SO_PATH)
    P, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "sg_create": (i32, [C.POINTER(_Config), C.POINTER(P)]),
        "sg_create_ex": (i32, [C.POINTER(_Config), P, C.POINTER(P)]),
        "sg_dsatur_colouring": (i32, [C.POINTER(_Lattice), P, C.POINTER(i32)]),
        "sg_destroy": (None, [P]),
        "sg_last_error": (C.c_char_p, [P]),
        "sg_sweep": (i32, [P, i32]),
        "sg_icm": (i32, [P, dbl, P]),
        "sg_energy": (i32, [P, P]),
        "sg_swap": (i32, [P, P]),
        "sg_run_apt": (i32, [P, i64, i32, dbl, i32, P]),
        "sg_run_apt_ex": (i32, [P, i64, C.POINTER(_AptOptions), P]),
        "sg_icm_ex": (i32, [P, C.POINTER(_AptOptions), P]),
        "sg_best": (i32, [P, P]),
        "sg_swap_counts": (i32, [P, P]),
        "sg_sqa_anneal": (i32, [P, P, i32, P, P]),
        "sg_sqa_trotter_agreement": (i32, [P, P]),
        "sg_get_launch_config": (i32, [P, P]),
        "sg_set_launch_config": (i32, [P, i32]),
        "sg_get_spins": (i32, [P, P]),
        "sg_get_spins_range": (i32, [P, i32, i32, i32, P]),
        "sg_set_spins": (i32, [P, P]),
        "sg_get_counters": (i32, [P, P]),
        "sg_get_state": (i32, [P, P, C.POINTER(C.c_size_t)]),
        "sg_set_state": (i32, [P, P, C.c_size_t]),
        "sg_timer_start": (i32, [P]),
        "sg_timer_stop": (i32, [P, C.POINTER(C.c_float)]),
        "sg_synchronize": (i32, [P]),
        "sg_kernel_timing": (i32, [P, i32]),
        "sg_kernel_time": (i32, [P, C.POINTER(C.c_float), C.POINTER(i32)]),
        "sg_adaptive_ladder": (i32, [C.POINTER(_Lattice), i32, C.POINTER(_Adaptive), u64, P, P, P, P]),
        "sg_mlp_create": (i32, [P, u64, P, C.POINTER(P)]),
        "sg_mlp_destroy": (None, [P]),
        "sg_instance_features": (i32, [C.POINTER(_Lattice), i32, P]),
        "sg_mlp_set_standardisation": (i32, [P, P, P]),
        "sg_mlp_loss_grad": (i32, [P, P, P, i32, P, P]),
        "sg_mlp_train": (i32, [P, P, P, i32, i32, i32, C.c_float, P]),
        "sg_mlp_get_params": (i32, [P, P]),
        "sg_ladder_predict": (i32, [P, C.POINTER(_Lattice), i32, P, P]),
        "sg_ladder_predict_noalloc": (i32, [P, C.POINTER(_Lattice), i32, P, P]),
        "sg_learned_ladders": (i32, [P, C.POINTER(_Lattice), i32, P, P, C.POINTER(_Adaptive), i32, i32,
                                     u64, P, P, P, P]),
        "sg_judge_ladders": (i32, [C.POINTER(_Lattice), i32, P, P, C.POINTER(_Adaptive), i32, i32, u64,
                                   P, P, P, P]),
        "sg_ladder_repair": (i32, [P, P, P, P, i32, C.c_double, P]),
        "sg_energy_dev": (i32, [P, P]),
        "sg_get_spins_dev": (i32, [P, P]),
        "sg_best_dev": (i32, [P, P]),
        "sg_sqa_anneal_dev": (i32, [P, P, i32, P, P]),
        "sg_threshold_heat_bath": (i32, [C.c_double, i32, P]),
        "sg_threshold_sqa": (i32, [C.c_double, i32, C.c_double, i32, i32, P]),
        "sg_threshold_swap": (i32, [C.c_double, C.c_double, C.c_int64, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dev(x):
    """A device address for the device-output calls: None, an int, or an object with
    data_ptr() (a framework tensor); the library checks that it is device memory."""
    if x is None:
        return None
    return C.c_void_p(int(x.data_ptr()) if hasattr(x, "data_ptr") else int(x))


def _lattices(instances):
    """instances: list of (J[Lz,Ly,Lx,3] int8, periodic, h or None)."""
    keep = []
    arr = (_Lattice * len(instances))()
    for i, inst in enumerate(instances):
        J, periodic, h = (tuple(inst) + (None,))[:3] if len(inst) < 3 else inst
        J = np.ascontiguousarray(J, dtype=np.int8)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.int8).reshape(-1)
        keep += [J, hh]
        Lz, Ly, Lx = J.shape[:3]
        arr[i] = _Lattice(Lx, Ly, Lz, int(periodic), J.ctypes.data,
                          None if hh is None else hh.ctypes.data)
    return arr, keep


class Context:
    """One libsg context (APT or DT-SQA) over a batch of instances."""

    def __init__(self, instances, mode, seed, beta=None, reps_per_beta=2, M=0, R=0, sqa_beta=0.0,
                 colours=None):
        """colours: optional list of per-instance colour maps ([n] int8 or None)."""
        self.lib = load()
        self._arr, self._keep = _lattices(instances)
        self.n_inst = len(instances)
        self.ns = [int(np.prod(np.asarray(inst[0]).shape[:3])) for inst in instances]
        self.n_max = max(self.ns)
        self.mode = mode
        bt = None
        if mode == SG_APT:
            bt = np.ascontiguousarray(beta, dtype=np.float64)
            if bt.ndim == 1:
                bt = np.ascontiguousarray(np.broadcast_to(bt, (self.n_inst, bt.size)))
            self.n_beta = bt.shape[1]
            self.reps = reps_per_beta
            self.n_slots = self.n_beta * self.reps
            self.beta = bt
        else:
            self.M, self.R = M, R
        cfg = _Config(mode, self.n_inst, self._arr, self.n_beta if mode == SG_APT else 0,
                      None if bt is None else bt.ctypes.data, reps_per_beta if mode == SG_APT else 0,
                      M, R, float(sqa_beta), int(seed) & (2 ** 64 - 1), None)
        self._cfg_keep = bt
        h = C.c_void_p()
        if colours is None:
            rc = self.lib.sg_create(C.byref(cfg), C.byref(h))
        else:
            maps = [None if m is None else np.ascontiguousarray(m, dtype=np.int8).reshape(-1)
                    for m in colours]
            if len(maps) != self.n_inst:
                raise ValueError("one colour map (or None) per instance expected")
            ptrs = (C.c_void_p * self.n_inst)(*[None if m is None else m.ctypes.data for m in maps])
            self._maps = (maps, ptrs)
            rc = self.lib.sg_create_ex(C.byref(cfg), ptrs, C.byref(h))
        if rc != SG_OK:
            raise SGError(rc, self.lib.sg_last_error(None).decode())
        self.h = h

    # -- plumbing
    def _check(self, rc):
        if rc != SG_OK:
            raise SGError(rc, self.lib.sg_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.sg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- APT
    def sweep(self, n=1):
        self._check(self.lib.sg_sweep(self.h, int(n)))

    def icm(self, cutoff, want_info=False):
        info = None
        if want_info:
            info = np.zeros((self.n_inst, self.n_beta, max(1, self.reps // 2), 4), np.int32)
        self._check(self.lib.sg_icm(self.h, float(cutoff), _p(info)))
        return info

    def energy(self):
        if self.mode == SG_APT:
            E = np.zeros((self.n_inst, self.n_slots), np.int64)
        else:
            E = np.zeros((self.n_inst, self.R, self.M), np.int64)
        self._check(self.lib.sg_energy(self.h, _p(E)))
        return E

    def swap(self, want_flags=True):
        acc = np.zeros((self.n_inst, (self.n_beta - 1) * self.reps), np.int32) if want_flags else None
        self._check(self.lib.sg_swap(self.h, _p(acc)))
        return acc

    def run_apt(self, n_cycles, sweeps_per_swap=1, icm_cutoff=float("inf"), record_every=0):
        tr = None
        if record_every > 0:
            tr = np.zeros((self.n_inst, n_cycles // record_every), np.int64)
        self._check(self.lib.sg_run_apt(self.h, int(n_cycles), int(sweeps_per_swap),
                                        float(icm_cutoff), int(record_every), _p(tr)))
        return tr

    def _options(self, sweeps_per_swap, icm_pairs, icm_cutoff, record_every):
        cut = np.asarray(icm_cutoff, dtype=np.float64)
        per = None
        if cut.ndim == 1:
            if cut.size != self.n_inst:
                raise ValueError("one ICM cutoff per instance expected")
            per = np.ascontiguousarray(cut)
        opt = _AptOptions(int(sweeps_per_swap), int(icm_pairs),
                          float(cut) if per is None else float("inf"),
                          None if per is None else per.ctypes.data, int(record_every))
        return opt, per

    def run_apt_ex(self, n_cycles, sweeps_per_swap=1, icm_cutoff=float("inf"), icm_pairs=2,
                   record_every=0):
        """sg_run_apt_ex: icm_cutoff is one value or one per instance; icm_pairs 2 or 1."""
        opt, keep = self._options(sweeps_per_swap, icm_pairs, icm_cutoff, record_every)
        tr = None
        if record_every > 0:
            tr = np.zeros((self.n_inst, n_cycles // record_every), np.int64)
        self._check(self.lib.sg_run_apt_ex(self.h, int(n_cycles), C.byref(opt), _p(tr)))
        return tr

    def icm_ex(self, icm_cutoff, icm_pairs=2, want_info=False):
        opt, keep = self._options(1, icm_pairs, icm_cutoff, 0)
        info = None
        if want_info:
            info = np.zeros((self.n_inst, self.n_beta, max(1, self.reps // 2), 4), np.int32)
        self._check(self.lib.sg_icm_ex(self.h, C.byref(opt), _p(info)))
        return info

    def best(self):
        b = np.zeros(self.n_inst, np.int64)
        self._check(self.lib.sg_best(self.h, _p(b)))
        return b

    def swap_counts(self):
        c = np.zeros((self.n_inst, (self.n_beta - 1) * self.reps), np.int64)
        self._check(self.lib.sg_swap_counts(self.h, _p(c)))
        return c

    # -- DT-SQA
    def sqa_anneal(self, gammas):
        g = np.ascontiguousarray(gammas, dtype=np.float64)
        bE = np.zeros(self.n_inst, np.int64)
        bs = np.zeros((self.n_inst, self.n_max), np.int8)
        self._check(self.lib.sg_sqa_anneal(self.h, _p(g), g.size, _p(bE), _p(bs)))
        return bE, bs

    # -- device outputs: `out` is a device address (int) or an object with data_ptr() on the
    #    context's device; the work is queued on the context's stream
    def energy_dev(self, out):
        self._check(self.lib.sg_energy_dev(self.h, _dev(out)))

    def spins_dev(self, out):
        self._check(self.lib.sg_get_spins_dev(self.h, _dev(out)))

    def best_dev(self, out):
        self._check(self.lib.sg_best_dev(self.h, _dev(out)))

    def sqa_anneal_dev(self, gammas, best_E=None, best_state=None):
        g = np.ascontiguousarray(gammas, dtype=np.float64)
        self._check(self.lib.sg_sqa_anneal_dev(self.h, _p(g), g.size, _dev(best_E), _dev(best_state)))

    def trotter_agreement(self):
        """DT-SQA: [n_inst, R, M] sites where slice k agrees with slice 0 of its replica."""
        a = np.zeros((self.n_inst, self.R, self.M), np.int32)
        self._check(self.lib.sg_sqa_trotter_agreement(self.h, _p(a)))
        return a

    def launch_config(self):
        """DT-SQA work-group size, or APT configuration code (1..15); 0 until the autotuner
        has run."""
        t = C.c_int32(0)
        self._check(self.lib.sg_get_launch_config(self.h, C.byref(t)))
        return t.value

    def set_launch_config(self, threads):
        self._check(self.lib.sg_set_launch_config(self.h, int(threads)))

    # -- state
    def spins(self):
        if self.mode == SG_APT:
            s = np.zeros((self.n_inst, self.n_slots, self.n_max), np.int8)
        else:
            s = np.zeros((self.n_inst, self.R, self.M, self.n_max), np.int8)
        self._check(self.lib.sg_get_spins(self.h, _p(s)))
        return s

    def spins_range(self, inst, first, count):
        """APT slots / DT-SQA replicas [first, first + count) of one instance."""
        n = int(self.ns[inst])
        shape = (count, n) if self.mode == SG_APT else (count, self.M, n)
        s = np.zeros(shape, np.int8)
        self._check(self.lib.sg_get_spins_range(self.h, int(inst), int(first), int(count), _p(s)))
        return s

    def set_spins(self, s):
        s = np.ascontiguousarray(s, dtype=np.int8)
        self._check(self.lib.sg_set_spins(self.h, _p(s)))

    def counters(self):
        c = np.zeros(3, np.uint32)
        self._check(self.lib.sg_get_counters(self.h, _p(c)))
        return c

    def get_state(self):
        n = C.c_size_t(0)
        self._check(self.lib.sg_get_state(self.h, None, C.byref(n)))
        blob = np.zeros(n.value, np.uint8)
        self._check(self.lib.sg_get_state(self.h, _p(blob), C.byref(n)))
        return blob

    def set_state(self, blob):
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        self._check(self.lib.sg_set_state(self.h, _p(b), b.size))

    def timer_start(self):
        self._check(self.lib.sg_timer_start(self.h))

    def timer_stop(self):
        ms = C.c_float(0)
        self._check(self.lib.sg_timer_stop(self.h, C.byref(ms)))
        return ms.value

    def synchronize(self):
        self._check(self.lib.sg_synchronize(self.h))

    def kernel_timing(self, enable=True):
        self._check(self.lib.sg_kernel_timing(self.h, 1 if enable else 0))

    def kernel_time(self):
        """(summed ms, launches) of the main kernels since the last query."""
        ms, n = C.c_float(0), C.c_int32(0)
        self._check(self.lib.sg_kernel_time(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value


def _threshold(fn, *args):
    lib = load()
    t = C.c_uint32(0)
    rc = getattr(lib, fn)(*args, C.byref(t))
    if rc != SG_OK:
        raise SGError(rc, lib.sg_last_error(None).decode())
    return t.value


def threshold_heat_bath(beta, I):
    """The library's heat-bath threshold (Eq. 6) for local field I at inverse temperature beta."""
    return _threshold("sg_threshold_heat_bath", float(beta), int(I))


def threshold_sqa(beta, M, gamma, s, tau):
    """The library's DT-SQA threshold (Supplementary Eq. S.3)."""
    return _threshold("sg_threshold_sqa", float(beta), int(M), float(gamma), int(s), int(tau))


def threshold_swap(beta_lo, beta_hi, d):
    """The library's swap threshold (Eq. 4) for an unfavourable energy change d >= 1."""
    return _threshold("sg_threshold_swap", float(beta_lo), float(beta_hi), int(d))


def apt(instances, beta, seed, reps_per_beta=2, colours=None):
    return Context(instances, SG_APT, seed, beta=beta, reps_per_beta=reps_per_beta, colours=colours)


def sqa(instances, M, R, beta, seed, colours=None):
    return Context(instances, SG_SQA, seed, M=M, R=R, sqa_beta=beta, colours=colours)


def dsatur(instance):
    """DSATUR colouring of one instance (J, periodic, h): (colour map [n] int8, colours)."""
    lib = load()
    arr, keep = _lattices([instance])
    n = arr[0].Lx * arr[0].Ly * arr[0].Lz
    col = np.zeros(n, np.int8)
    nc = C.c_int32(0)
    rc = lib.sg_dsatur_colouring(arr, _p(col), C.byref(nc))
    if rc != SG_OK:
        raise SGError(rc, lib.sg_last_error(None).decode())
    return col, nc.value


def adaptive_ladder(instances, seed, beta0=0.5, alpha=1.25, tol=0.5, n_chains=100, sweeps=10000,
                    tail=1000, max_steps=64):
    lib = load()
    arr, keep = _lattices(instances)
    p = _Adaptive(beta0, alpha, tol, n_chains, sweeps, tail, max_steps)
    n = len(instances)
    b = np.zeros((n, max_steps), np.float64)
    sg_ = np.zeros((n, max_steps), np.float64)
    ln = np.zeros(n, np.int32)
    rc = lib.sg_adaptive_ladder(arr, n, C.byref(p), int(seed), None, _p(b), _p(sg_), _p(ln))
    if rc != SG_OK:
        raise SGError(rc, lib.sg_last_error(None).decode())
    return [(b[i, :ln[i]].copy(), sg_[i, :ln[i]].copy()) for i in range(n)]
