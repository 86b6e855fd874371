"""Plain CPU oracle for the spin-glass Monte Carlo hot path -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never calls it and shares no code
with it.  The C source (``sg_oracle.c``) holds the arithmetic; this module only
marshals numpy arrays through ctypes.

Every function follows a step of arXiv:2503.10302 (Eqs. 1, 4-8, Supplementary
Eqs. S.1-S.3, Algorithms S1 and S2); see the comments in ``sg_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SG_ORACLE_SO names a separately built copy of the oracle (the planted-mistake tests
# load mutated builds this way); it is loaded as is, never rebuilt.
_VARIANT = os.environ.get("SG_ORACLE_SO")
_SO = _VARIANT or os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sg_oracle.c")

TAG_APT_INIT, TAG_APT_SWEEP, TAG_SWAP, TAG_ICM_PAIR, TAG_ICM_PICK = 1, 2, 3, 4, 5
TAG_SQA_INIT, TAG_SQA_SWEEP, TAG_ADAPT_INIT, TAG_ADAPT_SWEEP = 6, 7, 8, 9
MLP_NPARAM = 64 * 4 + 64 + 64 * 64 + 64 + 33 * 64 + 33


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if _VARIANT:
        return _SO
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Lattice(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("Lz", C.c_int32),
                ("periodic", C.c_uint32), ("J", C.c_void_p), ("h", C.c_void_p),
                ("colour", C.c_void_p), ("n_map_colours", C.c_int32)]


class _AdaptiveParams(C.Structure):
    _fields_ = [("beta0", C.c_double), ("alpha", C.c_double), ("tol", C.c_double),
                ("n_chains", C.c_int32), ("sweeps", C.c_int32), ("tail", C.c_int32),
                ("max_steps", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        P = C.c_void_p
        i32, u32, u64, i64, dbl = C.c_int32, C.c_uint32, C.c_uint64, C.c_int64, C.c_double
        LP = C.POINTER(_Lattice)
        sig = {
            "sgo_philox4x32_10": (None, [P, P, P]),
            "sgo_word": (u32, [u64, u32, u32, u32, u32, u32, C.c_int]),
            "sgo_n_sites": (i32, [LP]),
            "sgo_neighbour": (i32, [LP, i32, i32, i32]),
            "sgo_bond": (i32, [LP, i32, i32, i32]),
            "sgo_n_colours": (i32, [LP, i32]),
            "sgo_colour": (i32, [LP, i32, i32, i32]),
            "sgo_local_field": (i32, [LP, P, i32]),
            "sgo_energy": (i64, [LP, P]),
            "sgo_heat_threshold": (u32, [dbl, i32]),
            "sgo_sqa_threshold": (u32, [dbl, i32, dbl, i32, i32]),
            "sgo_swap_accept": (i32, [dbl, dbl, i64, i64, u32]),
            "sgo_apt_init": (None, [LP, u32, i32, u64, u32, P]),
            "sgo_apt_sweep": (None, [LP, u32, i32, P, u64, u32, u32, P]),
            "sgo_apt_icm": (i32, [LP, u32, i32, i32, P, dbl, i32, u64, u32, P, P]),
            "sgo_apt_swap": (None, [u32, i32, i32, P, u64, u32, i32, P, P, P]),
            "sgo_apt_run": (i32, [LP, u32, i32, i32, P, u64, i64, i32, dbl, i32, i32, P, P, P,
                                  P, P, P]),
            "sgo_sqa_init": (None, [LP, u32, i32, i32, i32, u64, P]),
            "sgo_sqa_step": (None, [LP, u32, i32, i32, i32, dbl, dbl, u64, u32, P]),
            "sgo_sqa_anneal": (None, [LP, u32, i32, i32, i32, dbl, P, i32, u64, u32, P, P, P, P]),
            "sgo_trotter_agreement": (None, [LP, i32, i32, P, P]),
            "sgo_adaptive_ladder": (i32, [LP, u32, C.POINTER(_AdaptiveParams), u64, P, P, P]),
            "sgo_sigma_from_moments": (dbl, [i64, i64, i64]),
            "sgo_instance_features": (None, [LP, P]),
            "sgo_mlp_loss_grad": (dbl, [P, P, P, i32, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Lattice:
    """An instance: couplings J[Lz, Ly, Lx, 3] (int8, bond to +x,+y,+z), fields h."""

    def __init__(self, J, periodic=7, h=None, colour=None):
        """colour: optional colour map [n] (a proper colouring of the coupled sites)."""
        self.J = np.ascontiguousarray(J, dtype=np.int8)
        assert self.J.ndim == 4 and self.J.shape[3] == 3
        self.Lz, self.Ly, self.Lx = self.J.shape[:3]
        self.periodic = int(periodic)
        self.h = None if h is None else np.ascontiguousarray(h, dtype=np.int8).reshape(-1)
        self.n = self.Lx * self.Ly * self.Lz
        self.colour = None if colour is None else np.ascontiguousarray(colour, dtype=np.int8).reshape(-1)
        ncol = 0 if self.colour is None else int(self.colour.max()) + 1
        self._c = _Lattice(self.Lx, self.Ly, self.Lz, self.periodic,
                           self.J.ctypes.data, None if self.h is None else self.h.ctypes.data,
                           None if self.colour is None else self.colour.ctypes.data, ncol)

    @property
    def c(self):
        return C.byref(self._c)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().sgo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def word(seed, c0, c1, c2, inst, tag, w):
    return lib().sgo_word(seed, c0, c1, c2, inst, tag, w)


def n_colours(lat, M=0):
    return lib().sgo_n_colours(lat.c, M)


def colour(lat, j, M=0, k=0):
    return lib().sgo_colour(lat.c, M, j, k)


def neighbour(lat, j, axis, direction):
    return lib().sgo_neighbour(lat.c, j, axis, direction)


def bond(lat, j, axis, direction):
    return lib().sgo_bond(lat.c, j, axis, direction)


def local_field(lat, spins, j):
    s = np.ascontiguousarray(spins, dtype=np.int8)
    return lib().sgo_local_field(lat.c, _ptr(s), j)


def energy(lat, spins):
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    assert s.size == lat.n
    return lib().sgo_energy(lat.c, _ptr(s))


def heat_threshold(beta, I):
    return lib().sgo_heat_threshold(float(beta), int(I))


def sqa_threshold(beta, M, gamma, s, tau):
    return lib().sgo_sqa_threshold(float(beta), int(M), float(gamma), int(s), int(tau))


def swap_accept(beta_lo, beta_hi, E_lo, E_hi, u):
    return lib().sgo_swap_accept(float(beta_lo), float(beta_hi), int(E_lo), int(E_hi), int(u))


def apt_init(lat, inst, n_slots, seed, tag=TAG_APT_INIT):
    s = np.zeros((n_slots, lat.n), np.int8)
    lib().sgo_apt_init(lat.c, inst, n_slots, seed, tag, _ptr(s))
    return s


def apt_sweep(lat, inst, slot_beta, seed, t, spins, tag=TAG_APT_SWEEP):
    """One coloured sweep of every slot, in place.  slot_beta[n_slots] (float64)."""
    sb = np.ascontiguousarray(slot_beta, dtype=np.float64)
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and spins.shape == (sb.size, lat.n)
    lib().sgo_apt_sweep(lat.c, inst, sb.size, _ptr(sb), seed, tag, t, _ptr(spins))
    return spins


def apt_icm(lat, inst, beta, R_lab, cutoff, seed, a, spins, pairs_per_call=2):
    b = np.ascontiguousarray(beta, dtype=np.float64)
    npair = max(1, R_lab // 2)
    info = np.full((b.size, npair, 4), -7, np.int32)
    rc = lib().sgo_apt_icm(lat.c, inst, b.size, R_lab, _ptr(b), float(cutoff), int(pairs_per_call),
                           seed, a, _ptr(spins), _ptr(info))
    return rc, info


def apt_swap(inst, beta, R_lab, seed, a, spins, E):
    b = np.ascontiguousarray(beta, dtype=np.float64)
    acc = np.zeros(((b.size - 1) * R_lab,), np.int32)
    n = spins.shape[1]
    lib().sgo_apt_swap(inst, b.size, R_lab, _ptr(b), seed, a, n, _ptr(spins), _ptr(E), _ptr(acc))
    return acc


def apt_run(lat, inst, beta, R_lab, seed, n_cycles, sweeps_per_swap, cutoff, record_every,
            counters, spins, E, best, icm_pairs=2):
    """APT cycles in place.  counters: uint32[3]; E: int64[n_slots]; best: int64[1]."""
    b = np.ascontiguousarray(beta, dtype=np.float64)
    ntr = n_cycles // record_every if record_every > 0 else 0
    trace = np.zeros(max(ntr, 1), np.int64)
    accc = np.zeros(max((b.size - 1) * R_lab, 1), np.int64)
    rc = lib().sgo_apt_run(lat.c, inst, b.size, R_lab, _ptr(b), seed, n_cycles, sweeps_per_swap,
                           float(cutoff), int(icm_pairs), record_every, _ptr(counters), _ptr(spins), _ptr(E),
                           _ptr(best), _ptr(trace), _ptr(accc))
    return rc, trace[:ntr], accc


def sqa_init(lat, inst, M, R, seed, r0=0):
    """Replicas r0 .. r0+R-1 of one instance, spins [R, M, n]."""
    s = np.zeros((R, M, lat.n), np.int8)
    lib().sgo_sqa_init(lat.c, inst, M, r0, R, seed, _ptr(s))
    return s


def sqa_step(lat, inst, M, R, beta, gamma, seed, t, spins, r0=0):
    assert spins.shape == (R, M, lat.n) and spins.dtype == np.int8 and spins.flags.c_contiguous
    lib().sgo_sqa_step(lat.c, inst, M, r0, R, float(beta), float(gamma), seed, t, _ptr(spins))
    return spins


def sqa_anneal(lat, inst, M, R, beta, gammas, seed, t0, spins, r0=0):
    assert spins.shape == (R, M, lat.n) and spins.dtype == np.int8 and spins.flags.c_contiguous
    g = np.ascontiguousarray(gammas, dtype=np.float64)
    sE = np.zeros((R, M), np.int64)
    bE = np.zeros(1, np.int64)
    bs = np.zeros(lat.n, np.int8)
    lib().sgo_sqa_anneal(lat.c, inst, M, r0, R, float(beta), _ptr(g), g.size, seed, t0,
                         _ptr(spins), _ptr(sE), _ptr(bE), _ptr(bs))
    return int(bE[0]), bs, sE


def trotter_agreement(lat, spins):
    """spins [R, M, n] -> agree [R, M]: sites where slice k agrees with slice 0."""
    s = np.ascontiguousarray(spins, dtype=np.int8)
    R, M, n = s.shape
    assert n == lat.n
    out = np.zeros((R, M), np.int32)
    lib().sgo_trotter_agreement(lat.c, M, R, _ptr(s), _ptr(out))
    return out


def adaptive_ladder(lat, inst, seed, beta0=0.5, alpha=1.25, tol=0.5, n_chains=100, sweeps=10000,
                    tail=1000, max_steps=64):
    p = _AdaptiveParams(beta0, alpha, tol, n_chains, sweeps, tail, max_steps)
    b = np.zeros(max_steps, np.float64)
    sg = np.zeros(max_steps, np.float64)
    mom = np.zeros((max_steps, n_chains, 2), np.int64)
    ln = lib().sgo_adaptive_ladder(lat.c, inst, C.byref(p), seed, _ptr(b), _ptr(sg), _ptr(mom))
    return b[:ln].copy(), sg[:ln].copy(), mom[:ln].copy()


def sigma_from_moments(S1, S2, N):
    return lib().sgo_sigma_from_moments(int(S1), int(S2), int(N))


def instance_features(lat):
    f = np.zeros(4, np.float64)
    lib().sgo_instance_features(lat.c, _ptr(f))
    return f


def mlp_loss_grad(params, x, y=None):
    p = np.ascontiguousarray(params, dtype=np.float64)
    assert p.size == MLP_NPARAM
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 4)
    B = xx.shape[0]
    yy = None if y is None else np.ascontiguousarray(y, dtype=np.float64).reshape(B, 33)
    g = np.zeros(MLP_NPARAM, np.float64)
    out = np.zeros((B, 33), np.float64)
    loss = lib().sgo_mlp_loss_grad(_ptr(p), _ptr(xx), _ptr(yy), B, _ptr(g), _ptr(out))
    return loss, g, out
