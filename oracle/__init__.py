"""CPU oracle for parallel flatPERM -- TEST INFRASTRUCTURE ONLY.

The plain, slow, obviously-correct reference the GPU path is checked against
(Campbell & Janse van Rensburg, "Parallel PERM": Sec. 1 Rosenbluth growth and
eqns (1)-(4); Sec. 2 flatPERM, eqn (6); Sec. 3 / Fig. 1 Algorithms 1 and 2).
Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library and never takes an input
produced by it.

The arithmetic lives in C (pperm_oracle.c, saw_enum.c); this module only
marshals numpy arrays into it.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

MODE_SHARED = 0        # Algorithm 2: pooled W
MODE_INDEPENDENT = 1   # Algorithm 1: independent sequences
MODE_ROSENBLUTH = 2    # plain Rosenbluth sampling (no prune / enrich)

STATS_FIELDS = ("steps", "events", "enrich", "copies", "prunes", "traps",
                "tours", "max_depth", "digest", "capped")
STATS_DTYPE = np.dtype([(f, np.uint64) for f in STATS_FIELDS])
# extended-range number m * 2^e (m in [0.5, 1), or m = 0 and e = 0)
GROUPS = 16          # sequence groups of the relative-error estimate (s mod 16)
XF_DTYPE = np.dtype([("m", np.float64), ("e", np.int32), ("pad", np.uint32)])


class XF_C(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("e", ctypes.c_int32), ("pad", ctypes.c_uint32)]


class _Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("n_max", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("step_cap", ctypes.c_uint64), ("n_pool", ctypes.c_uint64)]


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        srcs = [os.path.join(_HERE, s) for s in _build.SOURCES]
        if not os.path.exists(path) or any(os.path.getmtime(s) > os.path.getmtime(path) for s in srcs):
            _build.build()
        L = ctypes.CDLL(path)
        u32p, u64p = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
        dblp, i64p = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.orc_xf_apply.argtypes = [ctypes.c_int, dblp, i32p, dblp, i32p, dblp, ctypes.c_int64, dblp, i32p]
        L.orc_xf_normalize.argtypes = [dblp, ctypes.c_int64, dblp, i32p]
        L.orc_xf_ratio.argtypes = [XF_C, XF_C]
        L.orc_xf_ratio.restype = ctypes.c_double
        L.orc_set_selftest.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64]
        L.orc_set_selftest.restype = ctypes.c_int64
        L.orc_stats_init.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        vp = ctypes.c_void_p
        L.orc_run_epoch.argtypes = [ctypes.POINTER(_Params), ctypes.c_int64, vp, u64p, u64p,
                                    ctypes.c_uint32, vp, u32p, u32p, vp,
                                    i64p, ctypes.c_int64, ctypes.c_int, vp]
        L.orc_run_epoch.restype = ctypes.c_int
        L.orc_merge.argtypes = [ctypes.POINTER(_Params), ctypes.c_int64, vp, u32p, u32p,
                                vp, u64p, u64p, vp, vp]
        L.orc_observable_r2.argtypes = [ctypes.c_int64, vp, vp, dblp]
        L.orc_group_sums.argtypes = [ctypes.POINTER(_Params), ctypes.c_int64, vp, u32p, vp, u64p]
        L.orc_log_estimates.argtypes = [ctypes.c_int64, vp, ctypes.c_uint64, dblp]
        L.orc_plain_recursive.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint32, vp, u32p]
        L.orc_plain_recursive.restype = ctypes.c_int
        L.orc_forced_enumerate.argtypes = [ctypes.c_int, ctypes.c_int64, u64p, u64p, u64p]
        L.orc_forced_enumerate.restype = ctypes.c_int
        L.saw_count.argtypes = [ctypes.c_int, ctypes.c_int, u64p]
        L.saw_count.restype = ctypes.c_int
        L.saw_count_r2.argtypes = [ctypes.c_int, ctypes.c_int, u64p, u64p]
        L.saw_count_r2.restype = ctypes.c_int
        _LIB = L
    return _LIB


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: ctr is 4 uint32 words, key is 2."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def xf_from_float(x):
    """Normalise doubles into extended-range numbers (m, e)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = np.zeros(len(x)); e = np.zeros(len(x), dtype=np.int32)
    lib().orc_xf_normalize(_ptr(x, ctypes.c_double), len(x), _ptr(m, ctypes.c_double), _ptr(e, ctypes.c_int32))
    return m, e


def xf_apply(op, am, ae, bm=None, be=None, k=None):
    """Elementwise extended-range add (op 'add'), multiply or divide by k ('mul', 'div')."""
    n = len(am)
    am = np.ascontiguousarray(am, dtype=np.float64); ae = np.ascontiguousarray(ae, dtype=np.int32)
    bm = np.ascontiguousarray(bm if bm is not None else np.zeros(n), dtype=np.float64)
    be = np.ascontiguousarray(be if be is not None else np.zeros(n), dtype=np.int32)
    k = np.ascontiguousarray(k if k is not None else np.ones(n), dtype=np.float64)
    om = np.zeros(n); oe = np.zeros(n, dtype=np.int32)
    code = {"add": 0, "mul": 1, "div": 2}[op]
    lib().orc_xf_apply(code, _ptr(am, ctypes.c_double), _ptr(ae, ctypes.c_int32), _ptr(bm, ctypes.c_double),
                       _ptr(be, ctypes.c_int32), _ptr(k, ctypes.c_double), n,
                       _ptr(om, ctypes.c_double), _ptr(oe, ctypes.c_int32))
    return om, oe


def xf_ratio(am, ae, bm, be):
    return float(lib().orc_xf_ratio(XF_C(am, ae, 0), XF_C(bm, be, 0)))


def xf_log(a):
    """Natural log of extended-range values (structured XF_DTYPE array)."""
    with np.errstate(divide="ignore"):
        return np.log(a["m"]) + a["e"].astype(np.float64) * np.log(2.0)


def saw_counts(dim, n_max):
    """Exact c_0..c_n_max by brute-force enumeration."""
    out = np.zeros(n_max + 1, dtype=np.uint64)
    if lib().saw_count(dim, n_max, _ptr(out, ctypes.c_uint64)) != 0:
        raise RuntimeError("saw_count failed")
    return out


def forced_enumerate(dim, n_max):
    """Drive the oracle's scan and weight update over every chain.

    Returns (count[n], bad, r2sum[n]) where count[n] is the number of chains of
    length n, bad counts chains whose weight differs from the exact product of
    a_+, and r2sum[n] sums the chains' squared end-to-end distances."""
    cnt = np.zeros(n_max + 1, dtype=np.uint64)
    bad = np.zeros(1, dtype=np.uint64)
    r2 = np.zeros(n_max + 1, dtype=np.uint64)
    if lib().orc_forced_enumerate(dim, n_max, _ptr(cnt, ctypes.c_uint64), _ptr(bad, ctypes.c_uint64),
                                  _ptr(r2, ctypes.c_uint64)) != 0:
        raise RuntimeError("forced_enumerate failed")
    return cnt, int(bad[0]), r2


def saw_counts_r2(dim, n_max):
    """Exact c_n and the exact sum of R^2 over the c_n walks, by brute force."""
    out = np.zeros(n_max + 1, dtype=np.uint64)
    r2 = np.zeros(n_max + 1, dtype=np.uint64)
    if lib().saw_count_r2(dim, n_max, _ptr(out, ctypes.c_uint64), _ptr(r2, ctypes.c_uint64)) != 0:
        raise RuntimeError("saw_count_r2 failed")
    return out, r2


def set_selftest(ops, xyz, max_items):
    ops = np.ascontiguousarray(ops, dtype=np.int32)
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1)
    out = np.zeros(int((ops == 2).sum()), dtype=np.int32)
    c = lib().orc_set_selftest(_ptr(ops, ctypes.c_int32), _ptr(xyz, ctypes.c_int32), len(ops),
                               _ptr(out, ctypes.c_int32), max_items)
    return out, int(c)


def plain_recursive(dim, n_max, seed, tours, mode=MODE_SHARED, stream=0):
    """Plain flatPERM (one sequence, one epoch) in recursive form."""
    p = _Params(dim, mode, n_max, seed, stream, 0, 0, 1)
    L = np.zeros(n_max + 1, dtype=XF_DTYPE)
    H = np.zeros(n_max + 1, dtype=np.uint32)
    if lib().orc_plain_recursive(ctypes.byref(p), tours, L.ctypes.data, _ptr(H, ctypes.c_uint32)) != 0:
        raise RuntimeError("plain_recursive failed")
    return L, H


class Oracle:
    """Parallel flatPERM state and its epoch schedule (run / merge calls)."""

    def __init__(self, dim, n_max, n_sequences, seed, mode=MODE_SHARED, stream=0,
                 step_cap=0, threads=0, group_stats=False, observables=False):
        self.params = _Params(dim, mode, n_max, seed & 0xFFFFFFFFFFFFFFFF, stream, 0, step_cap,
                              n_sequences)
        self.dim, self.n_max, self.N, self.mode = dim, n_max, n_sequences, mode
        self.threads = threads
        n1 = n_max + 1
        gshape = (n_sequences, n1) if mode == MODE_INDEPENDENT else (n1,)
        self.G = np.zeros(gshape, dtype=XF_DTYPE)
        self.HG = np.zeros(gshape, dtype=np.uint64)
        self.MG = np.zeros(n_sequences if mode == MODE_INDEPENDENT else 1, dtype=np.uint64)
        self.t = np.zeros(n_sequences, dtype=np.uint64)
        self.L = np.zeros((n_sequences, n1), dtype=XF_DTYPE)
        self.H = np.zeros((n_sequences, n1), dtype=np.uint32)
        self.m = np.zeros(n_sequences, dtype=np.uint32)
        self.stats = np.zeros(n_sequences, dtype=STATS_DTYPE)
        lib().orc_stats_init(self.stats.ctypes.data, n_sequences)
        self.group_stats = group_stats
        self.observables = observables
        self.LR = np.zeros((n_sequences, n1), dtype=XF_DTYPE) if observables else None
        self.GR = np.zeros(gshape, dtype=XF_DTYPE) if observables else None
        self.gsum = np.zeros(GROUPS, dtype=XF_DTYPE)
        self.gtours = np.zeros(GROUPS, dtype=np.uint64)

    def run_tours(self, tours, ids=None):
        """Every sequence (or only `ids`) runs `tours` more tours. Returns True if capped."""
        idp, nid = None, 0
        if ids is not None:
            ids = np.ascontiguousarray(ids, dtype=np.int64)
            idp, nid = _ptr(ids, ctypes.c_int64), len(ids)
        rc = lib().orc_run_epoch(ctypes.byref(self.params), self.N, self.G.ctypes.data,
                                 _ptr(self.MG, ctypes.c_uint64), _ptr(self.t, ctypes.c_uint64),
                                 tours, self.L.ctypes.data, _ptr(self.H, ctypes.c_uint32),
                                 _ptr(self.m, ctypes.c_uint32), self.stats.ctypes.data,
                                 idp, nid, self.threads,
                                 self.LR.ctypes.data if self.observables else None)
        return bool(rc)

    def merge_epoch(self):
        if self.group_stats:
            lib().orc_group_sums(ctypes.byref(self.params), self.N, self.L.ctypes.data,
                                 _ptr(self.m, ctypes.c_uint32), self.gsum.ctypes.data,
                                 _ptr(self.gtours, ctypes.c_uint64))
        lib().orc_merge(ctypes.byref(self.params), self.N, self.L.ctypes.data,
                        _ptr(self.H, ctypes.c_uint32), _ptr(self.m, ctypes.c_uint32),
                        self.G.ctypes.data, _ptr(self.HG, ctypes.c_uint64),
                        _ptr(self.MG, ctypes.c_uint64),
                        self.LR.ctypes.data if self.observables else None,
                        self.GR.ctypes.data if self.observables else None)

    def log_estimates(self):
        """log c_n: the pooled average (shared mode) or, in independent mode, the
        log of the mean over sequences of each sequence's average (eqn (7))."""
        if self.mode == MODE_INDEPENDENT:
            per = xf_log(self.G) - np.log(self.MG.astype(np.float64))[:, None]
            top = per.max(axis=0)
            with np.errstate(invalid="ignore"):
                return top + np.log(np.exp(per - top).sum(axis=0)) - np.log(self.N)
        out = np.zeros(self.n_max + 1)
        lib().orc_log_estimates(self.n_max, self.G.ctypes.data, int(self.MG[0]), _ptr(out, ctypes.c_double))
        return out

    def error_estimate(self):
        """Relative error estimate of c_{n_max} from the 16 group sums: the
        sample standard deviation of the group averages A_k / C_k over 4 times
        their mean (+inf while a group is empty or has no weight at n_max).
        The averages are taken relative to the largest group exponent,
        g_k = ldexp(m_k / C_k, e_k - e_max), and summed in group order, so the
        value is a fixed sequence of correctly rounded operations."""
        if np.any(self.gtours == 0) or np.any(self.gsum["m"] == 0.0):
            return math.inf
        e_top = int(self.gsum["e"].max())
        g = [math.ldexp(float(self.gsum["m"][k]) / float(self.gtours[k]), int(self.gsum["e"][k]) - e_top)
             for k in range(GROUPS)]
        total = 0.0
        for x in g:
            total += x
        mean = total / GROUPS
        ss = 0.0
        for x in g:
            ss += (x - mean) * (x - mean)
        return math.sqrt(ss / (GROUPS - 1)) / (4.0 * mean)

    def observable_r2(self):
        """<R^2_n> by the ratio estimator of eqn (5) (shared mode), NaN where no sample."""
        out = np.zeros(self.n_max + 1)
        lib().orc_observable_r2(self.n_max, self.G.ctypes.data, self.GR.ctypes.data, _ptr(out, ctypes.c_double))
        return out

    def walk_steps(self):
        return int(self.stats["steps"].sum())
