"""CPU oracle for population annealing of the 2D Ising model.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU product path never imports
this package.

Thin ctypes wrapper over ``liboracle.so`` (built from ``pa_oracle.c``, plain
serial C, FP64 without contraction).  See ``pa_oracle.c`` for the algorithm and
the paper sections each function follows.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force=True):
    """Compile liboracle.so with gcc (always recompiles when force is set)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Obs(ctypes.Structure):
    _fields_ = [
        ("beta", ctypes.c_double), ("e", ctypes.c_double), ("C", ctypes.c_double),
        ("abs_m", ctypes.c_double), ("m2", ctypes.c_double), ("m4", ctypes.c_double),
        ("betaF_per_N", ctypes.c_double), ("S_per_N", ctypes.c_double), ("lnQ", ctypes.c_double),
        ("R", ctypes.c_int64),
        ("sumE", ctypes.c_int64), ("sumE2", ctypes.c_int64), ("sumAbsM", ctypes.c_int64),
        ("sumM2", ctypes.c_int64), ("sumM4_lo", ctypes.c_uint64), ("sumM4_hi", ctypes.c_uint64),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["sumM4"] = (d.pop("sumM4_hi") << 64) | d.pop("sumM4_lo")
        return d


_lib = None


def lib():
    """The oracle library (built on first use if missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load(_LIB)
    return _lib


def load(path):
    """Load an oracle shared library from ``path`` and declare its signatures."""
    L = ctypes.CDLL(path)
    vp, i32, u32, u64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "philox4x32_10": (None, [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]),
        "orc_new": (vp, [i32, i32, i32, u64, u32]),
        "orc_free": (None, [vp]),
        "orc_init": (None, [vp]),
        "orc_thresholds": (None, [dbl, P(u64), P(u64)]),
        "orc_hb_thresholds": (None, [dbl, P(u64), P(u64)]),
        "orc_set_heatbath": (None, [vp, i32]),
        "orc_set_threads": (None, [vp, i32]),
        "orc_set_lcg": (None, [vp, i32]),
        "orc_sweep": (None, [vp, i32]),
        "orc_resample": (i32, [vp, dbl, P(dbl), P(ctypes.c_int32)]),
        "orc_alpha": (dbl, [vp, dbl]),
        "orc_adapt_beta": (i32, [vp, dbl, dbl, P(dbl)]),
        "orc_measure": (None, [vp, P(Obs)]),
        "orc_reweight": (None, [vp, P(dbl), i32, P(Obs)]),
        "orc_population": (i32, [vp]),
        "orc_step": (i32, [vp]),
        "orc_sweeps": (u64, [vp]),
        "orc_beta": (dbl, [vp]),
        "orc_lnZ": (dbl, [vp]),
        "orc_get_population": (None, [vp, vp, vp, vp]),
        "orc_get_counts": (i32, [vp, vp]),
        "orc_set_population": (i32, [vp, i32, vp, i32, u64, dbl, dbl]),
        "orc_recount": (None, [vp, i32, P(ctypes.c_int32), P(ctypes.c_int32)]),
        "orc_tables": (dbl, [i32, i32, i32, vp, dbl, vp, vp]),
        "orc_set_slots": (None, [vp, vp]),
        "orc_word_uniforms": (None, [vp, u64, i32, i32, i32, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(counter, key, lib_=None):
    """Philox4x32-10 block: 4-word counter, 2-word key -> 4 uint32 words."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in counter])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    (lib_ or lib()).philox4x32_10(c, k, o)
    return [int(x) for x in o]


def thresholds(beta, lib_=None):
    """Metropolis thresholds (T_2, T_4) = ceil(2^32 exp(-2 beta k)), k = 2, 4."""
    t2, t4 = ctypes.c_uint64(), ctypes.c_uint64()
    (lib_ or lib()).orc_thresholds(float(beta), ctypes.byref(t2), ctypes.byref(t4))
    return t2.value, t4.value


def hb_thresholds(beta, lib_=None):
    """Heat-bath thresholds (U_2, U_4) = ceil(2^32 / (1 + exp(2 beta k))), k = 2, 4."""
    u2, u4 = ctypes.c_uint64(), ctypes.c_uint64()
    (lib_ or lib()).orc_hb_thresholds(float(beta), ctypes.byref(u2), ctypes.byref(u4))
    return u2.value, u4.value


def tables(N, R, Rprev, hist, dbeta, lib_=None):
    """Resampling tables (base, thr) and ln Q for an energy histogram."""
    hist = np.ascontiguousarray(hist, dtype=np.int64)
    assert hist.shape == (N + 1,)
    base = np.zeros(N + 1, np.uint32)
    thr = np.zeros(N + 1, np.uint32)
    lnQ = (lib_ or lib()).orc_tables(N, R, Rprev, _ptr(hist), float(dbeta), _ptr(base), _ptr(thr))
    return base, thr, lnQ


def default_capacity(R):
    return R + int(np.ceil(10.0 * np.sqrt(R))) + 64


class Run:
    """One PA run held by the oracle."""

    def __init__(self, L, R, seed, run_id=0, capacity=0, lib_=None, heatbath=False, lcg=False):
        self.L, self.N, self.R = L, L * L, R
        self.capacity = capacity or default_capacity(R)
        self.lib = lib_ or lib()
        self.heatbath = bool(heatbath)
        self.h = self.lib.orc_new(L, R, self.capacity, seed, run_id)
        if not self.h:
            raise ValueError("invalid oracle parameters")
        self.lib.orc_set_heatbath(self.h, 1 if self.heatbath else 0)
        self.lcg = bool(lcg)
        self.lib.orc_set_lcg(self.h, 1 if self.lcg else 0)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_free(self.h)
            self.h = None

    def set_threads(self, n):
        """Share the replicas of init and sweeps out among n threads (timing)."""
        self.lib.orc_set_threads(self.h, int(n))

    def init(self):
        self.lib.orc_init(self.h)

    def sweep(self, nsweeps):
        self.lib.orc_sweep(self.h, int(nsweeps))

    def resample(self, beta_next):
        lnq = ctypes.c_double()
        emin = ctypes.c_int32()
        rn = self.lib.orc_resample(self.h, float(beta_next), ctypes.byref(lnq), ctypes.byref(emin))
        if rn == -1:
            raise OverflowError("population exceeds capacity")
        if rn < 0:
            raise ArithmeticError("no replica would survive")
        return {"R_new": rn, "lnQ": lnq.value, "E_min": emin.value}

    def alpha(self, beta_prime):
        return self.lib.orc_alpha(self.h, float(beta_prime))

    def adapt_beta(self, alpha_star, beta_f):
        out = ctypes.c_double()
        st = self.lib.orc_adapt_beta(self.h, float(alpha_star), float(beta_f), ctypes.byref(out))
        if st != 0:
            raise ValueError("no temperature step reaches the overlap target")
        return out.value

    def measure(self):
        o = Obs()
        self.lib.orc_measure(self.h, ctypes.byref(o))
        return o.as_dict()

    def reweight(self, betas):
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        out = (Obs * len(betas))()
        self.lib.orc_reweight(self.h, betas.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(betas), out)
        return [o.as_dict() for o in out]

    @property
    def population(self):
        return self.lib.orc_population(self.h)

    @property
    def step(self):
        return self.lib.orc_step(self.h)

    @property
    def sweeps(self):
        return self.lib.orc_sweeps(self.h)

    @property
    def beta(self):
        return self.lib.orc_beta(self.h)

    @property
    def lnZ(self):
        return self.lib.orc_lnZ(self.h)

    def get_population(self):
        """(spins int8 [R_i, L, L], E int32 [R_i], M int32 [R_i])."""
        n = self.population
        s = np.empty((n, self.L, self.L), np.int8)
        E = np.empty(n, np.int32)
        M = np.empty(n, np.int32)
        self.lib.orc_get_population(self.h, _ptr(s), _ptr(E), _ptr(M))
        return s, E, M

    def get_counts(self):
        buf = np.empty(self.capacity, np.uint32)
        n = self.lib.orc_get_counts(self.h, _ptr(buf))
        return buf[:n].copy()

    def set_population(self, spins, step=0, sweeps=0, beta=0.0, lnZ=0.0):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        n = spins.shape[0]
        assert spins.shape[1:] == (self.L, self.L)
        st = self.lib.orc_set_population(self.h, n, _ptr(spins), int(step), int(sweeps), float(beta), float(lnZ))
        if st != 0:
            raise ValueError("population does not fit")

    def set_slots(self, slots):
        """Random-stream slot of each replica for later sweeps (None: identity)."""
        if slots is None:
            self.lib.orc_set_slots(self.h, None)
        else:
            self._slots = np.ascontiguousarray(slots, dtype=np.int32)
            assert len(self._slots) == self.population
            self.lib.orc_set_slots(self.h, _ptr(self._slots))

    def word_uniforms(self, g, c, j, v):
        """The 32 site uniforms (uint32) of word v, colour c, slot j, sweep g."""
        out = np.empty(32, np.uint32)
        self.lib.orc_word_uniforms(self.h, int(g), int(c), int(j), int(v), _ptr(out))
        return out

    def recount(self, j):
        e, m = ctypes.c_int32(), ctypes.c_int32()
        self.lib.orc_recount(self.h, int(j), ctypes.byref(e), ctypes.byref(m))
        return e.value, m.value
