"""Population annealing for the 2D Ising model on one MI355X (gfx950).

Thin ctypes binding over ``libpa.so`` (C ABI in ``include/pa.h``).  The
binding only marshals arguments: every step of the method runs in the
library's HIP kernels.  PyTorch provides the device workspace and the stream.

Loading requires the HIP extension: if ``libpa.so`` has not been built, or no
GPU is present when a run is started, an error is raised; there is no CPU
fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpa.so")

PA_OK, PA_EINVAL, PA_ENOMEM, PA_ECAPACITY, PA_EHIP, PA_ESTATE, PA_EEXTINCT = 0, -1, -2, -3, -4, -5, -6
PA_SPIN_INT8, PA_SPIN_BITS, PA_SPIN_INTERLEAVED = 0, 1, 2
PA_FLAG_MHR = 1
PA_FLAG_HEATBATH = 2
PA_FLAG_LCG = 4
PA_STATS_AUTO, PA_STATS_EPILOGUE, PA_STATS_PASS = 0, 1, 2
STATS_PATHS = {"auto": PA_STATS_AUTO, "epilogue": PA_STATS_EPILOGUE, "pass": PA_STATS_PASS}
LAYOUTS = {"int8": PA_SPIN_INT8, "bits": PA_SPIN_BITS, "interleaved": PA_SPIN_INTERLEAVED}
SUPPORTED_L = (16, 32, 64, 128, 256)


class PaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class CapacityError(PaError):
    pass


class ExtinctError(PaError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("R", ctypes.c_int32), ("capacity", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("seed", ctypes.c_uint64), ("run_id", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


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


class ResampleInfo(ctypes.Structure):
    _fields_ = [("lnQ", ctypes.c_double), ("R_new", ctypes.c_int64), ("E_min", ctypes.c_int32)]


class StateInfo(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int64), ("step", ctypes.c_int32), ("sweeps", ctypes.c_uint64),
                ("beta", ctypes.c_double), ("lnZ", ctypes.c_double)]


class Schedule(ctypes.Structure):
    _fields_ = [("beta_f", ctypes.c_double), ("dbeta", ctypes.c_double), ("alpha_star", ctypes.c_double),
                ("alpha_tol", ctypes.c_double), ("theta", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("leader", ctypes.c_int32)]


PA_STEP_FIXED, PA_STEP_ADAPTIVE, PA_STEP_LEARNED, PA_STEP_FOLLOW = 0, 1, 2, 3
STEP_MODES = {"fixed": PA_STEP_FIXED, "adaptive": PA_STEP_ADAPTIVE, "learned": PA_STEP_LEARNED,
              "follow": PA_STEP_FOLLOW}


# Every symbol declared in include/pa.h, with its ctypes signature.
_P = ctypes.POINTER
_vp = ctypes.c_void_p
SIGNATURES = {
    "pa_workspace_bytes": (ctypes.c_size_t, [_P(Params)]),
    "pa_init": (ctypes.c_int, [_P(Params), _vp, ctypes.c_size_t, _vp, _P(_vp)]),
    "pa_sweep": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pa_weighted_average": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp]),
    "pa_anneal": (ctypes.c_int, [_vp, _P(Schedule), ctypes.c_int32, _vp, _vp, ctypes.c_int32, _P(ctypes.c_int32)]),
    "pa_resample": (ctypes.c_int, [_vp, ctypes.c_double, _P(ResampleInfo)]),
    "pa_adapt_beta": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, _P(ctypes.c_double), _P(ctypes.c_double)]),
    "pa_alpha": (ctypes.c_int, [_vp, ctypes.c_double, _P(ctypes.c_double)]),
    "pa_observables": (ctypes.c_int, [_vp, _P(Obs)]),
    "pa_reweight": (ctypes.c_int, [_vp, _P(ctypes.c_double), ctypes.c_int32, _P(Obs)]),
    "pa_state": (ctypes.c_int, [_vp, _P(StateInfo)]),
    "pa_free": (ctypes.c_int, [_vp]),
    "pa_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pa_last_error": (ctypes.c_char_p, [_vp]),
    "pa_download_population": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pa_download_replicas": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "pa_upload_population": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, ctypes.c_int32, ctypes.c_uint64,
                                            ctypes.c_double, ctypes.c_double]),
    "pa_download_counts": (ctypes.c_int, [_vp, _vp, _P(ctypes.c_int32)]),
    "pa_set_tie_queue_cap": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pa_set_stats_path": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pa_batch_init_ex": (ctypes.c_int, [_P(Params), _P(Schedule), ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp,
                                        _P(_vp)]),
    "pa_batch_waves_per_block": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int32)]),
    "pa_batch_set_tie_queue_cap": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pa_batch_workspace_bytes": (ctypes.c_size_t, [_P(Params), ctypes.c_int32]),
    "pa_batch_init": (ctypes.c_int, [_P(Params), _P(Schedule), ctypes.c_int32, _vp, ctypes.c_size_t, _vp, _P(_vp)]),
    "pa_batch_step": (ctypes.c_int, [_vp, _P(ctypes.c_int32)]),
    "pa_batch_run": (ctypes.c_int, [_vp]),
    "pa_batch_run_status": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pa_batch_state": (ctypes.c_int, [_vp, ctypes.c_int32, _P(StateInfo)]),
    "pa_batch_history": (ctypes.c_int, [_vp, ctypes.c_int32, _P(Obs), ctypes.c_int32, _P(ctypes.c_int32)]),
    "pa_batch_reweight": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_double), ctypes.c_int32, _P(Obs)]),
    "pa_batch_download_population": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp]),
    "pa_batch_free": (ctypes.c_int, [_vp]),
    "pa_batch_set_model": (ctypes.c_int, [_vp, _vp, _vp]),
    "pa_batch_training_pairs": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, _P(ctypes.c_int32)]),
    "pa_batch_features": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _P(ctypes.c_int32), _P(ctypes.c_float)]),
    "pa_batch_learned_stats": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    "pa_batch_choice_stats": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_double)]),
    "pa_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "pa_mlp_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_uint64, _vp, ctypes.c_size_t, _vp, _P(_vp)]),
    "pa_mlp_set_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "pa_mlp_get_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "pa_mlp_fit_norm": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32]),
    "pa_mlp_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, ctypes.c_int32]),
    "pa_mlp_gradient": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, _vp, _P(ctypes.c_float)]),
    "pa_mlp_train": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_uint64, _vp]),
    "pa_mlp_last_error": (ctypes.c_char_p, [_vp]),
    "pa_mlp_free": (ctypes.c_int, [_vp]),
    "pa_observables_static": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _vp, _vp, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, _vp, _P(Obs)]),
    "pa_static_scratch_bytes": (ctypes.c_size_t, []),
}

MLP_PARAMS, MLP_NORM = 4801, 18
PA_STATIC_MAX_R = 1 << 20

_lib = None


def lib():
    """Load libpa.so.  torch is imported first so that the library binds to the
    same HIP runtime instance torch uses."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpa.so is not built (run python paper_1703_03676_amd/build.py)")
        import torch  # noqa: F401  (binds the HIP runtime before libpa is loaded)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(status):
    return lib().pa_strerror(status).decode()


def _check(status, handle=None):
    if status == PA_OK:
        return
    msg = strerror(status)
    if handle:
        extra = lib().pa_last_error(handle)
        if extra:
            msg += ": " + extra.decode()
    if status == PA_ECAPACITY:
        raise CapacityError(status, msg)
    if status == PA_EEXTINCT:
        raise ExtinctError(status, msg)
    raise PaError(status, msg)


def make_params(L, R, seed, run_id=0, capacity=0, layout="bits", mhr=False, heatbath=False, lcg=False):
    return Params(L=int(L), R=int(R), capacity=int(capacity), layout=LAYOUTS[layout] if isinstance(layout, str) else int(layout),
                  seed=int(seed), run_id=int(run_id),
                  flags=(PA_FLAG_MHR if mhr else 0) | (PA_FLAG_HEATBATH if heatbath else 0) | (PA_FLAG_LCG if lcg else 0))


def workspace_bytes(params):
    return lib().pa_workspace_bytes(ctypes.byref(params))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _obs_struct(d):
    o = Obs()
    for name, _ in Obs._fields_:
        if name in ("sumM4_lo", "sumM4_hi"):
            continue
        if name in d:
            setattr(o, name, d[name])
    m4 = int(d.get("sumM4", 0))
    o.sumM4_lo, o.sumM4_hi = m4 & ((1 << 64) - 1), m4 >> 64
    return o


def weighted_average(runs, N):
    """Free-energy-weighted average of independent runs (lists of observable
    dicts at the same temperatures); N = L * L.  Host arithmetic in libpa."""
    nruns, nb = len(runs), len(runs[0]) if runs else 0
    if any(len(r) != nb for r in runs):
        raise PaError(PA_EINVAL, "runs measured at different numbers of temperatures")
    flat = (Obs * (nruns * nb))(*[_obs_struct(o) for r in runs for o in r])
    out = (Obs * max(nb, 1))()
    _check(lib().pa_weighted_average(int(N), nruns, nb, ctypes.cast(flat, _vp), ctypes.cast(out, _vp)))
    return [o.as_dict() for o in out[:nb]]


def observables_static(L, E, M, beta=0.0, lnZ=0.0, lnQ=0.0, stream=None):
    """pa_observables_static: observables of the population whose energies and
    magnetisations are the int32 device tensors E and M (same length R), with
    no allocation in the library (its static device array holds the
    statistics).  Returns the observables as a dict."""
    import torch
    if E.dtype != torch.int32 or M.dtype != torch.int32 or not E.is_cuda or not M.is_cuda:
        raise PaError(PA_EINVAL, "E and M must be int32 device tensors")
    if E.dim() != 1 or E.shape != M.shape or not E.is_contiguous() or not M.is_contiguous():
        raise PaError(PA_EINVAL, "E and M must be contiguous 1-d tensors of equal length")
    if E.shape[0] > PA_STATIC_MAX_R:
        raise PaError(PA_EINVAL, "pa_observables_static takes at most %d replicas (its static device scratch "
                                 "is sized for that); got %d" % (PA_STATIC_MAX_R, E.shape[0]))
    s = stream if stream is not None else torch.cuda.current_stream(E.device)
    o = Obs()
    with torch.cuda.device(E.device):
        _check(lib().pa_observables_static(int(L), int(E.shape[0]), ctypes.c_void_p(E.data_ptr()),
                                           ctypes.c_void_p(M.data_ptr()), float(beta), float(lnZ), float(lnQ),
                                           ctypes.c_void_p(s.cuda_stream), ctypes.byref(o)))
    return o.as_dict()


class Run:
    """One PA run on the current GPU (C-ABI handle + torch-owned workspace)."""

    def __init__(self, L, R, seed, run_id=0, capacity=0, layout="bits", mhr=False, stream=None, device=None,
                 heatbath=False, lcg=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: libpa runs on the GPU only")
        self.params = make_params(L, R, seed, run_id, capacity, layout, mhr, heatbath, lcg)
        nbytes = workspace_bytes(self.params)
        if nbytes == 0:
            raise PaError(PA_EINVAL, "invalid parameters")
        self.L, self.N, self.R = L, L * L, R
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        _check(lib().pa_init(ctypes.byref(self.params), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.capacity = self.params.capacity or default_capacity(R)

    def close(self):
        if getattr(self, "h", None):
            lib().pa_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # --- the method -------------------------------------------------------
    def sweep(self, nsweeps):
        _check(lib().pa_sweep(self.h, int(nsweeps)), self.h)

    def anneal(self, beta_f=1.0, dbeta=0.0, alpha_star=0.0, theta=1, mode="fixed", max_steps=1 << 30, cap=4096,
               sweep_times=False):
        """Temperature steps until beta_f (fixed dbeta or adaptive alpha_star),
        each resample + theta sweeps + measurement; returns the observables
        after every step (at most cap of them), and with sweep_times also the
        sweep launch durations in ms."""
        sched = make_schedule(beta_f=beta_f, dbeta=dbeta, alpha_star=alpha_star, theta=theta, mode=mode)
        out = (Obs * cap)()
        ms = np.zeros(cap, np.float32)
        n = ctypes.c_int32()
        st = lib().pa_anneal(self.h, ctypes.byref(sched), int(max_steps), ctypes.cast(out, _vp),
                             _ptr(ms) if sweep_times else None, int(cap), ctypes.byref(n))
        k = min(n.value, cap)
        res = [o.as_dict() for o in out[:k]]
        _check(st, self.h)
        return (res, ms[:k].tolist()) if sweep_times else res

    def resample(self, beta_next):
        info = ResampleInfo()
        _check(lib().pa_resample(self.h, float(beta_next), ctypes.byref(info)), self.h)
        return {"R_new": info.R_new, "lnQ": info.lnQ, "E_min": info.E_min}

    def adapt_beta(self, alpha_star, beta_f):
        b, a = ctypes.c_double(), ctypes.c_double()
        _check(lib().pa_adapt_beta(self.h, float(alpha_star), float(beta_f), ctypes.byref(b), ctypes.byref(a)), self.h)
        return b.value

    def alpha(self, beta_prime):
        a = ctypes.c_double()
        _check(lib().pa_alpha(self.h, float(beta_prime), ctypes.byref(a)), self.h)
        return a.value

    def observables(self):
        o = Obs()
        _check(lib().pa_observables(self.h, ctypes.byref(o)), self.h)
        return o.as_dict()

    def reweight(self, betas):
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        out = (Obs * max(len(betas), 1))()
        _check(lib().pa_reweight(self.h, betas.ctypes.data_as(_P(ctypes.c_double)), len(betas), out), self.h)
        return [out[k].as_dict() for k in range(len(betas))]

    def state(self):
        s = StateInfo()
        _check(lib().pa_state(self.h, ctypes.byref(s)), self.h)
        return {"R": s.R, "step": s.step, "sweeps": s.sweeps, "beta": s.beta, "lnZ": s.lnZ}

    # --- test hooks ---------------------------------------------------------
    def download_population(self):
        n = self.state()["R"]
        s = np.empty((n, self.L, self.L), np.int8)
        E = np.empty(n, np.int32)
        M = np.empty(n, np.int32)
        _check(lib().pa_download_population(self.h, _ptr(s), _ptr(E), _ptr(M)), self.h)
        return s, E, M

    def download_energies(self):
        """(E int32 [R_i], M int32 [R_i]) without the spins."""
        n = self.state()["R"]
        E = np.empty(n, np.int32)
        M = np.empty(n, np.int32)
        _check(lib().pa_download_population(self.h, None, _ptr(E), _ptr(M)), self.h)
        return E, M

    def download_replicas(self, idx):
        """Spins (int8 [n, L, L]), E and M of the replicas idx."""
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        n = len(idx)
        s = np.empty((n, self.L, self.L), np.int8)
        E = np.empty(n, np.int32)
        M = np.empty(n, np.int32)
        _check(lib().pa_download_replicas(self.h, _ptr(idx), n, _ptr(s), _ptr(E), _ptr(M)), self.h)
        return s, E, M

    def upload_population(self, spins, step=0, sweeps=0, beta=0.0, lnZ=0.0):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        assert spins.ndim == 3 and spins.shape[1:] == (self.L, self.L)
        _check(lib().pa_upload_population(self.h, spins.shape[0], _ptr(spins), int(step), int(sweeps),
                                          float(beta), float(lnZ)), self.h)

    def download_counts(self, capacity):
        buf = np.empty(capacity, np.uint32)
        n = ctypes.c_int32()
        _check(lib().pa_download_counts(self.h, _ptr(buf), ctypes.byref(n)), self.h)
        return buf[: n.value].copy()

    def set_tie_queue_cap(self, cap):
        """Limit the LDS-path tie queue to cap entries, one per word with a
        tied site (0: every lane decides its own ties); 128 or more restores
        the default."""
        _check(lib().pa_set_tie_queue_cap(self.h, int(cap)), self.h)

    def set_stats_path(self, path):
        """Where the statistics of a swept population are taken: "auto",
        "epilogue" (the sweep's epilogue) or "pass" (a separate pass)."""
        _check(lib().pa_set_stats_path(self.h, STATS_PATHS.get(path, path)), self.h)


def make_schedule(beta_f=1.0, dbeta=0.0, alpha_star=0.0, alpha_tol=0.0, theta=1, mode="fixed", leader=0):
    return Schedule(beta_f=float(beta_f), dbeta=float(dbeta), alpha_star=float(alpha_star),
                    alpha_tol=float(alpha_tol), theta=int(theta),
                    mode=STEP_MODES[mode] if isinstance(mode, str) else int(mode), leader=int(leader))


class BatchOptions(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32)]


class Batch:
    """Many independent PA runs advanced together (one graph replay per step).

    runs: list of dicts with keys L, R, seed and optional run_id, capacity,
    layout, mhr, heatbath, lcg.  schedules: list of dicts for make_schedule (or one dict for
    all runs).  waves_per_block: 0 (timed choice) or a forced sweep shape."""

    def __init__(self, runs, schedules, stream=None, device=None, waves_per_block=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: libpa runs on the GPU only")
        n = len(runs)
        if isinstance(schedules, dict):
            schedules = [schedules] * n
        self.specs = [dict(r) for r in runs]
        self.params = (Params * n)(*[make_params(r["L"], r["R"], r["seed"], r.get("run_id", 0), r.get("capacity", 0),
                                                 r.get("layout", "bits"), r.get("mhr", False),
                                                 r.get("heatbath", False), r.get("lcg", False)) for r in runs])
        self.sched = (Schedule * n)(*[make_schedule(**sc) for sc in schedules])
        nbytes = lib().pa_batch_workspace_bytes(self.params, n)
        if nbytes == 0:
            raise PaError(PA_EINVAL, "invalid run parameters")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        self.options = BatchOptions(waves_per_block=int(waves_per_block))
        _check(lib().pa_batch_init_ex(self.params, self.sched, n, ctypes.byref(self.options),
                                      ctypes.c_void_p(self.workspace.data_ptr()), nbytes, sp, ctypes.byref(h)))
        self.h = h
        self.n = n

    def close(self):
        if getattr(self, "h", None):
            lib().pa_batch_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def step(self):
        n = ctypes.c_int32()
        _check(lib().pa_batch_step(self.h, ctypes.byref(n)))
        return n.value

    def run(self):
        _check(lib().pa_batch_run(self.h))

    def status(self, run):
        return lib().pa_batch_run_status(self.h, int(run))

    def state(self, run):
        s = StateInfo()
        _check(lib().pa_batch_state(self.h, int(run), ctypes.byref(s)))
        return {"R": s.R, "step": s.step, "sweeps": s.sweeps, "beta": s.beta, "lnZ": s.lnZ}

    def history(self, run):
        n = ctypes.c_int32()
        _check(lib().pa_batch_history(self.h, int(run), None, 0, ctypes.byref(n)))
        out = (Obs * max(n.value, 1))()
        _check(lib().pa_batch_history(self.h, int(run), out, n.value, ctypes.byref(n)))
        return [out[k].as_dict() for k in range(n.value)]

    def reweight(self, run, betas):
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        out = (Obs * max(len(betas), 1))()
        _check(lib().pa_batch_reweight(self.h, int(run), betas.ctypes.data_as(_P(ctypes.c_double)), len(betas), out))
        return [out[k].as_dict() for k in range(len(betas))]

    def set_model(self, params, norm):
        params = np.ascontiguousarray(params, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float32)
        assert params.shape == (MLP_PARAMS,) and norm.shape == (MLP_NORM,)
        _check(lib().pa_batch_set_model(self.h, _ptr(params), _ptr(norm)))

    def training_pairs(self):
        n = ctypes.c_int32()
        _check(lib().pa_batch_training_pairs(self.h, None, None, 0, ctypes.byref(n)))
        x = np.empty((max(n.value, 1), 8), np.float32)
        t = np.empty(max(n.value, 1), np.float32)
        _check(lib().pa_batch_training_pairs(self.h, _ptr(x), _ptr(t), n.value, ctypes.byref(n)))
        return x[: n.value], t[: n.value]

    def features(self, run):
        x = np.empty(8, np.float32)
        v = ctypes.c_int32()
        pr = ctypes.c_float()
        _check(lib().pa_batch_features(self.h, int(run), _ptr(x), ctypes.byref(v), ctypes.byref(pr)))
        return x, bool(v.value), pr.value

    def waves_per_block(self, run):
        w = ctypes.c_int32()
        _check(lib().pa_batch_waves_per_block(self.h, int(run), ctypes.byref(w)))
        return w.value

    def set_tie_queue_cap(self, cap):
        _check(lib().pa_batch_set_tie_queue_cap(self.h, int(cap)))

    def choice_stats(self, run):
        """(overlap evaluations, host seconds) spent choosing run's temperatures."""
        n, t = ctypes.c_int64(), ctypes.c_double()
        _check(lib().pa_batch_choice_stats(self.h, int(run), ctypes.byref(n), ctypes.byref(t)))
        return n.value, t.value

    def learned_stats(self, run):
        p, a = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pa_batch_learned_stats(self.h, int(run), ctypes.byref(p), ctypes.byref(a)))
        return p.value, a.value

    def download_population(self, run):
        L = self.specs[run]["L"]
        n = self.state(run)["R"]
        s = np.empty((n, L, L), np.int8)
        E = np.empty(n, np.int32)
        M = np.empty(n, np.int32)
        _check(lib().pa_batch_download_population(self.h, int(run), _ptr(s), _ptr(E), _ptr(M)))
        return s, E, M


class Mlp:
    """The learned step proposer (MLP 8 -> 64 -> 64 -> 1) with its device
    training and inference kernels.  Data arguments are torch CUDA tensors."""

    def __init__(self, max_batch=1024, seed=0, stream=None, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: libpa runs on the GPU only")
        nbytes = lib().pa_mlp_workspace_bytes(int(max_batch))
        if nbytes == 0:
            raise PaError(PA_EINVAL, "invalid max_batch")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        _check(lib().pa_mlp_create(self.max_batch, int(seed), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().pa_mlp_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _err(self, st):
        if st != PA_OK:
            raise PaError(st, strerror(st) + ": " + lib().pa_mlp_last_error(self.h).decode())

    @staticmethod
    def _dev(t):
        import torch
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    def params(self):
        p = np.empty(MLP_PARAMS, np.float32)
        n = np.empty(MLP_NORM, np.float32)
        self._err(lib().pa_mlp_get_params(self.h, _ptr(p), _ptr(n)))
        return p, n

    def set_params(self, params=None, norm=None):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        n = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        self._err(lib().pa_mlp_set_params(self.h, None if p is None else _ptr(p), None if n is None else _ptr(n)))

    def fit_norm(self, x, t):
        self._err(lib().pa_mlp_fit_norm(self.h, self._dev(x), self._dev(t), int(x.shape[0])))

    def forward(self, x, bf16=True):
        import torch
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        self._err(lib().pa_mlp_forward(self.h, self._dev(x), int(x.shape[0]), self._dev(y), 1 if bf16 else 0))
        return y

    def gradient(self, x, t):
        g = np.empty(MLP_PARAMS, np.float32)
        loss = ctypes.c_float()
        self._err(lib().pa_mlp_gradient(self.h, self._dev(x), self._dev(t), int(x.shape[0]), _ptr(g),
                                        ctypes.byref(loss)))
        return g, loss.value

    def train(self, x, t, batch=256, epochs=10, lr=1e-2, momentum=0.9, seed=0):
        losses = np.empty(max(int(epochs), 1), np.float32)
        self._err(lib().pa_mlp_train(self.h, self._dev(x), self._dev(t), int(x.shape[0]), int(batch), int(epochs),
                                     float(lr), float(momentum), int(seed), _ptr(losses)))
        return losses[: int(epochs)]


def default_capacity(R):
    return R + int(np.ceil(10.0 * np.sqrt(R))) + 64
