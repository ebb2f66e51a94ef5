"""ctypes binding of libhz.so (C ABI in include/hz.h); argument marshalling only.

Every computation runs in the library's HIP kernels. torch provides device memory and
streams: vectors are complex128 CUDA tensors, the stream is torch's current stream.
torch is imported before the library so that both share one HIP runtime.
"""

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhz.so")

HZ_OK, HZ_EINVAL, HZ_ENOMEM, HZ_EDEVICE, HZ_ESINGULAR, HZ_EBUSY = range(6)
HZ_FP64, HZ_MIXED = 0, 1
OPS = {"A0": 0, "AEPS": 1, "JACOBI": 2, "RESTRICT": 3, "PROLONG": 4, "VCYCLE": 5,
       "COARSE_SOLVE": 6, "COARSE_A": 7, "RESID_RESTRICT": 8}
_PREC = {"fp64": HZ_FP64, "mixed": HZ_MIXED, HZ_FP64: HZ_FP64, HZ_MIXED: HZ_MIXED}


class HZError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hz status {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int), ("omega", ctypes.c_double), ("restart", ctypes.c_int),
                ("maxit", ctypes.c_int), ("tol", ctypes.c_double), ("prec", ctypes.c_int),
                ("timing", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("vcycles", ctypes.c_long), ("coarse_solves", ctypes.c_long),
                ("coarse_solve_ms", ctypes.c_double), ("factor_ms", ctypes.c_double),
                ("coarse_bytes", ctypes.c_double), ("graph_rounds", ctypes.c_long),
                ("coarse_systems", ctypes.c_long), ("factor_flop", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_res_true", ctypes.c_double), ("rel_res_est", ctypes.c_double),
                ("setup_s", ctypes.c_double), ("solve_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class C64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class EngineConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_int),
                ("setup_threads", ctypes.c_int)]


class EngineResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_long), ("status", ctypes.c_int), ("result", Result),
                ("queue_s", ctypes.c_double), ("latency_s", ctypes.c_double),
                ("message", ctypes.c_char * 120)]

    def as_dict(self):
        d = self.result.as_dict()
        d.update(id=self.id, status=self.status, queue_s=self.queue_s,
                 latency_s=self.latency_s, message=self.message.decode())
        return d


class EngineInfo(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int), ("admitted", ctypes.c_int),
                ("bytes_in_use", ctypes.c_size_t), ("hbm_budget", ctypes.c_size_t),
                ("submitted", ctypes.c_long), ("completed", ctypes.c_long)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SearchSample(ctypes.Structure):
    _fields_ = [("k", ctypes.c_double), ("h", ctypes.c_double), ("p", ctypes.c_int)]


class SearchResult(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("rho", ctypes.c_double),
                ("sigma_best", ctypes.c_double), ("evaluations", ctypes.c_int),
                ("status", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = ctypes.c_void_p
_SIGS = {
    "hz_default_options": (ctypes.c_int, [ctypes.POINTER(Options)]),
    "hz_create_problem": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int, C64,
                                         ctypes.POINTER(Options), _P, ctypes.POINTER(_P)]),
    "hz_problem_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_long),
                                       ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_size_t)]),
    "hz_footprint_estimate": (ctypes.c_size_t, [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                ctypes.POINTER(Options)]),
    "hz_planewave_rhs": (ctypes.c_int, [_P, ctypes.c_double, _P, _P]),
    "hz_create_problem_cells": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int,
                                               ctypes.POINTER(Options), _P, ctypes.POINTER(_P)]),
    "hz_gaussian_rhs": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _P, _P]),
    "hz_solve": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(Options), ctypes.POINTER(Result),
                                ctypes.POINTER(ctypes.c_double), _P]),
    "hz_apply": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_int, _P]),
    "hz_apply_noalloc": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_int, _P]),
    "hz_solve_batched": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_P),
                                        ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(Options),
                                        ctypes.POINTER(Result), _P]),
    "hz_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                   ctypes.c_int, ctypes.POINTER(Options)]),
    "hz_problem_stats": (ctypes.c_int, [_P, ctypes.POINTER(Stats), ctypes.c_int]),
    "hz_destroy_problem": (None, [_P]),
    "hz_engine_default_config": (ctypes.c_int, [ctypes.POINTER(EngineConfig)]),
    "hz_engine_create": (ctypes.c_int, [ctypes.POINTER(EngineConfig), ctypes.POINTER(Options),
                                        ctypes.POINTER(_P)]),
    "hz_engine_submit": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int, C64,
                                        ctypes.c_double, _P, _P, ctypes.c_long]),
    "hz_engine_poll": (ctypes.c_int, [_P, ctypes.POINTER(EngineResult), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "hz_engine_info": (ctypes.c_int, [_P, ctypes.POINTER(EngineInfo)]),
    "hz_engine_destroy": (None, [_P]),
    "hz_last_error": (ctypes.c_char_p, []),
    "hz_shift_search": (ctypes.c_int, [ctypes.POINTER(SearchSample), ctypes.c_int,
                                       ctypes.POINTER(_P), ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.POINTER(EngineConfig),
                                       ctypes.POINTER(Options), ctypes.POINTER(SearchResult)]),
}

_lib = None


def lib():
    """Loads libhz.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2104_01439_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != HZ_OK:
        raise HZError(status, lib().hz_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


def options(nu=2, omega=0.6, restart=50, maxit=5000, tol=1e-8, prec="fp64", timing=False):
    o = Options()
    _check(lib().hz_default_options(ctypes.byref(o)))
    o.nu, o.omega, o.restart, o.maxit, o.tol, o.prec = nu, omega, restart, maxit, tol, _PREC[prec]
    o.timing = 1 if timing else 0
    return o


def footprint_estimate(k, h, p, **kw):
    o = options(**kw)
    return int(lib().hz_footprint_estimate(k, h, p, ctypes.byref(o)))


def batch_workspace_bytes(h, p, nprob, nrhs_per_prob, **kw):
    o = options(**kw)
    return int(lib().hz_batch_workspace_bytes(h, p, nprob, nrhs_per_prob, ctypes.byref(o)))


def sizes(n, p):
    """(fine lattice M, fine dofs, coarse lattice Mc, coarse dofs) for n cells per side."""
    M, Mc = p * n + 1, p * (n // 2) + 1
    return M, M * M, Mc, Mc * Mc


class Problem:
    """create_problem(k, h, p, s): tables, coarse factor and Krylov workspace on the GPU."""

    def __init__(self, k, h, p, s, nu=2, omega=0.6, restart=50, maxit=5000, tol=1e-8,
                 prec="fp64", timing=False):
        self.k, self.h, self.p, self.s = float(k), float(h), int(p), complex(s)
        self.n = int(round(1.0 / h))
        self.opts = options(nu, omega, restart, maxit, tol, prec, timing)
        self._h = ctypes.c_void_p()
        _check(lib().hz_create_problem(self.k, self.h, self.p, C64(self.s.real, self.s.imag),
                                       ctypes.byref(self.opts), _stream(), ctypes.byref(self._h)))
        self.M, self.N, self.Mc, self.Nc = sizes(self.n, self.p)

    @classmethod
    def cells(cls, k_cell, s_cell, h, p, nu=2, omega=0.6, restart=50, maxit=5000, tol=1e-8,
              prec="fp64", timing=False):
        """create_problem_cells: k and the shift multiplier per cell of the n x n fine mesh
        (arrays indexed [row j (y), column i (x)])."""
        self = cls.__new__(cls)
        self.h, self.p = float(h), int(p)
        self.n = int(round(1.0 / h))
        kc = np.ascontiguousarray(k_cell, dtype=np.float64)
        sc = np.ascontiguousarray(s_cell, dtype=np.complex128)
        if kc.shape != (self.n, self.n) or sc.shape != (self.n, self.n):
            raise ValueError(f"cell arrays must be {self.n} x {self.n}")
        self.k, self.s = float(kc.max()), None
        self.opts = options(nu, omega, restart, maxit, tol, prec, timing)
        self._h = ctypes.c_void_p()
        _check(lib().hz_create_problem_cells(kc.ctypes.data, sc.ctypes.data, self.h, self.p,
                                             ctypes.byref(self.opts), _stream(),
                                             ctypes.byref(self._h)))
        self.M, self.N, self.Mc, self.Nc = sizes(self.n, self.p)
        return self

    @property
    def handle(self):
        return self._h

    def info(self):
        n, nc, fp = ctypes.c_long(), ctypes.c_long(), ctypes.c_size_t()
        _check(lib().hz_problem_info(self._h, ctypes.byref(n), ctypes.byref(nc), ctypes.byref(fp)))
        return {"n_dofs": n.value, "n_coarse": nc.value, "footprint_bytes": fp.value}

    def stats(self, reset=False):
        st = Stats()
        _check(lib().hz_problem_stats(self._h, ctypes.byref(st), 1 if reset else 0))
        return st.as_dict()

    def empty(self, coarse=False):
        return torch.empty(self.Nc if coarse else self.N, dtype=torch.complex128, device="cuda")

    def planewave_rhs(self, theta, out=None):
        F = self.empty() if out is None else out
        _check(lib().hz_planewave_rhs(self._h, float(theta), _ptr(F), _stream()))
        return F

    def gaussian_rhs(self, center, amp=2.0, width=1000.0, out=None):
        F = self.empty() if out is None else out
        _check(lib().hz_gaussian_rhs(self._h, float(center[0]), float(center[1]), float(amp),
                                     float(width), _ptr(F), _stream()))
        return F

    def solve(self, F, u=None, tol=None, restart=None, maxit=None, prec=None, history=True):
        o = Options.from_buffer_copy(self.opts)
        if tol is not None:
            o.tol = tol
        if restart is not None:
            o.restart = restart
        if maxit is not None:
            o.maxit = maxit
        if prec is not None:
            o.prec = _PREC[prec]
        u = self.empty() if u is None else u
        res = Result()
        hist = (ctypes.c_double * o.maxit)() if history else None
        _check(lib().hz_solve(self._h, _ptr(F), _ptr(u), ctypes.byref(o), ctypes.byref(res),
                              hist, _stream()))
        out = res.as_dict()
        if history:
            out["hist"] = list(hist[: res.iterations])
        return u, out

    def apply(self, op, x, f=None, prec="fp64", y=None, noalloc=False):
        """y = op(x[, f]) by hz_apply, or by hz_apply_noalloc (the library allocates nothing;
        y is allocated here unless given)."""
        op_id = OPS[op]
        coarse_out = op in ("RESTRICT", "COARSE_SOLVE", "COARSE_A", "RESID_RESTRICT")
        y = self.empty(coarse=coarse_out) if y is None else y
        fn = lib().hz_apply_noalloc if noalloc else lib().hz_apply
        _check(fn(self._h, op_id, _ptr(x), _ptr(f), _ptr(y), _PREC[prec], _stream()))
        return y

    def close(self):
        if self._h:
            lib().hz_destroy_problem(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batched(problems, Fs, nrhs_per_prob, us=None, tol=None, restart=None, maxit=None,
                  prec=None):
    """Lockstep solves: Fs[i*nrhs + r] with problems[i]; returns (us, [result dict])."""
    o = Options.from_buffer_copy(problems[0].opts)
    if tol is not None:
        o.tol = tol
    if restart is not None:
        o.restart = restart
    if maxit is not None:
        o.maxit = maxit
    if prec is not None:
        o.prec = _PREC[prec]
    nsol = len(problems) * nrhs_per_prob
    assert len(Fs) == nsol
    us = [problems[i // nrhs_per_prob].empty() for i in range(nsol)] if us is None else us
    P = (ctypes.c_void_p * len(problems))(*[p.handle.value for p in problems])
    FF = (ctypes.c_void_p * nsol)(*[F.data_ptr() for F in Fs])
    UU = (ctypes.c_void_p * nsol)(*[u.data_ptr() for u in us])
    res = (Result * nsol)()
    _check(lib().hz_solve_batched(P, len(problems), FF, nrhs_per_prob, UU, ctypes.byref(o), res,
                                  _stream()))
    return us, [r.as_dict() for r in res]


class Engine:
    """Serving engine (continuous batching of independent solves, admission by device
    memory); see hz_engine_* in include/hz.h. Solutions land in complex128 CUDA tensors
    that the caller provides or that submit() allocates; they are complete once poll()
    has returned the request."""

    def __init__(self, hbm_budget=0, max_active=64, setup_threads=2, **opts):
        self.opts = options(**opts)
        c = EngineConfig()
        _check(lib().hz_engine_default_config(ctypes.byref(c)))
        c.hbm_budget, c.max_active, c.setup_threads = int(hbm_budget), max_active, setup_threads
        self._h = ctypes.c_void_p()
        _check(lib().hz_engine_create(ctypes.byref(c), ctypes.byref(self.opts), ctypes.byref(self._h)))
        self._out = {}

    def submit(self, req_id, k, h, p, s, theta=0.0, F=None, u=None):
        n = int(round(1.0 / h))
        if u is None:
            u = torch.empty(sizes(n, p)[1], dtype=torch.complex128, device="cuda")
        self._out[req_id] = (u, F)
        if F is not None:
            # the engine copies F on its own stream: the work producing F must be complete
            torch.cuda.current_stream().synchronize()
        _check(lib().hz_engine_submit(self._h, float(k), float(h), int(p),
                                      C64(complex(s).real, complex(s).imag), float(theta),
                                      _ptr(F), _ptr(u), int(req_id)))
        return u

    def poll(self, max_results=256, wait_ms=0):
        """[(result dict, u tensor)] of finished requests."""
        buf = (EngineResult * max_results)()
        n = ctypes.c_int()
        _check(lib().hz_engine_poll(self._h, buf, max_results, ctypes.byref(n), int(wait_ms)))
        out = []
        for i in range(n.value):
            d = buf[i].as_dict()
            u, _ = self._out.pop(d["id"], (None, None))
            out.append((d, u))
        return out

    def info(self):
        i = EngineInfo()
        _check(lib().hz_engine_info(self._h, ctypes.byref(i)))
        return i.as_dict()

    def close(self):
        if self._h:
            lib().hz_engine_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shift_search(samples, Fs, sigma_lo=1.0, sigma_hi=2.0, tol=1e-2, solve_tol=1e-8, maxit=50,
                 restart=50, prec="fp64", max_active=64, setup_threads=4, hbm_budget=0):
    """Golden-section search of the shift exponent for every sample (hz_shift_search):
    samples = [(k, h, p)], Fs = matching complex128 CUDA right-hand sides. Returns one result
    dict per sample (sigma, rho, sigma_best, evaluations, status)."""
    n = len(samples)
    assert len(Fs) == n and n > 0
    S = (SearchSample * n)(*[SearchSample(float(k), float(h), int(p)) for k, h, p in samples])
    FF = (ctypes.c_void_p * n)(*[_ptr(F).value for F in Fs])
    o = options(restart=restart, maxit=maxit, tol=solve_tol, prec=prec)
    c = EngineConfig()
    _check(lib().hz_engine_default_config(ctypes.byref(c)))
    c.hbm_budget, c.max_active, c.setup_threads = int(hbm_budget), max_active, setup_threads
    out = (SearchResult * n)()
    # the engine reads the right-hand sides on its own streams
    torch.cuda.current_stream().synchronize()
    _check(lib().hz_shift_search(S, n, FF, sigma_lo, sigma_hi, tol, ctypes.byref(c),
                                 ctypes.byref(o), out))
    return [r.as_dict() for r in out]
