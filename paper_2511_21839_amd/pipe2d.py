"""ctypes binding of the 2D conducting-pipe PIC (include/dpic2d.h) and of
the Twiss / matching library (include/dtwiss.h). Argument marshalling only;
the kernels do the arithmetic, PyTorch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import dpic

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_I64 = ctypes.POINTER(ctypes.c_int64)

GRID_RHO, GRID_PHI, GRID_E = 0, 1, 2
STAGE_DEPOSIT, STAGE_SOLVE, STAGE_FIELD = 0, 1, 2


class dpic2d_dims(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int64), ("ntan", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("flags", ctypes.c_int32)]


SYMBOLS_2D = (
    "dpic2d_query_workspace", "dpic2d_create", "dpic2d_destroy", "dpic2d_last_error", "dpic2d_set_beam",
    "dpic2d_set_pipe", "dpic2d_set_lattice", "dpic2d_set_params", "dpic2d_init_beam", "dpic2d_step",
    "dpic2d_read_emittance", "dpic2d_read_particles", "dpic2d_stage", "dpic2d_read_grid", "dpic2d_write_grid",
    "dpic2d_counters",
)
SYMBOLS_TWISS = ("dtwiss_query_workspace", "dtwiss_eval", "dtwiss_match")

_SIGS = {
    "dpic2d_query_workspace": ([ctypes.POINTER(dpic2d_dims), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "dpic2d_create": ([ctypes.POINTER(dpic2d_dims), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "dpic2d_destroy": ([_P], ctypes.c_int),
    "dpic2d_last_error": ([_P, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "dpic2d_set_beam": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double], ctypes.c_int),
    "dpic2d_set_pipe": ([_P, ctypes.c_double, ctypes.c_double], ctypes.c_int),
    "dpic2d_set_lattice": ([_P, ctypes.c_int, _I, _I, _D, _D, _I, _I, ctypes.c_int], ctypes.c_int),
    "dpic2d_set_params": ([_P, ctypes.c_int, _D, _D], ctypes.c_int),
    "dpic2d_init_beam": ([_P, ctypes.c_int64, _P, _D, _D], ctypes.c_int),
    "dpic2d_step": ([_P, ctypes.c_int], ctypes.c_int),
    "dpic2d_read_emittance": ([_P, _D], ctypes.c_int),
    "dpic2d_read_particles": ([_P, _D], ctypes.c_int),
    "dpic2d_stage": ([_P, ctypes.c_int], ctypes.c_int),
    "dpic2d_read_grid": ([_P, ctypes.c_int, _D], ctypes.c_int),
    "dpic2d_write_grid": ([_P, ctypes.c_int, _D], ctypes.c_int),
    "dpic2d_counters": ([_P, _I64, _I64], ctypes.c_int),
    "dtwiss_query_workspace": ([ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "dtwiss_eval": ([_P, ctypes.c_size_t, _P, ctypes.c_int, _I, _D, _D, _I, _I, ctypes.c_int, ctypes.c_int, _D, _D, _D,
                     _D, _D], ctypes.c_int),
    "dtwiss_match": ([_P, ctypes.c_size_t, _P, ctypes.c_int, _I, _D, _D, _I, _I, ctypes.c_int, _D, _D, _D,
                      ctypes.c_double, ctypes.c_int, _D, _D, _I, _D], ctypes.c_int),
}

_bound = False


def lib():
    global _bound
    L = dpic.lib()
    if not _bound:
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _bound = True
    return L


def _check(ctx, rc, err_fn="dpic2d_last_error"):
    if rc != dpic.DPIC_OK:
        msg = ""
        if ctx:
            buf = ctypes.create_string_buffer(512)
            getattr(lib(), err_fn)(ctx, buf, 512)
            msg = buf.value.decode(errors="replace")
        raise dpic.DpicError(rc, msg)


def _d(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


class Pipe2D:
    """One 2D pipe context with its torch-owned workspace on torch's current stream."""

    def __init__(self, n_particles: int, ntan: int, nx: int, ny: int, device: str = "cuda"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("dpic2d needs a ROCm GPU")
        self.torch = torch
        self.ntan, self.nx, self.ny = int(ntan), int(nx), int(ny)
        self.dims = dpic2d_dims(int(n_particles), self.ntan, self.nx, self.ny, 0)
        b = ctypes.c_size_t(0)
        _check(None, lib().dpic2d_query_workspace(ctypes.byref(self.dims), ctypes.byref(b)))
        self.workspace = torch.empty(b.value + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream()
        ctx = _P()
        _check(None, lib().dpic2d_create(ctypes.byref(self.dims), _P(ptr), b.value,
                                         _P(self.stream.cuda_stream) if self.stream.cuda_stream else None,
                                         ctypes.byref(ctx)))
        self.ctx = ctx
        self.n = 0

    def close(self):
        if getattr(self, "ctx", None):
            lib().dpic2d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_beam(self, kinetic_eV, rest_eV, charge_e, current_A):
        _check(self.ctx, lib().dpic2d_set_beam(self.ctx, kinetic_eV, rest_eV, charge_e, current_A))

    def set_pipe(self, a, b):
        _check(self.ctx, lib().dpic2d_set_pipe(self.ctx, a, b))

    def set_lattice(self, kind, n_steps, L, k, L_param, k_param, n_periods):
        kind, n_steps, L_param, k_param = _i(kind), _i(n_steps), _i(L_param), _i(k_param)
        L, k = _d(L), _d(k)
        _check(self.ctx, lib().dpic2d_set_lattice(self.ctx, len(kind), kind.ctypes.data_as(_I), n_steps.ctypes.data_as(_I),
                                                  _dp(L), _dp(k), L_param.ctypes.data_as(_I), k_param.ctypes.data_as(_I),
                                                  int(n_periods)))

    def set_params(self, p, seed=None):
        p = _d(p)
        s = _d(seed) if seed is not None and np.size(seed) else None
        _check(self.ctx, lib().dpic2d_set_params(self.ctx, len(p), _dp(p), _dp(s)))

    def init_beam(self, xi, sigma, sigma_seed=None):
        xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 4)
        self._xi = self.torch.from_numpy(xi).to(self.workspace.device)
        self.n = xi.shape[0]
        _check(self.ctx, lib().dpic2d_init_beam(self.ctx, self.n, _P(self._xi.data_ptr()), _dp(_d(sigma)),
                                                _dp(_d(sigma_seed))))

    def step(self, n):
        _check(self.ctx, lib().dpic2d_step(self.ctx, int(n)))

    def stage(self, s):
        _check(self.ctx, lib().dpic2d_stage(self.ctx, int(s)))

    def emittance(self):
        out = np.empty((2, self.ntan + 1))
        _check(self.ctx, lib().dpic2d_read_emittance(self.ctx, _dp(out)))
        return out

    def particles(self):
        out = np.empty((self.n, 4, self.ntan + 1))
        _check(self.ctx, lib().dpic2d_read_particles(self.ctx, _dp(out)))
        return out

    def _shape(self, which):
        base = (self.nx + 1, self.ny + 1)
        return base + ((2,) if which == GRID_E else ()) + (self.ntan + 1,)

    def read_grid(self, which):
        out = np.empty(self._shape(which))
        _check(self.ctx, lib().dpic2d_read_grid(self.ctx, int(which), _dp(out)))
        return out

    def write_grid(self, which, data):
        data = _d(data)
        _check(self.ctx, lib().dpic2d_write_grid(self.ctx, int(which), _dp(data)))

    def counters(self):
        lost, steps = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(self.ctx, lib().dpic2d_counters(self.ctx, ctypes.byref(lost), ctypes.byref(steps)))
        return lost.value, steps.value


class Twiss:
    """Twiss evaluations and matching on the GPU for one line of elements."""

    def __init__(self, kind, L, k, L_param, k_param, nmax: int = 1, device: str = "cuda"):
        import torch

        self.torch = torch
        self.kind, self.L_param, self.k_param = _i(kind), _i(L_param), _i(k_param)
        self.L, self.k = _d(L), _d(k)
        self.nmax = int(nmax)
        b = ctypes.c_size_t(0)
        _check(None, lib().dtwiss_query_workspace(self.nmax, ctypes.byref(b)))
        self.bytes = b.value
        self.workspace = torch.empty(b.value + 256, dtype=torch.uint8, device=device)
        self.ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream().cuda_stream

    def _line(self):
        return (len(self.kind), self.kind.ctypes.data_as(_I), _dp(self.L), _dp(self.k),
                self.L_param.ctypes.data_as(_I), self.k_param.ctypes.data_as(_I))

    def eval(self, p, twiss0=None, target=None):
        """p [nb][np] -> twiss [nb][4][1+np] (and f [nb][1+np] with a target)."""
        p = _d(np.atleast_2d(p))
        nb, npar = p.shape
        tw = np.empty((nb, 4, npar + 1))
        f = np.empty((nb, npar + 1)) if target is not None else None
        t0, tg = _d(twiss0), _d(target)
        _check(None, lib().dtwiss_eval(_P(self.ptr), self.bytes, _P(self.stream) if self.stream else None, *self._line(),
                                       npar, nb, _dp(p), _dp(t0), _dp(tg), _dp(tw), _dp(f)))
        return (tw, f) if target is not None else tw

    def match(self, p0, twiss0, target, tol=1e-12, max_eval=2000):
        """BFGS on the matching objective and its dual-number gradient."""
        p0 = _d(p0)
        out = np.empty_like(p0)
        f = ctypes.c_double(0.0)
        ne = ctypes.c_int(0)
        hist = np.zeros(max_eval)
        _check(None, lib().dtwiss_match(_P(self.ptr), self.bytes, _P(self.stream) if self.stream else None,
                                        *self._line(), len(p0), _dp(p0), _dp(_d(twiss0)), _dp(_d(target)), tol,
                                        int(max_eval), _dp(out), ctypes.byref(f), ctypes.byref(ne), _dp(hist)))
        return out, f.value, ne.value, hist[:ne.value]
