"""ctypes binding of libdpic.so (the C ABI in include/dpic.h).

Argument marshalling only: every function forwards to the entry point of the
same name; the HIP kernels do all the arithmetic. PyTorch supplies device
memory (the caller-owned workspace) and the stream. The binding raises
instead of falling back to anything else when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpic.so")

DPIC_OK = 0
DPIC_EINVAL = -1
DPIC_ESTATE = -2
DPIC_EHIP = -3
DPIC_ENONFINITE = -4
DPIC_EUNSUPPORTED = -5

GRID_RHO, GRID_PHI, GRID_E = 0, 1, 2
STAGE_DEPOSIT, STAGE_SOLVE, STAGE_FIELD = 0, 1, 2
OPT_SORT_EVERY, OPT_STAGE_TIMING, OPT_CHUNK, OPT_PART_BLOCKS, OPT_GRAPH, OPT_CHECK_FINITE = 1, 2, 3, 4, 5, 6
OPT_DETERMINISTIC = 7
SEG = 1024  # each setting of a batch starts on a multiple of this many storage slots
N_STAGE_TIMERS = 4
STAGE_TIMER_NAMES = ("particles", "solve", "field", "sort")

_ERRNAMES = {
    DPIC_EINVAL: "DPIC_EINVAL", DPIC_ESTATE: "DPIC_ESTATE", DPIC_EHIP: "DPIC_EHIP",
    DPIC_ENONFINITE: "DPIC_ENONFINITE", DPIC_EUNSUPPORTED: "DPIC_EUNSUPPORTED",
}

# exported symbols, in header order (the CPU tests check that each is present)
SYMBOLS = (
    "dpic_version", "dpic_query_workspace", "dpic_create", "dpic_destroy", "dpic_last_error",
    "dpic_set_beam", "dpic_set_grid", "dpic_set_lattice", "dpic_set_params", "dpic_set_params_batch",
    "dpic_init_beam", "dpic_init_beam_batch", "dpic_step", "dpic_read_moments", "dpic_read_emittance",
    "dpic_read_emittance_noalloc", "dpic_read_particles", "dpic_counters", "dpic_batch_counters", "dpic_stage", "dpic_read_grid",
    "dpic_write_grid", "dpic_state_bytes", "dpic_save_state", "dpic_load_state", "dpic_set_option",
    "dpic_get_option", "dpic_autotune", "dpic_stage_times",
    "dpic_adjoint_query", "dpic_adjoint_bind", "dpic_adjoint_backward",
)


class DpicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class dpic_dims(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int64), ("ntan", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("nbatch", ctypes.c_int32)]


_lib = None

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_I64 = ctypes.POINTER(ctypes.c_int64)

_SIGS = {
    "dpic_version": ([], ctypes.c_int),
    "dpic_query_workspace": ([ctypes.POINTER(dpic_dims), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "dpic_create": ([ctypes.POINTER(dpic_dims), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "dpic_destroy": ([_P], ctypes.c_int),
    "dpic_last_error": ([_P, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "dpic_set_beam": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double], ctypes.c_int),
    "dpic_set_grid": ([_P, _D, _D], ctypes.c_int),
    "dpic_set_lattice": ([_P, ctypes.c_int, _I, _I, _D, _D, _I, _I, ctypes.c_int], ctypes.c_int),
    "dpic_set_params": ([_P, ctypes.c_int, _D, _D], ctypes.c_int),
    "dpic_set_params_batch": ([_P, ctypes.c_int, ctypes.c_int, _D, _D], ctypes.c_int),
    "dpic_init_beam": ([_P, ctypes.c_int64, _P, _D, _D], ctypes.c_int),
    "dpic_init_beam_batch": ([_P, ctypes.c_int, _I64, _P, _D, _D], ctypes.c_int),
    "dpic_step": ([_P, ctypes.c_int], ctypes.c_int),
    "dpic_read_moments": ([_P, _D], ctypes.c_int),
    "dpic_read_emittance": ([_P, ctypes.c_int, _D], ctypes.c_int),
    "dpic_read_particles": ([_P, _D], ctypes.c_int),
    "dpic_counters": ([_P, _I64, _I64, _D], ctypes.c_int),
    "dpic_batch_counters": ([_P, _I64], ctypes.c_int),
    "dpic_stage": ([_P, ctypes.c_int], ctypes.c_int),
    "dpic_read_grid": ([_P, ctypes.c_int, _D], ctypes.c_int),
    "dpic_write_grid": ([_P, ctypes.c_int, _D], ctypes.c_int),
    "dpic_state_bytes": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "dpic_save_state": ([_P, _P], ctypes.c_int),
    "dpic_load_state": ([_P, _P], ctypes.c_int),
    "dpic_set_option": ([_P, ctypes.c_int, ctypes.c_int64], ctypes.c_int),
    "dpic_get_option": ([_P, ctypes.c_int, _I64], ctypes.c_int),
    "dpic_autotune": ([_P, _P, ctypes.c_size_t, ctypes.c_int, _I64, _D], ctypes.c_int),
    "dpic_stage_times": ([_P, _D, _I64], ctypes.c_int),
    "dpic_read_emittance_noalloc": ([_P, ctypes.c_int, _P], ctypes.c_int),
    "dpic_adjoint_query": ([ctypes.POINTER(dpic_dims), ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                           ctypes.c_int),
    "dpic_adjoint_bind": ([_P, _P, ctypes.c_size_t, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "dpic_adjoint_backward": ([_P, _D, _D, _D], ctypes.c_int),
}


def lib() -> ctypes.CDLL:
    """Load libdpic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2511_21839_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


def _f64(a, shape=None) -> np.ndarray:
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        out = out.reshape(shape)
    return out


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _check(ctx, rc: int):
    if rc != DPIC_OK:
        msg = ""
        if ctx:
            buf = ctypes.create_string_buffer(512)
            lib().dpic_last_error(ctx, buf, 512)
            msg = buf.value.decode(errors="replace")
        raise DpicError(rc, msg)


# ---------------------------------------------------------------- one-to-one wrappers
def dpic_version() -> int:
    return lib().dpic_version()


def make_dims(n_particles: int, ntan: int, grid: Sequence[int], nbatch: int = 1) -> dpic_dims:
    return dpic_dims(int(n_particles), int(ntan), int(grid[0]), int(grid[1]), int(grid[2]), 0, int(nbatch))


def batch_capacity(ns: Sequence[int]) -> int:
    """Storage slots that settings with these particle counts need."""
    ns = [int(v) for v in ns]
    return sum((v + SEG - 1) // SEG * SEG for v in ns[:-1]) + (ns[-1] if ns else 0)


def dpic_query_workspace(dims: dpic_dims) -> int:
    b = ctypes.c_size_t(0)
    _check(None, lib().dpic_query_workspace(ctypes.byref(dims), ctypes.byref(b)))
    return b.value


def dpic_create(dims: dpic_dims, workspace_ptr: int, workspace_bytes: int, stream: int):
    ctx = _P()
    _check(None, lib().dpic_create(ctypes.byref(dims), _P(workspace_ptr), workspace_bytes,
                                   _P(stream) if stream else None, ctypes.byref(ctx)))
    return ctx


def dpic_destroy(ctx) -> None:
    _check(None, lib().dpic_destroy(ctx))


def dpic_set_beam(ctx, kinetic_eV: float, rest_eV: float, charge_e: float, bunch_charge_C: float):
    _check(ctx, lib().dpic_set_beam(ctx, kinetic_eV, rest_eV, charge_e, bunch_charge_C))


def dpic_set_grid(ctx, lo, hi):
    lo, hi = _f64(lo, (3,)), _f64(hi, (3,))
    _check(ctx, lib().dpic_set_grid(ctx, _dp(lo), _dp(hi)))


def dpic_set_lattice(ctx, kind, n_steps, L, k, L_param, k_param, n_periods: int):
    kind, n_steps = _i32(kind), _i32(n_steps)
    L, k = _f64(L), _f64(k)
    L_param, k_param = _i32(L_param), _i32(k_param)
    n = len(kind)
    for a in (n_steps, L, k, L_param, k_param):
        if len(a) != n:
            raise ValueError("lattice arrays must have one entry per element")
    _check(ctx, lib().dpic_set_lattice(ctx, n, kind.ctypes.data_as(_I), n_steps.ctypes.data_as(_I),
                                       _dp(L), _dp(k), L_param.ctypes.data_as(_I),
                                       k_param.ctypes.data_as(_I), int(n_periods)))


def dpic_set_params(ctx, p, seed=None, ntan: Optional[int] = None):
    p = _f64(p)
    s = None
    if seed is not None:
        s = _f64(seed)
        if s.size == 0:
            s = None
    _check(ctx, lib().dpic_set_params(ctx, len(p), _dp(p), _dp(s)))


def dpic_set_params_batch(ctx, p, seed=None):
    p = _f64(p)
    if p.ndim != 2:
        raise ValueError("p must be [nbatch][np]")
    s = None
    if seed is not None:
        s = _f64(seed)
        if s.size == 0:
            s = None
    _check(ctx, lib().dpic_set_params_batch(ctx, p.shape[0], p.shape[1], _dp(p), _dp(s)))


def dpic_init_beam_batch(ctx, ns, xi_dev_ptr: int, sigma, sigma_seed=None):
    n = np.ascontiguousarray(np.asarray(ns, dtype=np.int64))
    sigma = _f64(sigma, (len(n), 6))
    ss = None if sigma_seed is None else _f64(sigma_seed)
    _check(ctx, lib().dpic_init_beam_batch(ctx, len(n), n.ctypes.data_as(_I64), _P(xi_dev_ptr) if xi_dev_ptr else None,
                                           _dp(sigma), _dp(ss)))


def dpic_init_beam(ctx, n: int, xi_dev_ptr: int, sigma, sigma_seed=None):
    sigma = _f64(sigma, (6,))
    ss = None if sigma_seed is None else _f64(sigma_seed)
    _check(ctx, lib().dpic_init_beam(ctx, int(n), _P(xi_dev_ptr) if xi_dev_ptr else None, _dp(sigma), _dp(ss)))


def dpic_step(ctx, n: int):
    _check(ctx, lib().dpic_step(ctx, int(n)))


def dpic_read_moments(ctx, ntan: int, nbatch: int = 1) -> np.ndarray:
    out = np.empty((nbatch, 3, 5, ntan + 1))
    _check(ctx, lib().dpic_read_moments(ctx, _dp(out)))
    return out


def dpic_read_emittance(ctx, ntan: int, centred: bool = False, nbatch: int = 1) -> np.ndarray:
    out = np.empty((nbatch, 3, ntan + 1))
    _check(ctx, lib().dpic_read_emittance(ctx, int(bool(centred)), _dp(out)))
    return out


def dpic_read_emittance_noalloc(ctx, centred: bool, out_dev_ptr: int):
    """Emittances into caller device memory [B][3][1+ntan] (float64),
    asynchronous, with no allocation (the library's static scratch)."""
    _check(ctx, lib().dpic_read_emittance_noalloc(ctx, int(bool(centred)), _P(out_dev_ptr)))


def dpic_read_particles(ctx, n: int, ntan: int) -> np.ndarray:
    out = np.empty((n, 6, ntan + 1))
    _check(ctx, lib().dpic_read_particles(ctx, _dp(out)))
    return out


def dpic_counters(ctx):
    oob, steps = ctypes.c_int64(0), ctypes.c_int64(0)
    ext = np.zeros(3)
    _check(ctx, lib().dpic_counters(ctx, ctypes.byref(oob), ctypes.byref(steps), _dp(ext)))
    return oob.value, steps.value, ext


def dpic_batch_counters(ctx, nbatch: int) -> np.ndarray:
    out = np.zeros(nbatch, dtype=np.int64)
    _check(ctx, lib().dpic_batch_counters(ctx, out.ctypes.data_as(_I64)))
    return out


def dpic_stage(ctx, stage: int):
    _check(ctx, lib().dpic_stage(ctx, int(stage)))


def grid_shape(which: int, grid: Sequence[int], ntan: int):
    nx, ny, nz = grid
    if which == GRID_RHO:
        return (nz, ny, nx, ntan + 1)
    if which == GRID_PHI:
        return (nz + 2, ny + 2, nx + 2, ntan + 1)
    if which == GRID_E:
        return (nz, ny, nx, 3, ntan + 1)
    raise ValueError(which)


def dpic_read_grid(ctx, which: int, grid, ntan: int, nbatch: int = 1) -> np.ndarray:
    out = np.empty((nbatch,) + grid_shape(which, grid, ntan))
    _check(ctx, lib().dpic_read_grid(ctx, int(which), _dp(out)))
    return out


def dpic_write_grid(ctx, which: int, data: np.ndarray):
    data = _f64(data)
    _check(ctx, lib().dpic_write_grid(ctx, int(which), _dp(data)))


def dpic_state_bytes(ctx) -> int:
    b = ctypes.c_size_t(0)
    _check(ctx, lib().dpic_state_bytes(ctx, ctypes.byref(b)))
    return b.value


def dpic_save_state(ctx, dev_ptr: int):
    _check(ctx, lib().dpic_save_state(ctx, _P(dev_ptr)))


def dpic_load_state(ctx, dev_ptr: int):
    _check(ctx, lib().dpic_load_state(ctx, _P(dev_ptr)))


def dpic_set_option(ctx, option: int, value: int):
    _check(ctx, lib().dpic_set_option(ctx, int(option), int(value)))


def dpic_get_option(ctx, option: int) -> int:
    v = ctypes.c_int64(0)
    _check(ctx, lib().dpic_get_option(ctx, int(option), ctypes.byref(v)))
    return v.value


def dpic_autotune(ctx, scratch_ptr: int, scratch_bytes: int, trial_steps: int):
    best = np.zeros(3, dtype=np.int64)
    ms = ctypes.c_double(0.0)
    _check(ctx, lib().dpic_autotune(ctx, _P(scratch_ptr), scratch_bytes, int(trial_steps),
                                    best.ctypes.data_as(_I64), ctypes.byref(ms)))
    return {"sort_every": int(best[0]), "chunk": int(best[1]), "part_blocks": int(best[2]), "ms": ms.value}


def dpic_stage_times(ctx):
    ms = np.zeros(N_STAGE_TIMERS)
    n = (ctypes.c_int64 * N_STAGE_TIMERS)()
    _check(ctx, lib().dpic_stage_times(ctx, _dp(ms), n))
    return ms, np.array(list(n), dtype=np.int64)


def dpic_adjoint_query(dims: dpic_dims, n_steps: int, checkpoint_every: int) -> int:
    b = ctypes.c_size_t(0)
    _check(None, lib().dpic_adjoint_query(ctypes.byref(dims), int(n_steps), int(checkpoint_every), ctypes.byref(b)))
    return b.value


def dpic_adjoint_bind(ctx, dev_ptr: int, nbytes: int, n_steps: int, checkpoint_every: int):
    _check(ctx, lib().dpic_adjoint_bind(ctx, _P(dev_ptr), nbytes, int(n_steps), int(checkpoint_every)))


def dpic_adjoint_backward(ctx, weights, n_params: int):
    w = _f64(weights, (3,))
    gp = np.zeros(max(n_params, 1))
    gs = np.zeros(6)
    _check(ctx, lib().dpic_adjoint_backward(ctx, _dp(w), _dp(gp), _dp(gs)))
    return gp[:n_params], gs


# ---------------------------------------------------------------- convenience
class Simulation:
    """One context with its torch-owned workspace, on torch's current stream.

    With nbatch > 1 the context runs that many settings together: use
    set_params_batch and init_beam_batch, and the readers return arrays with a
    leading setting index. n_particles is the storage capacity (see
    batch_capacity)."""

    def __init__(self, n_particles: int, ntan: int, grid: Sequence[int], device: str = "cuda", nbatch: int = 1):
        import torch  # device memory and streams only

        if not torch.cuda.is_available():
            raise RuntimeError("dpic needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.ntan = int(ntan)
        self.grid = tuple(int(g) for g in grid)
        self.capacity = int(n_particles)
        self.nbatch = int(nbatch)
        self.dims = make_dims(n_particles, ntan, grid, nbatch)
        nbytes = dpic_query_workspace(self.dims)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream()
        self.ctx = dpic_create(self.dims, self._ws_ptr, nbytes, self.stream.cuda_stream)
        self.n = 0
        self._xi = None

    def close(self):
        if getattr(self, "ctx", None):
            dpic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ----------------------------------------------------------
    def set_beam(self, kinetic_eV, rest_eV, charge_e, bunch_charge_C):
        dpic_set_beam(self.ctx, kinetic_eV, rest_eV, charge_e, bunch_charge_C)

    def set_grid(self, lo, hi):
        dpic_set_grid(self.ctx, lo, hi)

    def set_lattice(self, kind, n_steps, L, k, L_param, k_param, n_periods):
        dpic_set_lattice(self.ctx, kind, n_steps, L, k, L_param, k_param, n_periods)

    def set_params(self, p, seed=None):
        dpic_set_params(self.ctx, p, seed)

    def set_params_batch(self, p, seed=None):
        dpic_set_params_batch(self.ctx, p, seed)

    def init_beam(self, xi: np.ndarray, sigma, sigma_seed=None):
        torch = self.torch
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        self._xi = torch.from_numpy(xi).to(device=self.workspace.device)
        self.n = xi.shape[0]
        dpic_init_beam(self.ctx, self.n, self._xi.data_ptr(), sigma, sigma_seed)

    def init_beam_batch(self, ns, xi, sigmas, sigma_seed=None):
        """Setting b takes rows [sum(ns[:b]), + ns[b]) of xi [sum ns][6] (numpy,
        or a float64 tensor on the device) and sizes sigmas[b]."""
        torch = self.torch
        if isinstance(xi, torch.Tensor):
            self._xi = xi.to(device=self.workspace.device, dtype=torch.float64).reshape(-1, 6).contiguous()
        else:
            xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 6)
            self._xi = torch.from_numpy(xi).to(device=self.workspace.device)
        if self._xi.shape[0] != int(np.sum(ns)):
            raise ValueError("xi must hold sum(ns) rows")
        self.n = int(self._xi.shape[0])
        self.ns = [int(v) for v in ns]
        dpic_init_beam_batch(self.ctx, ns, self._xi.data_ptr(), sigmas, sigma_seed)

    # -- run --------------------------------------------------------------
    def step(self, n: int):
        dpic_step(self.ctx, n)

    def stage(self, stage: int):
        dpic_stage(self.ctx, stage)

    # -- read ---------------------------------------------------------------
    def _unbatch(self, a):
        return a[0] if self.nbatch == 1 else a

    def moments(self):
        return self._unbatch(dpic_read_moments(self.ctx, self.ntan, self.nbatch))

    def emittance(self, centred=False):
        return self._unbatch(dpic_read_emittance(self.ctx, self.ntan, centred, self.nbatch))

    def particles(self):
        return dpic_read_particles(self.ctx, self.n, self.ntan)

    def counters(self):
        return dpic_counters(self.ctx)

    def batch_counters(self):
        return dpic_batch_counters(self.ctx, self.nbatch)

    def read_grid(self, which):
        return self._unbatch(dpic_read_grid(self.ctx, which, self.grid, self.ntan, self.nbatch))

    def write_grid(self, which, data):
        dpic_write_grid(self.ctx, which, data)

    def set_option(self, option, value):
        dpic_set_option(self.ctx, option, value)

    def get_option(self, option):
        return dpic_get_option(self.ctx, option)

    def stage_times(self):
        return dpic_stage_times(self.ctx)

    def autotune(self, trial_steps: int):
        """Time candidate work-item sizes, grid sizes and sort cadences from the
        current state (which is restored) and keep the fastest."""
        nbytes = dpic_state_bytes(self.ctx)
        scratch = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.workspace.device)
        ptr = (scratch.data_ptr() + 255) // 256 * 256
        return dpic_autotune(self.ctx, ptr, nbytes, trial_steps)

    def synchronize(self):
        self.stream.synchronize()

    # -- reverse mode (value-only contexts) --------------------------------
    def bind_adjoint(self, n_steps: int, checkpoint_every: int):
        """Allocate (torch) and attach the reverse-mode workspace; call before init_beam."""
        nbytes = dpic_adjoint_query(self.dims, n_steps, checkpoint_every)
        self.adjoint_workspace = self.torch.empty(nbytes + 256, dtype=self.torch.uint8,
                                                  device=self.workspace.device)
        ptr = (self.adjoint_workspace.data_ptr() + 255) // 256 * 256
        dpic_adjoint_bind(self.ctx, ptr, nbytes, n_steps, checkpoint_every)

    def backward(self, weights, n_params: int):
        return dpic_adjoint_backward(self.ctx, weights, n_params)
