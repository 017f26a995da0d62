"""ctypes binding of the emittance surrogate (include/dmlp.h) and its
workflow: PIC-generated training data (values and 13-component gradients
from a batched forward-mode run), Sobolev training on the GPU, screening of
optimizer candidates, and the PIC judge and fallback.

Argument marshalling only: the network, its loss and its gradients run in
the library's kernels; the PIC runs in dpic's. PyTorch supplies device
memory and the stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import dpic

NIN, NOUT, HIDDEN, LAYERS = 13, 2, 256, 5
WIDTHS = (NIN, HIDDEN, HIDDEN, HIDDEN, HIDDEN, NOUT)

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)

SYMBOLS = (
    "dmlp_param_count", "dmlp_query_workspace", "dmlp_create", "dmlp_destroy", "dmlp_last_error",
    "dmlp_set_normalization", "dmlp_set_params", "dmlp_get_params", "dmlp_predict", "dmlp_loss_grad",
    "dmlp_train_step", "dmlp_set_adam", "dmlp_read_loss",
)

_SIGS = {
    "dmlp_param_count": ([], ctypes.c_int),
    "dmlp_query_workspace": ([ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "dmlp_create": ([ctypes.c_int, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "dmlp_destroy": ([_P], ctypes.c_int),
    "dmlp_last_error": ([_P, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "dmlp_set_normalization": ([_P, _D, _D, _D, _D], ctypes.c_int),
    "dmlp_set_params": ([_P, _F], ctypes.c_int),
    "dmlp_get_params": ([_P, _F], ctypes.c_int),
    "dmlp_predict": ([_P, ctypes.c_int, _P, _P, _P], ctypes.c_int),
    "dmlp_loss_grad": ([_P, ctypes.c_int, _P, _P, _P, ctypes.c_double, ctypes.c_double, _D, _F], ctypes.c_int),
    "dmlp_train_step": ([_P, ctypes.c_int, _P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double],
                        ctypes.c_int),
    "dmlp_set_adam": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_double], ctypes.c_int),
    "dmlp_read_loss": ([_P, _D], ctypes.c_int),
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


def _check(ctx, rc):
    if rc != dpic.DPIC_OK:
        msg = ""
        if ctx:
            buf = ctypes.create_string_buffer(512)
            lib().dmlp_last_error(ctx, buf, 512)
            msg = buf.value.decode(errors="replace")
        raise dpic.DpicError(rc, msg)


def param_count() -> int:
    return lib().dmlp_param_count()


def query_workspace(nmax: int) -> int:
    b = ctypes.c_size_t(0)
    _check(None, lib().dmlp_query_workspace(int(nmax), ctypes.byref(b)))
    return b.value


def init_params(rng: np.random.Generator) -> np.ndarray:
    """Packed FP32 parameters, uniform within +-1/sqrt(fan_in) (drawn here, on the host)."""
    parts = []
    for i in range(LAYERS):
        lim = 1.0 / np.sqrt(WIDTHS[i])
        parts.append(rng.uniform(-lim, lim, size=WIDTHS[i + 1] * WIDTHS[i]))
        parts.append(rng.uniform(-lim, lim, size=WIDTHS[i + 1]))
    return np.concatenate(parts).astype(np.float32)


class Surrogate:
    """One network with its torch-owned workspace for batches of up to nmax samples."""

    def __init__(self, nmax: int, device: str = "cuda"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate needs a ROCm GPU")
        self.torch = torch
        self.nmax = int(nmax)
        nbytes = query_workspace(self.nmax)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream()
        ctx = _P()
        _check(None, lib().dmlp_create(self.nmax, _P(ptr), nbytes, _P(self.stream.cuda_stream)
                                       if self.stream.cuda_stream else None, ctypes.byref(ctx)))
        self.ctx = ctx
        self.device = device

    def close(self):
        if getattr(self, "ctx", None):
            lib().dmlp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ------------------------------------------------------------
    def set_normalization(self, in_center, in_scale, out_center, out_scale):
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (in_center, in_scale, out_center, out_scale)]
        _check(self.ctx, lib().dmlp_set_normalization(self.ctx, *[v.ctypes.data_as(_D) for v in a]))
        self.norm = a

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != param_count():
            raise ValueError(f"expected {param_count()} parameters")
        _check(self.ctx, lib().dmlp_set_params(self.ctx, p.ctypes.data_as(_F)))

    def get_params(self) -> np.ndarray:
        p = np.empty(param_count(), dtype=np.float32)
        _check(self.ctx, lib().dmlp_get_params(self.ctx, p.ctypes.data_as(_F)))
        return p

    def set_adam(self, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(self.ctx, lib().dmlp_set_adam(self.ctx, beta1, beta2, eps))

    # -- device tensors -----------------------------------------------------
    def to_device(self, a):
        torch = self.torch
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=torch.float64).contiguous()
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)

    # -- run ----------------------------------------------------------------
    def predict_dev(self, x, eps, jac=None):
        """x [n][13], eps [n][2], jac [n][2][13]: float64 device tensors (asynchronous)."""
        n = x.shape[0]
        _check(self.ctx, lib().dmlp_predict(self.ctx, n, _P(x.data_ptr()), _P(eps.data_ptr()),
                                            _P(jac.data_ptr()) if jac is not None else None))

    def predict(self, x, with_jacobian: bool = True):
        torch = self.torch
        xd = self.to_device(x)
        n = xd.shape[0]
        eps = torch.empty((n, NOUT), dtype=torch.float64, device=self.device)
        jac = torch.empty((n, NOUT, NIN), dtype=torch.float64, device=self.device) if with_jacobian else None
        self.predict_dev(xd, eps, jac)
        return eps.cpu().numpy(), (jac.cpu().numpy() if jac is not None else None)

    def loss_grad(self, x, eps, jac, wv: float, wj: float):
        xd, ed, jd = self.to_device(x), self.to_device(eps), self.to_device(jac)
        loss = ctypes.c_double(0.0)
        g = np.empty(param_count(), dtype=np.float32)
        _check(self.ctx, lib().dmlp_loss_grad(self.ctx, xd.shape[0], _P(xd.data_ptr()), _P(ed.data_ptr()),
                                              _P(jd.data_ptr()), wv, wj, ctypes.byref(loss), g.ctypes.data_as(_F)))
        return loss.value, g

    def train_step_dev(self, x, eps, jac, wv: float, wj: float, lr: float):
        _check(self.ctx, lib().dmlp_train_step(self.ctx, x.shape[0], _P(x.data_ptr()), _P(eps.data_ptr()),
                                               _P(jac.data_ptr()), wv, wj, lr))

    def read_loss(self) -> float:
        v = ctypes.c_double(0.0)
        _check(self.ctx, lib().dmlp_read_loss(self.ctx, ctypes.byref(v)))
        return v.value

    def fit(self, x, eps, jac, epochs: int, batch: int, lr: float, wv: float = 1.0, wj: float = 1.0,
            seed: int = 0, lr_final: Optional[float] = None, log_every: int = 0):
        """Adam over shuffled mini-batches (the order is drawn on the host);
        cosine decay from lr to lr_final. Returns the loss of the last batch
        of every epoch."""
        torch = self.torch
        xd, ed, jd = self.to_device(x), self.to_device(eps), self.to_device(jac)
        n = xd.shape[0]
        rng = np.random.default_rng(seed)
        lr_final = lr * 0.05 if lr_final is None else lr_final
        steps_per_epoch = max(1, n // batch)
        total = epochs * steps_per_epoch
        hist = []
        k = 0
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).to(self.device)
            xs, es, js = xd[perm], ed[perm], jd[perm]
            for b in range(steps_per_epoch):
                sl = slice(b * batch, (b + 1) * batch)
                a = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * k / max(total - 1, 1)))
                self.train_step_dev(xs[sl], es[sl], js[sl], wv, wj, a)
                k += 1
            hist.append(self.read_loss())
            if log_every and (ep + 1) % log_every == 0:
                print(f"epoch {ep + 1}: loss {hist[-1]:.4e}", flush=True)
        return hist


# ---------------------------------------------------------------- PIC side
@dataclass
class PicSetup:
    """What the PIC needs besides the 13 inputs: grid, box, beam and lattice
    (the lattice parameters 0..6 and the beam sizes are the inputs)."""
    grid: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    beam: Sequence[float]      # kinetic_eV, rest_eV, charge_e, bunch_charge_C
    lattice: Sequence          # kind, n_steps, L, k, L_param, k_param, n_periods
    n_steps: int


def pic_targets(setup: PicSetup, x: np.ndarray, xi: np.ndarray, batch: int = 256, graph: bool = True):
    """Final (eps_x, eps_y) and their gradients with respect to the 13 inputs
    for every row of x [n][13] (7 lattice parameters, 6 beam sizes), from
    batched forward-mode runs with 13 tangents. Every run starts from the
    same normals xi [n_particles][6]. Returns eps [n][2], jac [n][2][13] and
    the out-of-box particle-steps per run."""
    import torch

    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    npart = int(xi.shape[0])
    eps = np.empty((n, NOUT))
    jac = np.empty((n, NOUT, NIN))
    oob = np.empty(n, dtype=np.int64)
    seed_p = np.zeros((7, 13))
    seed_p[np.arange(7), np.arange(7)] = 1.0
    seed_s = np.zeros((6, 13))
    seed_s[np.arange(6), 7 + np.arange(6)] = 1.0
    xi_d = torch.from_numpy(np.ascontiguousarray(xi, dtype=np.float64)).to("cuda")
    sim = None
    for b0 in range(0, n, batch):
        b1 = min(n, b0 + batch)
        nb = b1 - b0
        if sim is None or sim.nbatch != nb:
            if sim is not None:
                sim.close()
            sim = dpic.Simulation(dpic.batch_capacity(np.full(nb, npart)), 13, setup.grid, nbatch=nb)
            sim.set_beam(*setup.beam)
            sim.set_grid(setup.lo, setup.hi)
            sim.set_lattice(*setup.lattice)
            if graph:
                sim.set_option(dpic.OPT_GRAPH, 1)
            xi_rep = xi_d.repeat(nb, 1)
        sim.set_params_batch(x[b0:b1, :7], seed_p)
        sim.init_beam_batch(np.full(nb, npart), xi_rep, x[b0:b1, 7:], seed_s)
        sim.step(setup.n_steps)
        e = sim.emittance()
        e = e if nb > 1 else e[None]
        eps[b0:b1] = e[:, :2, 0]
        jac[b0:b1] = e[:, :2, 1:14]
        oob[b0:b1] = sim.batch_counters()
    if sim is not None:
        sim.close()
    return eps, jac, oob


def objective(eps):
    """J = eps_x + eps_y (the optimisation objective of the screening)."""
    return eps[:, 0] + eps[:, 1]


def screen(net: Surrogate, candidates: np.ndarray, top_k: int):
    """Rank candidates [m][13] by the surrogate's J (one inference batch per
    nmax rows); return the indices of the top_k smallest, their predicted J
    and predicted gradients dJ/dx [top_k][13]."""
    Js, grads = [], []
    for b0 in range(0, candidates.shape[0], net.nmax):
        e, jc = net.predict(candidates[b0:b0 + net.nmax])
        Js.append(objective(e))
        grads.append(jc[:, 0] + jc[:, 1])
    J = np.concatenate(Js)
    G = np.concatenate(grads)
    idx = np.argsort(J)[:top_k]
    return idx, J[idx], G[idx]


def judge(g_surrogate: np.ndarray, g_pic: np.ndarray, rtol: float = 1e-3):
    """The PIC gradient judges the surrogate's: relative error (max norm) and
    whether it is within rtol; a caller falls back to the PIC gradient
    when it is not."""
    err = float(np.abs(g_surrogate - g_pic).max() / np.abs(g_pic).max())
    return err <= rtol, err
