"""CPU FP64 oracle of the emittance surrogate: an MLP with its input
Jacobian and the Sobolev loss, and the loss gradient with respect to every
weight and bias.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network (the surrogate of the learned extension: 13 inputs, 4 hidden layers
of width 256 with SiLU, 2 outputs; any widths are accepted here):
    a_0 = u,  z_l = W_l a_{l-1} + b_l,  a_l = silu(z_l)   (l = 1 .. L-1)
    o   = W_L a_{L-1} + b_L
with silu(z) = z s(z), s the logistic function. The input Jacobian J = do/du
follows the chain rule as tangent matrices T_l = da_l/du:
    T_0 = I,  T_l = diag(silu'(z_l)) W_l T_{l-1},  J = W_L T_{L-1}.

Sobolev loss over n samples with value targets y and gradient targets G:
    loss = (1/n) sum_s [ wv |o_s - y_s|^2 + wj |J_s - G_s|_F^2 ].

Its gradient is reverse mode through the pair (a_l, T_l): with
Zt_l = W_l T_{l-1},
    zbar  = silu'(z_l) abar_l + silu''(z_l) sum_t Tbar_l[:, t] Zt_l[:, t]
    Ztbar = silu'(z_l) Tbar_l
    Wbar_l += zbar a_{l-1}^T + Ztbar T_{l-1}^T,  bbar_l += zbar
    abar_{l-1} = W_l^T zbar,  Tbar_{l-1} = W_l^T Ztbar.

`bf16=True` evaluates the same formulas with the rounding points of a BF16
matrix-core implementation: the inputs u, every hidden activation and
tangent column a_l, T_l, and every backward product (zbar, Ztbar, and the
output-layer (obar, Jbar)) are rounded to bfloat16 (round to nearest even,
through float32); all arithmetic in between stays FP64. Weights are used as
given (a caller comparing with a BF16 implementation passes BF16-exact
weights).

Pins (tests/test_oracle_mlp.py): silu' and silu'' against central
differences of silu; J against central differences of the network; the loss
gradient against central differences of the loss for every parameter of a
small network; a one-hidden-unit network against its hand-derived closed
form; the BF16 rounding against exactly representable values and ties.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

Params = List[Tuple[np.ndarray, np.ndarray]]  # [(W_l [out][in], b_l [out])]


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def d2silu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), via float32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(widths: Sequence[int], rng: np.random.Generator) -> Params:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    out = []
    for i in range(len(widths) - 1):
        lim = 1.0 / np.sqrt(widths[i])
        out.append((rng.uniform(-lim, lim, size=(widths[i + 1], widths[i])),
                    rng.uniform(-lim, lim, size=widths[i + 1])))
    return out


def _r(x, bf16):
    return round_bf16(x) if bf16 else x


def forward(params: Params, u: np.ndarray, bf16: bool = False):
    """u [n][n_in] -> o [n][n_out], J [n][n_out][n_in], and the per-layer
    values needed by the backward pass."""
    u = np.asarray(u, dtype=np.float64)
    n, n_in = u.shape
    a = _r(u, bf16)
    T = np.broadcast_to(np.eye(n_in), (n, n_in, n_in)).copy()  # [n][features][inputs]
    cache = []
    for l, (W, b) in enumerate(params):
        z = a @ W.T + b
        Zt = np.einsum("ij,njt->nit", W, T)
        last = l == len(params) - 1
        cache.append((a, T, z, Zt))
        if last:
            return z, Zt, cache
        a = _r(silu(z), bf16)
        T = _r(dsilu(z)[:, :, None] * Zt, bf16)
    raise ValueError("empty network")


def sobolev_loss(o, J, y, G, wv: float, wj: float) -> float:
    n = o.shape[0]
    return float((wv * np.sum((o - y) ** 2) + wj * np.sum((J - G) ** 2)) / n)


def loss_and_grad(params: Params, u, y, G, wv: float, wj: float, bf16: bool = False):
    """Sobolev loss and its gradient [(dW_l, db_l)] by the reverse sweep above."""
    o, J, cache = forward(params, u, bf16)
    n = o.shape[0]
    loss = sobolev_loss(o, J, y, G, wv, wj)
    zbar = _r(2.0 * wv * (o - y) / n, bf16)  # output layer: z = o, Zt = J
    Ztbar = _r(2.0 * wj * (J - G) / n, bf16)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        a_prev, T_prev, _, _ = cache[l]
        dW = zbar.T @ a_prev + np.einsum("nit,njt->ij", Ztbar, T_prev)
        db = zbar.sum(axis=0)
        grads[l] = (dW, db)
        if l == 0:
            break
        abar = zbar @ W  # W^T zbar per sample
        Tbar = np.einsum("ji,njt->nit", W, Ztbar)
        _, _, z, Zt = cache[l - 1]
        zbar = _r(dsilu(z) * abar + d2silu(z) * np.sum(Tbar * Zt, axis=2), bf16)
        Ztbar = _r(dsilu(z)[:, :, None] * Tbar, bf16)
    return loss, grads


def flatten(params: Params) -> np.ndarray:
    """Packed parameter vector: W_1 (row-major), b_1, W_2, b_2, ..."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflatten(vec: np.ndarray, widths: Sequence[int]) -> Params:
    out, k = [], 0
    for i in range(len(widths) - 1):
        nw = widths[i + 1] * widths[i]
        W = vec[k:k + nw].reshape(widths[i + 1], widths[i])
        k += nw
        b = vec[k:k + widths[i + 1]]
        k += widths[i + 1]
        out.append((W.copy(), b.copy()))
    return out
