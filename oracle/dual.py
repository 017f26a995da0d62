"""First-order dual numbers (the paper's order-1 truncated power series, Sec. 2).

A dual number is the vector F = (f, f_x1, ..., f_xn): the value followed by
its partial derivatives with respect to n independent variables. It is stored
as a numpy array whose LAST axis has length 1+n; leading axes index particles
or grid nodes, so one Dual object holds many dual numbers at once.

Rules implemented (Sec. 2, the four equations for sum, product, quotient and
function of a dual variable):
  F + G  = (f + g, f_x + g_x)
  F G    = (f g,   g f_x + f g_x)
  F / G  = (f / g, (f_x g - g_x f) / g^2)
  h(F)   = (h(f),  h'(f) f_x)

Pins: tests/test_oracle_dual.py (the paper's five-variable worked example in
Sec. 3 against its hand-derived gradient; every rule against complex-step
derivatives, which use no dual arithmetic).
"""
from __future__ import annotations

import numpy as np


class Dual:
    __slots__ = ("a",)
    __array_priority__ = 1000  # make numpy defer to Dual's reflected operators

    def __init__(self, a):
        self.a = np.asarray(a, dtype=np.float64)

    # -- constructors -----------------------------------------------------
    @staticmethod
    def const(v, n: int) -> "Dual":
        """Dual with value v (scalar or array) and all n derivatives zero."""
        v = np.asarray(v, dtype=np.float64)
        a = np.zeros(v.shape + (1 + n,))
        a[..., 0] = v
        return Dual(a)

    @staticmethod
    def var(v, i: int, n: int) -> "Dual":
        """Independent variable X_i = (x_i, 0, .., 1, .., 0): 1 in slot i+1."""
        d = Dual.const(v, n)
        d.a[..., 1 + i] = 1.0
        return d

    @staticmethod
    def seeded(v, seed_row) -> "Dual":
        """Value v with derivative row given explicitly (length n)."""
        seed_row = np.asarray(seed_row, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        a = np.zeros(v.shape + (1 + seed_row.shape[-1],))
        a[..., 0] = v
        a[..., 1:] = seed_row
        return Dual(a)

    # -- accessors ---------------------------------------------------------
    @property
    def v(self) -> np.ndarray:
        return self.a[..., 0]

    @property
    def d(self) -> np.ndarray:
        return self.a[..., 1:]

    @property
    def n(self) -> int:
        return self.a.shape[-1] - 1

    def __getitem__(self, idx) -> "Dual":
        if not isinstance(idx, tuple):
            idx = (idx,)
        return Dual(self.a[idx + (slice(None),)])

    def copy(self) -> "Dual":
        return Dual(self.a.copy())

    def __repr__(self) -> str:
        return f"Dual({self.a!r})"

    # -- helpers -----------------------------------------------------------
    @staticmethod
    def _lift(x, like: "Dual") -> "Dual":
        if isinstance(x, Dual):
            return x
        return Dual.const(x, like.n)

    # -- sum rule ----------------------------------------------------------
    def __add__(self, o):
        o = Dual._lift(o, self)
        return Dual(self.a + o.a)

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.a)

    def __sub__(self, o):
        o = Dual._lift(o, self)
        return Dual(self.a - o.a)

    def __rsub__(self, o):
        return Dual._lift(o, self) - self

    # -- product rule ------------------------------------------------------
    def __mul__(self, o):
        if not isinstance(o, Dual):
            # a plain number g has zero derivatives: (f g, g f_x)
            return Dual(self.a * np.asarray(o, dtype=np.float64)[..., None])
        f, g = self.v, o.v
        out = np.empty(np.broadcast_shapes(self.a.shape, o.a.shape))
        out[..., 0] = f * g
        out[..., 1:] = g[..., None] * self.d + f[..., None] * o.d
        return Dual(out)

    __rmul__ = __mul__

    # -- quotient rule -----------------------------------------------------
    def __truediv__(self, o):
        if not isinstance(o, Dual):
            return Dual(self.a / np.asarray(o, dtype=np.float64)[..., None])
        f, g = self.v, o.v
        out = np.empty(np.broadcast_shapes(self.a.shape, o.a.shape))
        out[..., 0] = f / g
        out[..., 1:] = (self.d * g[..., None] - o.d * f[..., None]) / (g * g)[..., None]
        return Dual(out)

    def __rtruediv__(self, o):
        return Dual._lift(o, self) / self

    # -- function rule -----------------------------------------------------
    def apply(self, h, dh) -> "Dual":
        """h(F) = (h(f), h'(f) f_x) for an elementary function h with derivative dh."""
        f = self.v
        out = np.empty(self.a.shape)
        out[..., 0] = h(f)
        out[..., 1:] = dh(f)[..., None] * self.d
        return Dual(out)

    def sqrt(self):
        return self.apply(np.sqrt, lambda f: 0.5 / np.sqrt(f))

    def sin(self):
        return self.apply(np.sin, np.cos)

    def cos(self):
        return self.apply(np.cos, lambda f: -np.sin(f))

    def sinh(self):
        return self.apply(np.sinh, np.cosh)

    def cosh(self):
        return self.apply(np.cosh, np.sinh)

    def exp(self):
        return self.apply(np.exp, np.exp)

    def log(self):
        return self.apply(np.log, lambda f: 1.0 / f)

    def __pow__(self, p):
        if isinstance(p, Dual):
            return (self.log() * p).exp()
        p = float(p)
        return self.apply(lambda f: f ** p, lambda f: p * f ** (p - 1.0))

    # -- reductions ----------------------------------------------------------
    def sum(self, axis=0) -> "Dual":
        """Sum over a leading axis: repeated application of the sum rule."""
        if axis < 0:
            raise ValueError("axis must index a leading (non-derivative) axis")
        return Dual(self.a.sum(axis=axis))


def sqrt(x: Dual) -> Dual:
    return x.sqrt()


def sin(x: Dual) -> Dual:
    return x.sin()


def cos(x: Dual) -> Dual:
    return x.cos()


def sinh(x: Dual) -> Dual:
    return x.sinh()


def cosh(x: Dual) -> Dual:
    return x.cosh()


def exp(x: Dual) -> Dual:
    return x.exp()


def log(x: Dual) -> Dual:
    return x.log()
