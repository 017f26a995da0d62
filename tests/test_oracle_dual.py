"""Pins of the oracle's dual algebra (Sec. 2 rules).

* The paper's worked example (Sec. 3, first example): the five-variable
  function at (3, 0.1, 0.1, 1, 1) against its gradient derived by hand.
* Every rule against complex-step differentiation, f'(x) = Im f(x + i h)/h,
  which involves no dual arithmetic and is exact to rounding.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle.dual import Dual


def _example(x1, x2, x3, x4, x5):
    return x3 * (2.0 * (x1 / x2).cos() + x1 / x2 + x2.exp()) + 2.0 * x4 + x4.sinh() + x5 * x5


def test_worked_example_value_and_gradient():
    pt = (3.0, 0.1, 0.1, 1.0, 1.0)
    xs = [Dual.var(v, i, 5) for i, v in enumerate(pt)]
    f = _example(*xs)
    x1, x2, x3, x4, x5 = pt
    r = x1 / x2
    value = x3 * (2 * math.cos(r) + r + math.exp(x2)) + 2 * x4 + math.sinh(x4) + x5 ** 2
    grad = [
        x3 * (-2 * math.sin(r) / x2 + 1 / x2),
        x3 * (2 * math.sin(r) * x1 / x2 ** 2 - x1 / x2 ** 2 + math.exp(x2)),
        2 * math.cos(r) + r + math.exp(x2),
        2 + math.cosh(x4),
        2 * x5,
    ]
    assert f.v == pytest.approx(value, rel=1e-15)
    np.testing.assert_allclose(f.d, grad, rtol=1e-14)
    # The numbers themselves, for a reader checking by eye.
    assert f.v == pytest.approx(7.31656857542888, rel=1e-13)
    np.testing.assert_allclose(
        f.d, [2.97606324818572, -89.1713803537641, 31.4136738178508, 3.54308063481524, 2.0],
        rtol=1e-13)


def _cs(fun, x, h=1e-30):
    return (fun(complex(x, h))).imag / h


_cfuncs = {
    "sqrt": (lambda d: d.sqrt(), lambda z: np.sqrt(z)),
    "sin": (lambda d: d.sin(), lambda z: np.sin(z)),
    "cos": (lambda d: d.cos(), lambda z: np.cos(z)),
    "sinh": (lambda d: d.sinh(), lambda z: np.sinh(z)),
    "cosh": (lambda d: d.cosh(), lambda z: np.cosh(z)),
    "exp": (lambda d: d.exp(), lambda z: np.exp(z)),
    "log": (lambda d: d.log(), lambda z: np.log(z)),
    "pow2.5": (lambda d: d ** 2.5, lambda z: z ** 2.5),
}


@pytest.mark.parametrize("name", sorted(_cfuncs))
@settings(max_examples=30, deadline=None)
@given(x=st.floats(0.05, 3.0))
def test_function_rule_matches_complex_step(name, x):
    dfun, cfun = _cfuncs[name]
    d = dfun(Dual.var(x, 0, 1))
    assert d.v == pytest.approx(cfun(complex(x, 0)).real, rel=1e-14)
    assert d.d[0] == pytest.approx(_cs(cfun, x), rel=1e-13, abs=1e-300)


@settings(max_examples=50, deadline=None)
@given(a=st.floats(-3, 3), b=st.floats(0.1, 3), c=st.floats(-3, 3))
def test_sum_product_quotient_against_complex_step(a, b, c):
    # g(a, b, c) = (a b + c) / b - a c, derivatives by complex step per variable
    def g(x, y, z):
        return (x * y + z) / y - x * z

    xs = [Dual.var(v, i, 3) for i, v in enumerate((a, b, c))]
    gd = g(*xs)
    for i in range(3):
        args = [complex(a), complex(b), complex(c)]
        args[i] += 1e-30j
        ref = g(*args).imag / 1e-30
        assert gd.d[i] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_constants_have_zero_derivatives_and_broadcast():
    x = Dual.var(np.array([1.0, 2.0, 3.0]), 1, 3)
    y = 2.0 * x + 1.0
    np.testing.assert_array_equal(y.d[:, 1], [2.0, 2.0, 2.0])
    np.testing.assert_array_equal(y.d[:, 0], 0.0)
    s = (x * x).sum()
    assert s.v == 14.0 and s.d[1] == 12.0
