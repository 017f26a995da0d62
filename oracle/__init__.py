"""CPU FP64 oracle for the forward-mode differentiable 3D PIC space-charge step.

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
GPU library is checked against. Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: it has its own dual-number type, its
own physical constants, its own Green's function and its own convolution
(a library FFT convolution of the zero-padded charge with the point kernel,
not the doubled-grid circular convolution the GPU uses).

Modules
  dual     -- first-order dual numbers F = (f, f_x1, ..., f_xn) (Sec. 2 rules)
  physics  -- constants, beam kinematics and kick coefficients
  lattice  -- per-element step sizes and half-step transfer maps (Sec. 4,
              quadrupole maps and their dual-variable form)
  green    -- open-boundary point Green's function with a cell-averaged
              self term
  pic      -- deposit, solve, field, gather, kick, split-operator step,
              moments and emittances (Sec. 4)
  pipe2d   -- the paper's own 2D PIC: rectangular conducting pipe, sine-series
              Poisson solver, bilinear deposit, perveance kick (Sec. 4)
  twiss    -- single-particle Twiss transport, matched Twiss of a cell, the
              matching objective and its BFGS optimiser (Sec. 3)
  mlp      -- the emittance surrogate: MLP with its input Jacobian, the
              Sobolev loss and its weight gradient (exact, and with the
              rounding points of a BF16 matrix-core implementation)

Every function is pinned by the tests in tests/test_oracle_*.py against
closed forms, brute force, invariants or finite differences; the pins are
listed per function in the module docstrings.
"""
from . import dual, physics, lattice, green, pic, pipe2d, twiss, mlp  # noqa: F401
