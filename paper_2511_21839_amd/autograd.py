"""Reverse-mode gradients of the final emittances behind torch.autograd.Function.

`AdjointRun` holds one value-only simulation (fixed beam draws, lattice,
grid and step count) with the reverse-mode workspace bound. Its forward takes
the lattice parameters and the six initial beam sizes, steps the beam with
checkpoints, and returns the raw emittances (eps_x, eps_y, eps_z). Its
backward sweeps the steps in reverse on the GPU and returns dJ/dparams and
dJ/dsigma for J = sum_plane w_plane eps_plane. `emittances()` wraps the pair
as an autograd function; every computation runs in the library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dpic


class AdjointRun:
    def __init__(self, n_particles: int, grid, lo, hi, beam, lattice, xi: np.ndarray, n_steps: int,
                 checkpoint_every: int = 50, sort_every: int = -1, graph: bool = False):
        """beam = (kinetic_eV, rest_eV, charge_e, bunch_charge_C);
        lattice = (kind, n_steps, L, k, L_param, k_param, n_periods);
        sort_every: the library option (-1, automatic: with the adjoint bound
        the beam is sorted once and the tiled kernels run);
        graph: capture the forward steps and the adjoint sweep in HIP graphs
        on first use and replay them afterwards."""
        self.sim = dpic.Simulation(n_particles, 0, grid)
        self.sim.set_beam(*beam)
        self.sim.set_grid(lo, hi)
        self.sim.set_lattice(*lattice)
        self.sim.set_option(dpic.OPT_SORT_EVERY, sort_every)
        if graph:
            self.sim.set_option(dpic.OPT_GRAPH, 1)
        self.sim.bind_adjoint(n_steps, checkpoint_every)
        self.xi = np.ascontiguousarray(xi, dtype=np.float64)
        self.n_steps = int(n_steps)
        self.n_params = 0
        self.generation = 0  # the run keeps one forward at a time for its backward

    def forward(self, params, sigma) -> np.ndarray:
        params = np.asarray(params, dtype=np.float64)
        self.n_params = len(params)
        self.sim.set_params(params, None)
        self.sim.init_beam(self.xi, np.asarray(sigma, dtype=np.float64))
        self.sim.step(self.n_steps)
        self.generation += 1
        return self.sim.emittance()[:, 0].copy()

    def backward(self, weights):
        return self.sim.backward(np.asarray(weights, dtype=np.float64), self.n_params)


class EmittanceFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, sigma: torch.Tensor, run: AdjointRun):
        eps = run.forward(params.detach().cpu().numpy(), sigma.detach().cpu().numpy())
        ctx.run = run
        ctx.generation = run.generation
        return torch.tensor(eps, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_eps: torch.Tensor):
        run = ctx.run
        if run.generation != ctx.generation:
            raise RuntimeError("AdjointRun was stepped again after this forward; "
                               "call backward before the next forward on the same run")
        gp, gs = run.backward(grad_eps.detach().cpu().numpy())
        return torch.from_numpy(np.array(gp)), torch.from_numpy(np.array(gs)), None


def emittances(params: torch.Tensor, sigma: torch.Tensor, run: AdjointRun) -> torch.Tensor:
    """(eps_x, eps_y, eps_z) with gradients to params and sigma through the GPU adjoint."""
    return EmittanceFunction.apply(params, sigma, run)
