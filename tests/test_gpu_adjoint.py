"""Reverse-mode adjoint of the whole run (GPU, through the C ABI and the
autograd wrapper) against the oracle's forward-mode gradient (13 tangents:
7 lattice parameters + 6 initial beam sizes), against central finite
differences, and against the zero-current closed forms.

The gradient of J = sum w_plane eps_plane is compared normwise per block
(lattice parameters; beam sizes) at 1e-9 relative, the paper's quantity being
the same derivative computed in the other accumulation order.
"""
import numpy as np
import pytest

import synth
from oracle import pic

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _run(w, K, n_steps=None, graph=False, sort_every=20):
    """sort_every 20 keeps the tiled kernels (the beam sorted once) at these
    small sizes, where the library's automatic choice would not tile."""
    from paper_2511_21839_amd.autograd import AdjointRun

    L = w.lattice
    return AdjointRun(w.n_particles, w.grid, w.lo, w.hi,
                      (w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C),
                      (L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods),
                      w.xi(), n_steps or w.total_steps(), checkpoint_every=K, graph=graph, sort_every=sort_every)


def _oracle_grad(w, weights):
    r = pic.simulate_workload(w.with_(ntan=13, sigma_tangents=True))
    eps = r.emittance
    g = sum(weights[pl] * eps[pl, 1:] for pl in range(3))
    return eps[:, 0], g


def _check(gp, gs, ref):
    for name, got, want in (("params", gp, ref[:7]), ("sigma", gs, ref[7:])):
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= GRAD_RTOL, (name, err, got, want)


@pytest.mark.parametrize("K", [4, 7, 100])
def test_adjoint_matches_oracle_forward_mode(K):
    w = synth.tiny(n_particles=2000, grid=16, steps_per_element=3, ntan=0)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    run = _run(w, K)
    eps = run.forward(w.params, w.sigma)
    gp, gs = run.backward([1.0, 1.0, 0.0])
    ref_eps, ref = _oracle_grad(w, (1.0, 1.0, 0.0))
    np.testing.assert_allclose(eps, ref_eps, rtol=1e-10)
    _check(gp, gs, ref)


def test_adjoint_weights_include_longitudinal_plane():
    w = synth.tiny(n_particles=1500, grid=16, steps_per_element=3, ntan=0)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    weights = (0.3, -1.2, 0.7)
    run = _run(w, 5)
    run.forward(w.params, w.sigma)
    gp, gs = run.backward(weights)
    _, ref = _oracle_grad(w, weights)
    _check(gp, gs, ref)


def test_adjoint_repeats_with_new_parameters():
    # the same run object differentiates a second parameter point correctly
    w = synth.tiny(n_particles=1200, grid=16, steps_per_element=2, ntan=0)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    run = _run(w, 3)
    run.forward(w.params, w.sigma)
    run.backward([1.0, 1.0, 0.0])
    p2 = tuple(np.asarray(w.params) * (1 + 0.03 * np.array([1, -1, 1, 1, -1, 1, -1])))
    s2 = tuple(np.asarray(w.sigma) * 1.02)
    run.forward(p2, s2)
    gp, gs = run.backward([1.0, 1.0, 0.0])
    _, ref = _oracle_grad(w.with_(params=p2, sigma=s2), (1.0, 1.0, 0.0))
    _check(gp, gs, ref)


def test_graph_replays_of_forward_and_adjoint_sweep_match_the_oracle():
    """With graph replay the forward steps and the adjoint sweep are captured
    on the first call and replayed afterwards: every call, at the first and
    at a second parameter point (new device-side values under the same
    graphs), gives the oracle's gradients, and the replayed result equals the
    captured one."""
    w = synth.tiny(n_particles=1200, grid=16, steps_per_element=2, ntan=0)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    run = _run(w, 3, graph=True)
    _, ref = _oracle_grad(w, (1.0, 1.0, 0.0))
    first = None
    for _ in range(2):
        run.forward(w.params, w.sigma)
        gp, gs = run.backward([1.0, 1.0, 0.0])
        _check(gp, gs, ref)
        if first is None:
            first = (gp, gs)
        else:
            np.testing.assert_allclose(gp, first[0], rtol=1e-11, atol=0)
            np.testing.assert_allclose(gs, first[1], rtol=1e-11, atol=0)
    p2 = tuple(np.asarray(w.params) * (1 + 0.03 * np.array([1, -1, 1, 1, -1, 1, -1])))
    s2 = tuple(np.asarray(w.sigma) * 1.02)
    run.forward(p2, s2)
    gp, gs = run.backward([1.0, 1.0, 0.0])
    _, ref2 = _oracle_grad(w.with_(params=p2, sigma=s2), (1.0, 1.0, 0.0))
    _check(gp, gs, ref2)


def test_adjoint_c1_workload_two_segments():
    # 1e4 particles, 32^3 grid, 100 steps, checkpoints every 50 steps
    w = synth.c1(ntan=0)
    run = _run(w, 50, sort_every=-1)  # the library's automatic choice (tiled while the adjoint is bound)
    eps = run.forward(w.params, w.sigma)
    gp, gs = run.backward([1.0, 1.0, 0.0])
    ref_eps, ref = _oracle_grad(w, (1.0, 1.0, 0.0))
    np.testing.assert_allclose(eps, ref_eps, rtol=1e-10)
    _check(gp, gs, ref)


def test_adjoint_matches_central_differences_of_gpu_runs():
    from paper_2511_21839_amd import dpic

    w = synth.tiny(n_particles=1500, grid=16, steps_per_element=3, ntan=0)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    run = _run(w, 6)
    run.forward(w.params, w.sigma)
    gp, gs = run.backward([1.0, 1.0, 0.0])

    sim = dpic.Simulation(w.n_particles, 0, w.grid)
    sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
    sim.set_grid(w.lo, w.hi)
    L = w.lattice
    sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
    xi = w.xi()

    def J(p, s):
        sim.set_params(p, None)
        sim.init_beam(xi, s)
        sim.step(w.total_steps())
        e = sim.emittance()
        return e[0, 0] + e[1, 0]

    p0, s0 = np.asarray(w.params, float), np.asarray(w.sigma, float)
    fd = []
    for j in range(13):
        vec = np.concatenate([p0, s0])
        h = 1e-6 * abs(vec[j])
        up, dn = vec.copy(), vec.copy()
        up[j] += h
        dn[j] -= h
        fd.append((J(up[:7], up[7:]) - J(dn[:7], dn[7:])) / (2 * h))
    fd = np.array(fd)
    for got, want in ((gp, fd[:7]), (gs, fd[7:])):
        assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max()


def test_autograd_function_backpropagates_the_adjoint():
    import torch
    from paper_2511_21839_amd.autograd import emittances

    w = synth.tiny(n_particles=1000, grid=16, steps_per_element=2, ntan=0)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    run = _run(w, 4)
    p = torch.tensor(w.params, dtype=torch.float64, requires_grad=True)
    s = torch.tensor(w.sigma, dtype=torch.float64, requires_grad=True)
    eps = emittances(p, s, run)
    loss = 2.0 * eps[0] + eps[1]
    loss.backward()
    _, ref = _oracle_grad(w, (2.0, 1.0, 0.0))
    _check(p.grad.numpy(), s.grad.numpy(), ref)


def test_zero_current_adjoint_closed_forms():
    # the emittance is invariant under the linear lattice: no lattice
    # sensitivity, and d eps_x / d sigma_j = eps_x / sigma_j for its own plane
    w = synth.tiny(n_particles=800, grid=16, steps_per_element=3, ntan=0).with_(bunch_charge_C=0.0)
    run = _run(w, 4)
    eps = run.forward(w.params, w.sigma)
    gp, gs = run.backward([1.0, 0.0, 0.0])
    assert np.all(np.abs(gp * np.asarray(w.params)) <= 1e-11 * eps[0])
    want = np.array([eps[0] / w.sigma[0], eps[0] / w.sigma[1], 0, 0, 0, 0])
    np.testing.assert_allclose(gs, want, rtol=1e-11, atol=1e-12 * eps[0] / w.sigma[0])


def test_adjoint_at_the_benchmark_beam_matches_forward_mode():
    """The 1e6-particle, 64^3 beam (tiled adjoint deposit, 2 segments of 10
    steps) against the GPU's own 13-tangent forward mode of the same steps,
    which the oracle pins at 1e-9 on smaller beams."""
    from gpu_util import make_sim

    w = synth.c2()
    T = 20
    run = _run(w.with_(ntan=0), 10, n_steps=T)
    run.forward(w.params, w.sigma)
    gp, gs = run.backward([1.0, 1.0, 0.0])
    run.sim.close()
    w13 = w.with_(ntan=13, sigma_tangents=True)
    sim = make_sim(w13)
    sim.step(T)
    e = sim.emittance()
    _check(gp, gs, e[0, 1:] + e[1, 1:])
