"""The allocation-free emittance read-back (dpic_read_emittance_noalloc)
against dpic_read_emittance, through the C ABI: two calls in a row on one
GPU, the second with a smaller beam, raw and centred, a batch with an empty
setting, and a context too large for the static scratch."""
import numpy as np
import pytest

import synth
from gpu_util import make_sim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_21839_amd import dpic

    dpic.lib()
    yield


def _noalloc(sim, centred):
    import torch
    from paper_2511_21839_amd import dpic

    out = torch.full((sim.nbatch, 3, sim.ntan + 1), float("nan"), dtype=torch.float64, device="cuda")
    dpic.dpic_read_emittance_noalloc(sim.ctx, centred, out.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_emittance_equals_read_emittance_on_two_calls():
    # call 1: 3000 particles, 13 tangents
    w = synth.tiny(n_particles=3000, grid=16, steps_per_element=3, ntan=13, sigma_tangents=True)
    sim = make_sim(w)
    sim.step(7)
    for centred in (False, True):
        want = sim.emittance(centred=centred)
        got = _noalloc(sim, centred)[0]
        # the same kernels sum in the same order: equal to the last bit
        np.testing.assert_array_equal(got, want)
    # call 2, smaller input: 400 particles in the same context
    xi = w.xi()[:400]
    sim.init_beam(xi, w.sigma, w.sigma_seed())
    sim.step(5)
    for centred in (True, False):
        want = sim.emittance(centred=centred)
        got = _noalloc(sim, centred)[0]
        np.testing.assert_array_equal(got, want)


def test_noalloc_batch_with_an_empty_setting():
    from paper_2511_21839_amd import dpic

    base = synth.tiny(n_particles=1000, grid=16, steps_per_element=2)
    ns = [700, 0, 300]
    bt = synth.perturbed_batch(base, ns, seed=5)
    sim = dpic.Simulation(dpic.batch_capacity(bt.ns), base.ntan, base.grid, nbatch=bt.nbatch)
    sim.set_beam(base.kinetic_eV, base.rest_eV, base.charge_e, base.bunch_charge_C)
    sim.set_grid(base.lo, base.hi)
    L = base.lattice
    sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
    sim.set_params_batch(bt.params, base.param_seed())
    sim.init_beam_batch(bt.ns, bt.xi(), bt.sigma, base.sigma_seed())
    sim.step(3)
    got = _noalloc(sim, False)
    want = sim.emittance()
    np.testing.assert_array_equal(got, want)
    assert not got[1].any()


def test_noalloc_rejects_a_context_beyond_its_scratch():
    from paper_2511_21839_amd import dpic

    base = synth.tiny(n_particles=200, grid=8, steps_per_element=1, ntan=13, sigma_tangents=True)
    ns = [200] * 256
    bt = synth.perturbed_batch(base, ns, seed=6)
    sim = dpic.Simulation(dpic.batch_capacity(bt.ns), base.ntan, base.grid, nbatch=bt.nbatch)
    sim.set_beam(base.kinetic_eV, base.rest_eV, base.charge_e, base.bunch_charge_C)
    sim.set_grid(base.lo, base.hi)
    L = base.lattice
    sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
    sim.set_params_batch(bt.params, base.param_seed())
    sim.init_beam_batch(bt.ns, bt.xi(), bt.sigma, base.sigma_seed())
    with pytest.raises(dpic.DpicError) as ei:
        _noalloc(sim, False)
    assert ei.value.code == dpic.DPIC_EINVAL
    # the context itself is unaffected
    assert np.isfinite(sim.emittance()).all()
