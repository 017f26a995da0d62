"""Failure witnesses of the library on the GPU: a non-finite value in the
state is reported with the first step that stored it.

The NaN is planted from the host, in a checkpoint buffer that is loaded back
(a value the method can then carry through every later step); no kernel is
made to fault.
"""
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


def _with_nan_tangent(sim, coord=1, channel=3):
    """Save the state, set one tangent of the particle in storage slot 0 to
    NaN (the state is the buffer's last 6 x capacity x NC doubles), load it."""
    import torch
    from paper_2511_21839_amd import dpic

    nbytes = dpic.dpic_state_bytes(sim.ctx)
    buf = torch.zeros(nbytes // 8 + 1, dtype=torch.float64, device="cuda")
    dpic.dpic_save_state(sim.ctx, buf.data_ptr())
    cap = sim.capacity
    nc = 1 if sim.ntan == 0 else (8 if sim.ntan <= 7 else 16)
    st0 = nbytes // 8 - 6 * cap * nc
    buf[st0 + (coord * cap + 0) * nc + channel] = float("nan")
    dpic.dpic_load_state(sim.ctx, buf.data_ptr())


def test_nonfinite_tangent_is_reported_at_its_step():
    from paper_2511_21839_amd import dpic

    w = synth.tiny(n_particles=1500, grid=16, steps_per_element=4)
    sim = make_sim(w)
    sim.set_option(dpic.OPT_CHECK_FINITE, 1)
    sim.step(3)  # a clean run passes the check after every call
    sim.step(2)
    assert sim.counters()[1] == 5
    _with_nan_tangent(sim)
    with pytest.raises(dpic.DpicError) as ei:
        sim.step(2)
    assert ei.value.code == dpic.DPIC_ENONFINITE
    assert "since step 5" in str(ei.value)
    # the read-backs report it too
    with pytest.raises(dpic.DpicError) as ei:
        sim.emittance()
    assert ei.value.code == dpic.DPIC_ENONFINITE


def test_nonfinite_without_the_option_surfaces_at_read_back():
    from paper_2511_21839_amd import dpic

    w = synth.tiny(n_particles=1200, grid=16, steps_per_element=3)
    sim = make_sim(w)
    sim.step(4)
    _with_nan_tangent(sim, coord=4, channel=1)
    sim.step(3)  # asynchronous: no error here
    with pytest.raises(dpic.DpicError) as ei:
        sim.moments()
    assert ei.value.code == dpic.DPIC_ENONFINITE
    assert "since step 4" in str(ei.value)
    # a new beam clears the record
    sim.init_beam(w.xi(), w.sigma, w.sigma_seed())
    sim.step(2)
    assert np.isfinite(sim.emittance()).all()
