"""Batched runs (several settings in one context, one launch per stage),
graph capture of step runs, the work-item and grid-size options and the
autotuner, all through the C ABI.

Every setting of a batch must reproduce the oracle's run of that setting
alone at the tolerances of gpu_util (values 1e-10, derivatives 1e-9
normwise), whatever its neighbours, its particle count (ragged, empty) and
the options; graph replays must reproduce the eager path.
"""
import numpy as np
import pytest

import synth
from oracle import green, physics, pic
from gpu_util import assert_moments_close, assert_outputs_close, assert_particles_close, normwise_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_21839_amd import dpic

    dpic.lib()
    yield


def _batch(ns, ntan=7, grid=16, steps_per_element=3, seed=5, perturb_sigma=True, **kw):
    base = synth.tiny(n_particles=max(ns), grid=grid, steps_per_element=steps_per_element, ntan=ntan, **kw)
    return synth.perturbed_batch(base, ns, seed, perturb_sigma=perturb_sigma)


def _make(batch, capacity=None, sort_every=5, graph=False, chunk=None, part_blocks=None):
    from paper_2511_21839_amd import dpic

    w = batch.base
    cap = capacity or dpic.batch_capacity(batch.ns)
    sim = dpic.Simulation(cap, w.ntan, w.grid, nbatch=batch.nbatch)
    sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
    sim.set_grid(w.lo, w.hi)
    L = w.lattice
    sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
    sim.set_params_batch(batch.params, w.param_seed())
    if sort_every is not None:
        sim.set_option(dpic.OPT_SORT_EVERY, sort_every)
    if chunk is not None:
        sim.set_option(dpic.OPT_CHUNK, chunk)
    if part_blocks is not None:
        sim.set_option(dpic.OPT_PART_BLOCKS, part_blocks)
    if graph:
        sim.set_option(dpic.OPT_GRAPH, 1)
    sim.init_beam_batch(batch.ns, batch.xi(), batch.sigma, w.sigma_seed())
    return sim


def _split(particles, ns):
    out, r = [], 0
    for n in ns:
        out.append(particles[r:r + n])
        r += n
    return out


def _check_against_oracle(sim, batch, nsteps=None):
    parts = _split(sim.particles(), batch.ns)
    mom = sim.moments()
    emit = sim.emittance()
    oob = sim.batch_counters()
    for b in range(batch.nbatch):
        n = int(batch.ns[b])
        if n == 0:
            assert np.all(emit[b] == 0.0) and oob[b] == 0
            continue
        w = batch.setting(b)
        ref = pic.simulate_workload(w, nsteps=nsteps)
        assert_particles_close(parts[b], ref.particles)
        assert_moments_close(mom[b], ref.moments, ref.particles)
        if w.bunch_charge_C != 0.0:
            assert_outputs_close(emit[b], ref.emittance, what=f"emittance of setting {b}")
        else:
            # linear maps leave the emittance invariant: its lattice derivatives
            # are rounding noise on both sides, checked on the scale eps / p
            for pl in range(3):
                e0 = ref.emittance[pl, 0]
                assert abs(emit[b, pl, 0] - e0) <= 1e-10 * e0
                assert np.all(np.abs(emit[b, pl, 1:8] * np.asarray(w.params)) <= 1e-11 * e0)
        assert oob[b] == ref.out_of_box


def test_batch_with_streamed_fields_matches_oracle():
    """24 settings on 32^3 grids: their fields (151 MB) are more than the
    particle kernel expects to stay in the caches, so it stages E on each
    tile's own nodes and deposits with the drift allowance in z (the other
    tests run the cached-field geometry). Sampled settings against their own
    oracle runs, every setting's out-of-box count against zero."""
    ns = [400 + 50 * k for k in range(24)]
    batch = _batch(ns, grid=32)
    w0 = batch.base
    assert len(ns) * w0.grid[0] * w0.grid[1] * w0.grid[2] * 3 * (w0.ntan + 1) * 8 > 128 * 2**20
    sim = _make(batch, sort_every=2)
    sim.step(w0.total_steps())
    parts = _split(sim.particles(), batch.ns)
    emit = sim.emittance()
    assert np.all(sim.batch_counters() == 0)
    for b in (0, 11, 23):
        w = batch.setting(b)
        ref = pic.simulate_workload(w)
        assert ref.out_of_box == 0
        assert_particles_close(parts[b], ref.particles)
        assert_outputs_close(emit[b], ref.emittance, what=f"emittance of setting {b}")


@pytest.mark.parametrize("sort_every", [None, 5, 0, 4])
def test_batch_settings_match_their_own_oracle_runs(sort_every):
    # ragged counts: one below a segment, one empty, one spanning three segments
    batch = _batch([1500, 0, 2600, 700])
    sim = _make(batch, sort_every=sort_every)
    sim.step(batch.base.total_steps())
    _check_against_oracle(sim, batch)


def test_batch_13_tangents_and_split_calls():
    batch = _batch([1100, 2049], ntan=13, sigma_tangents=True)
    sim = _make(batch, sort_every=3)
    T = batch.base.total_steps()
    sim.step(4)
    sim.step(T - 4)
    _check_against_oracle(sim, batch)


def test_batch_zero_current():
    batch = _batch([900, 1800, 333])
    batch = synth.Batch(base=batch.base.with_(bunch_charge_C=0.0), params=batch.params, sigma=batch.sigma,
                        ns=batch.ns, seeds=batch.seeds)
    sim = _make(batch)
    sim.step(batch.base.total_steps())
    _check_against_oracle(sim, batch)


def test_batch_stages_per_setting():
    from paper_2511_21839_amd import dpic

    batch = _batch([1300, 2500, 10])
    sim = _make(batch)
    sim.stage(dpic.STAGE_DEPOSIT)
    rho = sim.read_grid(dpic.GRID_RHO)
    rng = np.random.default_rng(3)
    for b in range(batch.nbatch):
        w = batch.setting(b)
        st = pic.initial_state(w.xi(), w.sigma, w.sigma_seed(), w.ntan)
        g = pic.Grid(w.grid, w.lo, w.hi)
        want = pic.deposit(pic.cic_weights(st, g), g, w.bunch_charge_C / w.n_particles, w.ntan)
        want = np.transpose(want, (2, 1, 0, 3))
        for ch in range(w.ntan + 1):
            assert normwise_err(rho[b, ..., ch], want[..., ch]) <= 1e-12, (b, ch)
    # solve: a different random charge per setting, each solved alone by the oracle
    nx = batch.base.grid[0]
    q = rng.normal(size=(batch.nbatch, nx, nx, nx, batch.base.ntan + 1)) * 1e-15
    sim.write_grid(dpic.GRID_RHO, q)
    sim.stage(dpic.STAGE_SOLVE)
    phi = sim.read_grid(dpic.GRID_PHI)
    g = pic.Grid(batch.base.grid, batch.base.lo, batch.base.hi)
    g0, _ = physics.gamma_beta(batch.base.kinetic_eV, batch.base.rest_eV)
    G = green.green_offsets(g.n, g.h, g0)
    for b in range(batch.nbatch):
        want = np.transpose(pic.solve(np.transpose(q[b], (2, 1, 0, 3)), G), (2, 1, 0, 3))
        for ch in range(batch.base.ntan + 1):
            assert normwise_err(phi[b, ..., ch], want[..., ch]) <= 1e-12, (b, ch)


@pytest.mark.parametrize("chunk,part_blocks", [(128, 0), (2048, 0), (1024, 1), (256, 7)])
def test_work_item_and_grid_options(chunk, part_blocks):
    batch = _batch([2100, 900])
    sim = _make(batch, chunk=chunk, part_blocks=part_blocks)
    sim.step(batch.base.total_steps())
    _check_against_oracle(sim, batch)


def test_graph_replays_match_the_oracle():
    from paper_2511_21839_amd import dpic

    batch = _batch([1700, 1200])
    sim = _make(batch, graph=True, sort_every=4)
    T = batch.base.total_steps()
    for rep in range(3):
        # the same calls from the start of the schedule: captured once, replayed after
        sim.init_beam_batch(batch.ns, batch.xi(), batch.sigma, batch.base.sigma_seed())
        sim.step(5)
        e_mid = sim.emittance()  # eager work between the graph launches
        assert np.isfinite(e_mid).all()
        sim.step(T - 5)
        _check_against_oracle(sim, batch)
    # new parameter values live in device memory: a replay picks them up
    batch2 = synth.Batch(base=batch.base, params=batch.params * 1.01, sigma=batch.sigma, ns=batch.ns,
                         seeds=batch.seeds)
    sim.set_params_batch(batch2.params, batch.base.param_seed())
    sim.init_beam_batch(batch.ns, batch.xi(), batch.sigma, batch.base.sigma_seed())
    sim.step(5)
    sim.step(T - 5)
    _check_against_oracle(sim, batch2)
    assert sim.get_option(dpic.OPT_GRAPH) == 1


def test_single_setting_graph_matches_eager():
    from paper_2511_21839_amd import dpic
    from gpu_util import make_sim

    w = synth.tiny(n_particles=2500, grid=16, steps_per_element=3)
    eager = make_sim(w)
    eager.step(w.total_steps())
    graphed = make_sim(w)
    graphed.set_option(dpic.OPT_GRAPH, 1)
    for _ in range(2):
        graphed.init_beam(w.xi(), w.sigma, w.sigma_seed())
        graphed.step(w.total_steps())
        # both sides differ only in the order of the deposit atomics
        assert_outputs_close(graphed.emittance(), eager.emittance(), vtol=1e-11, dtol=1e-9)


def _expected_sorts(calls, sort_every):
    """Re-sorts of dpic_step calls of the given lengths from a fresh beam
    (dpic_init_beam already stored it sorted): one after every step s with
    (s + 1) % sort_every == 0 except a call's last."""
    n, s0 = 0, 0
    for c in calls:
        n += sum(1 for s in range(s0, s0 + c - 1) if (s + 1) % sort_every == 0)
        s0 += c
    return n


def test_stage_timing_counts_launches_and_keeps_results():
    """Stage timing binds events to the stages' own kernels: every stage
    launch is counted, every time is positive, and the run is unchanged."""
    from paper_2511_21839_amd import dpic
    from gpu_util import make_sim

    w = synth.tiny(n_particles=2500, grid=16, steps_per_element=3)
    T = w.total_steps()
    calls = [T // 2, T - T // 2]
    plain = make_sim(w, sort_every=5)
    for c in calls:
        plain.step(c)
    timed = make_sim(w, sort_every=5)
    timed.set_option(dpic.OPT_STAGE_TIMING, 1)
    timed.stage_times()
    for c in calls:
        timed.step(c)
    ms, launches = timed.stage_times()
    want = {"particles": T + len(calls), "solve": T, "field": T, "sort": _expected_sorts(calls, 5)}
    for i, name in enumerate(dpic.STAGE_TIMER_NAMES):
        assert launches[i] == want[name], name
        assert ms[i] > 0.0, name
    ms2, launches2 = timed.stage_times()  # read-back resets
    assert all(v == 0 for v in launches2) and all(v == 0.0 for v in ms2)
    assert_outputs_close(timed.emittance(), plain.emittance(), vtol=1e-11, dtol=1e-9)
    # mode 2 times the particle stage only
    part = make_sim(w, sort_every=5)
    part.set_option(dpic.OPT_STAGE_TIMING, 2)
    part.stage_times()
    for c in calls:
        part.step(c)
    ms3, launches3 = part.stage_times()
    assert list(launches3) == [T + len(calls), 0, 0, 0] and ms3[0] > 0.0
    assert_outputs_close(part.emittance(), plain.emittance(), vtol=1e-11, dtol=1e-9)
    # mode 3 times the plain particle launches only: with a re-sort every 5
    # steps some launches write keys or store in sorted order
    plain3 = make_sim(w, sort_every=5)
    plain3.set_option(dpic.OPT_STAGE_TIMING, 3)
    plain3.stage_times()
    for c in calls:
        plain3.step(c)
    ms4, launches4 = plain3.stage_times()
    assert 0 < launches4[0] < T + len(calls) and list(launches4[1:]) == [0, 0, 0] and ms4[0] > 0.0
    assert_outputs_close(plain3.emittance(), plain.emittance(), vtol=1e-11, dtol=1e-9)
    with pytest.raises(dpic.DpicError):
        part.set_option(dpic.OPT_STAGE_TIMING, 4)


def test_autotune_keeps_the_state_and_picks_a_candidate():
    from paper_2511_21839_amd import dpic

    batch = _batch([2600, 1900], steps_per_element=4)
    sim = _make(batch)
    T = batch.base.total_steps()
    sim.step(3)
    res = sim.autotune(trial_steps=8)
    assert res["chunk"] in (256, 512, 768, 1024, 2048)
    assert res["sort_every"] in (0, 5, 10, 12, 20, 40)
    assert res["part_blocks"] >= 0 and res["ms"] > 0
    assert sim.get_option(dpic.OPT_CHUNK) == res["chunk"]
    assert sim.counters()[1] == 3  # state and step counter restored
    sim.step(T - 3)
    _check_against_oracle(sim, batch)


def test_batch_checkpoint_roundtrip():
    batch = _batch([1500, 0, 1100])
    sim = _make(batch)
    T = batch.base.total_steps()
    sim.step(6)
    import torch
    from paper_2511_21839_amd import dpic

    nbytes = dpic.dpic_state_bytes(sim.ctx)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = (buf.data_ptr() + 255) // 256 * 256
    dpic.dpic_save_state(sim.ctx, ptr)
    sim.step(T - 6)
    first = sim.particles()
    dpic.dpic_load_state(sim.ctx, ptr)
    assert sim.counters()[1] == 6
    sim.step(T - 6)
    assert_particles_close(sim.particles(), first, vtol=1e-12, dtol=1e-11)


def test_c4_sized_settings_match_single_runs():
    """Four settings of the 64-setting workload (64^3 grid, 1e5..1e6
    particles) for 40 steps: each equals the same setting run alone on the
    GPU (1e-9 relative on the emittance gradients), and the smallest one
    equals the oracle over its first 2 steps."""
    from paper_2511_21839_amd import dpic

    full = synth.c4()
    idx = [int(np.argmin(full.ns)), 1, 2, int(np.argmax(full.ns))]
    batch = synth.Batch(base=full.base, params=full.params[idx], sigma=full.sigma[idx], ns=full.ns[idx],
                        seeds=full.seeds[idx])
    sim = _make(batch)
    sim.step(40)
    eb = sim.emittance()
    assert sim.batch_counters().sum() == 0
    for b in range(batch.nbatch):
        w = batch.setting(b)
        one = dpic.Simulation(w.n_particles, w.ntan, w.grid)
        one.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
        one.set_grid(w.lo, w.hi)
        L = w.lattice
        one.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
        one.set_params(w.params, w.param_seed())
        one.init_beam(w.xi(), w.sigma)
        one.step(40)
        assert_outputs_close(eb[b], one.emittance(), vtol=1e-10, dtol=1e-9, what=f"setting {b}")
        one.close()
    small = _make(synth.Batch(base=batch.base, params=batch.params[:1], sigma=batch.sigma[:1],
                              ns=batch.ns[:1], seeds=batch.seeds[:1]))
    small.step(2)
    ref = pic.simulate_workload(batch.setting(0), nsteps=2)
    assert_outputs_close(small.emittance(), ref.emittance, what="c4 smallest setting, 2 steps")
