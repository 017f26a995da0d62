"""Choose a workload's fixed grid box from value-only pre-passes on the GPU.

The box is fixed for a run and never differentiated, so it must contain
every particle at every step. Starting from a wide box, the script runs the
nominal lattice value-only (no tangents), reads the largest |x|, |y|, |z|
seen at deposit time and repeats with the box set to 1.1 times that extent,
until the extent settles. The result is what synth records as the workload's
box.

    python -m synth.box_prepass c2      # needs a GPU and the built library
    python -m synth.box_prepass c4      # every setting of a batched workload
"""
from __future__ import annotations

import sys

import numpy as np


def prepass(w, start_half=(0.05, 0.05, 0.05), iters=4, margin=1.1):
    from paper_2511_21839_amd import dpic

    half = np.asarray(start_half, dtype=np.float64)
    xi = w.xi()
    hist = []
    for _ in range(iters):
        sim = dpic.Simulation(w.n_particles, 0, w.grid)
        sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
        sim.set_grid(-half, half)
        L = w.lattice
        sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
        sim.set_params(w.params, None)
        sim.init_beam(xi, w.sigma)
        sim.step(w.total_steps())
        oob, _, ext = sim.counters()
        sim.close()
        hist.append((half.copy(), ext.copy(), oob))
        half = margin * ext
    return half, hist


def prepass_batch(bt, start_half=(0.05, 0.05, 0.05), iters=4, margin=1.1):
    """The same for every setting of a batch at once (value-only, one
    context): the box must hold all of them."""
    from paper_2511_21839_amd import dpic

    w = bt.base
    half = np.asarray(start_half, dtype=np.float64)
    xi = bt.xi()
    hist = []
    for _ in range(iters):
        sim = dpic.Simulation(dpic.batch_capacity(bt.ns), 0, w.grid, nbatch=bt.nbatch)
        sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
        sim.set_grid(-half, half)
        L = w.lattice
        sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
        sim.set_params_batch(bt.params, None)
        sim.init_beam_batch(bt.ns, xi, bt.sigma)
        sim.step(w.total_steps())
        oob, _, ext = sim.counters()
        sim.close()
        hist.append((half.copy(), ext.copy(), oob))
        half = margin * ext
    return half, hist


def c5_batch(n_settings=1024):
    """Settings spanning the surrogate's input box (13 inputs uniform within
    +-5% of nominal) on the 1e4-particle, 32^3-grid, 100-step workload."""
    import synth

    base = synth.c1(ntan=0)
    x = synth.c5_inputs(n_settings, seed=99)
    return synth.Batch(base=base, params=x[:, :7], sigma=x[:, 7:], ns=np.full(n_settings, base.n_particles),
                       seeds=base.seed + 5000 + np.arange(n_settings))


def main(argv):
    import synth

    name = argv[1] if len(argv) > 1 else "c2"
    if name == "c4":
        half, hist = prepass_batch(synth.c4())
    elif name == "c5":
        half, hist = prepass_batch(c5_batch())
    else:
        half, hist = prepass(getattr(synth, name)())
    for h, e, oob in hist:
        print(f"box half {h} -> extent {e} (out-of-box particle-steps {oob})")
    print("recommended half-widths:", tuple(float(f"{v:.4g}") for v in half))


if __name__ == "__main__":
    main(sys.argv)
