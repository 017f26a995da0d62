#!/usr/bin/env python3
"""Throughput of the forward-mode differentiable 3D PIC space-charge step.

Workload (one GPU): 1e6 protons at 1 GeV, 6D Gaussian beam, 64^3 CIC grid
with the open-boundary Hockney solve on the 128^3 doubled grid, 10 FODO
cells of 5 elements x 40 steps (2000 steps), 7 tangents (3 drift lengths,
2 quadrupole lengths, 2 quadrupole strengths), FP64, beam current set for a
tune ratio of 0.3. A bench "step" is one full PIC step (push, deposit, solve,
field, gather, kick) over all particles; the timed region is K steps from the
start of the lattice schedule with the beam already resident on the GPU.

Prints one JSON line: value = particles * steps / seconds, the roofline of
the dominant kernel (the fused particle kernel, 768 algorithmic bytes per
particle per step: read and write 6 coordinates x 8 channels x 8 B), timed
with HIP events on the library's stream, and the CPU oracle timed on a short
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _log(msg):
    """Progress on stderr (the result is the one JSON line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)
BYTES_PER_PARTICLE_STEP = 6 * 8 * 8 * 2  # 6 coords x 8 channels x 8 B, read + write


def _cpu_baseline(w, xi, steps: int):
    """The oracle on a bounded sample: the first `steps` steps of the same workload."""
    from oracle import pic

    t0 = time.perf_counter()
    pic.simulate_workload(w, nsteps=steps, xi=xi)
    dt = time.perf_counter() - t0
    return {
        "value": w.n_particles * steps / dt,
        "unit": "dual particle-steps/s",
        "cores": int(pic.FFT_WORKERS),
        "kind": "oracle",
        "sample": (f"first {steps} of {w.total_steps()} steps of the same workload "
                   f"({w.n_particles} particles, 7 tangents), {dt:.1f} s; numpy FP64, "
                   f"elementwise work on 1 thread, FFT convolution on {pic.FFT_WORKERS} threads"),
    }


PROFILE_RECORD = os.path.join(ROOT, "profiles", "k_particles_tiled_c2.md")


def _particle_launch_mix(n: int, sort_every: int) -> dict:
    """Particle-kernel launches of one dpic_step(n) call from a fresh beam, by
    kernel, following the library's step loop (1e6 particles on 64^3 nodes:
    tiled kernels with the E tile's drift allowance): the opening half-step
    deposit, then per step the plain fused launch, the launch that also
    writes the sort keys (two steps before a re-sort), the launch that stores
    the state in sorted order (the step before), and the call's last launch
    (no deposit)."""
    R = sort_every
    if R == 0:  # no re-sort: the storage-order kernel, deposit by global atomics
        return {k: v for k, v in (("k_particles<8, 6>", 1), ("k_particles<8, 7>", n - 1),
                                   ("k_particles<8, 3>", 1)) if v}
    mix = {"k_particles_tiled<8, 6>": 1}
    counted = False
    for s in range(n):
        last = s == n - 1
        sort_next = R > 0 and not last and (s + 1) % R == 0
        scatter = sort_next and counted
        early = R >= 2 and s + 2 < n and (s + 2) % R == 0
        keys = (sort_next and not scatter) or early
        if last:
            name = "k_particles_tiled<8, 19>"
        elif scatter:
            name = "k_particles_sorted<8, 87>"
        elif keys:
            name = "k_particles_tiled<8, 55>"
        else:
            name = "k_particles_tiled<8, 23>"
        mix[name] = mix.get(name, 0) + 1
        if scatter:
            counted = False
        elif early and not sort_next:
            counted = True
    return mix


def _recorded_traffic(mix: dict):
    """HBM bytes per launch averaged over the launches in `mix` (kernel ->
    count), from the committed counter summary (FETCH_SIZE and WRITE_SIZE per
    kernel, scaled by a plain copy); None when the kernels' sources changed
    since the counters were taken or a kernel has no record."""
    import hashlib
    import re

    try:
        text = open(PROFILE_RECORD).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        h = hashlib.sha256()
        for p in rec["sources"]:
            h.update(open(os.path.join(ROOT, p), "rb").read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        per = rec["traffic_bytes_per_launch"]
        total = sum(mix.values())
        return sum(float(per[k]) * c for k, c in mix.items()) / total if total else None
    except (OSError, AttributeError, KeyError, ValueError, TypeError):
        return None


def _median_ms(fn, reps=3):
    import torch

    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(sorted(ts)[len(ts) // 2])


def _adjoint_timing():
    """Gradient of eps_x + eps_y w.r.t. 7 lattice parameters + 6 beam sizes on
    the 1e4-particle, 32^3, 100-step workload: reverse mode (checkpoint every
    50 steps) against forward mode with 13 tangents and the value-only run."""
    import synth
    from paper_2511_21839_amd import dpic
    from paper_2511_21839_amd.autograd import AdjointRun

    w = synth.c1(ntan=13, sigma_tangents=True)
    L = w.lattice
    xi = w.xi()

    def plain(ntan, graph):
        sim = dpic.Simulation(w.n_particles, ntan, w.grid)
        sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
        sim.set_grid(w.lo, w.hi)
        sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
        sim.set_params(w.params, w.param_seed() if ntan else None)
        sim.set_option(dpic.OPT_GRAPH, int(graph))
        ss = w.sigma_seed() if ntan else None

        def go():
            sim.init_beam(xi, w.sigma, ss)
            sim.step(w.total_steps())
        return go, sim

    out = {"workload": "1e4 protons, 32^3 grid, 100 steps, J = eps_x + eps_y, 13 gradient components",
           "checkpoint_every": 50}
    # eager launches, and every run replayed from HIP graphs (at this size
    # the runs are bound by launch overhead)
    for mode, graph in (("", False), ("graph_", True)):
        go13, s13 = plain(13, graph)
        go0, s0 = plain(0, graph)
        run = AdjointRun(w.n_particles, w.grid, w.lo, w.hi, (w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C),
                         (L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods), xi, w.total_steps(),
                         checkpoint_every=50, graph=graph)

        def adj():
            run.forward(w.params, w.sigma)
            run.backward([1.0, 1.0, 0.0])

        t13, t0, ta = _median_ms(go13), _median_ms(go0), _median_ms(adj)
        out.update({f"{mode}t_forward_13_tangents_ms": t13, f"{mode}t_value_only_ms": t0, f"{mode}t_adjoint_ms": ta,
                    f"{mode}adjoint_over_forward_13": ta / t13, f"{mode}adjoint_over_value_only": ta / t0})
    return out


def _c1_timing(reps=5):
    """The 1e4-particle, 32^3-grid, 100-step workload with 7 tangents (one
    FODO cell), each whole run (beam initialisation and 100 steps) replayed
    from HIP graphs, and with eager launches."""
    import synth
    from paper_2511_21839_amd import dpic

    w = synth.c1()
    xi = w.xi()
    out = {"workload": w.name}
    for mode, graph in (("graph", True), ("eager", False)):
        sim = _sim_for(w, w.n_particles)
        sim.set_params(w.params, w.param_seed())
        sim.set_option(dpic.OPT_GRAPH, int(graph))

        def go():
            sim.init_beam(xi, w.sigma, w.sigma_seed())
            sim.step(w.total_steps())

        ms = _median_ms(go, reps)
        out[mode] = {"ms_per_run": ms, "ms_per_step": ms / w.total_steps(),
                     "dual_particle_steps_per_s": w.n_particles * w.total_steps() / (ms * 1e-3)}
        sim.close()
    # algorithmic bytes per step: particle state read and write, plus one
    # write and read of rho, phi and E and the Ghat octant
    n = w.grid[0]
    grid_bytes = 2 * 8 * 8 * (n ** 3 + (n + 2) ** 3 + 3 * n ** 3) + 8 * (n + 1) ** 3
    step_bytes = w.n_particles * BYTES_PER_PARTICLE_STEP + grid_bytes
    g = out["graph"]["ms_per_step"] * 1e-3
    out["roofline"] = {"bound": "hbm", "algorithmic_bytes_per_step": step_bytes,
                       "achieved": step_bytes / g / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": step_bytes / g / 1e9 / HBM_PEAK_GBS,
                       "note": "whole step; at this size the step is bound by launch and latency, not bytes"}
    return out


def _deterministic_timing(steps=20):
    """The 1e6-particle, 64^3 workload in the deterministic mode (fixed-order
    deposit, no re-sorting) against the default mode, `steps` steps from the
    start of the schedule; a second run in the mode must match the first to
    the bit."""
    import numpy as np
    import torch

    import synth
    from paper_2511_21839_amd import dpic

    w = synth.c2()
    xi = w.xi()
    out = {"workload": f"{w.name}, first {steps} steps"}
    emits = []
    for mode in ("default", "deterministic", "deterministic"):
        sim = _sim_for(w, w.n_particles)
        sim.set_params(w.params, w.param_seed())
        sim.set_option(dpic.OPT_DETERMINISTIC, int(mode == "deterministic"))
        sim.init_beam(xi, w.sigma, w.sigma_seed())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        out[f"{mode}_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
        emits.append(sim.emittance())
        sim.close()
    out["deterministic_over_default"] = out["deterministic_ms_per_step"] / out["default_ms_per_step"]
    out["bit_identical_runs"] = emits[1].tobytes() == emits[2].tobytes()
    out["max_rel_diff_vs_default"] = float(np.max(np.abs(emits[1] - emits[0]) / np.abs(emits[0]).max(axis=-1, keepdims=True)))
    return out


def _copy_rate():
    """Achievable streaming rate: a device-to-device copy of the particle
    state's size (384 MiB read and written), GB/s of read + write."""
    import torch

    n = 384 * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / 20 * 1e3
    del a, b
    torch.cuda.empty_cache()
    return {"bytes": 2 * n * 8, "us": us, "GBps": 2 * n * 8 / (us * 1e-6) / 1e9}


def _adjoint_scale_timing(steps=100):
    """Reverse mode where the state streams from HBM: the 1e6-particle, 64^3
    beam over its first `steps` steps, J = eps_x + eps_y, gradients w.r.t.
    the 7 lattice parameters and the 6 beam sizes, checkpoint every 50
    steps; against forward mode with 13 tangents and the value-only run
    (both fused, re-sorted every 5 steps), and the gradients against the
    13-tangent forward mode."""
    import numpy as np
    import synth
    from paper_2511_21839_amd import dpic
    from paper_2511_21839_amd.autograd import AdjointRun

    w = synth.c2(ntan=13, sigma_tangents=True)
    L = w.lattice
    xi = w.xi()
    out = {"workload": f"1e6 protons, 64^3 grid, first {steps} steps of the 2000-step schedule, J = eps_x + eps_y, "
                       "13 gradient components", "checkpoint_every": 50}

    def forward(ntan):
        sim = _sim_for(w.with_(ntan=ntan), w.n_particles)
        sim.set_params(w.params, w.param_seed() if ntan else None)
        ss = w.sigma_seed() if ntan else None

        def go():
            sim.init_beam(xi, w.sigma, ss)
            sim.step(steps)
        return go, sim

    go13, s13 = forward(13)
    t13 = _median_ms(go13, 3)
    e13 = s13.emittance()
    s13.close()
    del s13
    go0, s0 = forward(0)
    t0 = _median_ms(go0, 3)
    s0.close()
    del s0
    run = AdjointRun(w.n_particles, w.grid, w.lo, w.hi, (w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C),
                     (L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods), xi, steps, checkpoint_every=50)
    grads = []

    def adj():
        run.forward(w.params, w.sigma)
        grads.append(run.backward([1.0, 1.0, 0.0]))

    ta = _median_ms(adj, 3)
    tf = _median_ms(lambda: run.forward(w.params, w.sigma), 3)
    gp, gs = grads[-1]
    g_adj = np.concatenate([gp, gs])
    g_fwd = e13[0, 1:] + e13[1, 1:]
    run.sim.close()
    out.update({"t_forward_13_tangents_ms": t13, "t_value_only_ms": t0, "t_adjoint_ms": ta,
                "t_adjoint_forward_part_ms": tf,
                "adjoint_over_forward_13": ta / t13, "adjoint_over_value_only": ta / t0,
                "grad_rel_err_vs_forward_13": float(np.abs(g_adj - g_fwd).max() / np.abs(g_fwd).max())})
    return out


def _sim_for(w, capacity, nbatch=1):
    from paper_2511_21839_amd import dpic

    sim = dpic.Simulation(capacity, w.ntan, w.grid, nbatch=nbatch)
    sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
    sim.set_grid(w.lo, w.hi)
    L = w.lattice
    sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
    return sim


def _batch_vs_singles(bt, steps, autotune_steps=0, graph=False):
    """One batched run of every setting of `bt` against the settings run one
    after another in a single-setting context (same inputs, same options).
    Returns timings, the autotuner's choice and the largest difference of the
    batched emittances (value per scalar, derivatives normwise) from the
    single runs."""
    import numpy as np
    import torch
    from paper_2511_21839_amd import dpic

    w = bt.base
    xi = bt.xi()
    seed = w.param_seed()
    sseed = w.sigma_seed()
    sim = _sim_for(w, dpic.batch_capacity(bt.ns), bt.nbatch)
    sim.set_params_batch(bt.params, seed)
    tuned = None
    if autotune_steps:
        sim.init_beam_batch(bt.ns, xi, bt.sigma, sseed)
        sim.step(1)
        tuned = sim.autotune(autotune_steps)
    if graph:
        sim.set_option(dpic.OPT_GRAPH, 1)
    opts = {k: sim.get_option(o) for k, o in (("sort_every", dpic.OPT_SORT_EVERY), ("chunk", dpic.OPT_CHUNK),
                                                ("part_blocks", dpic.OPT_PART_BLOCKS))}
    runs = []
    for _ in range(2 if graph else 1):  # with graphs: capture, then the timed replay
        sim.init_beam_batch(bt.ns, xi, bt.sigma, sseed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    t_batch = runs[-1]
    eb = sim.emittance()
    oob = sim.batch_counters()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    one = _sim_for(w, int(bt.ns.max()))
    for k, o in (("sort_every", dpic.OPT_SORT_EVERY), ("chunk", dpic.OPT_CHUNK), ("part_blocks", dpic.OPT_PART_BLOCKS)):
        one.set_option(o, opts[k])
    if graph:
        one.set_option(dpic.OPT_GRAPH, 1)
    t_single = 0.0
    ev = ed = 0.0
    row = 0
    for b in range(bt.nbatch):
        n = int(bt.ns[b])
        xb = xi[row:row + n]
        row += n
        one.set_params(bt.params[b], seed)
        reps = 2 if graph else 1
        for _ in range(reps):
            one.init_beam(xb, bt.sigma[b], sseed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            one.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        t_single += dt
        e1 = one.emittance()
        for pl in range(2):
            ev = max(ev, abs(eb[b, pl, 0] - e1[pl, 0]) / abs(e1[pl, 0]))
            ed = max(ed, float(np.abs(eb[b, pl, 1:] - e1[pl, 1:]).max() / np.abs(e1[pl, 1:]).max()))
    one.close()
    return {"t_batched_s": t_batch, "t_sum_single_s": t_single, "batched_over_singles": t_batch / t_single,
            "options": opts, "autotune": tuned, "out_of_box": int(oob.sum()),
            "max_rel_err_value": ev, "max_rel_err_derivatives": ed}


def _batched_timing():
    """The 64-setting workload (64^3 grid, 1e5-1e6 particles per setting, 500
    steps, 7 tangents), autotuned, and 256 settings of the 1e4-particle 32^3
    workload with 13 tangents over 100 steps (the surrogate's training runs),
    with graph replay."""
    import synth

    c4 = synth.c4()
    r4 = _batch_vs_singles(c4, c4.base.total_steps(), autotune_steps=20, graph=True)
    r4["workload"] = c4.base.name + ", graph replay"
    r4["dual_particle_steps_per_s"] = float(c4.ns.sum()) * c4.base.total_steps() / r4["t_batched_s"]
    b5 = synth.c5_batch(256, seed=7)
    r5 = _batch_vs_singles(b5, b5.base.total_steps(), graph=True)
    r5["workload"] = "256 settings of 1e4 protons, 32^3 grid, 100 steps, 13 tangents (inputs +-5%), graph replay"
    return {"c4": r4, "c1x256": r5}


MFMA_BF16_PEAK_TFLOPS = 2500.0
# network 13 -> 4 x 256 -> 2 on 14 columns per sample (value + 13 tangents)
SURROGATE_MACS_PER_COLUMN = 13 * 256 + 3 * 256 * 256 + 256 * 2
SURROGATE_FLOPS_PER_SAMPLE = 2 * 14 * SURROGATE_MACS_PER_COLUMN


def _surrogate_setup(nmax):
    import numpy as np
    import synth
    from paper_2511_21839_amd import surrogate as sg

    nom = np.concatenate([synth.NOMINAL_PARAMS, synth.SIGMA_NOMINAL])
    net = sg.Surrogate(nmax)
    net.set_normalization(nom, 0.05 * np.abs(nom), [1.2e-6, 1.4e-6], [5e-8, 5e-8])
    net.set_params(sg.init_params(np.random.default_rng(31)))
    return net, nom


def _surrogate_timing(reps=20):
    """Inference of 65536 samples (values and 2 x 13 Jacobians) and Adam
    training steps on batches of 4096, BF16 MFMA with FP32 accumulation;
    achieved TFLOP/s on the algorithmic flops (14 columns per sample, no
    padding) against the dense BF16 matrix-core peak."""
    import numpy as np
    import torch
    import synth

    n = 65536
    net, nom = _surrogate_setup(n)
    x = net.to_device(synth.c5_inputs(n, seed=32))
    eps = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    jac = torch.empty((n, 2, 13), dtype=torch.float64, device="cuda")
    for _ in range(3):
        net.predict_dev(x, eps, jac)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.predict_dev(x, eps, jac)
    e1.record()
    torch.cuda.synchronize()
    t_inf = e0.elapsed_time(e1) / reps / 1e3
    bt = 4096
    rng = np.random.default_rng(33)
    xt = x[:bt]
    et = net.to_device(1.3e-6 + 5e-8 * rng.normal(size=(bt, 2)))
    jt = net.to_device(1e-6 * rng.normal(size=(bt, 2, 13)))
    for _ in range(3):
        net.train_step_dev(xt, et, jt, 1.0, 1.0, 1e-4)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        net.train_step_dev(xt, et, jt, 1.0, 1.0, 1e-4)
    e1.record()
    torch.cuda.synchronize()
    t_tr = e0.elapsed_time(e1) / reps / 1e3
    achieved = SURROGATE_FLOPS_PER_SAMPLE * n / t_inf / 1e12
    net.close()
    return {
        "inference": {"batch": n, "ms": t_inf * 1e3, "samples_per_s": n / t_inf,
                      "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": achieved / MFMA_BF16_PEAK_TFLOPS,
                                   "flops_per_sample": SURROGATE_FLOPS_PER_SAMPLE}},
        "train_step": {"batch": bt, "ms": t_tr * 1e3, "samples_per_s": bt / t_tr,
                       "tflops": 3 * SURROGATE_FLOPS_PER_SAMPLE * bt / t_tr / 1e12},
    }


def _surrogate_full(n_train=20000, epochs=1000):
    """The learned extension end to end: PIC training data (n_train runs of
    the 1e4-particle, 32^3, 100-step workload with 13 tangents, batched),
    Sobolev training, held-out accuracy, screening of 65536 candidates
    against random search at equal PIC cost, and the PIC adjoint as judge
    of the predicted gradient at the best point."""
    import numpy as np
    import torch
    import synth
    from paper_2511_21839_amd import surrogate as sg
    from paper_2511_21839_amd.autograd import AdjointRun

    base = synth.c5_base()
    L = base.lattice
    setup = sg.PicSetup(grid=base.grid, lo=base.lo, hi=base.hi,
                        beam=(base.kinetic_eV, base.rest_eV, base.charge_e, base.bunch_charge_C),
                        lattice=(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods),
                        n_steps=base.total_steps())
    xi = base.xi()
    nom = np.concatenate([synth.NOMINAL_PARAMS, synth.SIGMA_NOMINAL])
    out = {"workload": base.name, "n_train": n_train}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xtr = synth.c5_inputs(n_train, seed=41)
    eps, jac, oob = sg.pic_targets(setup, xtr, xi, batch=512)
    torch.cuda.synchronize()
    out["t_pic_data_s"] = time.perf_counter() - t0
    out["out_of_box"] = int(oob.sum())
    net = sg.Surrogate(65536)
    net.set_normalization(nom, 0.05 * np.abs(nom), eps.mean(axis=0), eps.std(axis=0))
    net.set_params(sg.init_params(np.random.default_rng(42)))
    t0 = time.perf_counter()
    # Sobolev weights 1 (values) and 4 (gradients), batches of 1024, Adam with
    # a cosine decay from 2e-3 to 1e-4 (on the same data, 60 epochs at batches
    # of 512 and equal weights gave a held-out median gradient error of
    # 2.1e-3; 2000 epochs at these settings 1.5e-3)
    hist = net.fit(xtr, eps, jac, epochs=epochs, batch=1024, lr=2e-3, wj=4.0, seed=43)
    torch.cuda.synchronize()
    out["t_train_s"] = time.perf_counter() - t0
    out["loss_first_last"] = [hist[0], hist[-1]]
    xte = synth.c5_inputs(1024, seed=44)
    ete, jte, _ = sg.pic_targets(setup, xte, xi, batch=512)
    ep, jp = net.predict(xte)
    j_err = np.abs(sg.objective(ep) - sg.objective(ete)) / sg.objective(ete)
    gt, gp_ = jte[:, 0] + jte[:, 1], jp[:, 0] + jp[:, 1]
    g_err = np.abs(gp_ - gt).max(axis=1) / np.abs(gt).max(axis=1)
    out["heldout"] = {"J_rel_err_median": float(np.median(j_err)), "J_rel_err_max": float(j_err.max()),
                      "grad_rel_err_median": float(np.median(g_err)), "grad_within_1e-3": float(np.mean(g_err <= 1e-3)),
                      "fallback_rate": float(np.mean(g_err > 1e-3))}
    cand = synth.c5_inputs(65536, seed=45)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, j_pred, g_pred = sg.screen(net, cand, 64)
    out["t_screen_65536_s"] = time.perf_counter() - t0
    e_s, _, _ = sg.pic_targets(setup, cand[idx], xi, batch=64)
    e_r, _, _ = sg.pic_targets(setup, cand[:64], xi, batch=64)
    js, jr = sg.objective(e_s), sg.objective(e_r)
    # random search: how many of 4096 PIC-evaluated random candidates beat the screened best
    e_rr, _, _ = sg.pic_targets(setup, cand[64:64 + 4096], xi, batch=512)
    jrr = sg.objective(e_rr)
    out["screening"] = {"best_J_screened_64": float(js.min()), "best_J_random_64": float(jr.min()),
                        "best_J_random_4096": float(jrr.min()),
                        "random_runs_beating_screened_best_of_4096": int(np.sum(jrr < js.min()))}
    b = int(np.argmin(js))
    xb = cand[idx[b]]
    run = AdjointRun(base.n_particles, base.grid, base.lo, base.hi,
                     (base.kinetic_eV, base.rest_eV, base.charge_e, base.bunch_charge_C),
                     (L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods), xi, base.total_steps(),
                     checkpoint_every=50)
    run.forward(xb[:7], xb[7:])
    gpar, gsig = run.backward([1.0, 1.0, 0.0])
    ok, err = sg.judge(g_pred[b], np.concatenate([gpar, gsig]))
    out["judge"] = {"grad_rel_err": err, "within_1e-3": ok, "used": "surrogate" if ok else "PIC adjoint (fallback)"}
    net.close()
    return out


def _pipe2d_timing():
    """The paper's own instance: 2D beam in a conducting pipe (sine-series
    solver), 1e5 protons, 64^2 cells, one FODO cell of 100 steps, 7 tangents;
    and the matching example minimised by BFGS on its dual-number gradient."""
    import numpy as np
    import torch
    import synth
    from paper_2511_21839_amd import pipe2d as p2

    w = synth.pipe2d(n_particles=100_000)
    sim = p2.Pipe2D(w.n_particles, w.ntan, w.nx, w.ny)
    sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.current_A)
    sim.set_pipe(w.a, w.b)
    L = w.lattice
    sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
    sim.set_params(w.params, w.param_seed())
    xi = w.xi()
    sim.init_beam(xi, w.sigma)
    sim.step(5)
    sim.init_beam(xi, w.sigma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(w.total_steps())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e = sim.emittance()
    rel = e[:, 1:] * np.asarray(w.params)[None, :] / e[:, :1]
    m = synth.matching()
    cell = [0, 1, 0, 1, 0]
    Lc = [0.1, 0.1, 0.2, 0.1, 0.1]

    def periodic(kq):
        tw = p2.Twiss(cell, Lc, [0.0, kq[0], 0.0, kq[1], 0.0], [-1] * 5, [-1] * 5)
        return tw.eval(np.zeros((1, 0)))[0][:, 0]

    t_from, t_to = periodic(m.cell_from), periodic(m.cell_to)
    tw = p2.Twiss(m.kind, m.L, [0.0] * len(m.kind), [-1] * len(m.kind), m.k_param)
    _, fb, nb, _ = tw.match(m.k0, t_from, t_to, tol=1e-12, max_eval=1000)
    sim.close()
    return {"workload": w.name, "dual_particle_steps_per_s": w.n_particles * w.total_steps() / dt,
            "ms_per_step": dt / w.total_steps() * 1e3,
            "relative_sensitivities_eps_x": [float(v) for v in rel[0]],
            "relative_sensitivities_eps_y": [float(v) for v in rel[1]],
            "matching": {"bfgs_evaluations": nb, "bfgs_f": fb}}


def _copy_calibration(mib: int) -> int:
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the
    factor that turns counter KiB into HBM bytes for the same profiler setup."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "copies": 3}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sort-every", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the reverse-mode and batched timings")
    ap.add_argument("--surrogate-full", action="store_true",
                    help="also run the learned extension end to end (20k PIC runs, training, screening)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (to scale HBM byte counters)")
    args = ap.parse_args(argv)
    if args.copy_calibration:
        return _copy_calibration(args.copy_calibration)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the step would shard)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_2511_21839_amd import dpic

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    w = synth.c2()
    K, W = int(args.steps), int(args.warmup)
    if K < 1 or K > w.total_steps() or W < 0 or W > w.total_steps():
        print(f"--steps must be 1..{w.total_steps()} and --warmup 0..{w.total_steps()}", file=sys.stderr)
        return 2
    xi = w.xi()
    sim = dpic.Simulation(w.n_particles, w.ntan, w.grid)
    sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
    sim.set_grid(w.lo, w.hi)
    L = w.lattice
    sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
    sim.set_params(w.params, w.param_seed())
    sim.set_option(dpic.OPT_SORT_EVERY, args.sort_every)

    # warm-up on a first copy of the beam
    sim.init_beam(xi, w.sigma, w.sigma_seed())
    if W:
        sim.step(W)
    torch.cuda.synchronize()

    # timed: K steps from the start of the schedule, beam resident in HBM,
    # with HIP events around every particle launch (mode 2: two event
    # records per step; the plain launches, the one that also writes the
    # sort keys, the one that stores in sorted order, and a call's first and
    # last launch each move the whole state once)
    sim.init_beam(xi, w.sigma, w.sigma_seed())
    sim.set_option(dpic.OPT_STAGE_TIMING, 2)
    sim.stage_times()  # reset the stage timers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches = sim.stage_times()
    dt = t1 - t0
    oob, steps_done, extent = sim.counters()
    emit = sim.emittance()

    # outside the timed region, the same steps again: events around the
    # plain particle launches only (mode 3), then around every stage
    sim.init_beam(xi, w.sigma, w.sigma_seed())
    sim.set_option(dpic.OPT_STAGE_TIMING, 3)
    sim.stage_times()
    sim.step(K)
    torch.cuda.synchronize()
    pms, plaunches = sim.stage_times()
    sim.init_beam(xi, w.sigma, w.sigma_seed())
    sim.set_option(dpic.OPT_STAGE_TIMING, 1)
    sim.stage_times()
    sim.step(K)
    torch.cuda.synchronize()
    sms, slaunches = sim.stage_times()
    sim.set_option(dpic.OPT_STAGE_TIMING, 0)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    copy = _copy_rate()

    mix = _particle_launch_mix(K, args.sort_every)
    part_avg_s = ms[0] / 1e3 / max(int(launches[0]), 1)
    achieved = w.n_particles * BYTES_PER_PARTICLE_STEP / part_avg_s / 1e9
    plain_avg_s = pms[0] / 1e3 / max(int(plaunches[0]), 1)
    plain_achieved = w.n_particles * BYTES_PER_PARTICLE_STEP / plain_avg_s / 1e9
    line = {
        "metric": "dual particle-steps/s (7 tangents)",
        "value": w.n_particles * K / dt,
        "unit": "dual particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "n_particles": w.n_particles,
            "grid": list(w.grid),
            "fft_grid": [2 * g for g in w.grid],
            "ntan": w.ntan,
            "schedule_steps": w.total_steps(),
            "bunch_charge_C": w.bunch_charge_C,
            "sort_every": args.sort_every,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": _recorded_traffic(mix),
            "kernel": "fused particle kernel (gather, kick, half-maps, deposit): every launch of the timed steps",
            "timed_launches": int(launches[0]),
            "launch_mix": mix,
            "avg_launch_us": part_avg_s * 1e6,
            "plain_launches_only": {"kernel": "k_particles_tiled<8, 23>", "launches": int(plaunches[0]),
                                    "avg_launch_us": plain_avg_s * 1e6, "achieved": plain_achieved,
                                    "frac": plain_achieved / HBM_PEAK_GBS,
                                    "traffic": _recorded_traffic({"k_particles_tiled<8, 23>": 1})},
            "copy_ceiling": {"what": "device-to-device copy, 384 MiB each way", "GBps": copy["GBps"],
                             "frac_of_peak": copy["GBps"] / HBM_PEAK_GBS,
                             "kernel_over_copy": achieved / copy["GBps"]},
        },
        "stages_ms": {n: float(sms[i]) for i, n in enumerate(dpic.STAGE_TIMER_NAMES)},
        "stage_launches": {n: int(slaunches[i]) for i, n in enumerate(dpic.STAGE_TIMER_NAMES)},
        "checks": {"out_of_box": int(oob), "steps_done": int(steps_done),
                   "emittance_x": float(emit[0, 0]), "emittance_y": float(emit[1, 0]),
                   "finite": bool(np.isfinite(emit).all())},
    }
    _log(f"c2: {K} steps in {dt:.3f} s")
    if not args.no_extensions:
        line["c1"] = _c1_timing()
        _log("1e4-particle workload timed")
        line["adjoint"] = _adjoint_timing()
        line["adjoint"]["at_1e6_particles"] = _adjoint_scale_timing()
        _log("reverse mode timed")
        line["batched"] = _batched_timing()
        _log("batched runs timed")
        line["deterministic"] = _deterministic_timing()
        _log("deterministic mode timed")
        line["surrogate"] = _surrogate_timing()
        _log("surrogate timed")
        line["pipe2d"] = _pipe2d_timing()
        _log("2D pipe instance timed")
    if args.surrogate_full:
        line["surrogate_full"] = _surrogate_full()
        _log("surrogate pipeline done")
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        line["cpu_baseline"] = _cpu_baseline(w, xi, args.cpu_steps)
        _log("oracle timed")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
