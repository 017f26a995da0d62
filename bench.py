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


def _recorded_traffic():
    """HBM bytes per launch of the particle kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when
    the kernel's sources changed since the counters were taken."""
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
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, AttributeError, KeyError, ValueError):
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

    def plain(ntan):
        sim = dpic.Simulation(w.n_particles, ntan, w.grid)
        sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
        sim.set_grid(w.lo, w.hi)
        sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
        sim.set_params(w.params, w.param_seed() if ntan else None)
        ss = w.sigma_seed() if ntan else None

        def go():
            sim.init_beam(xi, w.sigma, ss)
            sim.step(w.total_steps())
        return go, sim

    go13, s13 = plain(13)
    go0, s0 = plain(0)
    run = AdjointRun(w.n_particles, w.grid, w.lo, w.hi, (w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C),
                     (L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods), xi, w.total_steps(),
                     checkpoint_every=50)

    def adj():
        run.forward(w.params, w.sigma)
        run.backward([1.0, 1.0, 0.0])

    t13, t0, ta = _median_ms(go13), _median_ms(go0), _median_ms(adj)
    return {"workload": "1e4 protons, 32^3 grid, 100 steps, J = eps_x + eps_y, 13 gradient components",
            "checkpoint_every": 50, "t_forward_13_tangents_ms": t13, "t_value_only_ms": t0,
            "t_adjoint_ms": ta, "adjoint_over_forward_13": ta / t13, "adjoint_over_value_only": ta / t0}


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
    r4 = _batch_vs_singles(c4, c4.base.total_steps(), autotune_steps=20)
    r4["workload"] = c4.base.name
    b5 = synth.c5_batch(256, seed=7)
    r5 = _batch_vs_singles(b5, b5.base.total_steps(), graph=True)
    r5["workload"] = "256 settings of 1e4 protons, 32^3 grid, 100 steps, 13 tangents (inputs +-5%), graph replay"
    return {"c4": r4, "c1x256": r5}


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
    ap.add_argument("--sort-every", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the reverse-mode and batched timings")
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

    # timed: K steps from the start of the schedule, beam resident in HBM
    sim.init_beam(xi, w.sigma, w.sigma_seed())
    sim.set_option(dpic.OPT_STAGE_TIMING, 1)
    sim.stage_times()  # reset the stage timers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches = sim.stage_times()
    sim.set_option(dpic.OPT_STAGE_TIMING, 0)
    dt = t1 - t0
    oob, steps_done, extent = sim.counters()
    emit = sim.emittance()

    part_avg_s = ms[0] / 1e3 / max(int(launches[0]), 1)
    achieved = w.n_particles * BYTES_PER_PARTICLE_STEP / part_avg_s / 1e9
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
            "traffic": _recorded_traffic(),
            "kernel": "k_particles (gather, kick, two half-maps, deposit)",
            "avg_launch_us": part_avg_s * 1e6,
        },
        "stages_ms": {n: float(ms[i]) for i, n in enumerate(dpic.STAGE_TIMER_NAMES)},
        "stage_launches": {n: int(launches[i]) for i, n in enumerate(dpic.STAGE_TIMER_NAMES)},
        "checks": {"out_of_box": int(oob), "steps_done": int(steps_done),
                   "emittance_x": float(emit[0, 0]), "emittance_y": float(emit[1, 0]),
                   "finite": bool(np.isfinite(emit).all())},
    }
    if not args.no_extensions:
        line["adjoint"] = _adjoint_timing()
        line["batched"] = _batched_timing()
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        line["cpu_baseline"] = _cpu_baseline(w, xi, args.cpu_steps)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
