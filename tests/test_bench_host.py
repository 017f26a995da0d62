"""Host logic of bench.py: the particle-launch mix it weights the recorded
per-kernel traffic with, against the step loop's rules (one launch per step
plus the call's opening half-step; a re-sort after step s when (s + 1) is a
multiple of the cadence, except on a call's last step; with a cadence of 2
or more the keys are written two steps before and the sorted store replaces
the scatter)."""
import bench


def _sorts(n, R):
    return sum(1 for s in range(n - 1) if R > 0 and (s + 1) % R == 0)


def test_mix_counts_every_launch():
    for n in (1, 2, 3, 7, 20, 2000):
        for R in (0, 1, 2, 5, 7):
            mix = bench._particle_launch_mix(n, R)
            assert sum(mix.values()) == n + 1, (n, R, mix)
            pre = "k_particles_tiled" if R else "k_particles"
            assert mix[pre + "<8, 6>"] == 1
            assert mix[pre + ("<8, 19>" if R else "<8, 3>")] == 1


def test_mix_of_the_benchmark_call():
    mix = bench._particle_launch_mix(20, 5)
    assert mix == {"k_particles_tiled<8, 6>": 1, "k_particles_tiled<8, 23>": 13, "k_particles_tiled<8, 55>": 3,
                   "k_particles_sorted<8, 87>": 3, "k_particles_tiled<8, 19>": 1}
    mix = bench._particle_launch_mix(2000, 5)
    assert mix["k_particles_sorted<8, 87>"] == _sorts(2000, 5) == 399


def test_mix_without_folded_sorts():
    # no re-sort: the storage-order kernel on every step (no traffic record)
    assert bench._particle_launch_mix(10, 0) == {"k_particles<8, 6>": 1, "k_particles<8, 7>": 9,
                                                 "k_particles<8, 3>": 1}
    assert bench._recorded_traffic(bench._particle_launch_mix(10, 0)) is None
    # every step: the launch writes the keys and a plain sort follows
    mix = bench._particle_launch_mix(10, 1)
    assert mix.get("k_particles_sorted<8, 87>", 0) == 0
    assert mix["k_particles_tiled<8, 55>"] == _sorts(10, 1) == 9
