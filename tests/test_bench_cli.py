"""The benchmark's command-line contract on the CPU: more than one GPU is refused with a
message (the multi-GPU path is not built), and the copy-calibration and argument parsing
need no GPU before that point."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_c1_cpu_baseline_runs_the_oracle_on_the_sound_wave():
    """The 16^3 degree-1 workload's CPU leg: the oracle on the modal sound wave, limiter
    only, enough steps for a stable figure; the state stays a small-amplitude wave."""
    import types

    import numpy as np

    sys.path.insert(0, ROOT)
    import bench
    import synthetic
    args = types.SimpleNamespace(workload="c1", seed=1, cpu_steps=10, cpu_cells=500, start_state=None,
                                 rho_floor_rel=0.1)
    rec = bench.run_cpu_baseline(args)
    assert rec["kind"] == "oracle" and rec["value"] > 0 and "200 SSP-RK3 steps" in rec["sample"]
    one = rec["one_core"]
    assert one["cores"] == 1 and one["value"] > 0 and one["all_cores_same_sample"] > 0 and "500 seeded cells" in one["sample"]
    assert bench._omp_threads() == rec["cores"]                   # the thread count is restored
    u = synthetic.c1_modal_state(1)
    assert u.shape == (4, 4, 16 ** 3)
    axis = synthetic.c1_axis(1)
    assert np.allclose(u[1 + axis, 0], u[0, 0] - 1.0)             # m = cs (rho - 1) for cs = 1
    assert np.abs(u[0, 0] - 1.0).max() <= 1e-3


def test_default_workload_is_the_largest_single_gpu_configuration():
    """With no flags the benchmark times 256^3 cells at degree 2 in FP64 (the plain method),
    from the seeded turbulence-like start state, 5 warm-up and 20 timed steps."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.DEFAULT_WORKLOAD == "c5" and bench.DEFAULT_WARMUP == 5
    N, k, prec, mach, _, spinup = bench.WORKLOADS["c5"]
    assert (N, k, prec, mach) == (256, 2, "fp64", 10.0) and bench.DEFAULT_WARMUP < spinup
