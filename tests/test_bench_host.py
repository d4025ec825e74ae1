"""Host logic of bench.py that needs no GPU: the one-GPU refusal, the
algorithmic flop count of a Newton launch with a plan, and the rule that the
HBM traffic figure is withdrawn once the profiled kernel source changes."""
import importlib.util
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_newton_flops_with_plan_by_hand():
    B = load_bench()
    # one BVP, N = 2, one iteration: 1 * 2 * 4422 solve + 2 * 3 * 220 residual
    # evaluations + 3 * 144 for the first step formed from the plan
    assert B.newton_flops_plan(2, np.array([1])) == 2 * 4422 + 2 * 3 * 220 + 3 * 144
    # a BVP converged at its test (0 iterations) still costs one evaluation
    assert B.newton_flops_plan(2, np.array([0])) == 3 * 220 + 3 * 144
    # per-BVP meshes
    assert B.newton_flops_plan(np.array([2, 4]), np.array([1, 0])) == (2 * 4422 + 6 * 220 + 3 * 144) + (5 * 220 + 5 * 144)


def test_traffic_is_withdrawn_when_the_kernel_source_changes(tmp_path):
    B = load_bench()
    src = tmp_path / "kernel.hip"
    src.write_text("// a kernel\n")
    import hashlib
    h = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "counters.md"
    summary.write_text("sha256: %s\ntraffic_bytes_per_launch: 3.31e+09\n" % h)
    B.COUNTERS_FILE, B.KERNEL_SOURCE = str(summary), str(src)
    assert B.measured_traffic() == 3.31e9
    src.write_text("// the kernel, edited\n")
    assert B.measured_traffic() is None


def test_newton_flops_per_interval_step():
    B = load_bench()
    # 6.5 kflop per interval and linear solve: iters + 1 solves without a
    # plan, iters with one
    assert B.newton_flops(256, np.array([3])) == 6500.0 * 256 * 4
    assert B.newton_flops(256, np.array([3]), plan=True) == 6500.0 * 256 * 3
    assert B.newton_flops(np.array([64, 128]), np.array([0, 2])) == 6500.0 * (64 + 128 * 3)


def test_eval_flops_per_query_algorithmic_counts():
    # 2 m M + sum over nodes of (non-trivial dimensions - 1) + 6 x 5 flops per
    # point of X^2..X^{level+1}: 810, 3,344, 12,242 and 40,928 flops per query
    # (m = 3) at levels 2..5
    from oracle import oracle as O
    B = load_bench()
    for level, want in ((2, 810), (3, 3344), (4, 12242), (5, 40928)):
        keys = O.grid(6, level).keys
        assert B.eval_flops_per_query(keys, level, 3) == want, level


def test_cpu_model_is_named():
    B = load_bench()
    assert isinstance(B.cpu_model(), str) and B.cpu_model()


def test_swept_steps_by_hand():
    B = load_bench()
    iters = np.array([0, 2, 3, 4] * 16)  # 64 BVPs: the first steps from the six unit states' (by doubling)
    r = B.swept_steps_roofline(256, iters, len(iters), 1.0)
    assert r["interval_steps"] == 256 * iters.sum()
    assert np.isclose(r["flops"], 6500.0 * r["interval_steps"])
    assert np.isclose(r["achieved"], r["flops"] / 1e-3 / 1e12) and np.isclose(r["frac"], r["achieved"] / 78.6)
    # below 64 BVPs every BVP sweeps its own first step: the per-BVP count
    small = B.swept_steps_roofline(256, iters[:63], 63, 1.0)
    assert small["interval_steps"] == 256 * (iters[:63] + 1).sum()
    assert np.isclose(small["flops"], B.newton_flops(256, iters[:63]))
