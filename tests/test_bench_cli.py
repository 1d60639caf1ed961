"""bench.py's command line on the CPU: more than one GPU is refused with a
message before any device work; the coarse kernel's algorithmic bytes follow
the multigrid hierarchy."""
import os
import subprocess
import sys

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_coarse_kernel_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    p = W.config2().params   # 256 x 64: levels 64x16 (1024 cells), 32x8, 16x4 (dense)
    levels, lg = bench.mg_levels(p.nx, p.ny, 1024)
    assert levels[lg] == (64, 16) and levels[-1] == (16, 4)
    coef = sum(a * b + a * (b + 1) for a, b in levels[lg:])   # x- and y-faces
    assert bench.algo_bytes_per_launch("mg_coarse", p) == 8 * (2 * 1024 + coef + 64 * 64)


def test_batch_bytes_sum_over_instances():
    """A batched launch covers every instance: its algorithmic bytes are the
    sum of the per-instance figures."""
    sys.path.insert(0, ROOT)
    import bench
    cases = W.config4()
    ps = [c.params for c in cases]
    assert bench.algo_bytes_per_launch("stage", ps) == sum(
        bench.algo_bytes_per_launch("stage", p) for p in ps)
    assert bench.algo_bytes_per_launch("mg_coarse", ps, 4096) == sum(
        bench.algo_bytes_per_launch("mg_coarse", p, 4096) for p in ps)
    assert sum(p.nx * p.ny for p in ps) == 3899904
