"""Host-side pieces of the benchmark that run without a GPU: the CPU
description reported with the oracle baseline and the line contract for
more than one GPU."""
import os
import subprocess
import sys

import bench


def _expand(mask: str):
    cpus = set()
    for part in mask.split(","):
        a, _, b = part.partition("-")
        cpus.update(range(int(a), int(b or a) + 1))
    return cpus


def test_host_cpu_affinity_round_trips():
    model, mask, nproc = bench.host_cpu()
    assert isinstance(model, str) and model
    assert _expand(mask) == set(os.sched_getaffinity(0))
    assert nproc == os.cpu_count()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
