"""bench.py's command-line contract on the host (no GPU): workload names,
the periodic box of any shape, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_periodic_workload_shape():
    name, bx, wg, ph = bench.workload("periodic:24x16x8")
    assert name == "periodic_24x16x8"
    assert (bx["nx"], bx["ny"], bx["nz"]) == (24, 16, 8)
    assert bx["bc"] == [0] * 6 and wg == []
    assert ph["kind"] == "lattice" and ph["u0"].shape == (3, 8, 16, 24)


@pytest.mark.parametrize("spec", ["periodic:24x16", "periodic:axbxc", "nosuch"])
def test_bad_workload_names(spec):
    with pytest.raises(SystemExit):
        bench.workload(spec)


def test_headline_workloads():
    assert bench.workload("cf")[0] == "clap_fling_256x192x192"
    assert bench.workload("large")[0] == "clap_fling_512x384x384"


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
