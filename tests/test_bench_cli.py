"""Host logic of bench.py that needs no GPU: the proposal comparison reports its own failure
in the record instead of losing the benchmark line, and --gpus above 1 is refused."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


class _NoNet:
    """Stands in for the binding: creating the network fails as it would on a broken device."""

    class Net:
        def __init__(self, shape):
            raise RuntimeError("no device")


def test_proposal_failure_is_recorded():
    rec = bench.proposal_run(_NoNet, (8, 8, 8), steps=10, volumes=2)
    assert rec["train_steps"] == 10
    assert rec["error"] == "RuntimeError: no device"
    assert "speedup" not in rec


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))
