"""Host logic of bench.py that needs no GPU: the proposal comparison reports its own failure
in the record instead of losing the benchmark line, --gpus above 1 is refused, and the work
counts behind the roofline fractions."""
import os
import subprocess
import sys

import numpy as np
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


def test_work_counts_of_the_roofline_accounting():
    """The per-class work figures: evaluated voxel-atom pairs (every lane of every wave box the
    cut ball meets), the certificate passes' traffic and a LASSO column's box."""
    shape = (20, 12, 32)  # (nz, ny, nx)
    # a wide atom at the centre meets every 16 x 4 x 8 wave box; one far outside meets none
    wide = [1.0, 16.0, 6.0, 10.0, 4.0, 1.2]
    far = [1.0, 500.0, 500.0, 500.0, 0.5, 3.0]
    boxes = (32 // 16) * (12 // 4) * 3  # z boxes of 8, 8 and 4 planes
    assert bench.evaluated_pairs(shape, [wide], (16, 4, 8)) == (32 // 16) * (12 // 4) * 64 * 20
    assert bench.evaluated_pairs(shape, [far], (16, 4, 8)) == 0
    assert boxes == 18
    # a narrow atom: the count is the hit boxes' lanes times their planes
    narrow = [1.0, 3.0, 1.0, 2.0, 0.6, 3.0]
    r = 0.6 * (2 * 110.0) ** (1 / 3.0) * 1.0001 + 1e-3  # its cut radius, about 3.6 voxels
    hits = 0
    for z0 in range(0, 20, 8):
        for y0 in range(0, 12, 4):
            for x0 in range(0, 32, 16):
                z1, y1, x1 = min(z0 + 8, 20) - 1, y0 + 3, x0 + 15
                dx = max(0.0, x0 - 3.0, 3.0 - x1)
                dy = max(0.0, y0 - 1.0, 1.0 - y1)
                dz = max(0.0, z0 - 2.0, 2.0 - z1)
                if dx * dx + dy * dy + dz * dz <= r * r:
                    hits += 64 * (z1 - z0 + 1)
    assert bench.evaluated_pairs(shape, [narrow], (16, 4, 8)) == hits > 0
    # certificate passes at the bench grid: forward x, y, z, then the inverse y and x of 6 pairs
    Nx, Ny, Nz, nz, ny, nx = 150, 150, 81, 64, 128, 128
    fwd = (4 * nx * ny * nz + 8 * Nx * ny * nz) + (8 * Nx * ny * nz + 8 * Nx * Ny * nz) \
        + (8 * Nx * Ny * nz + 8 * Nx * Ny * Nz)
    inv = 6 * 8 * (Nx * Ny * nz + Nx * ny * nz) + 6 * 8 * Nx * ny * nz
    assert bench.cert_pass_bytes((nz, ny, nx), (Nx, Ny, Nz), 6) == fwd + inv
    # a column box inside the volume: 2 (radius + 1 + PSF half-width) + 1 per axis, x widened
    # to multiples of 4
    th = [60.0, 50.0, 30.0, 1.0, 2.0]
    R = 1.0 * (2 * 28.0) ** 0.5 + 1.0
    ext = [int(np.ceil(m + R + c) + 1) - int(np.floor(m - R - c))
           for m, c in zip(th[:3], (4.0, 4.0, 7.0))]
    lo_x = int(np.floor(60.0 - R - 4.0)) & ~3
    hi_x = (int(np.ceil(60.0 + R + 4.0) + 1) + 3) & ~3
    assert bench.column_box_voxels((64, 128, 128), th, (15, 9, 9)) == \
        (hi_x - lo_x) * ext[1] * ext[2]
