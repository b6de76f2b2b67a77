"""sfw_eta_points_noalloc (no workspace, fixed device scratch) against sfw_eta_points (workspace)
through the C ABI: two calls in a row, the second on a smaller volume with fewer points, each
within the float32 bars (eta relative 1e-5, gradient relative L2 1e-4) of the workspace path;
and the host-side rejections of sizes beyond the scratch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05473_amd import _lib
    return _lib


def _case(L, shape, npts, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    q = torch.from_numpy(rng.standard_normal(shape).astype(np.float32)).cuda()
    th = np.zeros((npts, 5), dtype=np.float32)
    th[:, 0] = rng.uniform(2, nx - 3, npts)
    th[:, 1] = rng.uniform(2, ny - 3, npts)
    th[:, 2] = rng.uniform(2, nz - 3, npts)
    th[:, 3] = rng.uniform(0.8, 2.5, npts)
    th[:, 4] = rng.uniform(1.3, 2.8, npts)
    return q, th


def test_noalloc_matches_workspace_path_twice(L):
    lam = 0.7
    for shape, npts, seed in (((64, 96, 128), 6, 71), ((32, 32, 32), 3, 72)):
        print("[case] sfw_eta_points_noalloc", shape, npts, flush=True)
        q, th = _case(L, shape, npts, seed)
        eta, grad = L.sfw_eta_points_noalloc(shape, q, lam, th)
        torch.cuda.synchronize()
        with L.Workspace(shape, (3, 3, 3), 16) as ws:
            eta_ref, grad_ref = L.sfw_eta_points(ws, shape, q, lam, th)
        eta, grad = eta.cpu().numpy(), grad.cpu().numpy()
        assert np.all(np.abs(eta - eta_ref) <= 1e-5 * np.abs(eta_ref) + 1e-12)
        assert np.linalg.norm(grad - grad_ref) <= 1e-4 * np.linalg.norm(grad_ref)


def test_noalloc_rejects_sizes_beyond_the_scratch(L):
    D = L.SfwDims
    th = np.ones((L.SFW_NOALLOC_MAX_POINTS + 1, 5), dtype=np.float32)
    out = torch.empty(16, dtype=torch.float64, device="cuda")
    q = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")
    args = lambda n: (D(8, 8, 8), ctypes.c_void_p(q.data_ptr()), 1.0,
                      th.ctypes.data_as(ctypes.c_void_p), n, ctypes.c_void_p(out.data_ptr()),
                      None, None)
    assert L.lib.sfw_eta_points_noalloc(*args(L.SFW_NOALLOC_MAX_POINTS + 1)) == L.SFW_EINVAL
    assert "SFW_NOALLOC_MAX_POINTS" in L.last_error()
    assert L.lib.sfw_eta_points_noalloc(*args(0)) == L.SFW_EINVAL
    # a volume whose tiles need more partials than the scratch holds: one point per 16 x 16 x 32
    # tile of a 4096 x 4096 x 64 volume with a very wide atom (no kernel is launched)
    wide = np.array([[2048, 2048, 32, 400.0, 1.2]], dtype=np.float32)
    assert L.lib.sfw_eta_points_noalloc(D(4096, 4096, 64), ctypes.c_void_p(q.data_ptr()), 1.0,
                                        wide.ctypes.data_as(ctypes.c_void_p), 1,
                                        ctypes.c_void_p(out.data_ptr()), None, None) == L.SFW_EINVAL
    assert "scratch" in L.last_error()
