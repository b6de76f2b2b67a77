"""CPU checks of the C ABI: the library loads, exports every declared entry point, and
rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfw.h")
LIB = os.path.join(ROOT, "paper_2009_05473_amd", "libsfw.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsfw.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfw_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sfw_forward", "sfw_residual_grad", "sfw_certificate", "sfw_lasso_weights",
              "sfw_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2009_05473_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_default_options():
    from paper_2009_05473_amd import _lib
    o = _lib.default_options()
    assert o.mode == _lib.SFW_MODE_BSFW
    assert o.n_sigma == 4 and o.n_d == 3
    assert list(o.d_grid)[:3] == [1.5, 2.0, 2.5]
    assert abs(o.sigma_grid[1] - 4.0 / 3.0) < 1e-6
    assert (o.sigma_lo, o.sigma_hi, o.d_lo, o.d_hi) == (0.5, 4.0, pytest.approx(1.2), 3.0)
    assert o.eta_tol == 1e-3 and o.prune_rel == 1e-6 and o.max_iter == 200
    o2 = _lib.default_options(mode="SFW", sigma_grid=[1, 2], d_grid=[2])
    assert o2.mode == _lib.SFW_MODE_SFW and o2.n_sigma == 2 and o2.n_d == 1


def test_workspace_create_rejects_bad_arguments():
    from paper_2009_05473_amd import _lib
    h = ctypes.c_void_p()
    D = _lib.SfwDims
    assert _lib.lib.sfw_workspace_create(ctypes.byref(h), D(0, 4, 4), D(3, 3, 3), 4, None) == _lib.SFW_EINVAL
    assert "positive" in _lib.last_error()
    assert _lib.lib.sfw_workspace_create(ctypes.byref(h), D(8, 8, 8), D(4, 3, 3), 4, None) == _lib.SFW_EINVAL
    assert "odd" in _lib.last_error()
    assert _lib.lib.sfw_workspace_create(ctypes.byref(h), D(8, 8, 8), D(3, 3, 3), 0, None) == _lib.SFW_EINVAL
    assert "max_atoms" in _lib.last_error()
    assert _lib.lib.sfw_workspace_create(None, D(8, 8, 8), D(3, 3, 3), 4, None) == _lib.SFW_EINVAL


def test_operators_reject_null_workspace_and_bad_lambda():
    from paper_2009_05473_amd import _lib
    D = _lib.SfwDims
    L = _lib.lib
    assert L.sfw_forward(None, None, D(3, 3, 3), D(8, 8, 8), None, 0, None) == _lib.SFW_EINVAL
    assert "workspace" in _lib.last_error()
    assert L.sfw_residual_grad(None, None, D(3, 3, 3), D(8, 8, 8), None, 1.0, None, 0, None, None,
                               None) == _lib.SFW_EINVAL
    assert L.sfw_certificate(None, None, D(3, 3, 3), D(8, 8, 8), None, 1.0, None, 1, None, 1, 12.0,
                             None, None) == _lib.SFW_EINVAL
    assert L.sfw_lasso_weights(None, None, D(3, 3, 3), D(8, 8, 8), None, 1.0, None, 1,
                               None) == _lib.SFW_EINVAL
    n = ctypes.c_int()
    assert L.sfw_solve(None, None, D(8, 8, 8), None, D(3, 3, 3), 1.0, None, None, 0, ctypes.byref(n),
                       None) == _lib.SFW_EINVAL
    assert L.sfw_default_options(None) == _lib.SFW_EINVAL
    assert L.sfw_workspace_set_stream(None, None) == _lib.SFW_EINVAL


def test_solve_batch_validates_before_touching_the_gpu():
    from paper_2009_05473_amd import _lib
    L = _lib.lib
    item = (_lib.SfwBatchItem * 1)()
    assert L.sfw_solve_batch(None, 0, None, 0, None) == _lib.SFW_OK  # nothing to solve
    assert L.sfw_solve_batch(None, 0, item, 1, None) == _lib.SFW_EINVAL
    assert "workspace" in _lib.last_error()
    assert L.sfw_solve_batch(None, 1, item, -1, None) == _lib.SFW_EINVAL
    nulls = (ctypes.c_void_p * 2)(None, None)
    assert L.sfw_solve_batch(nulls, 2, item, 1, None) == _lib.SFW_EINVAL
    assert "NULL" in _lib.last_error()
    fake = (ctypes.c_void_p * 2)(0x1000, 0x1000)  # never dereferenced: rejected as a repeat
    assert L.sfw_solve_batch(fake, 2, item, 1, None) == _lib.SFW_EINVAL
    assert "twice" in _lib.last_error()


def test_last_error_is_thread_local():
    import threading
    from paper_2009_05473_amd import _lib
    D = _lib.SfwDims
    _lib.lib.sfw_forward(None, None, D(3, 3, 3), D(8, 8, 8), None, 0, None)
    seen = {}

    def worker():
        seen["msg"] = _lib.last_error()

    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert seen["msg"] == ""
    assert "workspace" in _lib.last_error()


def test_net_entry_points_validate_before_touching_the_gpu():
    from paper_2009_05473_amd import _lib
    L = _lib.lib
    D = _lib.SfwDims
    # per layer weights [co][ci][3][3][3] then biases: (32, 1), (32, 32), (32, 32), (3, 32)
    assert L.sfw_net_num_params() == (32 * 27 + 32) + 2 * (32 * 32 * 27 + 32) + (3 * 32 * 27 + 3)
    assert L.sfw_net_create(None, D(8, 8, 8), None) == _lib.SFW_EINVAL
    assert L.sfw_net_set_params(None, None, 0) == _lib.SFW_EINVAL
    assert L.sfw_net_get_params(None, None, 0) == _lib.SFW_EINVAL
    assert L.sfw_net_forward(None, None, D(8, 8, 8), 1.0, None) == _lib.SFW_EINVAL
    assert "net" in _lib.last_error()
    assert L.sfw_net_gradients(None, None, D(8, 8, 8), 1.0, None, 0, None, None) == _lib.SFW_EINVAL
    assert L.sfw_net_train_step(None, None, D(8, 8, 8), 1.0, None, 0, 1e-3, None) == _lib.SFW_EINVAL
    assert L.sfw_net_propose(None, None, D(8, 8, 8), 1.0, None, None) == _lib.SFW_EINVAL
    L.sfw_net_destroy(None)  # no-op


def test_nnqp_batch_validates_before_touching_the_gpu():
    from paper_2009_05473_amd import _lib
    L = _lib.lib
    text = open(HEADER).read()
    assert int(re.search(r"#define SFW_NNQP_MAX_K (\d+)", text).group(1)) == _lib.SFW_NNQP_MAX_K
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below fails its host checks
    assert L.sfw_nnqp_batch(fake, fake, None, _lib.SFW_NNQP_MAX_K + 1, 1, fake, None, None) == _lib.SFW_EINVAL
    assert "SFW_NNQP_MAX_K" in _lib.last_error()
    assert L.sfw_nnqp_batch(fake, fake, None, 4, -1, fake, None, None) == _lib.SFW_EINVAL
    assert L.sfw_nnqp_batch(fake, fake, None, -1, 1, fake, None, None) == _lib.SFW_EINVAL
    assert L.sfw_nnqp_batch(None, fake, None, 4, 1, fake, None, None) == _lib.SFW_EINVAL
    assert L.sfw_nnqp_batch(fake, fake, None, 4, 1, None, None, None) == _lib.SFW_EINVAL
    assert "NULL" in _lib.last_error()
    assert L.sfw_nnqp_batch(None, None, None, 4, 0, None, None, None) == _lib.SFW_OK  # no-op
    assert L.sfw_nnqp_batch(None, None, None, 0, 3, None, None, None) == _lib.SFW_OK
