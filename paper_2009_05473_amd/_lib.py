"""ctypes binding of libsfw (include/sfw.h): argument marshalling only.

Every entry point of the C ABI is exposed under the same name. Volumes, PSFs and atom
arrays are torch tensors on the GPU (float32, contiguous); torch supplies device memory
and the current HIP stream, all arithmetic runs in libsfw's kernels. There is no CPU
fallback: importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SFW_LIB_PATH: another build of the same library (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("SFW_LIB_PATH") or os.path.join(_HERE, "libsfw.so")

SFW_OK, SFW_EINVAL, SFW_ENOMEM, SFW_EHIP, SFW_ECAP, SFW_ENOCONV = 0, -1, -2, -3, -4, -5
SFW_MODE_BSFW, SFW_MODE_SFW = 0, 1
SFW_MAX_GRID = 16
SFW_CERT_MAX_KERNELS, SFW_CERT_MAX_RADIUS = 16, 40

EXPORTED = (
    "sfw_default_options", "sfw_workspace_create", "sfw_workspace_destroy",
    "sfw_workspace_set_stream", "sfw_last_error", "sfw_forward", "sfw_residual_grad",
    "sfw_adjoint", "sfw_forward_vjp", "sfw_certificate", "sfw_eta_points", "sfw_lasso_weights",
    "sfw_solve", "sfw_solve_batch", "sfw_profile_begin", "sfw_profile_end",
    "sfw_net_num_params", "sfw_net_create", "sfw_net_destroy", "sfw_net_set_params",
    "sfw_net_get_params", "sfw_net_forward", "sfw_net_gradients", "sfw_net_train_step",
    "sfw_net_propose", "sfw_eta_points_noalloc", "sfw_nnqp_batch",
)
SFW_NOALLOC_SCRATCH_BYTES, SFW_NOALLOC_MAX_POINTS = 1 << 20, 8
SFW_NNQP_MAX_K = 128
SFW_PROF_KINDS = 16


class SfwDims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class SfwAtom(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("w", "mx", "my", "mz", "sigma", "d")]


class SfwArgmax(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_float), ("i_sigma", ctypes.c_int32), ("i_d", ctypes.c_int32),
                ("x", ctypes.c_int32), ("y", ctypes.c_int32), ("z", ctypes.c_int32)]


class SfwOptions(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("n_sigma", ctypes.c_int32), ("n_d", ctypes.c_int32),
        ("sigma_grid", ctypes.c_float * SFW_MAX_GRID), ("d_grid", ctypes.c_float * SFW_MAX_GRID),
        ("sigma_lo", ctypes.c_float), ("sigma_hi", ctypes.c_float),
        ("d_lo", ctypes.c_float), ("d_hi", ctypes.c_float), ("trunc_T", ctypes.c_float),
        ("eta_tol", ctypes.c_double), ("prune_rel", ctypes.c_double), ("merge_tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("ascent_max_iter", ctypes.c_int32),
        ("slide_max_iter", ctypes.c_int32), ("ascent_gtol", ctypes.c_double),
        ("slide_gtol", ctypes.c_double), ("ftol", ctypes.c_double),
        ("lbfgs_memory", ctypes.c_int32), ("check_finite", ctypes.c_int32),
        ("verbose", ctypes.c_int32), ("proposal", ctypes.c_void_p),
        ("init_atoms", ctypes.c_void_p), ("n_init", ctypes.c_int32),
        ("slide_slope_tol", ctypes.c_double), ("graphs", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
    ]


class SfwStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("n_atoms", ctypes.c_int32),
        ("n_eval_cgrad", ctypes.c_int32), ("n_eval_eta", ctypes.c_int32),
        ("n_certificates", ctypes.c_int32), ("max_support", ctypes.c_int32),
        ("criterion", ctypes.c_double), ("last_eta", ctypes.c_double),
        ("seconds_total", ctypes.c_double), ("seconds_certificate", ctypes.c_double),
        ("seconds_ascent", ctypes.c_double), ("seconds_lasso", ctypes.c_double),
        ("seconds_slide", ctypes.c_double), ("n_proposals", ctypes.c_int32),
        ("n_fallbacks", ctypes.c_int32), ("n_graph_replays", ctypes.c_int32),
        ("n_tunings", ctypes.c_int32), ("n_ascent_iterations", ctypes.c_int32),
        ("n_slide_iterations", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class SfwBatchItem(ctypes.Structure):
    _fields_ = [
        ("y", ctypes.c_void_p), ("vol", SfwDims), ("H", ctypes.c_void_p), ("psf", SfwDims),
        ("lam", ctypes.c_float), ("atoms_out", ctypes.c_void_p), ("cap", ctypes.c_int32),
        ("n_out", ctypes.c_void_p), ("stats", ctypes.c_void_p), ("status", ctypes.c_int32),
    ]


class SfwProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int32), ("ms", ctypes.c_double)]


class SfwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsfw error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
    D = SfwDims
    sig = {
        "sfw_default_options": (i32, [ctypes.POINTER(SfwOptions)]),
        "sfw_workspace_create": (i32, [ctypes.POINTER(vp), D, D, i32, vp]),
        "sfw_workspace_destroy": (None, [vp]),
        "sfw_workspace_set_stream": (i32, [vp, vp]),
        "sfw_last_error": (ctypes.c_char_p, []),
        "sfw_forward": (i32, [vp, vp, D, D, vp, i32, vp]),
        "sfw_residual_grad": (i32, [vp, vp, D, D, vp, f32, vp, i32, vp, vp, vp]),
        "sfw_adjoint": (i32, [vp, vp, D, D, vp, vp]),
        "sfw_forward_vjp": (i32, [vp, vp, D, D, vp, vp, i32, vp]),
        "sfw_certificate": (i32, [vp, vp, D, D, vp, f32, vp, i32, vp, i32, f32, vp, vp]),
        "sfw_eta_points": (i32, [vp, D, vp, f32, vp, i32, vp, vp]),
        "sfw_eta_points_noalloc": (i32, [D, vp, f32, vp, i32, vp, vp, vp]),
        "sfw_nnqp_batch": (i32, [vp, vp, vp, i32, i32, vp, vp, vp]),
        "sfw_lasso_weights": (i32, [vp, vp, D, D, vp, f32, vp, i32, vp]),
        "sfw_solve": (i32, [vp, vp, D, vp, D, f32, ctypes.POINTER(SfwOptions), vp, i32,
                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(SfwStats)]),
        "sfw_solve_batch": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(SfwBatchItem), i32,
                                  ctypes.POINTER(SfwOptions)]),
        "sfw_profile_begin": (i32, [vp, ctypes.c_char_p]),
        "sfw_net_num_params": (i32, []),
        "sfw_net_create": (i32, [ctypes.POINTER(vp), D, vp]),
        "sfw_net_destroy": (None, [vp]),
        "sfw_net_set_params": (i32, [vp, vp, i32]),
        "sfw_net_get_params": (i32, [vp, vp, i32]),
        "sfw_net_forward": (i32, [vp, vp, D, f32, vp]),
        "sfw_net_gradients": (i32, [vp, vp, D, f32, vp, i32, vp, vp]),
        "sfw_net_train_step": (i32, [vp, vp, D, f32, vp, i32, f32, vp]),
        "sfw_net_propose": (i32, [vp, vp, D, f32, vp, vp]),
        "sfw_profile_end": (i32, [vp, ctypes.POINTER(SfwProfEntry), ctypes.POINTER(ctypes.c_int)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return (lib.sfw_last_error() or b"").decode()


def check(code: int, allow=()) -> int:
    if code != SFW_OK and code not in allow:
        raise SfwError(code, last_error())
    return code


def dims(shape) -> SfwDims:
    """(nz, ny, nx) -> sfw_dims."""
    nz, ny, nx = (int(v) for v in shape)
    return SfwDims(nx, ny, nz)


def _dev_ptr(t, dtype_name, what):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what}: must live on the GPU")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise ValueError(f"{what}: dtype must be {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def default_options(**overrides) -> SfwOptions:
    o = SfwOptions()
    check(lib.sfw_default_options(ctypes.byref(o)))
    for k, v in overrides.items():
        if k in ("sigma_grid", "d_grid"):
            vals = list(v)
            if len(vals) > SFW_MAX_GRID:
                raise ValueError(f"{k}: at most {SFW_MAX_GRID} values")
            arr = getattr(o, k)
            for i, x in enumerate(vals):
                arr[i] = float(x)
            setattr(o, "n_sigma" if k == "sigma_grid" else "n_d", len(vals))
        elif k == "mode" and isinstance(v, str):
            o.mode = {"BSFW": SFW_MODE_BSFW, "SFW": SFW_MODE_SFW}[v]
        else:
            setattr(o, k, v)
    return o


class Workspace:
    """Owns an sfw_workspace bound to the current device and to a stream: torch's current
    stream, or `stream` (a torch.cuda.Stream). Calls enqueue on that stream and return before
    their kernels finish; with a stream of its own, order it against the tensors' stream
    (torch.cuda.synchronize, events) before reading results or handing it new inputs."""

    def __init__(self, vol_max, psf_max, max_atoms, stream=None):
        self.handle = ctypes.c_void_p()
        self.vol_max = tuple(vol_max)
        self.psf_max = tuple(psf_max)
        self.max_atoms = int(max_atoms)
        check(lib.sfw_workspace_create(ctypes.byref(self.handle), dims(vol_max), dims(psf_max),
                                       int(max_atoms), _stream_handle(stream)))

    def close(self):
        if self.handle:
            lib.sfw_workspace_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------- entry points (same names)

def sfw_forward(ws: Workspace, H, atoms, vol_shape, phi_mu=None):
    import torch
    n = 0 if atoms is None else int(atoms.shape[0])
    if phi_mu is None:
        phi_mu = torch.empty(tuple(vol_shape), dtype=torch.float32, device="cuda")
    check(lib.sfw_forward(ws.handle, _dev_ptr(H, "float32", "H"), dims(H.shape), dims(vol_shape),
                          _dev_ptr(atoms, "float32", "atoms") if n else None, n,
                          _dev_ptr(phi_mu, "float32", "phi_mu")))
    return phi_mu


def sfw_residual_grad(ws: Workspace, H, y, lam, atoms, r_out=None, want_r=True, loss_out=None,
                      grad_out=None):
    """Returns (r, loss[1] float64 tensor, grad[n, 6] tensor). Output tensors may be passed in."""
    import torch
    n = 0 if atoms is None else int(atoms.shape[0])
    if want_r and r_out is None:
        r_out = torch.empty_like(y)
    loss = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float64, device="cuda")
    grad = grad_out if grad_out is not None else torch.empty((max(n, 1), 6), dtype=torch.float32,
                                                             device="cuda")
    check(lib.sfw_residual_grad(ws.handle, _dev_ptr(H, "float32", "H"), dims(H.shape),
                                dims(y.shape), _dev_ptr(y, "float32", "y"), float(lam),
                                _dev_ptr(atoms, "float32", "atoms") if n else None, n,
                                _dev_ptr(r_out, "float32", "r_out") if want_r else None,
                                _dev_ptr(loss, "float64", "loss"),
                                _dev_ptr(grad, "float32", "grad")))
    return r_out, loss, grad[:n]


def sfw_adjoint(ws: Workspace, H, r, q_out=None):
    import torch
    if q_out is None:
        q_out = torch.empty_like(r)
    check(lib.sfw_adjoint(ws.handle, _dev_ptr(H, "float32", "H"), dims(H.shape), dims(r.shape),
                          _dev_ptr(r, "float32", "r"), _dev_ptr(q_out, "float32", "q_out")))
    return q_out


def sfw_forward_vjp(ws: Workspace, H, g, atoms, grad_out=None):
    """Returns grad[n, 6] = d<g, Phi mu>/d(w, mx, my, mz, sigma, d) per atom."""
    import torch
    n = 0 if atoms is None else int(atoms.shape[0])
    grad = grad_out if grad_out is not None else torch.empty((max(n, 1), 6), dtype=torch.float32,
                                                             device="cuda")
    check(lib.sfw_forward_vjp(ws.handle, _dev_ptr(H, "float32", "H"), dims(H.shape),
                              dims(g.shape), _dev_ptr(g, "float32", "g"),
                              _dev_ptr(atoms, "float32", "atoms") if n else None, n,
                              _dev_ptr(grad, "float32", "grad") if n else None))
    return grad[:n]


def sfw_certificate(ws: Workspace, H, r, lam, sigma_grid, d_grid, trunc_T=12.0, want_eta=False,
                    vol_shape=None):
    """Returns (eta [ns, nd, nz, ny, nx] or None, argmax dict). r=None reuses the workspace's
    last q (then vol_shape is required)."""
    import torch
    sg = (ctypes.c_float * len(sigma_grid))(*[float(v) for v in sigma_grid])
    dg = (ctypes.c_float * len(d_grid))(*[float(v) for v in d_grid])
    vol = tuple(r.shape) if r is not None else tuple(vol_shape)
    eta = None
    if want_eta:
        eta = torch.empty((len(sigma_grid), len(d_grid)) + vol, dtype=torch.float32, device="cuda")
    best = SfwArgmax()  # host: the library synchronises and fills it
    check(lib.sfw_certificate(ws.handle, _dev_ptr(H, "float32", "H"), dims(H.shape), dims(vol),
                              _dev_ptr(r, "float32", "r"), float(lam),
                              ctypes.cast(sg, ctypes.c_void_p), len(sigma_grid),
                              ctypes.cast(dg, ctypes.c_void_p), len(d_grid), float(trunc_T),
                              _dev_ptr(eta, "float32", "eta") if want_eta else None,
                              ctypes.byref(best)))
    return eta, {"eta": float(best.eta), "i_sigma": int(best.i_sigma), "i_d": int(best.i_d),
                 "x": int(best.x), "y": int(best.y), "z": int(best.z)}


def sfw_eta_points(ws: Workspace, vol_shape, q, lam, thetas):
    """thetas: host array [n, 5]; q: device volume or None (workspace's q). Returns (eta, grad)."""
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float32).reshape(-1, 5))
    n = th.shape[0]
    eta = np.zeros(n, dtype=np.float64)
    grad = np.zeros((n, 5), dtype=np.float64)
    check(lib.sfw_eta_points(ws.handle, dims(vol_shape),
                             _dev_ptr(q, "float32", "q") if q is not None else None, float(lam),
                             th.ctypes.data_as(ctypes.c_void_p), n,
                             eta.ctypes.data_as(ctypes.c_void_p),
                             grad.ctypes.data_as(ctypes.c_void_p)))
    return eta, grad


def sfw_eta_points_noalloc(vol_shape, q, lam, thetas, eta_out=None, grad_out=None, stream=None):
    """thetas: host array [n, 5]; q: device volume; eta_out / grad_out: device float64 tensors
    [n] / [n, 5] (allocated here when None; the library call itself allocates nothing).
    Enqueues on `stream` (torch's current stream by default) and returns (eta, grad)."""
    import torch
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float32).reshape(-1, 5))
    n = th.shape[0]
    if eta_out is None:
        eta_out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    if grad_out is None:
        grad_out = torch.empty((max(n, 1), 5), dtype=torch.float64, device="cuda")
    check(lib.sfw_eta_points_noalloc(dims(vol_shape), _dev_ptr(q, "float32", "q"), float(lam),
                                     th.ctypes.data_as(ctypes.c_void_p), n,
                                     _dev_ptr(eta_out, "float64", "eta_out"),
                                     _dev_ptr(grad_out, "float64", "grad_out"),
                                     _stream_handle(stream)))
    return eta_out[:n], grad_out[:n]


def sfw_nnqp_batch(G, c, k=None, w_out=None, info_out=None, stream=None):
    """G: device float64 [count, kmax, kmax] (symmetric blocks), c: device float64
    [count, kmax], k: device int32 [count] or None (every problem of size kmax). Enqueues the
    batched weights QP on `stream` (torch's current stream by default); returns (w, info),
    device tensors [count, kmax] float64 and [count] int32 (allocated here when None)."""
    import torch
    if G.dim() != 3 or G.shape[1] != G.shape[2]:
        raise ValueError("G: expected [count, kmax, kmax]")
    count, kmax = int(G.shape[0]), int(G.shape[1])
    if tuple(c.shape) != (count, kmax):
        raise ValueError("c: expected [count, kmax]")
    if k is not None and tuple(k.shape) != (count,):
        raise ValueError("k: expected [count]")
    if w_out is None:
        w_out = torch.empty((count, kmax), dtype=torch.float64, device=G.device)
    if info_out is None:
        info_out = torch.empty(count, dtype=torch.int32, device=G.device)
    check(lib.sfw_nnqp_batch(_dev_ptr(G, "float64", "G"), _dev_ptr(c, "float64", "c"),
                             _dev_ptr(k, "int32", "k"), kmax, count,
                             _dev_ptr(w_out, "float64", "w_out"),
                             _dev_ptr(info_out, "int32", "info_out"), _stream_handle(stream)))
    return w_out, info_out


def sfw_lasso_weights(ws: Workspace, H, y, lam, atoms, w_out=None):
    import torch
    n = int(atoms.shape[0])
    w = w_out if w_out is not None else torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
    check(lib.sfw_lasso_weights(ws.handle, _dev_ptr(H, "float32", "H"), dims(H.shape),
                                dims(y.shape), _dev_ptr(y, "float32", "y"), float(lam),
                                _dev_ptr(atoms, "float32", "atoms"), n, _dev_ptr(w, "float64", "w")))
    return w[:n]


def atoms_host(atoms):
    """Host array [n, 6] (w, mx, my, mz, sigma, d) -> ctypes sfw_atom array (keep it alive)."""
    a = np.asarray(atoms, dtype=np.float64).reshape(-1, 6)
    arr = (SfwAtom * max(a.shape[0], 1))()
    for i, row in enumerate(a):
        arr[i] = SfwAtom(*[float(v) for v in row])
    return arr, a.shape[0]


def sfw_solve(ws: Workspace, y, H, lam, opts: SfwOptions | None = None, cap: int | None = None,
              init_atoms=None):
    """Returns (atoms [n, 6] float64 numpy, stats dict, status code). init_atoms: host array
    [k, 6] the solve starts from (sets opts.init_atoms / n_init for this call)."""
    cap = ws.max_atoms if cap is None else int(cap)
    init = None
    if init_atoms is not None:
        opts = opts if opts is not None else default_options()
        init, k = atoms_host(init_atoms)
        opts.init_atoms = ctypes.cast(init, ctypes.c_void_p)
        opts.n_init = k
    out = (SfwAtom * max(cap, 1))()
    n_out = ctypes.c_int(0)
    stats = SfwStats()
    code = lib.sfw_solve(ws.handle, _dev_ptr(y, "float32", "y"), dims(y.shape),
                         _dev_ptr(H, "float32", "H"), dims(H.shape), float(lam),
                         ctypes.byref(opts) if opts is not None else None,
                         ctypes.cast(out, ctypes.c_void_p), cap, ctypes.byref(n_out),
                         ctypes.byref(stats))
    check(code, allow=(SFW_ENOCONV,))
    n = n_out.value
    arr = np.array([[a.w, a.mx, a.my, a.mz, a.sigma, a.d] for a in out[:n]], dtype=np.float64)
    return arr.reshape(-1, 6), stats.as_dict(), code


def sfw_solve_batch(workspaces, problems, opts: SfwOptions | None = None, cap: int | None = None):
    """Independent solves: problems is a sequence of (y, H, lam) (device tensors, float);
    workspaces a sequence of Workspace, one host thread each. Returns one (atoms [n, 6] float64
    numpy, stats dict, status code) per problem, in order; raises on the first item (in
    order) whose status is neither SFW_OK nor SFW_ENOCONV."""
    wss = list(workspaces)
    cap = min(w.max_atoms for w in wss) if cap is None else int(cap)
    n = len(problems)
    items = (SfwBatchItem * max(n, 1))()
    outs, counts, stats = [], [], []
    for i, (y, H, lam) in enumerate(problems):
        out = (SfwAtom * max(cap, 1))()
        cnt = ctypes.c_int32(0)
        st = SfwStats()
        outs.append(out)
        counts.append(cnt)
        stats.append(st)
        it = items[i]
        it.y = _dev_ptr(y, "float32", "y")
        it.vol = dims(y.shape)
        it.H = _dev_ptr(H, "float32", "H")
        it.psf = dims(H.shape)
        it.lam = float(lam)
        it.atoms_out = ctypes.cast(out, ctypes.c_void_p)
        it.cap = cap
        it.n_out = ctypes.cast(ctypes.byref(cnt), ctypes.c_void_p)
        it.stats = ctypes.cast(ctypes.byref(st), ctypes.c_void_p)
        it.status = 0
    handles = (ctypes.c_void_p * len(wss))(*[w.handle.value for w in wss])
    lib.sfw_solve_batch(handles, len(wss), items, n, ctypes.byref(opts) if opts is not None else None)
    msg = last_error()
    res = []
    for i in range(n):
        code = items[i].status
        if code not in (SFW_OK, SFW_ENOCONV):
            raise SfwError(code, msg)
        k = counts[i].value
        arr = np.array([[a.w, a.mx, a.my, a.mz, a.sigma, a.d] for a in outs[i][:k]],
                       dtype=np.float64)
        res.append((arr.reshape(-1, 6), stats[i].as_dict(), code))
    return res


class Net:
    """The proposal network (sfw_net_*): parameters as one float32 vector in the library's
    master layout (per layer weights [co][ci][tz][ty][tx], then biases)."""

    def __init__(self, vol_max, stream=None):
        self.handle = ctypes.c_void_p()
        self.vol_max = tuple(vol_max)
        check(lib.sfw_net_create(ctypes.byref(self.handle), dims(vol_max), _stream_handle(stream)))
        self.num_params = int(lib.sfw_net_num_params())

    def close(self):
        if self.handle:
            lib.sfw_net_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        check(lib.sfw_net_set_params(self.handle, p.ctypes.data_as(ctypes.c_void_p), p.size))

    def get_params(self):
        p = np.zeros(self.num_params, dtype=np.float32)
        check(lib.sfw_net_get_params(self.handle, p.ctypes.data_as(ctypes.c_void_p), p.size))
        return p

    def forward(self, x, scale):
        """[(nz+1)/2, (ny+1)/2, (nx+1)/2, 4] float32 tensor (heatmap logit, sigma, d, unused)."""
        import torch
        half = tuple((n + 1) // 2 for n in x.shape)
        out = torch.empty(half + (4,), dtype=torch.float32, device="cuda")
        check(lib.sfw_net_forward(self.handle, _dev_ptr(x, "float32", "x"), dims(x.shape),
                                  float(scale), _dev_ptr(out, "float32", "out")))
        return out

    @staticmethod
    def _atoms(atoms):
        a = np.ascontiguousarray(np.asarray(atoms, dtype=np.float32).reshape(-1, 6))
        return a, a.shape[0]

    def gradients(self, x, scale, atoms):
        """(loss, grads float32 [num_params]) against the atoms still to be found."""
        a, k = self._atoms(atoms)
        loss = ctypes.c_double(0.0)
        g = np.zeros(self.num_params, dtype=np.float32)
        check(lib.sfw_net_gradients(self.handle, _dev_ptr(x, "float32", "x"), dims(x.shape),
                                    float(scale), a.ctypes.data_as(ctypes.c_void_p), k,
                                    ctypes.byref(loss), g.ctypes.data_as(ctypes.c_void_p)))
        return loss.value, g

    def train_step(self, x, scale, atoms, lr, want_loss=False):
        a, k = self._atoms(atoms)
        loss = ctypes.c_double(0.0)
        check(lib.sfw_net_train_step(self.handle, _dev_ptr(x, "float32", "x"), dims(x.shape),
                                     float(scale), a.ctypes.data_as(ctypes.c_void_p), k,
                                     float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def propose(self, x, scale):
        """(theta [5] = mx, my, mz, sigma, d, score)."""
        th = np.zeros(5, dtype=np.float64)
        sc = ctypes.c_double(0.0)
        check(lib.sfw_net_propose(self.handle, _dev_ptr(x, "float32", "x"), dims(x.shape),
                                  float(scale), th.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(sc)))
        return th, sc.value


def sfw_profile_begin(ws: Workspace, classes=None):
    """Time the named kernel classes (an iterable of names or a comma-separated string; None
    = every class) until sfw_profile_end."""
    if classes is not None and not isinstance(classes, str):
        classes = ",".join(classes)
    check(lib.sfw_profile_begin(ws.handle, classes.encode() if classes else None))


def sfw_profile_end(ws: Workspace):
    """Returns {class name: (launches, total ms)}."""
    arr = (SfwProfEntry * SFW_PROF_KINDS)()
    n = ctypes.c_int(0)
    check(lib.sfw_profile_end(ws.handle, arr, ctypes.byref(n)))
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].ms)) for i in range(n.value)}
