"""MI355X (gfx950) hot path of the boosted Sliding Frank-Wolfe solver for 3D deconvolution.

The compute path is libsfw.so (HIP kernels behind the C ABI of include/sfw.h); the
``_lib`` module is its ctypes binding. ``synth`` draws seeded synthetic workloads and
holds none of the solver's arithmetic. The binding is imported lazily so that the
drawer can be used on machines without the built library.
"""


def lib():
    """Return the ctypes binding, loading libsfw.so (raises ImportError if not built)."""
    from . import _lib
    return _lib
