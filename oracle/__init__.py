"""FP64 CPU oracle for the boosted Sliding Frank-Wolfe (BSFW) 3D deconvolution hot path.

TEST INFRASTRUCTURE ONLY. This package is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``,
and by nothing else. The GPU library never imports, links or calls it, and
it imports nothing from the GPU library: the two share only the seeded input
drawer (``paper_2009_05473_amd.synth``), which holds none of the method's
arithmetic.

Every function cites the passage of Courbot & Colicchio, "Boosting the
Sliding Frank-Wolfe solver for 3D deconvolution" (arXiv:2009.05473) that it
follows. Parity status of each function is listed in ``oracle.sfw``'s header.
"""
from .sfw import *  # noqa: F401,F403
