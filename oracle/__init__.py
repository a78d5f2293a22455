"""CPU oracle for polynomial-preconditioned CG (test infrastructure only).

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark use
this package.  The GPU library never imports, links or calls it.
"""
from .oracle import *  # noqa: F401,F403
from . import mlp  # noqa: F401,E402
