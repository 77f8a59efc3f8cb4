"""CPU oracle for the Helmholtz Krylov path -- TEST INFRASTRUCTURE ONLY.

Imported by ``tests/``, the package smoke check and the CPU-baseline leg of
``bench.py``; never by the GPU library or its binding.
"""

from .oracle import *  # noqa: F401,F403
from .oracle import lib, STATUS_NAMES  # noqa: F401
