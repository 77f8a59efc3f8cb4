"""Seeded random draws shared by every workload.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).  The
draw order of each builder is fixed and documented where it is used.
"""

from __future__ import annotations

import numpy as np


def make_rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


def cn_vector(rng: np.random.Generator, n: int, std: float = 1.0 / np.sqrt(2.0)) -> np.ndarray:
    """Complex normal vector: real parts drawn first, then imaginary parts.

    ``std`` is the standard deviation of each of the real and imaginary
    parts; the default gives the circular CN(0, 1) law, E|z|^2 = 1.
    """
    re = rng.standard_normal(n) * std
    im = rng.standard_normal(n) * std
    return (re + 1j * im).astype(np.complex128)
