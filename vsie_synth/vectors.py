"""Seeded random test vectors."""
import numpy as np


def complex_normal(n, seed=1234, nrhs=None):
    """x ~ CN(0, 1): real and imaginary parts i.i.d. N(0, 1/2). Shape (n,) or (nrhs, n)."""
    rng = np.random.default_rng(seed)
    shape = (n,) if nrhs is None else (nrhs, n)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
