"""Voxel phantoms: a homogeneous sphere and a head-like set of nested seeded ellipsoids."""
from dataclasses import dataclass

import numpy as np


@dataclass
class Grid:
    """Uniform voxel grid with a complex-permittivity description per voxel.

    ``eps_r`` and ``sigma`` have shape (n3, n2, n1); air is eps_r = 1, sigma = 0.
    ``labels`` is 0 for air and 1..5 for tissue classes (informational).
    """
    n: tuple
    h: float
    origin: np.ndarray
    eps_r: np.ndarray
    sigma: np.ndarray
    labels: np.ndarray

    @property
    def n_v(self):
        return int(self.n[0] * self.n[1] * self.n[2])

    def centres(self):
        """Voxel-centre coordinates, shape (n3, n2, n1, 3)."""
        i1 = self.origin[0] + (np.arange(self.n[0]) + 0.5) * self.h
        i2 = self.origin[1] + (np.arange(self.n[1]) + 0.5) * self.h
        i3 = self.origin[2] + (np.arange(self.n[2]) + 0.5) * self.h
        z, y, x = np.meshgrid(i3, i2, i1, indexing="ij")
        return np.stack([x, y, z], axis=-1)

    def tissue(self):
        """Boolean mask of voxels that carry polarisation current (eps_r != 1 or sigma != 0)."""
        return (self.eps_r != 1.0) | (self.sigma != 0.0)


def sphere_phantom(n=(16, 16, 16), h=5e-3, radius=35e-3, eps_r=52.0, sigma=0.55):
    """Homogeneous sphere centred in a box of n voxels; voxels whose centre lies inside are tissue."""
    n = tuple(int(v) for v in n)
    origin = -0.5 * h * np.array(n, dtype=np.float64)
    g = Grid(n, float(h), origin, np.ones(n[::-1]), np.zeros(n[::-1]), np.zeros(n[::-1], np.int32))
    c = g.centres()
    inside = (c ** 2).sum(-1) < radius ** 2
    g.eps_r[inside] = eps_r
    g.sigma[inside] = sigma
    g.labels[inside] = 1
    return g


def random_block(n, h=5e-3, seed=0):
    """Every voxel of an n-voxel box is tissue with eps_r ~ U[1.5, 80] and sigma ~ U[0, 0.9] S/m
    (seeded): a body with no air, for grids of any shape."""
    n = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    origin = -0.5 * h * np.array(n, dtype=np.float64)
    eps = 1.5 + 78.5 * rng.random(n[::-1])
    sig = 0.9 * rng.random(n[::-1])
    return Grid(n, float(h), origin, eps, sig, np.ones(n[::-1], np.int32))


def head_phantom(seed, n=(96, 112, 128), h=2e-3):
    """Five nested seeded ellipsoids, labels 1..5 from outside in, air outside.

    Outer semi-axes 0.8 * half-extent * (1 + 0.05 U(-1, 1)); inner ellipsoids scaled by
    (0.85, 0.65, 0.45, 0.25) * (1 + 0.05 U) with centres jittered by up to 0.1 of the outer
    semi-axes and resampled until contained in their parent. Per label eps_r ~ U[40, 80] and
    sigma ~ U[0.3, 0.9] S/m.
    """
    rng = np.random.default_rng(seed)
    n = tuple(int(v) for v in n)
    half = 0.5 * h * np.array(n, dtype=np.float64)
    origin = -half
    a0 = 0.8 * half * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, 3))
    axes = [a0]
    centres = [np.zeros(3)]
    for s in (0.85, 0.65, 0.45, 0.25):
        for _ in range(1000):
            a = s * a0 * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, 3))
            c = centres[-1] + 0.1 * a0 * rng.uniform(-1.0, 1.0, 3)
            # contained in the parent: every point of the child box hull lies inside the parent
            pa, pc = axes[-1], centres[-1]
            if np.all(np.abs(c - pc) + a < pa * 0.98):
                break
        axes.append(a)
        centres.append(c)
    g = Grid(n, float(h), origin, np.ones(n[::-1]), np.zeros(n[::-1]), np.zeros(n[::-1], np.int32))
    x = g.centres()
    for lab, (a, c) in enumerate(zip(axes, centres), start=1):
        inside = ((((x - c) / a) ** 2).sum(-1)) < 1.0
        g.labels[inside] = lab
    eps = rng.uniform(40.0, 80.0, 5)
    sig = rng.uniform(0.3, 0.9, 5)
    for lab in range(1, 6):
        m = g.labels == lab
        g.eps_r[m] = eps[lab - 1]
        g.sigma[m] = sig[lab - 1]
    return g
