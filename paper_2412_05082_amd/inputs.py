"""Seeded synthetic input vectors (shared by the tests, the bench and the
smoke run; holds none of the method's arithmetic).

Every vector is ``numpy.random.default_rng(seed).uniform(-1, 1, n)`` over the
(kN+1)^d nodes in lexicographic order (x fastest), float64, with the
boundary-node entries then set to 0.
"""
from __future__ import annotations

import numpy as np


def boundary_nodes(dim: int, degree: int, n_cells: int) -> np.ndarray:
    n1 = degree * n_cells + 1
    idx = np.arange(n1)
    edge = (idx == 0) | (idx == n1 - 1)
    if dim == 2:
        return (edge[None, :] | edge[:, None]).ravel()
    return (edge[None, None, :] | edge[None, :, None] | edge[:, None, None]).ravel()


def seeded_vector(dim: int, degree: int, n_cells: int, seed: int) -> np.ndarray:
    n1 = degree * n_cells + 1
    v = np.random.default_rng(seed).uniform(-1.0, 1.0, n1 ** dim)
    v[boundary_nodes(dim, degree, n_cells)] = 0.0
    return v
