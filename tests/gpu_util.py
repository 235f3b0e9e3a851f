"""Helpers shared by the GPU tests (device vectors, oracle caches)."""
import functools
import sys

import numpy as np

import oracle as O
from paper_2412_05082_amd.inputs import seeded_vector


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(v, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(v))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.double().cpu().numpy()


def rel_l2(a, b):
    d = np.linalg.norm(a - b)
    n = np.linalg.norm(b)
    return d / n if n else d


@functools.lru_cache(maxsize=None)
def oracle_ops(dim, k, N):
    A = O.assemble(dim, k, N)
    At = O.assemble(dim, k, N, bulk="diag")
    pidx = O.patch_indices(dim, k, N)
    return A, O.patch_blocks(At, pidx), pidx


def vectors(dim, k, N):
    return seeded_vector(dim, k, N, 1), seeded_vector(dim, k, N, 0)
