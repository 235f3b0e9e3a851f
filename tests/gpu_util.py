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


EPS64 = np.finfo(np.float64).eps


@functools.lru_cache(maxsize=None)
def patch_condition(dim, k, N):
    """Largest 2-norm condition number of the separable patch matrices."""
    _, blocks, _ = oracle_ops(dim, k, N)
    return float(max(np.linalg.cond(blocks[i]) for i in range(0, len(blocks), max(1, len(blocks) // 16))))


def fp64_tol(dim, k, N):
    """1e-12, or 2 kappa(A~_v) eps where the local solves are worse
    conditioned: two correct float64 inverses of A~_v then differ by up to
    about kappa eps in relative terms."""
    return max(1e-12, 2.0 * patch_condition(dim, k, min(N, 8)) * EPS64)


EPS32 = float(np.finfo(np.float32).eps)


def fp32_tol(dim, k, N):
    """1e-5, or 0.05 kappa(A~_v) eps32 where the patch matrices are worse
    conditioned (k >= 5): a float32 residual of a high-frequency input has
    rounding error ~eps32 |r| in every mode, and the local solve amplifies
    its low modes by up to kappa; measured errors are 0.01-0.07 kappa eps32."""
    return max(1e-5, 0.05 * patch_condition(dim, k, min(N, 8)) * EPS32)
