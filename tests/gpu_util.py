"""Helpers shared by the GPU tests (device vectors, oracle caches, and the
parity bars with the measurements behind them)."""
import functools
import math
import sys

import numpy as np
import scipy.sparse as sp

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


def check(name, err, bar):
    """Assert err <= bar and print both (the GPU log keeps the measured
    errors that the tolerance tables are built from)."""
    say(f"  [{name}] err {err:.3e} bar {bar:.3e}")
    assert err <= bar, (name, err, bar)


@functools.lru_cache(maxsize=None)
def oracle_ops(dim, k, N):
    A = O.assemble(dim, k, N)
    At = O.assemble(dim, k, N, bulk="diag")
    pidx = O.patch_indices(dim, k, N)
    return A, O.patch_blocks(At, pidx), pidx


def vectors(dim, k, N):
    return seeded_vector(dim, k, N, 1), seeded_vector(dim, k, N, 0)


EPS64 = float(np.finfo(np.float64).eps)
EPS32 = float(np.finfo(np.float32).eps)


@functools.lru_cache(maxsize=None)
def patch_condition(dim, k, N):
    """Largest 2-norm condition number of the separable patch matrices."""
    _, blocks, _ = oracle_ops(dim, k, N)
    return float(max(np.linalg.cond(blocks[i]) for i in range(0, len(blocks), max(1, len(blocks) // 16))))


def _small_N(dim, k, N):
    """The mesh on which a rounding floor is measured: the test's own mesh
    when the oracle handles it in a second or two, else the largest smaller
    one (the floors depend on k, hardly on N)."""
    cap = 60_000 if dim == 2 else 25_000
    while N > 2 and (k * N + 1) ** dim > cap:
        N //= 2
    return N


def fp64_tol(dim, k, N):
    """1e-12, or 2 kappa(A~_v) eps where the local solves are worse
    conditioned (k >= 5): two correct float64 inverses of A~_v differ by up
    to about kappa eps in relative terms (the oracle's LU and Cholesky local
    solvers agree far inside it: tests/test_oracle_precision.py)."""
    return max(1e-12, 2.0 * patch_condition(dim, k, min(N, 8)) * EPS64)


def fp64_vcycle_tol(dim, k, N, pre=1, post=1):
    """Bar for a float64 V-cycle: every smoothing step adds at most the
    smoother bar, the transfers and the coarse solve a few eps, and the
    V-cycle's error propagation does not amplify earlier errors (its
    iteration operator is a contraction), so the errors add at most
    linearly over the L (pre + post) steps (L levels above the coarse one)."""
    L = int(round(math.log2(N))) - 1
    return (L * (pre + post) + 1) * fp64_tol(dim, k, N)


@functools.lru_cache(maxsize=None)
def fp32_residual_floor(dim, k, N, omega):
    """Rounding floor of a float32 smoother step S(x, b) on the seeded
    inputs: the error of x + omega sum_v R_v^T A~_v^{-1} R_v fl32(b - A x)
    -- residual formed in float32, local solves exact (float64 LU) --
    against the float64 step on the same float32-rounded inputs.  Any
    float32 residual of a high-frequency x carries ~eps32 |A||x| rounding in
    every mode, which a local solve amplifies by up to kappa(A~_v); this is
    the part of the error no float32 smoother can avoid.  Measured (2D,
    omega 1/4): 5e-7, 3.4e-6, 1.2e-5, 3.7e-5, 8.6e-5, 1.8e-4 for k = 2..7."""
    N = _small_N(dim, k, N)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x32, b32 = (v.astype(np.float32) for v in vectors(dim, k, N))
    x, b = x32.astype(np.float64), b32.astype(np.float64)
    ref = O.avs_apply(A, blocks, pidx, x, b, omega, 1)
    r32 = (b32 - A.astype(np.float32) @ x32).astype(np.float64)
    u = np.linalg.solve(blocks, r32[pidx][..., None])[..., 0]
    corr = np.zeros_like(x)
    np.add.at(corr, pidx.ravel(), u.ravel())
    return rel_l2(x + omega * corr, ref)


def fp32_tol(dim, k, N, omega=None):
    """Bar for a float32 smoother step S(x, b): 1e-5 (the target), or twice
    the float32-residual floor above where that floor exceeds it (k >= 4 in
    2D): no float32 step can beat the floor, so the 1e-5 target is out of
    reach there, and the bar asks for the floor's accuracy."""
    if omega is None:
        omega = 0.25 if dim == 2 else 0.1
    return max(1e-5, 2.0 * fp32_residual_floor(dim, k, N, omega))


def _row_order_shuffled(A, rng):
    """A with the entries of each row stored in a random order.  SciPy sums
    a CSR row in stored order, so products with the result are the same
    float32 inner products under another summation order."""
    A = A.tocsr()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    o = np.lexsort((rng.random(A.nnz), rows))
    return sp.csr_matrix((A.data[o], A.indices[o], A.indptr), shape=A.shape)


@functools.lru_cache(maxsize=None)
def fp32_vcycle_floor(dim, k, N, omega, pre=1, post=1, smoother="avs"):
    """Error of the oracle's own float32 V-cycle (float32 matrices, float32
    dense-LU patch solves and transfers, float64 coarse solve) against its
    float64 V-cycle, on the float32-rounded seeded right-hand side: the
    largest over the stored summation order of its sparse products and
    three random ones.  The float32 residual's rounding depends on the
    order each row is summed in, and at high degree that alone moves the
    V-cycle's error several-fold (2D Q7 on 4 x 4 cells: 7e-5 to 4e-4), so a
    single order is no floor for another implementation's arithmetic."""
    _, b = vectors(dim, k, N)
    b = b.astype(np.float32).astype(np.float64)
    kw = dict(omega=omega, pre=pre, post=post, smoother=smoother)
    ref = O.Hierarchy(dim, k, N, **kw).vcycle(b)
    low = O.Hierarchy(dim, k, N, dtype=np.float32, **kw)
    errs = [rel_l2(low.vcycle(b), ref)]
    stored = list(low.Alow)
    for seed in range(3):
        rng = np.random.default_rng(seed)
        low.Alow = [_row_order_shuffled(A, rng) for A in stored]
        errs.append(rel_l2(low.vcycle(b), ref))
    return max(errs)


def fp32_vcycle_tol(dim, k, N, omega=None, pre=1, post=1, smoother="avs"):
    """Bar for a float32 V-cycle against the float64 oracle: 1e-5, or twice
    the worst the oracle's own float32 V-cycle reaches on the same input
    over the summation orders above."""
    if omega is None:
        omega = 0.25 if dim == 2 else 0.1
    return max(1e-5, 2.0 * fp32_vcycle_floor(dim, k, N, omega, pre, post, smoother))


@functools.lru_cache(maxsize=None)
def mvs_ops(dim, k, N):
    A, blocks, pidx = oracle_ops(dim, k, N)
    return A, blocks, pidx, O.mvs_colors(dim, N)


def fp64_mvs_tol(dim, k, N, steps=1):
    """Bar for float64 coloured multiplicative steps: one smoother bar per
    colour sweep (2^(dim+1) sequential sub-steps per step, each a local
    solve whose rounding adds at most the additive bar; the sub-steps'
    error propagation is a contraction)."""
    return steps * (2 ** (dim + 1)) * fp64_tol(dim, k, N)


@functools.lru_cache(maxsize=None)
def fp32_mvs_floor(dim, k, N, omega):
    """Error of the oracle's coloured multiplicative step run entirely in
    float32 (float32 A and residuals, float32 dense-LU local solves) against
    float64, on the float32-rounded seeded inputs."""
    N = _small_N(dim, k, N)
    A, blocks, pidx, col = mvs_ops(dim, k, N)
    x, b = (v.astype(np.float32).astype(np.float64) for v in vectors(dim, k, N))
    ref = O.mvs_apply(A, blocks, pidx, col, x, b, omega)
    low = O.mvs_apply(A.astype(np.float32), blocks.astype(np.float32), pidx, col, x, b, omega)
    return rel_l2(low.astype(np.float64), ref)


def fp32_mvs_tol(dim, k, N, omega):
    return max(1e-5, 2.0 * fp32_mvs_floor(dim, k, N, omega))


@functools.lru_cache(maxsize=None)
def exact_ops(dim, k, N):
    """Oracle operator with the exact local matrices A[I_v, I_v] as patch blocks."""
    A = O.assemble(dim, k, N)
    pidx = O.patch_indices(dim, k, N)
    return A, O.patch_blocks(A, pidx), pidx, O.mvs_colors(dim, N)


def fp64_exact_tol(dim, k, N):
    """1e-12, or 2 kappa(A_v) eps for the exact local matrices."""
    _, blocks, _, _ = exact_ops(dim, k, min(N, 8))
    kap = max(np.linalg.cond(blocks[i]) for i in range(0, len(blocks), max(1, len(blocks) // 16)))
    return max(1e-12, 2.0 * kap * EPS64)


@functools.lru_cache(maxsize=None)
def fp32_exact_floor(dim, k, N, omega):
    """Float32 floor of an additive step with exact local solves: float32
    residual, exact (float64) solves, against the float64 step."""
    N = _small_N(dim, k, N)
    A, blocks, pidx, _ = exact_ops(dim, k, N)
    x32, b32 = (v.astype(np.float32) for v in vectors(dim, k, N))
    x, b = x32.astype(np.float64), b32.astype(np.float64)
    ref = O.avs_apply(A, blocks, pidx, x, b, omega, 1)
    r32 = (b32 - A.astype(np.float32) @ x32).astype(np.float64)
    u = np.linalg.solve(blocks, r32[pidx][..., None])[..., 0]
    corr = np.zeros_like(x)
    np.add.at(corr, pidx.ravel(), u.ravel())
    return rel_l2(x + omega * corr, ref)
