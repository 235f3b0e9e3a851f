"""Precision floors of the oracle's own definitions, and the coarse-solver
branch of its hierarchy (no GPU).

Why these exist: the GPU tests compare float32 results with the float64
oracle.  Whether a given bar can be met at all is a property of float32
arithmetic applied to the method, not of any kernel.  Here the oracle
evaluates the same definitions entirely in float32 (float32 matrices, dense
LU patch solves in float32, float32 vectors; Sec. 3 and the mixed-precision
V-cycle of Sec. 5.2) and the error against its float64 evaluation on the
same seeded input is measured.  That error is the floor a textbook float32
implementation reaches; the GPU float32 bars (tests/gpu_util.py) are
max(1e-5, that floor).

The floor follows from the patch conditioning: a float32 residual of a
high-frequency input carries rounding error ~eps32 |A||x| in every mode, and
a local solve amplifies low modes by up to kappa(A~_v) (eq. inverse is exact
in exact arithmetic, so no method avoids this).  Measured: error / (kappa
eps32) between 0.03 and 0.25 for k = 2..7, above 1e-5 from k = 4 on.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from paper_2412_05082_amd.inputs import seeded_vector

EPS32 = float(np.finfo(np.float32).eps)
EPS64 = float(np.finfo(np.float64).eps)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _ops(dim, k, N):
    A = O.assemble(dim, k, N)
    At = O.assemble(dim, k, N, bulk="diag")
    pidx = O.patch_indices(dim, k, N)
    return A, O.patch_blocks(At, pidx), pidx


def _kappa(blocks):
    return max(np.linalg.cond(blocks[i]) for i in range(0, len(blocks), max(1, len(blocks) // 16)))


@pytest.mark.parametrize("k,N", [(2, 32), (3, 32), (4, 16), (5, 8), (6, 8), (7, 8)])
def test_float32_lu_smoother_floor(k, N):
    """The oracle's float32 S(x, b) (float32 A, float32 dense-LU patch solves)
    against its float64 S(x, b) on the float32-rounded inputs: the error is
    a fixed fraction of kappa(A~_v) eps32, below 1e-5 for k <= 3 and above it
    for k >= 5 (so a 1e-5 bar for k >= 5 is out of reach of float32)."""
    dim = 2
    A, blocks, pidx = _ops(dim, k, N)
    x = seeded_vector(dim, k, N, 1).astype(np.float32).astype(np.float64)
    b = seeded_vector(dim, k, N, 0).astype(np.float32).astype(np.float64)
    ref = O.avs_apply(A, blocks, pidx, x, b, 0.25, 1)
    s32 = O.avs_apply(A.astype(np.float32), blocks.astype(np.float32), pidx, x, b, 0.25, 1).astype(np.float64)
    err = _rel(s32, ref)
    ratio = err / (_kappa(blocks) * EPS32)
    assert 0.01 <= ratio <= 0.5, (err, ratio)
    if k <= 3:
        assert err < 1e-5
    if k >= 5:
        assert err > 1e-5


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (2, 5), (3, 2), (3, 3)])
def test_coarse_smoother_mode_is_separable_solve(dim, k):
    """coarse='smoother' (one smoothing step with omega = 1 from 0 on the
    2^dim-cell level, reading of Sec. 5.1) equals the dense solve of the
    separable matrix of eq. localsolverbila on the free nodes: on that level
    the single vertex patch holds every free node."""
    H = O.Hierarchy(dim, k, 2, coarse="smoother")
    b = seeded_vector(dim, k, 2, 0)
    got = H.coarse_solve(b)
    At = O.assemble(dim, k, 2, bulk="diag").toarray()
    free = ~O.boundary_mask(dim, k, 2)
    want = np.zeros_like(b)
    want[free] = np.linalg.solve(At[np.ix_(free, free)], b[free])
    assert _rel(got, want) <= 1e-13
    # and differs from the exact coarse solve (the dropped mixed term matters)
    exact = O.Hierarchy(dim, k, 2).coarse_solve(b)
    assert _rel(got, exact) > 1e-3


@pytest.mark.parametrize("k,N", [(2, 16), (3, 16), (4, 16), (5, 8)])
def test_float32_hierarchy_within_its_rounding_floor(k, N):
    """The float32 V-cycle (Sec. 5.2) differs from the float64 one by the
    float32 rounding of its smoothing steps: within a small multiple of the
    float32 smoother floor above, and far from float64 agreement."""
    dim = 2
    b = seeded_vector(dim, k, N, 0).astype(np.float32).astype(np.float64)
    H64 = O.Hierarchy(dim, k, N, omega=0.25)
    H32 = O.Hierarchy(dim, k, N, omega=0.25, dtype=np.float32)
    err = _rel(H32.vcycle(b), H64.vcycle(b))
    kap = _kappa(H64.blocks[-1])
    assert 1e-8 < err <= kap * EPS32 * 2.0, (err, kap)


@pytest.mark.parametrize("k,N", [(2, 16), (3, 64), (5, 8), (7, 8)])
def test_float64_vcycle_is_well_determined(k, N):
    """Two valid float64 local solvers (LU, Cholesky) give V-cycles that agree
    far inside the per-step forward-error bound 2 kappa(A~_v) eps64 used by
    the GPU tests; the V-cycle bar (levels x steps x that bound) therefore
    measures the local solver's rounding, not an ambiguity of Algorithm 1."""
    import oracle.c0ip_oracle as OM
    dim = 2
    b = seeded_vector(dim, k, N, 0)
    ref = O.Hierarchy(dim, k, N, omega=0.25).vcycle(b)

    def avs_cholesky(A, blocks, pidx, x, b, omega, steps=1, x_is_zero=False):
        x = np.zeros_like(b) if x_is_zero else np.array(x, dtype=np.float64)
        for s in range(steps):
            r = b if (x_is_zero and s == 0) else b - A @ x
            corr = np.zeros_like(x)
            for p in range(len(blocks)):
                u = sla.cho_solve(sla.cho_factor(blocks[p]), r[pidx[p]])
                np.add.at(corr, pidx[p], u)
            x = x + omega * corr
        return x

    saved = OM.avs_apply
    OM.avs_apply = avs_cholesky
    try:
        alt = O.Hierarchy(dim, k, N, omega=0.25).vcycle(b)
    finally:
        OM.avs_apply = saved
    H = O.Hierarchy(dim, k, N, omega=0.25)
    kap = _kappa(H.blocks[-1])
    err = _rel(alt, ref)
    assert err <= 0.1 * 2 * kap * EPS64 + 1e-15, (err, kap)
