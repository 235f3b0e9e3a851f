"""The single-workgroup tail of the 2D V-cycle (levels 0..LT in one launch,
vectors in LDS) against the oracle's V-cycle, and against the same problem
with the tail switched off, in both precisions, for meshes whose whole
hierarchy fits in the tail and for meshes where the tiled levels hand over
to it.  Tolerances as for the V-cycle parity tests (tests/gpu_util.py).
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import check, dev, fp32_vcycle_tol, fp64_tol, fp64_vcycle_tol, host, rel_l2, say, vectors

pytestmark = pytest.mark.gpu

CASES = [(2, 4), (2, 16), (2, 64), (3, 8), (3, 16), (3, 64), (4, 16), (4, 32)]


def _vcycle(k, N, dtype, b, **kw):
    pb = P.Problem(2, N, k, omega=0.25, vcycle_dtype=dtype, **kw)
    tdt = torch.float64 if dtype == P.C0IP_F64 else torch.float32
    xd = torch.empty(b.size, dtype=tdt, device="cuda")
    pb.vcycle(dev(b), xd)
    torch.cuda.synchronize()
    out = host(xd).astype(np.float64)
    pb.close()
    return out


@pytest.mark.parametrize("k,N", CASES)
@pytest.mark.parametrize("dtype", [P.C0IP_F64, P.C0IP_F32])
def test_tail_vcycle_matches_oracle(k, N, dtype):
    say("tail vcycle", k, N, dtype)
    _, b = vectors(2, k, N)
    if dtype == P.C0IP_F32:
        b = b.astype(np.float32)
    ref = O.Hierarchy(2, k, N, omega=0.25).vcycle(b.astype(np.float64))
    tol = fp64_vcycle_tol(2, k, N) if dtype == P.C0IP_F64 else fp32_vcycle_tol(2, k, N)
    outs = {t: _vcycle(k, N, dtype, b, tail_levels=t) for t in (-1, 0, 2, 3)}
    for t, x in outs.items():
        check(f"tail {t}", rel_l2(x, ref), tol)
    # tail on and off agree with each other to rounding
    check("tail on/off", rel_l2(outs[-1], outs[0]), tol)


@pytest.mark.parametrize("pre,post,coarse", [(0, 1, 0), (2, 2, 0), (1, 1, 1), (3, 0, 0), (0, 0, 0)])
@pytest.mark.parametrize("N", [16, 64])
def test_tail_smoothing_steps_and_coarse_modes(pre, post, coarse, N):
    k = 3
    say("tail steps", pre, post, coarse, N)
    _, b = vectors(2, k, N)
    H = O.Hierarchy(2, k, N, omega=0.25, pre=pre, post=post, coarse="cholesky" if coarse == 0 else "smoother")
    ref = H.vcycle(b)
    x = _vcycle(k, N, P.C0IP_F64, b, pre_steps=pre, post_steps=post, coarse_mode=coarse)
    check("tail steps", rel_l2(x, ref), fp64_vcycle_tol(2, k, N, pre, post))


def test_tail_inside_solve():
    """The mixed-precision FGMRES solve with and without the tail: the
    iteration counts agree to one, and both meet the residual target."""
    k, N = 3, 32
    say("tail solve", k, N)
    A = O.assemble(2, k, N)
    _, b = vectors(2, k, N)
    its = []
    for t in (-1, 0):
        pb = P.Problem(2, N, k, omega=0.25, tail_levels=t)
        xd = torch.zeros(b.size, dtype=torch.float64, device="cuda")
        info = pb.solve(dev(b), xd, rtol=1e-8)
        torch.cuda.synchronize()
        assert info["converged"] == 1
        assert np.linalg.norm(b - A @ host(xd)) / np.linalg.norm(b) <= 1.05e-8
        its.append(info["iterations"])
        pb.close()
    assert abs(its[0] - its[1]) <= 1


def test_tail_rejects_bad_option():
    with pytest.raises(P.C0ipError):
        P.Problem(2, 16, 3, tail_levels=-2)
