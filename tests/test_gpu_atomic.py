"""The atomic-scatter smoother (scatter_mode 1: each patch solved once, its
correction added with floating-point atomics) against the oracle's AVS step,
V-cycle and solve.  Same tolerances as the owner-computes kernels (the
summation order of overlapping patches is not fixed, so agreement is to
rounding)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import check, dev, fp32_tol, fp64_tol, fp64_vcycle_tol, host, oracle_ops, rel_l2, say, vectors

pytestmark = pytest.mark.gpu

CASES = [(2, 16), (3, 32), (4, 16), (5, 8), (7, 8), (3, 2)]


@pytest.mark.parametrize("k,N", CASES)
def test_atomic_smoother_step_matches_oracle(k, N):
    dim = 2
    say("atomic smoother", k, N)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=0.25, scatter_mode=1)
    xo = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.smoother_step(dev(b), dev(x), xo)
    x0 = torch.empty_like(xo)
    pb.smoother_step(dev(b), None, x0)
    xi = dev(x.copy())
    pb.apply_smoother(dev(b), xi)  # in place
    torch.cuda.synchronize()
    ref = O.avs_apply(A, blocks, pidx, x, b, 0.25, 1)
    ref0 = O.avs_apply(A, blocks, pidx, None, b, 0.25, 1, x_is_zero=True)
    assert rel_l2(host(xo), ref) <= fp64_tol(dim, k, N)
    assert rel_l2(host(xi), ref) <= fp64_tol(dim, k, N)
    assert rel_l2(host(x0), ref0) <= fp64_tol(dim, k, N)
    b32, x32 = b.astype(np.float32), x.astype(np.float32)
    xo32 = torch.empty(x.size, dtype=torch.float32, device="cuda")
    pb.smoother_step(dev(b32), dev(x32), xo32)
    torch.cuda.synchronize()
    ref32 = O.avs_apply(A, blocks, pidx, x32.astype(np.float64), b32.astype(np.float64), 0.25, 1)
    assert rel_l2(host(xo32), ref32) <= fp32_tol(dim, k, N)


@pytest.mark.parametrize("k,N", [(2, 32), (3, 16)])
def test_atomic_vcycle_and_solve(k, N):
    dim = 2
    say("atomic vcycle", k, N)
    _, b = vectors(dim, k, N)
    ref = O.Hierarchy(dim, k, N, omega=0.25).vcycle(b)
    pb = P.Problem(dim, N, k, omega=0.25, vcycle_dtype=P.C0IP_F64, scatter_mode=1)
    xd = torch.empty(b.size, dtype=torch.float64, device="cuda")
    pb.vcycle(dev(b), xd)
    torch.cuda.synchronize()
    check("atomic vcycle f64", rel_l2(host(xd), ref), fp64_vcycle_tol(dim, k, N))
    its = []
    for mode in (0, 1):
        pm = P.Problem(dim, N, k, omega=0.25, scatter_mode=mode)
        x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
        info = pm.solve(dev(b), x)
        assert info["converged"] == 1
        its.append(info["iterations"])
    assert abs(its[0] - its[1]) <= 1


def test_atomic_mode_not_batched():
    with pytest.raises(P.C0ipError) as e:
        P.Batch([(8, 2)], [1], scatter_mode=1)
    assert e.value.status == -6
