"""GPU parity of the exact local solvers (local_solver 1: dense inverses of
A_v = R_v A R_v^T, the paper's Table 1) against the oracle's smoothers with
the blocks A[I_v, I_v] of its quadrature-assembled operator: additive and
coloured multiplicative steps in both precisions, V-cycles and solves."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import check, dev, exact_ops, fp32_exact_floor, fp64_exact_tol, host, rel_l2, say, vectors

pytestmark = pytest.mark.gpu

CASES = [(2, 2, 16), (2, 3, 8), (2, 3, 32), (2, 4, 16), (2, 5, 8), (2, 7, 8), (2, 2, 2), (2, 3, 4)]


@pytest.mark.parametrize("dim,k,N", CASES)
def test_exact_avs_step(dim, k, N):
    say("exact AVS step", dim, k, N)
    A, blocks, pidx, _ = exact_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=0.25, local_solver=1)
    xo = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.smoother_step(dev(b), dev(x), xo)
    x0 = torch.empty_like(xo)
    pb.smoother_step(dev(b), None, x0)
    xs = dev(x)
    pb.apply_smoother(dev(b), xs)
    x32, b32 = x.astype(np.float32), b.astype(np.float32)
    xo32 = torch.empty(x.size, dtype=torch.float32, device="cuda")
    pb.smoother_step(dev(b32), dev(x32), xo32)
    torch.cuda.synchronize()
    bar = fp64_exact_tol(dim, k, N)
    ref = O.avs_apply(A, blocks, pidx, x, b, 0.25, 1)
    check("exact S(x,b) f64", rel_l2(host(xo), ref), bar)
    check("exact S(x,b) in place", rel_l2(host(xs), ref), bar)
    check("exact S(0,b) f64", rel_l2(host(x0), O.avs_apply(A, blocks, pidx, None, b, 0.25, 1, x_is_zero=True)), bar)
    ref32 = O.avs_apply(A, blocks, pidx, x32.astype(np.float64), b32.astype(np.float64), 0.25, 1)
    check("exact S(x,b) f32", rel_l2(host(xo32), ref32), max(1e-5, 2 * fp32_exact_floor(dim, k, N, 0.25)))


@pytest.mark.parametrize("dim,k,N", [(2, 2, 16), (2, 3, 8), (2, 4, 16), (2, 5, 8), (2, 7, 8), (2, 3, 4)])
def test_exact_mvs_step(dim, k, N):
    say("exact MVS step", dim, k, N)
    A, blocks, pidx, col = exact_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=1.0, smoother=1, local_solver=1, vcycle_dtype=P.C0IP_F64)
    xo = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.smoother_step(dev(b), dev(x), xo)
    x0 = torch.empty_like(xo)
    pb.smoother_step(dev(b), None, x0)
    torch.cuda.synchronize()
    bar = 2 ** (dim + 1) * fp64_exact_tol(dim, k, N)
    check("exact MVS S(x,b)", rel_l2(host(xo), O.mvs_apply(A, blocks, pidx, col, x, b, 1.0)), bar)
    check("exact MVS S(0,b)", rel_l2(host(x0), O.mvs_apply(A, blocks, pidx, col, None, b, 1.0, x_is_zero=True)), bar)


@pytest.mark.parametrize("smoother,steps,omega,k,N", [(0, 2, 0.25, 2, 16), (0, 2, 0.25, 3, 32), (1, 1, 1.0, 3, 32),
                                                      (1, 1, 1.0, 4, 16), (0, 1, 0.25, 5, 8)])
def test_exact_vcycle_and_solve(smoother, steps, omega, k, N):
    """V-cycle and MG-FGMRES with exact local solvers: the oracle's
    V-cycle (Hierarchy with local='exact') and its iteration count."""
    dim = 2
    say("exact vcycle/solve", smoother, steps, k, N)
    kind = "mvs" if smoother else "avs"
    H = O.Hierarchy(dim, k, N, omega=omega, pre=steps, post=steps, local="exact", smoother=kind)
    _, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=omega, pre_steps=steps, post_steps=steps, smoother=smoother, local_solver=1,
                   vcycle_dtype=P.C0IP_F64)
    xd = torch.empty(b.size, dtype=torch.float64, device="cuda")
    pb.vcycle(dev(b), xd)
    torch.cuda.synchronize()
    L = int(round(np.log2(N))) - 1
    bar = (2 ** (dim + 1) if smoother else 1) * (L * 2 * steps + 1) * fp64_exact_tol(dim, k, N)
    check("exact vcycle f64", rel_l2(host(xd), H.vcycle(b)), bar)
    A = O.assemble(dim, k, N)
    _, info_r = O.fgmres(A, b, H.vcycle, rtol=1e-8, restart=50)
    xs = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    info = pb.solve(dev(b), xs)
    say(f"  iterations oracle {info_r['iterations']} gpu {info['iterations']}")
    assert info["converged"] == 1 and info["iterations"] == info_r["iterations"]
    assert np.linalg.norm(b - A @ host(xs)) / np.linalg.norm(b) <= 1.05e-8


def test_exact_options_rejected():
    for kw in [dict(dim=3, N=4, k=2, local_solver=1), dict(dim=2, N=8, k=2, local_solver=1, scatter_mode=1)]:
        with pytest.raises(P.C0ipError) as e:
            P.Problem(kw.pop("dim"), kw.pop("N"), kw.pop("k"), **kw)
        assert e.value.status == -6
    with pytest.raises(P.C0ipError) as e:
        P.Problem(2, 8, 2, local_solver=2)
    assert e.value.status == -1
    with pytest.raises(P.C0ipError) as e:
        P.Batch([(8, 2)], [1], local_solver=1)
    assert e.value.status == -6
