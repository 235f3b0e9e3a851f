"""Degenerate meshes: the coarsest mesh the library accepts (2^d cells, one
vertex patch, the coarse level alone) and the next one, at the lowest and
highest degree, through every entry point: A x in both precisions, the
additive, multiplicative and exact-local-solver smoother steps, the V-cycle
in both precisions, and the FGMRES and flexible-CG solves (true residual
from the oracle's assembled matrix)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import (check, dev, exact_ops, fp32_vcycle_tol, fp64_exact_tol, fp64_mvs_tol, fp64_tol,
                            fp64_vcycle_tol, host, mvs_ops, oracle_ops, rel_l2, say, vectors)

pytestmark = pytest.mark.gpu

CASES = [(2, 2, 2), (2, 7, 2), (2, 7, 4), (3, 2, 2), (3, 4, 2), (3, 3, 4)]


@pytest.mark.parametrize("dim,k,N", CASES)
def test_degenerate_meshes_every_entry_point(dim, k, N):
    say("degenerate", dim, k, N)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    om = 0.25 if dim == 2 else 0.1
    pb = P.Problem(dim, N, k, omega=om, vcycle_dtype=P.C0IP_F64)
    # operator, both precisions
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    y32 = torch.empty(x.size, dtype=torch.float32, device="cuda")
    x32 = x.astype(np.float32)
    pb.apply_A(dev(x32), y32)
    torch.cuda.synchronize()
    check("A x f64", rel_l2(host(y), A @ x), 1e-12)
    check("A x f32", rel_l2(host(y32), A @ x32.astype(np.float64)), 1e-5)
    # additive smoother step
    xd = dev(x)
    pb.apply_smoother(dev(b), xd)
    torch.cuda.synchronize()
    check("AVS S(x,b)", rel_l2(host(xd), O.avs_apply(A, blocks, pidx, x, b, om, 1)), fp64_tol(dim, k, N))
    # V-cycle, float64 then float32
    H = O.Hierarchy(dim, k, N, omega=om)
    ref = H.vcycle(b)
    z = torch.empty(b.size, dtype=torch.float64, device="cuda")
    pb.vcycle(dev(b), z)
    torch.cuda.synchronize()
    check("V-cycle f64", rel_l2(host(z), ref), fp64_vcycle_tol(dim, k, N))
    z32 = torch.empty(b.size, dtype=torch.float32, device="cuda")
    b32 = b.astype(np.float32)
    pb.vcycle(dev(b32), z32)
    torch.cuda.synchronize()
    check("V-cycle f32", rel_l2(host(z32), H.vcycle(b32.astype(np.float64))), fp32_vcycle_tol(dim, k, N, omega=om))
    # solves to 1e-8 in both V-cycle precisions; residual from the oracle's matrix
    for dt in (P.C0IP_F64, P.C0IP_F32):
        ps = P.Problem(dim, N, k, omega=om, vcycle_dtype=dt)
        for fcg in (False, True):
            xs = torch.zeros(b.size, dtype=torch.float64, device="cuda")
            info = ps.solve_fcg(dev(b), xs) if fcg else ps.solve(dev(b), xs)
            torch.cuda.synchronize()
            assert info["converged"] == 1, (dt, fcg, info)
            res = np.linalg.norm(b * ~O.boundary_mask(dim, k, N) - A @ host(xs)) / np.linalg.norm(
                b * ~O.boundary_mask(dim, k, N))
            check(f"solve dtype {dt} fcg {fcg}", res, 1.05e-8)
        ps.close()
    pb.close()


@pytest.mark.parametrize("dim,k,N", [(2, 2, 2), (2, 7, 2), (3, 2, 2), (3, 4, 2)])
def test_degenerate_meshes_multiplicative_and_exact(dim, k, N):
    say("degenerate MVS / exact", dim, k, N)
    A, blocks, pidx, col = mvs_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=1.0, smoother=1, vcycle_dtype=P.C0IP_F64)
    xd = dev(x)
    pb.apply_smoother(dev(b), xd)
    torch.cuda.synchronize()
    check("MVS S(x,b)", rel_l2(host(xd), O.mvs_apply(A, blocks, pidx, col, x, b, 1.0)), fp64_mvs_tol(dim, k, N))
    pb.close()
    if dim == 2:  # exact local solvers are built for 2D
        Ae, be, pe, _ = exact_ops(dim, k, N)
        pe_ = P.Problem(dim, N, k, omega=0.25, local_solver=1, vcycle_dtype=P.C0IP_F64)
        xe = dev(x)
        pe_.apply_smoother(dev(b), xe)
        torch.cuda.synchronize()
        check("exact S(x,b)", rel_l2(host(xe), O.avs_apply(Ae, be, pe, x, b, 0.25, 1)), fp64_exact_tol(dim, k, N))
        pe_.close()
