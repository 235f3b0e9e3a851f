"""GPU flexible CG preconditioned by the V-cycle (Sec. 5.1: the paper's
Krylov method for the additive smoother) against the oracle's flexible CG
with its V-cycle: iteration counts, the residual of the returned solution
from the oracle's matrix, the float32 V-cycle, 3D, and the error paths."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import dev, host, say, vectors

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,k,N,pre", [(2, 2, 16, 1), (2, 3, 32, 1), (2, 3, 32, 2), (2, 5, 8, 1), (2, 4, 16, 2),
                                         (3, 2, 8, 1), (3, 3, 4, 1)])
def test_fcg_matches_oracle(dim, k, N, pre):
    say("fcg", dim, k, N, pre)
    om = 0.25 if dim == 2 else 0.1
    A = O.assemble(dim, k, N)
    _, b = vectors(dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=om, pre=pre, post=pre)
    xr, info_r = O.fcg(A, b, H.vcycle, rtol=1e-8)
    assert info_r["converged"]
    its = {}
    for dt in (P.C0IP_F64, P.C0IP_F32):
        pb = P.Problem(dim, N, k, omega=om, pre_steps=pre, post_steps=pre, vcycle_dtype=dt)
        xd = torch.zeros(b.size, dtype=torch.float64, device="cuda")
        info = pb.solve_fcg(dev(b), xd, rtol=1e-8)
        xh = host(xd)
        res = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
        say(f"  dtype {dt}: its {info['iterations']} (oracle {info_r['iterations']}), est {info['rel_res_est']:.2e} "
            f"true {info['rel_res_true']:.2e} oracle-res {res:.2e}")
        assert info["converged"] == 1 and info["rel_res_est"] <= 1e-8
        assert res <= 2e-8 and abs(info["rel_res_true"] - res) <= 1e-3 * res + 1e-15
        its[dt] = info["iterations"]
        if dt == P.C0IP_F64:
            assert abs(its[dt] - info_r["iterations"]) <= 1
            assert np.linalg.norm(xh - xr) <= 1e-6 * np.linalg.norm(xr)
    assert its[P.C0IP_F32] <= info_r["iterations"] + 2


def test_fcg_start_from_x_and_statuses():
    dim, k, N = 2, 3, 16
    say("fcg statuses")
    A = O.assemble(dim, k, N)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=0.25)
    xd = dev(x)
    info = pb.solve_fcg(dev(b), xd, x0_is_zero=False)
    assert info["converged"] == 1
    assert np.linalg.norm(b - A @ host(xd)) / np.linalg.norm(b) <= 2e-8
    xd = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    info = pb.solve_fcg(dev(b), xd, max_iters=2, raise_on_nonconv=False)
    assert info["iterations"] == 2 and info["converged"] == 0
    bn = b.copy()
    bn[50] = np.inf
    with pytest.raises(P.C0ipError) as e:
        pb.solve_fcg(dev(bn), xd)
    assert e.value.status == -5
    with pytest.raises(P.C0ipError) as e:
        pb.solve_fcg(dev(b), xd, rtol=0.0)
    assert e.value.status == -1
