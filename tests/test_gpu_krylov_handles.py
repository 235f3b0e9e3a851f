"""Regression: Krylov solves of handles created and destroyed one after
another in one process (pinned host memory freed by one handle is reused by
the next) give the iterations and residuals of the same solves run first."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from paper_2412_05082_amd.inputs import seeded_vector
from tests.gpu_util import host, say

pytestmark = pytest.mark.gpu

CASES = [(16, 2), (8, 3), (32, 3), (16, 4), (4, 2), (64, 2), (8, 4), (8, 2)]


def _solve(N, k, dtype, seed, fcg=False):
    pb = P.Problem(2, N, k, omega=0.25, vcycle_dtype=dtype)
    b = torch.from_numpy(seeded_vector(2, k, N, seed)).cuda()
    x = torch.zeros_like(b)
    info = pb.solve_fcg(b, x, rtol=1e-8) if fcg else pb.solve(b, x, rtol=1e-8)
    pb.close()
    return info, host(b), host(x)


@pytest.mark.parametrize("dtype", [P.C0IP_F32, P.C0IP_F64])
def test_sequential_handles_repeat_their_solves(dtype):
    say("sequential handles", dtype)
    first = [_solve(N, k, dtype, 700 + i) for i, (N, k) in enumerate(CASES)]
    for rnd in range(2):
        for i, (N, k) in enumerate(CASES):
            info, bh, xh = _solve(N, k, dtype, 700 + i, fcg=(rnd == 1 and i % 2 == 1))
            if rnd == 1 and i % 2 == 1:
                continue  # interleaved flexible-CG solves only reuse the memory
            assert info["iterations"] == first[i][0]["iterations"], (rnd, i, info, first[i][0])
            assert np.array_equal(xh, first[i][2]), (rnd, i)
            A = O.assemble(2, k, N)
            assert np.linalg.norm(bh - A @ xh) <= 1.05e-8 * np.linalg.norm(bh), (rnd, i)
