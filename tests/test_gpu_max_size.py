"""The largest meshes the library accepts, just under 2^31 DoFs per vector:
2D Q2 16384^2 (1,073,807,361 DoFs) and 3D Q2 512^3 (1,076,890,625 DoFs);
the next mesh of either (twice the cells per direction) is refused.  A x
and one smoother step S(x, b) in float64 are compared with the windowed
oracle at sampled DoFs (next to the corners, on the boundary, at tile
seams, in the last rows and at random).  The inputs are drawn on the device
(seeded); the oracle reads only the windows it needs from them."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import check, fp64_tol, say

pytestmark = pytest.mark.gpu


class _OnDevice:
    """Read access to entries of a device vector, one window at a time."""

    def __init__(self, t):
        self.t = t

    def __getitem__(self, idx):
        if isinstance(idx, (int, np.integer)):
            return float(self.t[int(idx)].item())
        i = torch.as_tensor(np.asarray(idx, dtype=np.int64), device=self.t.device)
        return self.t[i].cpu().numpy()


def _nodes(dim, k, N, count, seed):
    n1 = k * N + 1
    rng = np.random.default_rng(seed)
    picks = [[1] * dim, [n1 - 2] * dim, [0] + [n1 // 2] * (dim - 1), [k] * dim, [2 * k + 1] * dim,
             [n1 // 2] * dim, [n1 - 1 - k] + [3] * (dim - 1), [48 * 5 + 1] + [24 * 7] * (dim - 1),
             [n1 - 2] + [1] * (dim - 1)]
    nodes = [sum(int(v) * n1 ** m for m, v in enumerate(p)) for p in picks]
    nodes += [int(v) for v in rng.integers(0, n1 ** dim, count)]
    return np.array(nodes, dtype=np.int64)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dim,k,N", [(2, 2, 16384), (3, 2, 512)])
def test_largest_meshes_sampled(dim, k, N):
    n1 = k * N + 1
    n = n1 ** dim
    assert n < 2 ** 31 <= (2 * k * N + 1) ** dim
    say("largest mesh", dim, k, N, n)
    with pytest.raises(P.C0ipError):
        P.Problem(dim, 2 * N, k)
    g = torch.Generator(device="cuda")
    g.manual_seed(2024 + dim)
    x = torch.rand(n, generator=g, dtype=torch.float64, device="cuda") * 2 - 1
    b = torch.rand(n, generator=g, dtype=torch.float64, device="cuda") * 2 - 1
    omega = 0.25 if dim == 2 else 0.1
    pb = P.Problem(dim, N, k, omega=omega, vcycle_dtype=P.C0IP_F64)
    y = torch.empty_like(x)
    pb.apply_A(x, y)
    xs = x.clone()
    pb.apply_smoother(b, xs)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all()) and bool(torch.isfinite(xs).all())
    nodes = _nodes(dim, k, N, 12 if dim == 3 else 20, 17)
    yh = y[torch.as_tensor(nodes, device="cuda")].cpu().numpy()
    ya = O.apply_rows_windowed(dim, k, N, _OnDevice(x), nodes)
    check("A x", np.abs(yh - ya).max() / np.abs(ya).max(), 1e-12)
    sh = xs[torch.as_tensor(nodes, device="cuda")].cpu().numpy()
    sa = O.avs_nodes_windowed(dim, k, N, _OnDevice(x), _OnDevice(b), omega, nodes)
    check("S(x,b)", np.abs(sh - sa).max() / np.abs(sa).max(), fp64_tol(dim, k, N))
    pb.close()
    del x, b, y, xs
    torch.cuda.empty_cache()
