"""GPU parity of the 3D HIP path (through the C ABI) against the CPU oracle:
operator, smoother, V-cycle and MG-FGMRES on small 3D meshes (several tiles,
ragged last tiles; for k >= 5 the patch kernel's tile is one cell and the
operator's 16 nodes, so N = 4 already spans several of both), and the
full-size 3D Q3 128^3 workload on sampled outputs from the windowed oracle.
Tolerances as in the 2D tests (tests/gpu_util.py)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import (check, dev, fp32_tol, fp32_vcycle_tol, fp64_tol, fp64_vcycle_tol, host, oracle_ops,
                            rel_l2, say, vectors)

pytestmark = pytest.mark.gpu

SMALL3 = [(3, 2, 2), (3, 2, 4), (3, 2, 8), (3, 3, 4), (3, 3, 8), (3, 4, 4), (3, 5, 2), (3, 6, 2), (3, 7, 2),
          (3, 5, 4), (3, 6, 4), (3, 7, 4)]


@pytest.mark.parametrize("dim,k,N", SMALL3)
def test_apply_A_3d(dim, k, N):
    say("3d apply_A", dim, k, N)
    A, _, _ = oracle_ops(dim, k, N)
    x, _ = vectors(dim, k, N)
    pb = P.Problem(dim, N, k)
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    y32 = torch.empty(x.size, dtype=torch.float32, device="cuda")
    x32 = x.astype(np.float32)
    pb.apply_A(dev(x32), y32)
    torch.cuda.synchronize()
    check("A f64", rel_l2(host(y), A @ x), 1e-12)
    check("A f32", rel_l2(host(y32), A @ x32.astype(np.float64)), 1e-5)


def test_apply_A_3d_k2_n16_full():
    """k = 2, 16^3 cells: two y tiles and two z chunks of the operator kernel,
    every output against the assembled matrix."""
    dim, k, N = 3, 2, 16
    say("3d apply_A full", dim, k, N)
    A = O.assemble(dim, k, N)
    x, _ = vectors(dim, k, N)
    pb = P.Problem(dim, N, k)
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    torch.cuda.synchronize()
    assert rel_l2(host(y), A @ x) <= 1e-12


def _tile_seam_nodes(k, N, rng, count):
    """Nodes next to the seams of the operator's tiles and z chunks (cells
    multiple of 4 and 16 in x, y and z), next to the boundary, and random."""
    n1 = k * N + 1
    seams = sorted({c * k + d for c in range(0, N + 1, 4) for d in (-1, 0, 1)} & set(range(n1)))
    pick = [(int(rng.choice(seams)), int(rng.choice(seams)), int(rng.choice(seams))) for _ in range(count)]
    pick += [(1, 1, 1), (n1 - 2, n1 - 2, n1 - 2), (0, 5, 5), (n1 - 1, 3, 4), (2, n1 - 1, n1 - 1)]
    return np.array([i + n1 * (j + n1 * l) for i, j, l in pick])


@pytest.mark.parametrize("k", [2, 3, 4])
def test_apply_A_3d_n32_sampled(k):
    """32^3 cells: several x and y tiles, ragged tiles and several z chunks;
    A x (float64 and float32) and one smoothing step at nodes on the seams."""
    dim, N = 3, 32
    say("3d apply_A sampled", dim, k, N)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=0.1)
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    x32 = x.astype(np.float32)
    y32 = torch.empty(x.size, dtype=torch.float32, device="cuda")
    pb.apply_A(dev(x32), y32)
    xs = dev(x)
    pb.apply_smoother(dev(b), xs)
    torch.cuda.synchronize()
    yh, y32h, sh = host(y), host(y32), host(xs)
    rng = np.random.default_rng(11)
    nodes = _tile_seam_nodes(k, N, rng, 24)
    ya = O.apply_rows_windowed(dim, k, N, x, nodes)
    scale = np.abs(ya).max()
    assert np.abs(yh[nodes] - ya).max() <= 1e-12 * scale
    ya32 = O.apply_rows_windowed(dim, k, N, x32.astype(np.float64), nodes)
    assert np.abs(y32h[nodes] - ya32).max() <= 1e-5 * scale
    sn = nodes[: {2: 4, 3: 2, 4: 1}[k]]
    sa = O.avs_nodes_windowed(dim, k, N, x, b, 0.1, sn)
    assert np.abs(sh[sn] - sa).max() <= fp64_tol(dim, k, 8) * np.abs(sa).max()
    # the float32 smoother step on the same nodes
    b32 = b.astype(np.float32)
    xs32 = dev(x32)
    pb.apply_smoother(dev(b32), xs32)
    torch.cuda.synchronize()
    sa32 = O.avs_nodes_windowed(dim, k, N, x32.astype(np.float64), b32.astype(np.float64), 0.1, sn)
    assert np.abs(host(xs32)[sn] - sa32).max() <= fp32_tol(dim, k, 8) * np.abs(sa32).max()
    assert np.isfinite(yh).all() and np.isfinite(y32h).all() and np.isfinite(sh).all()


@pytest.mark.parametrize("k", [3, 2])
def test_apply_A_3d_ring_chunks_sampled(k):
    """64^3 cells: ring z chunks of 4 planes (N / 16) and interior chunks of
    8; float64 and float32 A x at nodes on the tile and chunk seams."""
    N = 64
    dim = 3
    say("3d apply_A ring chunks", dim, k, N)
    x, _ = vectors(dim, k, N)
    pb = P.Problem(dim, N, k)
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    x32 = x.astype(np.float32)
    y32 = torch.empty(x.size, dtype=torch.float32, device="cuda")
    pb.apply_A(dev(x32), y32)
    torch.cuda.synchronize()
    yh, y32h = host(y), host(y32)
    nodes = _tile_seam_nodes(k, N, np.random.default_rng(13), 32)
    ya = O.apply_rows_windowed(dim, k, N, x, nodes)
    scale = np.abs(ya).max()
    assert np.abs(yh[nodes] - ya).max() <= 1e-12 * scale
    ya32 = O.apply_rows_windowed(dim, k, N, x32.astype(np.float64), nodes)
    assert np.abs(y32h[nodes] - ya32).max() <= 1e-5 * scale
    assert np.isfinite(yh).all() and np.isfinite(y32h).all()


@pytest.mark.parametrize("k,N", [(2, 8), (3, 4), (4, 4)])
def test_apply_A_and_smoother_3d_other_penalty(k, N):
    """A penalty other than k(k+1): the operator takes the table-driven path
    (no compile-time reference rows); operator and smoother against the
    oracle assembled with the same penalty."""
    dim, gamma, om = 3, 2.5 * k * (k + 1), 0.1
    say("3d other penalty", dim, k, N, gamma)
    A = O.assemble(dim, k, N, gamma)
    At = O.assemble(dim, k, N, gamma, bulk="diag")
    pidx = O.patch_indices(dim, k, N)
    blocks = O.patch_blocks(At, pidx)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, gamma=gamma, omega=om)
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    xd = dev(x)
    pb.apply_smoother(dev(b), xd)
    torch.cuda.synchronize()
    check("A f64", rel_l2(host(y), A @ x), 1e-12)
    ref = O.avs_apply(A, blocks, pidx, x, b, om, 1)
    check("S f64", rel_l2(host(xd), ref), fp64_tol(dim, k, N))


@pytest.mark.parametrize("dim,k,N", SMALL3)
@pytest.mark.parametrize("x_is_zero", [False, True])
def test_smoother_3d(dim, k, N, x_is_zero):
    say("3d smoother", dim, k, N, x_is_zero)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    om = 0.1
    pb = P.Problem(dim, N, k, omega=om)
    ref = O.avs_apply(A, blocks, pidx, x, b, om, 1, x_is_zero=x_is_zero)
    xd = dev(x)
    pb.apply_smoother(dev(b), xd, x_is_zero=x_is_zero)
    x32, b32 = x.astype(np.float32), b.astype(np.float32)
    ref32 = O.avs_apply(A, blocks, pidx, x32.astype(np.float64), b32.astype(np.float64), om, 1, x_is_zero=x_is_zero)
    xd32 = dev(x32)
    pb.apply_smoother(dev(b32), xd32, x_is_zero=x_is_zero)
    torch.cuda.synchronize()
    check("S f64", rel_l2(host(xd), ref), fp64_tol(dim, k, N))
    check("S f32", rel_l2(host(xd32), ref32), 1e-5 if x_is_zero else fp32_tol(dim, k, N))


@pytest.mark.parametrize("dim,k,N", [(3, 2, 8), (3, 3, 8), (3, 4, 4)])
def test_vcycle_3d(dim, k, N):
    say("3d vcycle", dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=0.1)
    _, b = vectors(dim, k, N)
    ref = H.vcycle(b)
    pb = P.Problem(dim, N, k, omega=0.1, vcycle_dtype=P.C0IP_F64)
    xd = torch.empty(b.size, dtype=torch.float64, device="cuda")
    pb.vcycle(dev(b), xd)
    b32 = b.astype(np.float32)
    ref32 = H.vcycle(b32.astype(np.float64))
    x32 = torch.empty(b.size, dtype=torch.float32, device="cuda")
    pb.vcycle(dev(b32), x32)
    torch.cuda.synchronize()
    check("vcycle f64", rel_l2(host(xd), ref), fp64_vcycle_tol(dim, k, N))
    check("vcycle f32", rel_l2(host(x32), ref32), fp32_vcycle_tol(dim, k, N))


@pytest.mark.parametrize("k,N", [(2, 8), (3, 8)])
def test_solve_3d(k, N):
    dim = 3
    say("3d solve", dim, k, N)
    A = O.assemble(dim, k, N)
    _, b = vectors(dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=0.1)
    xr, info_r = O.fgmres(A, b, H.vcycle, rtol=1e-8, restart=50)
    for dt in (P.C0IP_F64, P.C0IP_F32):
        pb = P.Problem(dim, N, k, omega=0.1, vcycle_dtype=dt)
        xd = torch.zeros(b.size, dtype=torch.float64, device="cuda")
        info = pb.solve(dev(b), xd, rtol=1e-8)
        assert info["converged"] == 1
        if dt == P.C0IP_F64:
            assert info["iterations"] == info_r["iterations"]
        else:
            assert info["iterations"] <= info_r["iterations"] + 2
        assert np.linalg.norm(b - A @ host(xd)) / np.linalg.norm(b) <= 1.05e-8


@pytest.mark.parametrize("dtype", [P.C0IP_F32, P.C0IP_F64])
def test_solve_3d_q3_n32_sampled_residual(dtype):
    """3D Q3, 32^3 cells (912,673 DoFs: interior and ring tiles of the
    operator, interior tiles of the smoother): MG-FGMRES to 1e-8; the
    residual of the returned solution at sampled rows, from the oracle's
    windowed rows, obeys |r_i| <= ||r||_2 <= 1e-8 ||b||_2."""
    dim, k, N = 3, 3, 32
    say("3d solve sampled residual", dim, k, N, dtype)
    _, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=0.1, vcycle_dtype=dtype)
    xd = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    info = pb.solve(dev(b), xd, rtol=1e-8)
    torch.cuda.synchronize()
    assert info["converged"] == 1
    xh = host(xd)
    n1 = k * N + 1
    rng = np.random.default_rng(3)
    rows = _tile_seam_nodes(k, N, rng, 16)
    i, j, l = rows % n1, (rows // n1) % n1, rows // (n1 * n1)
    rows = rows[(i > 0) & (i < n1 - 1) & (j > 0) & (j < n1 - 1) & (l > 0) & (l < n1 - 1)]
    r = b[rows] - O.apply_rows_windowed(dim, k, N, xh, rows)
    assert np.abs(r).max() <= 1.05e-8 * np.linalg.norm(b)
    assert np.isfinite(xh).all()


def test_full_size_3d_q3_128_sampled():
    """3D Q3, 128^3 cells (57,066,625 DoFs): A x and S(x,b) at sampled DoFs
    (corners, edges, faces, interior) against the windowed oracle."""
    dim, k, N = 3, 3, 128
    say("3d full size", dim, k, N)
    x, b = vectors(dim, k, N)
    n1 = k * N + 1
    pb = P.Problem(dim, N, k, omega=0.1)
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    xs = dev(x)
    pb.apply_smoother(dev(b), xs)
    torch.cuda.synchronize()
    yh, sh = host(y), host(xs)
    rng = np.random.default_rng(7)
    picks = [(1, 1, 1), (n1 - 2, n1 - 2, n1 - 2), (1, n1 // 2, 3), (k, k, k), (2 * k, 2 * k + 1, 5),
             (n1 // 2, n1 // 2, n1 // 2), (n1 - 1 - k, 3, n1 // 3)]
    nodes = [i + n1 * (j + n1 * l) for i, j, l in picks] + list(rng.integers(0, n1 ** 3, 1))
    nodes = np.array(nodes)
    ya = O.apply_rows_windowed(dim, k, N, x, nodes)
    assert np.abs(yh[nodes] - ya).max() <= 1e-12 * np.abs(ya).max()
    sa = O.avs_nodes_windowed(dim, k, N, x, b, 0.1, nodes)
    check("S f64 sampled", np.abs(sh[nodes] - sa).max() / np.abs(sa).max(), fp64_tol(dim, k, 8))
    assert np.isfinite(yh).all() and np.isfinite(sh).all()


def _smoother_seam_nodes(k, N, rng, count):
    """Nodes on the seams of the 3D smoother's tiles (6 x 6 cells in x and
    y) and of the operator's (multiples of 4 and 16 cells), next to the
    boundary and next to the domain corners."""
    n1 = k * N + 1
    seams = sorted({c * k + d for c in set(range(0, N + 1, 6)) | set(range(0, N + 1, 16)) for d in (-1, 0, 1, 2)}
                   & set(range(1, n1 - 1)))
    pick = [(int(rng.choice(seams)), int(rng.choice(seams)), int(rng.choice(seams))) for _ in range(count)]
    pick += [(1, 1, 1), (n1 - 2, n1 - 2, n1 - 2), (1, n1 // 2, 2), (n1 - 2, 6 * k, 6 * k + 1),
             (6 * k - 1, 1, n1 - 3), (k, k, k)]
    return np.array([i + n1 * (j + n1 * l) for i, j, l in pick])


def test_full_size_3d_q3_128_f32_smoother_sampled():
    """The float32 smoother step of the 3D Q3 128^3 workload (the precision
    of its V-cycle) at 22 nodes on tile seams and the boundary, against the
    windowed oracle on the float32-rounded inputs."""
    dim, k, N = 3, 3, 128
    say("3d full size f32 smoother", dim, k, N)
    x, b = vectors(dim, k, N)
    x32, b32 = x.astype(np.float32), b.astype(np.float32)
    pb = P.Problem(dim, N, k, omega=0.1)
    xo = torch.empty(x.size, dtype=torch.float32, device="cuda")
    pb.smoother_step(dev(b32), dev(x32), xo)
    torch.cuda.synchronize()
    sh = host(xo)
    assert np.isfinite(sh).all()
    nodes = _smoother_seam_nodes(k, N, np.random.default_rng(17), 16)
    sa = O.avs_nodes_windowed(dim, k, N, x32.astype(np.float64), b32.astype(np.float64), 0.1, nodes)
    check("S f32 sampled 128^3", np.abs(sh[nodes] - sa).max() / np.abs(sa).max(), fp32_tol(dim, k, 8))


@pytest.mark.timeout(600)
def test_3d_k5_n8_full():
    """3D Q5 on 8^3 cells (68,921 DoFs): several operator tiles with ragged
    last tiles and 512 patch tiles; A x, S(x, b) and S(0, b) in float64 and
    S(x, b) in float32 against the full oracle."""
    dim, k, N = 3, 5, 8
    say("3d k5 n8 full (oracle assembly ~1 min)", dim, k, N)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=0.1, vcycle_dtype=P.C0IP_F64)
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    xs = dev(x)
    pb.apply_smoother(dev(b), xs)
    x0 = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.smoother_step(dev(b), None, x0)
    x32, b32 = x.astype(np.float32), b.astype(np.float32)
    xs32 = dev(x32)
    pb.apply_smoother(dev(b32), xs32)
    torch.cuda.synchronize()
    check("A f64", rel_l2(host(y), A @ x), 1e-12)
    check("S(x,b) f64", rel_l2(host(xs), O.avs_apply(A, blocks, pidx, x, b, 0.1, 1)), fp64_tol(dim, k, N))
    check("S(0,b) f64", rel_l2(host(x0), O.avs_apply(A, blocks, pidx, None, b, 0.1, 1, x_is_zero=True)),
          fp64_tol(dim, k, N))
    ref32 = O.avs_apply(A, blocks, pidx, x32.astype(np.float64), b32.astype(np.float64), 0.1, 1)
    check("S(x,b) f32", rel_l2(host(xs32), ref32), fp32_tol(dim, k, N))
