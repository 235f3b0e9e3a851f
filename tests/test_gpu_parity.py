"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances (tests/gpu_util.py): float64 results within 1e-12 relative l2
of the oracle, or 2 kappa(A~_v) eps where the patch matrices are worse
conditioned (k >= 6: two correct float64 local solves differ by up to
~kappa eps); float64 V-cycles within (L (pre + post) + 1) times that;
float32 operator applies and S(0, b) within 1e-5; float32 S(x, b) within
1e-5 or twice the floor that a float32 residual with exact local solves
reaches on the same input (above 1e-5 from k = 4 on); float32 V-cycles
within 1e-5 or twice the oracle's own float32 V-cycle error.  Sizes span several tiles and ragged last tiles; the full-size
workloads (2D Q3 512^2 and the degree sweep) are checked on sampled
outputs computed by the windowed oracle.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import (check, dev, fp32_tol, fp32_vcycle_tol, fp64_tol, fp64_vcycle_tol, host, oracle_ops,
                            rel_l2, say, vectors)

pytestmark = pytest.mark.gpu

SMALL = [(2, 2, 16), (2, 2, 32), (2, 3, 8), (2, 3, 32), (2, 4, 16), (2, 5, 8), (2, 6, 8), (2, 7, 8), (2, 7, 16),
         (2, 3, 2), (2, 5, 4)]


def _problem(dim, k, N, **kw):
    return P.Problem(dim, N, k, **kw)


@pytest.mark.parametrize("dim,k,N", SMALL)
def test_apply_A_f64_matches_oracle(dim, k, N):
    say("apply_A f64", dim, k, N)
    A, _, _ = oracle_ops(dim, k, N)
    x, _ = vectors(dim, k, N)
    x_in = x.copy()
    x_in[O.boundary_mask(dim, k, N)] = 7.0  # boundary inputs are ignored
    pb = _problem(dim, k, N)
    y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x_in), y)
    torch.cuda.synchronize()
    assert rel_l2(host(y), A @ x) <= 1e-12


@pytest.mark.parametrize("dim,k,N", [(2, 2, 32), (2, 3, 32), (2, 5, 8), (2, 7, 16)])
def test_apply_A_f32_matches_oracle(dim, k, N):
    say("apply_A f32", dim, k, N)
    A, _, _ = oracle_ops(dim, k, N)
    x, _ = vectors(dim, k, N)
    x32 = x.astype(np.float32)
    pb = _problem(dim, k, N)
    y = torch.empty(A.shape[0], dtype=torch.float32, device="cuda")
    pb.apply_A(dev(x32), y)
    torch.cuda.synchronize()
    assert rel_l2(host(y), A @ x32.astype(np.float64)) <= 1e-5


@pytest.mark.parametrize("dim,k,N", [(2, 3, 16), (2, 5, 8)])
def test_apply_A_on_every_level(dim, k, N):
    pb = _problem(dim, k, N)
    for lev in range(pb.num_levels()):
        Nl = 2 ** (lev + 1)
        say("apply_A level", lev, Nl)
        A, _, _ = oracle_ops(dim, k, Nl)
        x, _ = vectors(dim, k, Nl)
        y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
        pb.apply_A(dev(x), y, level=lev)
        torch.cuda.synchronize()
        assert rel_l2(host(y), A @ x) <= 1e-12


@pytest.mark.parametrize("dim,k,N", SMALL)
@pytest.mark.parametrize("x_is_zero", [False, True])
def test_smoother_f64_matches_oracle(dim, k, N, x_is_zero):
    say("smoother f64", dim, k, N, x_is_zero)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    om = 0.25
    ref = O.avs_apply(A, blocks, pidx, x, b, om, 1, x_is_zero=x_is_zero)
    pb = _problem(dim, k, N, omega=om)
    xd = dev(x)
    pb.apply_smoother(dev(b), xd, x_is_zero=x_is_zero)
    torch.cuda.synchronize()
    check("S f64", rel_l2(host(xd), ref), fp64_tol(dim, k, N))


@pytest.mark.parametrize("dim,k,N", [(2, 2, 32), (2, 3, 32), (2, 4, 16), (2, 5, 8), (2, 6, 8), (2, 7, 8)])
def test_smoother_f32_matches_oracle(dim, k, N):
    say("smoother f32", dim, k, N)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    x32, b32 = x.astype(np.float32), b.astype(np.float32)
    ref = O.avs_apply(A, blocks, pidx, x32.astype(np.float64), b32.astype(np.float64), 0.25, 1)
    pb = _problem(dim, k, N, omega=0.25)
    xd = dev(x32)
    pb.apply_smoother(dev(b32), xd)
    torch.cuda.synchronize()
    check("S(x,b) f32", rel_l2(host(xd), ref), fp32_tol(dim, k, N))
    x0 = torch.zeros(x.size, dtype=torch.float32, device="cuda")
    pb.apply_smoother(dev(b32), x0, x_is_zero=True)
    ref0 = O.avs_apply(A, blocks, pidx, None, b32.astype(np.float64), 0.25, 1, x_is_zero=True)
    torch.cuda.synchronize()
    check("S(0,b) f32", rel_l2(host(x0), ref0), 1e-5)


@pytest.mark.parametrize("dim,k,N", [(2, 2, 16), (2, 3, 16), (2, 5, 8), (2, 7, 4), (2, 2, 64), (2, 3, 64),
                                     (2, 5, 32), (2, 7, 16)])
def test_vcycle_f64_matches_oracle(dim, k, N):
    say("vcycle f64", dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=0.25)
    _, b = vectors(dim, k, N)
    ref = H.vcycle(b)
    pb = _problem(dim, k, N, omega=0.25, vcycle_dtype=P.C0IP_F64)
    xd = torch.empty(b.size, dtype=torch.float64, device="cuda")
    pb.vcycle(dev(b), xd)
    torch.cuda.synchronize()
    check("vcycle f64", rel_l2(host(xd), ref), fp64_vcycle_tol(dim, k, N))


@pytest.mark.parametrize("dim,k,N", [(2, 2, 16), (2, 3, 16), (2, 3, 64), (2, 4, 32), (2, 5, 8), (2, 6, 8),
                                     (2, 7, 8), (2, 7, 16)])
def test_vcycle_f32_matches_oracle(dim, k, N):
    say("vcycle f32", dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=0.25)
    _, b = vectors(dim, k, N)
    b32 = b.astype(np.float32)
    ref = H.vcycle(b32.astype(np.float64))
    pb = _problem(dim, k, N, omega=0.25)
    xd = torch.empty(b.size, dtype=torch.float32, device="cuda")
    pb.vcycle(dev(b32), xd)
    torch.cuda.synchronize()
    check("vcycle f32", rel_l2(host(xd), ref), fp32_vcycle_tol(dim, k, N))


@pytest.mark.parametrize("k,N", [(2, 16), (3, 16)])
def test_solve_f64_matches_oracle_iterations(k, N):
    dim = 2
    say("solve f64", dim, k, N)
    A = O.assemble(dim, k, N)
    _, b = vectors(dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=0.25)
    xr, info_r = O.fgmres(A, b, H.vcycle, rtol=1e-8, restart=50)
    pb = _problem(dim, k, N, omega=0.25, vcycle_dtype=P.C0IP_F64)
    xd = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    info = pb.solve(dev(b), xd, rtol=1e-8)
    assert info["converged"] == 1
    assert info["iterations"] == info_r["iterations"]
    assert info["rel_res_true"] <= 1.05e-8
    res = np.linalg.norm(b - A @ host(xd)) / np.linalg.norm(b)
    assert res <= 1.05e-8
    assert rel_l2(host(xd), xr) <= 1e-6


@pytest.mark.parametrize("k,N", [(2, 16), (3, 32), (5, 8)])
def test_solve_mixed_precision(k, N):
    dim = 2
    say("solve mixed", dim, k, N)
    A = O.assemble(dim, k, N)
    _, b = vectors(dim, k, N)
    p64 = _problem(dim, k, N, omega=0.25, vcycle_dtype=P.C0IP_F64)
    p32 = _problem(dim, k, N, omega=0.25, vcycle_dtype=P.C0IP_F32)
    x64 = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    x32 = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    i64 = p64.solve(dev(b), x64)
    i32 = p32.solve(dev(b), x32)
    assert i32["converged"] == 1 and i64["converged"] == 1
    assert i32["iterations"] <= i64["iterations"] + 2
    for xx in (x64, x32):
        assert np.linalg.norm(b - A @ host(xx)) / np.linalg.norm(b) <= 1.05e-8
    free = ~O.boundary_mask(dim, k, N)
    import scipy.sparse.linalg as spla
    xs = np.zeros(b.size)
    xs[free] = spla.spsolve(A[free][:, free].tocsc(), b[free])
    kappa_bound = 1e-8 * 1e6  # error <= cond(A) * residual; cond of these systems < 1e6
    assert rel_l2(host(x32), xs) <= kappa_bound


def _sample_nodes(dim, k, N, count, seed):
    n1 = k * N + 1
    rng = np.random.default_rng(seed)
    picks = [(1, 1), (n1 - 2, n1 - 2), (1, n1 // 2), (k, k), (2 * k, 2 * k + 1), (n1 // 2, n1 // 2),
             (n1 - 1 - k, 3), (0, 5)]
    nodes = [i + n1 * j for i, j in picks]
    nodes += list(rng.integers(0, n1 * n1, count))
    return np.array(nodes)


FULL = [(3, 512), (2, 512), (4, 512), (7, 256)]


@pytest.mark.parametrize("k,N", FULL)
def test_full_size_sampled_parity(k, N):
    """Full-size 2D workloads in the bench's launch configuration: A x and
    S(x, b) at sampled DoFs against the windowed oracle."""
    dim = 2
    say("full size sampled", dim, k, N)
    x, b = vectors(dim, k, N)
    nodes = _sample_nodes(dim, k, N, 24, 11)
    pb = _problem(dim, k, N, omega=0.25)
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.apply_A(dev(x), y)
    xs = dev(x)
    pb.apply_smoother(dev(b), xs)
    torch.cuda.synchronize()
    yh, sh = host(y), host(xs)
    ya = O.apply_rows_windowed(dim, k, N, x, nodes)
    scale = np.abs(ya).max()
    assert np.abs(yh[nodes] - ya).max() <= 1e-12 * scale
    sa = O.avs_nodes_windowed(dim, k, N, x, b, 0.25, nodes)
    assert np.abs(sh[nodes] - sa).max() <= fp64_tol(dim, k, N) * np.abs(sa).max()
    # boundary rows are exactly zero; no non-finite values anywhere
    assert np.isfinite(yh).all() and np.isfinite(sh).all()
    bd = O.boundary_mask(dim, k, N) if N <= 256 else None
    if bd is not None:
        assert np.all(yh[bd] == 0) and np.all(sh[bd] == 0)


@pytest.mark.parametrize("k,N", [(3, 512), (2, 512), (4, 512), (7, 256)])
def test_full_size_f32_smoother_variants_sampled(k, N):
    """The float32 fused smoother step at the bench's full sizes, in every
    compiled tile variant (the autotuner picks among them for the bench and
    the mixed-precision solve) and in the variant the autotuner picked, at
    sampled DoFs against the windowed oracle on the float32-rounded inputs."""
    dim = 2
    say("full size f32 variants", k, N)
    x, b = vectors(dim, k, N)
    x, b = x.astype(np.float32), b.astype(np.float32)
    nodes = _sample_nodes(dim, k, N, 16, 5)
    sa = O.avs_nodes_windowed(dim, k, N, x.astype(np.float64), b.astype(np.float64), 0.25, nodes)
    scale = np.abs(sa).max()
    bar = fp32_tol(dim, k, N)
    pb = _problem(dim, k, N, omega=0.25)
    xd, bd = dev(x), dev(b)
    variants = []
    for v in range(3):
        try:
            pb.set_variant(v, dtype=P.C0IP_F32)
        except P.C0ipError:
            break
        variants.append(v)
    pb.autotune()
    tuned = pb.tuned_variant(dtype=P.C0IP_F32)
    say("  tuned f32 variant", tuned)
    for v in variants + ["tuned"]:
        pb.set_variant(tuned if v == "tuned" else v, dtype=P.C0IP_F32)
        xo = torch.empty(x.size, dtype=torch.float32, device="cuda")
        pb.smoother_step(bd, xd, xo)
        torch.cuda.synchronize()
        sh = host(xo)
        check(f"variant {v}", np.abs(sh[nodes] - sa).max() / scale, bar)
        assert np.isfinite(sh).all()


@pytest.mark.parametrize("dim,k,N", [(2, 3, 64), (2, 5, 16), (3, 3, 8), (3, 2, 32)])
def test_owner_computes_is_deterministic(dim, k, N):
    """Owner computes writes every DoF once in a fixed order: two runs of
    the smoother step and of the V-cycle (both precisions) give bitwise
    equal results."""
    say("determinism", dim, k, N)
    x, b = vectors(dim, k, N)
    pb = _problem(dim, k, N)
    for tdt in (torch.float64, torch.float32):
        xd, bd = dev(x, tdt), dev(b, tdt)
        outs = []
        for rep in range(2):
            xo = torch.empty_like(xd)
            pb.smoother_step(bd, xd, xo)
            z = torch.empty_like(xd)
            pb.vcycle(bd, z)
            torch.cuda.synchronize()
            outs.append((xo.cpu().numpy(), z.cpu().numpy()))
        assert np.array_equal(outs[0][0], outs[1][0])
        assert np.array_equal(outs[0][1], outs[1][1])


def test_abi_rejects_bad_arguments():
    say("abi errors")
    for kw in [dict(dim=4, N=8, k=3), dict(dim=2, N=6, k=3), dict(dim=3, N=40, k=2), dict(dim=2, N=8, k=1),
               dict(dim=2, N=8, k=8)]:
        with pytest.raises(P.C0ipError) as e:
            P.Problem(kw["dim"], kw["N"], kw["k"])
        assert e.value.status == -1
    with pytest.raises(P.C0ipError) as e:
        P.Problem(2, 8, 3, omega=-1.0)
    assert e.value.status == -1
    with pytest.raises(P.C0ipError) as e:
        P.Problem(2, 8, 3, scatter_mode=2)
    assert e.value.status == -1
    with pytest.raises(P.C0ipError) as e:
        P.Problem(3, 4, 3, scatter_mode=1)
    assert e.value.status == -6
    pb = P.Problem(2, 8, 3)
    with pytest.raises(ValueError):
        pb.apply_A(torch.zeros(10, dtype=torch.float64, device="cuda"),
                   torch.zeros(10, dtype=torch.float64, device="cuda"))
    lib = P.load_library()
    assert lib.c0ip_apply_A(pb._h, 0, 0, None, None) == -1
    assert lib.c0ip_apply_A(pb._h, 99, 0, 1, 2) == -1


def test_solve_not_converged_and_nan():
    dim, k, N = 2, 2, 16
    say("solve status", dim, k, N)
    _, b = vectors(dim, k, N)
    pb = _problem(dim, k, N)
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    info = pb.solve(dev(b), x, max_iters=3, raise_on_nonconv=False)
    assert info["iterations"] == 3 and info["converged"] == 0
    bn = b.copy()
    bn[100] = np.nan
    with pytest.raises(P.C0ipError) as e:
        pb.solve(dev(bn), x)
    assert e.value.status == -5


@pytest.mark.parametrize("dim,k,N", [(2, 2, 32), (2, 3, 32), (2, 4, 16), (2, 5, 8), (2, 7, 8), (3, 2, 4), (3, 3, 4)])
def test_smoother_step_out_of_place(dim, k, N):
    """c0ip_smoother_step: x_out = S(x_in, b) (fused in 2D), x_in untouched."""
    say("smoother_step", dim, k, N)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    om = 0.25 if dim == 2 else 0.1
    pb = _problem(dim, k, N, omega=om)
    xi = dev(x)
    xo = torch.empty_like(xi)
    pb.smoother_step(dev(b), xi, xo)
    x0 = torch.empty_like(xi)
    pb.smoother_step(dev(b), None, x0)
    torch.cuda.synchronize()
    assert np.array_equal(host(xi), x)
    assert rel_l2(host(xo), O.avs_apply(A, blocks, pidx, x, b, om, 1)) <= fp64_tol(dim, k, N)
    assert rel_l2(host(x0), O.avs_apply(A, blocks, pidx, None, b, om, 1, x_is_zero=True)) <= fp64_tol(dim, k, N)
    with pytest.raises(P.C0ipError):
        pb.smoother_step(dev(b), xi, xi)


@pytest.mark.parametrize("pre,post", [(2, 2), (1, 3), (0, 1), (3, 0)])
def test_vcycle_smoothing_steps(pre, post):
    """V-cycles with several (or no) pre/post steps: the fused out-of-place
    steps alternate buffers; the result must land in x."""
    dim, k, N = 2, 3, 32
    say("vcycle steps", pre, post)
    H = O.Hierarchy(dim, k, N, omega=0.25, pre=pre, post=post)
    _, b = vectors(dim, k, N)
    ref = H.vcycle(b)
    pb = _problem(dim, k, N, omega=0.25, pre_steps=pre, post_steps=post, vcycle_dtype=P.C0IP_F64)
    xd = torch.empty(b.size, dtype=torch.float64, device="cuda")
    pb.vcycle(dev(b), xd)
    torch.cuda.synchronize()
    check("vcycle f64 steps", rel_l2(host(xd), ref), fp64_vcycle_tol(dim, k, N, pre, post))


@pytest.mark.parametrize("k,N", [(2, 64), (3, 64), (3, 32), (4, 16), (4, 32), (5, 8), (5, 16), (6, 8), (6, 16), (7, 8),
                                 (7, 16)])
@pytest.mark.parametrize("dtype", [P.C0IP_F64, P.C0IP_F32])
def test_every_fused_tile_variant_and_autotune(k, N, dtype):
    """Each compiled tile size of the fused smoother gives the oracle's
    S(x, b) in both precisions (meshes with several tiles and a ragged last
    tile for every size); the autotuner picks one of them, and the step
    with the variant it picked is checked again."""
    dim = 2
    say("fused variants", k, N, dtype)
    A, blocks, pidx = oracle_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    tdt = torch.float64 if dtype == P.C0IP_F64 else torch.float32
    if dtype == P.C0IP_F32:
        x, b = x.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
        bar = fp32_tol(dim, k, N)
    else:
        bar = fp64_tol(dim, k, N)
    ref = O.avs_apply(A, blocks, pidx, x, b, 0.25, 1)
    pb = _problem(dim, k, N, omega=0.25)
    nvar = 0
    for v in range(3):
        try:
            pb.set_variant(v, dtype=dtype)
        except P.C0ipError:
            break
        nvar += 1
        xo = torch.empty(x.size, dtype=tdt, device="cuda")
        pb.smoother_step(dev(b, tdt), dev(x, tdt), xo)
        torch.cuda.synchronize()
        check(f"variant {v}", rel_l2(host(xo), ref), bar)
    assert nvar >= 2
    pb.autotune()
    assert 0 <= pb.tuned_variant(dtype=dtype) < nvar
    xo = torch.empty(x.size, dtype=tdt, device="cuda")
    pb.smoother_step(dev(b, tdt), dev(x, tdt), xo)
    torch.cuda.synchronize()
    check("autotuned", rel_l2(host(xo), ref), bar)
