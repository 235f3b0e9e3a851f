"""GPU parity of the coloured multiplicative vertex-patch smoother (MVS,
Sec. 3 and Fig. 2: 8 colours in 2D, a residual per colour) against the
oracle's coloured sweep (itself pinned to the one-patch-at-a-time
definition on the CPU): smoother steps in both precisions, the V-cycle
with MVS, and the MVS-preconditioned FGMRES solve, in 2D (8 colours) and
3D (16 colours); in 2D both places a colour's residual can be formed (in
the colour's launch, or a full residual pass) are checked, also on a mesh
above the automatic switch between them.  Bars in tests/gpu_util.py."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import (check, dev, exact_ops, fp32_exact_floor, fp32_mvs_tol, fp32_vcycle_tol, fp64_exact_tol,
                            fp64_mvs_tol, fp64_vcycle_tol, host, mvs_ops, rel_l2, say, vectors)

pytestmark = pytest.mark.gpu

CASES = [(2, 2, 16), (2, 3, 8), (2, 3, 32), (2, 4, 16), (2, 5, 8), (2, 6, 8), (2, 7, 8), (2, 2, 2), (2, 3, 4),
         (3, 2, 2), (3, 2, 4), (3, 2, 8), (3, 3, 4), (3, 4, 4), (3, 5, 2), (3, 6, 2)]


@pytest.mark.parametrize("dim,k,N", CASES)
@pytest.mark.parametrize("omega", [1.0, 0.7])
def test_mvs_step_f64(dim, k, N, omega):
    say("mvs step f64", dim, k, N, omega)
    A, blocks, pidx, col = mvs_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    pb = P.Problem(dim, N, k, omega=omega, smoother=1, vcycle_dtype=P.C0IP_F64)
    xd = dev(x)
    pb.apply_smoother(dev(b), xd)
    x0 = torch.empty(x.size, dtype=torch.float64, device="cuda")
    pb.smoother_step(dev(b), None, x0)
    xo = torch.empty_like(x0)
    xi = dev(x)
    pb.smoother_step(dev(b), xi, xo)
    torch.cuda.synchronize()
    ref = O.mvs_apply(A, blocks, pidx, col, x, b, omega)
    ref0 = O.mvs_apply(A, blocks, pidx, col, None, b, omega, x_is_zero=True)
    bar = fp64_mvs_tol(dim, k, N)
    check("MVS S(x,b)", rel_l2(host(xd), ref), bar)
    check("MVS S(0,b)", rel_l2(host(x0), ref0), bar)
    check("MVS step out of place", rel_l2(host(xo), ref), bar)
    assert np.array_equal(host(xi), x)  # x_in untouched


@pytest.mark.parametrize("dim,k,N", [(2, 2, 32), (2, 3, 32), (2, 4, 16), (2, 5, 8), (2, 7, 8), (3, 2, 8), (3, 3, 4)])
def test_mvs_step_f32(dim, k, N):
    say("mvs step f32", dim, k, N)
    A, blocks, pidx, col = mvs_ops(dim, k, N)
    x, b = vectors(dim, k, N)
    x32, b32 = x.astype(np.float32), b.astype(np.float32)
    om = 1.0 if dim == 2 else 0.7
    pb = P.Problem(dim, N, k, omega=om, smoother=1)
    xd = dev(x32)
    pb.apply_smoother(dev(b32), xd)
    torch.cuda.synchronize()
    ref = O.mvs_apply(A, blocks, pidx, col, x32.astype(np.float64), b32.astype(np.float64), om)
    check("MVS S(x,b) f32", rel_l2(host(xd), ref), fp32_mvs_tol(dim, k, N, om))


@pytest.mark.parametrize("dim,k,N,omega", [(2, 2, 16, 1.0), (2, 3, 16, 1.0), (2, 3, 64, 1.0), (2, 4, 32, 1.0),
                                           (2, 5, 8, 1.0), (3, 2, 8, 0.7), (3, 3, 4, 0.7)])
def test_mvs_vcycle(dim, k, N, omega):
    say("mvs vcycle", dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=omega, smoother="mvs")
    _, b = vectors(dim, k, N)
    ref = H.vcycle(b)
    pb = P.Problem(dim, N, k, omega=omega, smoother=1, vcycle_dtype=P.C0IP_F64)
    xd = torch.empty(b.size, dtype=torch.float64, device="cuda")
    pb.vcycle(dev(b), xd)
    b32 = b.astype(np.float32)
    x32 = torch.empty(b.size, dtype=torch.float32, device="cuda")
    pb.vcycle(dev(b32), x32)
    torch.cuda.synchronize()
    check("MVS vcycle f64", rel_l2(host(xd), ref), 2 ** (dim + 1) * fp64_vcycle_tol(dim, k, N))
    ref32 = H.vcycle(b32.astype(np.float64))
    check("MVS vcycle f32", rel_l2(host(x32), ref32), fp32_vcycle_tol(dim, k, N, omega, smoother="mvs"))


@pytest.mark.parametrize("dim,k,N,omega", [(2, 2, 16, 1.0), (2, 3, 32, 1.0), (2, 4, 16, 1.0), (2, 5, 8, 1.0),
                                           (3, 2, 8, 0.7), (3, 3, 4, 0.7)])
def test_mvs_solve(dim, k, N, omega):
    """MG-FGMRES with the MVS V-cycle: the oracle's iteration count with the
    float64 V-cycle (at most 2 more with the float32 one), a true residual
    <= 1.05e-8, and fewer iterations than with the additive smoother."""
    say("mvs solve", dim, k, N)
    A = O.assemble(dim, k, N)
    _, b = vectors(dim, k, N)
    H = O.Hierarchy(dim, k, N, omega=omega, smoother="mvs")
    _, info_r = O.fgmres(A, b, H.vcycle, rtol=1e-8, restart=50)
    its = {}
    for dt in (P.C0IP_F64, P.C0IP_F32):
        pb = P.Problem(dim, N, k, omega=omega, smoother=1, vcycle_dtype=dt)
        xd = torch.zeros(b.size, dtype=torch.float64, device="cuda")
        info = pb.solve(dev(b), xd, rtol=1e-8)
        assert info["converged"] == 1
        assert np.linalg.norm(b - A @ host(xd)) / np.linalg.norm(b) <= 1.05e-8
        its[dt] = info["iterations"]
    say(f"  iterations oracle {info_r['iterations']} f64 {its[P.C0IP_F64]} f32 {its[P.C0IP_F32]}")
    assert its[P.C0IP_F64] == info_r["iterations"]
    assert its[P.C0IP_F32] <= info_r["iterations"] + 2
    pa = P.Problem(dim, N, k, omega=0.25 if dim == 2 else 0.1, vcycle_dtype=P.C0IP_F64)
    xa = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    assert pa.solve(dev(b), xa)["iterations"] > its[P.C0IP_F64]


def _mvs_outputs(dim, k, N, mode, x, b, tdt, local_solver=0):
    """S(x, b), S(0, b) and a V-cycle of b with the given mvs_residual mode."""
    pb = P.Problem(dim, N, k, omega=1.0, smoother=1, local_solver=local_solver, mvs_residual=mode,
                   vcycle_dtype=P.C0IP_F32 if tdt == torch.float32 else P.C0IP_F64)
    xs = x.clone()
    pb.apply_smoother(b, xs)
    x0 = torch.empty_like(x)
    pb.smoother_step(b, None, x0)
    z = torch.empty_like(x)
    pb.vcycle(b, z)
    torch.cuda.synchronize()
    pb.close()
    return [t.cpu().double().numpy() for t in (xs, x0, z)]


def _mode_bars(k, N, tdt, local_solver=0):
    """Bars for S(x,b), S(0,b) and the V-cycle: the oracle bars of the tests above."""
    if local_solver == 1:  # one exact-solver bar per colour sub-step, as fp64_mvs_tol does for the separable one
        one = fp64_exact_tol(2, k, N) if tdt == torch.float64 else max(1e-5, 2 * fp32_exact_floor(2, k, N, 1.0))
        return 8 * one, 8 * one, None
    if tdt == torch.float64:
        return fp64_mvs_tol(2, k, N), fp64_mvs_tol(2, k, N), 8 * fp64_vcycle_tol(2, k, N)
    return (fp32_mvs_tol(2, k, N, 1.0), fp32_mvs_tol(2, k, N, 1.0),
            fp32_vcycle_tol(2, k, N, 1.0, smoother="mvs"))


@pytest.mark.parametrize("k,N,local_solver", [(2, 16, 0), (3, 32, 0), (4, 8, 0), (5, 8, 0), (7, 4, 0), (2, 2, 0),
                                              (3, 16, 1), (5, 4, 1), (7, 4, 1)])
@pytest.mark.parametrize("tdt", [torch.float64, torch.float32])
def test_mvs_residual_modes_match_oracle(k, N, local_solver, tdt):
    """2D: each colour's residual formed in the colour's launch (mode 1), by
    a full residual pass (mode 2), or by the automatic choice (mode 0, which
    is mode 1 at these sizes): S(x, b), S(0, b) and the V-cycle of each mode
    against the oracle, at the bars of the tests above."""
    say("mvs residual modes", k, N, local_solver, tdt)
    if local_solver == 1:
        A, blocks, pidx, _ = exact_ops(2, k, N)
        col = O.mvs_colors(2, N)
    else:
        A, blocks, pidx, col = mvs_ops(2, k, N)
    x, b = vectors(2, k, N)
    if tdt == torch.float32:
        x, b = x.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
    ref = O.mvs_apply(A, blocks, pidx, col, x, b, 1.0)
    ref0 = O.mvs_apply(A, blocks, pidx, col, None, b, 1.0, x_is_zero=True)
    refz = None
    if local_solver == 0:
        refz = O.Hierarchy(2, k, N, omega=1.0, smoother="mvs").vcycle(b)
    bars = _mode_bars(k, N, tdt, local_solver)
    for m in (0, 1, 2):
        xs, x0, z = _mvs_outputs(2, k, N, m, dev(x, tdt), dev(b, tdt), tdt, local_solver)
        check(f"mode {m} S(x,b)", rel_l2(xs, ref), bars[0])
        check(f"mode {m} S(0,b)", rel_l2(x0, ref0), bars[1])
        if refz is not None:
            check(f"mode {m} V-cycle", rel_l2(z, refz), bars[2])


@pytest.mark.parametrize("k,N", [(3, 32), (7, 8)])
@pytest.mark.parametrize("tdt", [torch.float64, torch.float32])
def test_mvs_in_launch_residual_is_deterministic(k, N, tdt):
    """The colour kernel updates x in place while other workgroups of the
    launch read x: two runs of S(x, b), S(0, b) and the V-cycle with the
    residual formed in the launch agree bit for bit (a workgroup reading a
    node another one writes would show up here as run-to-run differences)."""
    say("mvs in-launch determinism", k, N, tdt)
    x, b = vectors(2, k, N)
    xd, bd = dev(x, tdt), dev(b, tdt)
    first = _mvs_outputs(2, k, N, 1, xd, bd, tdt)
    second = _mvs_outputs(2, k, N, 1, xd, bd, tdt)
    for name, u, v in zip(("S(x,b)", "S(0,b)", "V-cycle"), first, second):
        assert np.array_equal(u, v), name


@pytest.mark.timeout(300)
def test_mvs_residual_modes_above_the_switch():
    """2D Q2 1024^2 (4,198,401 DoFs, above the 1.5 * 2^20 switch): the automatic
    mode uses the full residual pass on the finest level and the in-launch
    residual below; the two fixed modes agree with it to the oracle bars of
    the tests above (taken on 64^2, the oracle's floors depend on k, hardly
    on N), in both precisions."""
    dim, k, N = 2, 2, 1024
    assert (k * N + 1) ** 2 >= 3 * 2 ** 19 > (k * N // 2 + 1) ** 2
    say("mvs residual modes above the switch", dim, k, N)
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    n = (k * N + 1) ** 2
    x = torch.rand(n, generator=g, dtype=torch.float64, device="cuda") * 2 - 1
    b = torch.rand(n, generator=g, dtype=torch.float64, device="cuda") * 2 - 1
    for tdt in (torch.float64, torch.float32):
        bars = _mode_bars(k, 64, tdt)
        outs = [_mvs_outputs(dim, k, N, m, x.to(tdt), b.to(tdt), tdt) for m in (0, 1, 2)]
        for m in (1, 2):
            for name, u, v, bar in zip(("S(x,b)", "S(0,b)", "V-cycle"), outs[0], outs[m], bars):
                check(f"{tdt} mode 0 vs {m} {name}", rel_l2(v, u), bar)
        assert np.isfinite(outs[0][2]).all()


def test_mvs_options_rejected():
    with pytest.raises(P.C0ipError) as e:
        P.Problem(2, 8, 2, smoother=1, scatter_mode=1)
    assert e.value.status == -1
    for mode in (-1, 3):
        with pytest.raises(P.C0ipError) as e:
            P.Problem(2, 8, 2, smoother=1, mvs_residual=mode)
        assert e.value.status == -1
    with pytest.raises(P.C0ipError) as e:
        P.Problem(2, 8, 2, smoother=2)
    assert e.value.status == -1
    with pytest.raises(P.C0ipError) as e:
        P.Batch([(8, 2)], [1], smoother=1)
    assert e.value.status == -6
