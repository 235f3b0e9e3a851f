"""c0ip_smoother_step_noalloc (the smoother step for callers that cannot
allocate: its residual work space is a fixed per-GPU array of the library)
against c0ip_smoother_step and the oracle, through the C ABI: two calls in
a row, the second on a smaller level; S(0, b); the 2D fused step (no work
space), the 3D step and the atomic-scatter step (work space used); sizes
above the fixed work space and float32 calls without float32 tables are
rejected."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
import paper_2412_05082_amd as P
from tests.gpu_util import check, dev, fp32_tol, fp64_tol, host, oracle_ops, rel_l2, say, vectors

pytestmark = pytest.mark.gpu


def _pair(pb, level, b, x_in):
    """(no-allocation step, reference step) on the same inputs."""
    n = b.numel()
    out_na = torch.full((n,), float("nan"), dtype=b.dtype, device="cuda")
    out_ref = torch.empty_like(out_na)
    pb.smoother_step_noalloc(b, x_in, out_na, level=level)
    pb.smoother_step(b, x_in, out_ref, level=level)
    torch.cuda.synchronize()
    return host(out_na), host(out_ref)


@pytest.mark.parametrize("dim,k,N,scatter", [(3, 3, 8, 0), (3, 2, 8, 0), (2, 3, 32, 0), (2, 3, 32, 1)])
@pytest.mark.parametrize("tdt", [torch.float64, torch.float32])
def test_noalloc_matches_smoother_step_two_calls(dim, k, N, scatter, tdt):
    say("noalloc", dim, k, N, scatter, tdt)
    om = 0.25 if dim == 2 else 0.1
    pb = P.Problem(dim, N, k, omega=om, vcycle_dtype=P.C0IP_F32, scatter_mode=scatter)
    L = pb.num_levels() - 1
    for level, Nl in ((L, N), (L - 1, N // 2)):  # second call: a smaller input
        A, blocks, pidx = oracle_ops(dim, k, Nl)
        x, b = vectors(dim, k, Nl)
        if tdt == torch.float32:
            x, b = x.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
        bar = fp64_tol(dim, k, Nl) if tdt == torch.float64 else fp32_tol(dim, k, Nl, om)
        for x_in in (x, None):
            na, ref = _pair(pb, level, dev(b, tdt), None if x_in is None else dev(x_in, tdt))
            assert np.isfinite(na).all()
            if scatter == 0:  # same kernels, fixed order: bitwise equal
                assert np.array_equal(na, ref), (level, x_in is None)
            else:  # atomic adds: equal to rounding
                check("noalloc vs step", rel_l2(na, ref), bar)
            want = O.avs_apply(A, blocks, pidx, x_in, b, om, 1, x_is_zero=x_in is None)
            check(f"noalloc vs oracle level {level}", rel_l2(na, want), bar if x_in is not None else
                  (fp64_tol(dim, k, Nl) if tdt == torch.float64 else 1e-5))


def test_noalloc_rejects_oversize_and_missing_tables():
    lib = P.load_library()
    # 3D Q4 on 64^3 cells: 257^3 DoFs, a float64 residual of 136 MB > 64 MiB
    say("noalloc rejections")
    pb = P.Problem(3, 64, 4, omega=0.1, vcycle_dtype=P.C0IP_F64)
    n = pb.num_dofs()
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    y = torch.zeros_like(b)
    st = lib.c0ip_smoother_step_noalloc(pb._h, -1, P.C0IP_F64, C.c_void_p(b.data_ptr()),
                                        C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    assert st == -1 and b"work space" in lib.c0ip_last_error()
    # S(0, b) needs no work space: accepted at the same size
    assert lib.c0ip_smoother_step_noalloc(pb._h, -1, P.C0IP_F64, C.c_void_p(b.data_ptr()), None,
                                          C.c_void_p(y.data_ptr())) == 0
    # a coarser level fits
    nl = pb.num_dofs(level=pb.num_levels() - 2)
    st = lib.c0ip_smoother_step_noalloc(pb._h, pb.num_levels() - 2, P.C0IP_F64, C.c_void_p(b.data_ptr()),
                                        C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    assert st == 0 and nl * 8 <= 64 << 20
    torch.cuda.synchronize()
    pb.close()
    # float32 without float32 tables (the handle's V-cycle is float64)
    pb = P.Problem(2, 16, 3, vcycle_dtype=P.C0IP_F64)
    n = pb.num_dofs()
    b32 = torch.zeros(n, dtype=torch.float32, device="cuda")
    x32 = torch.zeros_like(b32)
    y32 = torch.zeros_like(b32)
    st = lib.c0ip_smoother_step_noalloc(pb._h, -1, P.C0IP_F32, C.c_void_p(b32.data_ptr()),
                                        C.c_void_p(x32.data_ptr()), C.c_void_p(y32.data_ptr()))
    assert st == -1 and b"float32 tables" in lib.c0ip_last_error()
    # overlapping output and input (shifted by one element) is rejected
    bb = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    st = lib.c0ip_smoother_step_noalloc(pb._h, -1, P.C0IP_F64, C.c_void_p(bb.data_ptr()), None,
                                        C.c_void_p(bb.data_ptr() + 8))
    assert st == -1
    pb.close()
