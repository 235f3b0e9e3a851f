"""ctypes binding of include/c0ip.h: same names, argument marshalling only.

Device vectors are torch tensors on the GPU (contiguous, float64/float32);
their data pointers go straight to the library.  Loading fails loudly when
the built library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

C0IP_F64 = 0
C0IP_F32 = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(_HERE, "libc0ip.so")


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_cells", C.c_int), ("degree", C.c_int), ("gamma", C.c_double)]


class MgOpts(C.Structure):
    _fields_ = [("omega", C.c_double), ("pre_steps", C.c_int), ("post_steps", C.c_int),
                ("vcycle_dtype", C.c_int), ("coarse_mode", C.c_int), ("scatter_mode", C.c_int),
                ("tail_levels", C.c_int), ("smoother", C.c_int), ("local_solver", C.c_int),
                ("mvs_residual", C.c_int)]


class KrylovOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iters", C.c_int), ("restart", C.c_int), ("x0_is_zero", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("rel_res_est", C.c_double),
                ("rel_res_true", C.c_double), ("frac_iters", C.c_double), ("seconds_total", C.c_double),
                ("seconds_vcycle", C.c_double), ("seconds_arnoldi", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


STATUS = {0: "C0IP_OK", -1: "C0IP_EINVAL", -2: "C0IP_ENOMEM", -3: "C0IP_EHIP", -4: "C0IP_NOT_CONVERGED",
          -5: "C0IP_ENAN", -6: "C0IP_EUNSUPPORTED"}


class C0ipError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_SIGS = {
    "c0ip_create": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(MgOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "c0ip_destroy": (C.c_int, [C.c_void_p]),
    "c0ip_num_levels": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "c0ip_num_dofs": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64)]),
    "c0ip_apply_A": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "c0ip_apply_smoother": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "c0ip_vcycle": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "c0ip_smoother_step": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "c0ip_smoother_step_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "c0ip_autotune": (C.c_int, [C.c_void_p, C.c_int]),
    "c0ip_tuned_variant": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "c0ip_set_variant": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "c0ip_solve": (C.c_int, [C.c_void_p, C.POINTER(KrylovOpts), C.c_void_p, C.c_void_p, C.POINTER(SolveInfo)]),
    "c0ip_solve_fcg": (C.c_int, [C.c_void_p, C.POINTER(KrylovOpts), C.c_void_p, C.c_void_p, C.POINTER(SolveInfo)]),
    "c0ip_last_error": (C.c_char_p, []),
    "c0ip_batch_create": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(C.c_int), C.c_int, C.POINTER(MgOpts), C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "c0ip_batch_num_systems": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "c0ip_batch_solve": (C.c_int, [C.c_void_p, C.POINTER(KrylovOpts), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(SolveInfo)]),
    "c0ip_batch_destroy": (C.c_int, [C.c_void_p]),
    "c0ip_host_matrices_1d": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "c0ip_host_patch_inverse": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_int),
                                          C.c_void_p]),
    "c0ip_host_patch_inverse_exact": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_int),
                                                C.c_void_p]),
}


def load_library():
    """Load libc0ip.so from the package directory (raises if it is not built)."""
    global _LIB
    if _LIB is None:
        p = lib_path()
        if not os.path.exists(p):
            raise ImportError(f"{p} is not built: run paper_2412_05082_amd.build.build() first")
        lib = C.CDLL(p)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def _check(st):
    if st != 0:
        raise C0ipError(st, load_library().c0ip_last_error().decode())


def _dt(t):
    import torch
    if t.dtype == torch.float64:
        return C0IP_F64
    if t.dtype == torch.float32:
        return C0IP_F32
    raise TypeError("float32 or float64 tensors only")


class Problem:
    """Owns a c0ip_problem handle (c0ip_create / c0ip_destroy)."""

    def __init__(self, dim, n_cells, degree, gamma=0.0, omega=None, pre_steps=1, post_steps=1,
                 vcycle_dtype=C0IP_F32, coarse_mode=0, scatter_mode=0, tail_levels=-1, smoother=0, local_solver=0,
                 mvs_residual=0, stream=None):
        """smoother: 0 = additive (AVS), 1 = coloured multiplicative (MVS);
        local_solver: 0 = separable (fast diagonalisation), 1 = exact (dense);
        mvs_residual: 2D MVS residual per colour, 0 = automatic, 1 = in the
        colour launch, 2 = a full residual pass."""
        lib = load_library()
        if omega is None:
            omega = 0.25 if dim == 2 else 0.1
        self.mesh = MeshDesc(dim, n_cells, degree, gamma)
        self.mg = MgOpts(omega, pre_steps, post_steps, vcycle_dtype, coarse_mode, scatter_mode, tail_levels,
                         smoother, local_solver, mvs_residual)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = C.c_void_p()
        _check(lib.c0ip_create(C.byref(self.mesh), C.byref(self.mg), C.c_void_p(stream), C.byref(h)))
        self._h = h
        self.dim, self.n_cells, self.degree = dim, n_cells, degree

    def close(self):
        if getattr(self, "_h", None):
            load_library().c0ip_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, reps=3):
        """Time the smoother's tile variants per level and keep the fastest."""
        _check(load_library().c0ip_autotune(self._h, reps))

    def tuned_variant(self, level=-1, dtype=C0IP_F32):
        v = C.c_int()
        _check(load_library().c0ip_tuned_variant(self._h, level, dtype, C.byref(v)))
        return v.value

    def set_variant(self, variant, level=-1, dtype=C0IP_F32):
        _check(load_library().c0ip_set_variant(self._h, level, dtype, variant))

    def num_levels(self) -> int:
        v = C.c_int()
        _check(load_library().c0ip_num_levels(self._h, C.byref(v)))
        return v.value

    def num_dofs(self, level=-1) -> int:
        v = C.c_int64()
        _check(load_library().c0ip_num_dofs(self._h, level, C.byref(v)))
        return v.value

    def _vec(self, t, level, dtype=None):
        import torch
        n = self.num_dofs(level)
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"expected a contiguous device tensor of {n} entries")
        if dtype is not None and _dt(t) != dtype:
            raise TypeError("dtype mismatch")
        return C.c_void_p(t.data_ptr())

    def apply_A(self, x, y, level=-1):
        d = _dt(x)
        _check(load_library().c0ip_apply_A(self._h, level, d, self._vec(x, level, d), self._vec(y, level, d)))

    def apply_smoother(self, b, x, level=-1, x_is_zero=False):
        d = _dt(b)
        _check(load_library().c0ip_apply_smoother(self._h, level, d, self._vec(b, level, d),
                                                  self._vec(x, level, d), int(bool(x_is_zero))))

    def smoother_step(self, b, x_in, x_out, level=-1):
        """x_out = S(x_in, b) (x_in None: S(0, b)); x_out must not overlap b or x_in."""
        d = _dt(b)
        xi = None if x_in is None else self._vec(x_in, level, d)
        _check(load_library().c0ip_smoother_step(self._h, level, d, self._vec(b, level, d), xi,
                                                 self._vec(x_out, level, d)))

    def smoother_step_noalloc(self, b, x_in, x_out, level=-1):
        """c0ip_smoother_step_noalloc: x_out = S(x_in, b) with no allocation
        (fixed per-GPU work space; see include/c0ip.h)."""
        d = _dt(b)
        xi = None if x_in is None else self._vec(x_in, level, d)
        _check(load_library().c0ip_smoother_step_noalloc(self._h, level, d, self._vec(b, level, d), xi,
                                                         self._vec(x_out, level, d)))

    def vcycle(self, b, x):
        d = _dt(b)
        _check(load_library().c0ip_vcycle(self._h, d, self._vec(b, -1, d), self._vec(x, -1, d)))

    def solve(self, b, x, rtol=1e-8, max_iters=500, restart=50, x0_is_zero=True, raise_on_nonconv=True):
        opts = KrylovOpts(rtol, max_iters, restart, int(bool(x0_is_zero)))
        info = SolveInfo()
        st = load_library().c0ip_solve(self._h, C.byref(opts), self._vec(b, -1, C0IP_F64),
                                       self._vec(x, -1, C0IP_F64), C.byref(info))
        if st in (-4, -5) and not raise_on_nonconv:  # NOT_CONVERGED / ENAN: info of the iterations done
            d = info.as_dict()
            d["status"] = st
            return d
        _check(st)
        return info.as_dict()

    def solve_fcg(self, b, x, rtol=1e-8, max_iters=500, x0_is_zero=True, raise_on_nonconv=True):
        """c0ip_solve_fcg: flexible CG preconditioned by the V-cycle."""
        opts = KrylovOpts(rtol, max_iters, 1, int(bool(x0_is_zero)))
        info = SolveInfo()
        st = load_library().c0ip_solve_fcg(self._h, C.byref(opts), self._vec(b, -1, C0IP_F64),
                                           self._vec(x, -1, C0IP_F64), C.byref(info))
        if st == -4 and not raise_on_nonconv:
            return info.as_dict()
        _check(st)
        return info.as_dict()


class Batch:
    """Owns a c0ip_batch: problems = [(n_cells, degree), ...] (2D), n_rhs per problem."""

    def __init__(self, problems, n_rhs, gamma=0.0, omega=0.25, pre_steps=1, post_steps=1, vcycle_dtype=C0IP_F32,
                 coarse_mode=0, tail_levels=-1, scatter_mode=0, smoother=0, local_solver=0, stream=None):
        lib = load_library()
        self.problems = list(problems)
        self.n_rhs = list(n_rhs)
        meshes = (MeshDesc * len(self.problems))(*[MeshDesc(2, N, k, gamma) for N, k in self.problems])
        rhs = (C.c_int * len(self.n_rhs))(*self.n_rhs)
        mg = MgOpts(omega, pre_steps, post_steps, vcycle_dtype, coarse_mode, scatter_mode, tail_levels, smoother,
                    local_solver)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _check(lib.c0ip_batch_create(meshes, rhs, len(self.problems), C.byref(mg), C.c_void_p(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().c0ip_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_systems(self):
        v = C.c_int()
        _check(load_library().c0ip_batch_num_systems(self._h, C.byref(v)))
        return v.value

    def solve(self, bs, xs, rtol=1e-8, max_iters=500, restart=50, x0_is_zero=True, raise_on_nonconv=True):
        """bs, xs: lists of contiguous float64 device tensors of shape (n_rhs[i], (k N + 1)^2)."""
        import torch
        if len(bs) != len(self.problems) or len(xs) != len(self.problems):
            raise ValueError("one b and one x tensor per problem")
        for (N, k), r, b, x in zip(self.problems, self.n_rhs, bs, xs):
            n = (k * N + 1) ** 2
            for t in (b, x):
                if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64
                        or not t.is_contiguous() or t.numel() != r * n):
                    raise ValueError(f"expected a contiguous float64 device tensor of {r} x {n} entries")
        bp = (C.c_void_p * len(bs))(*[t.data_ptr() for t in bs])
        xp = (C.c_void_p * len(xs))(*[t.data_ptr() for t in xs])
        ns = self.num_systems()
        infos = (SolveInfo * ns)()
        opts = KrylovOpts(rtol, max_iters, restart, int(bool(x0_is_zero)))
        st = load_library().c0ip_batch_solve(self._h, C.byref(opts), bp, xp, infos)
        if not (st == -4 and not raise_on_nonconv):
            _check(st)
        return [infos[i].as_dict() for i in range(ns)]


def host_matrices_1d(degree, n_cells, gamma=0.0):
    """Library's 1D factors (M, L, B) of a level, computed on the host."""
    n1 = degree * n_cells + 1
    M, L, B = (np.zeros((n1, n1)) for _ in range(3))
    _check(load_library().c0ip_host_matrices_1d(degree, n_cells, gamma, M.ctypes.data, L.ctypes.data,
                                                B.ctypes.data))
    return M, L, B


def host_patch_inverse(dim, degree, n_cells, vertex, gamma=0.0):
    """Library's fast-diagonalisation inverse of one separable patch matrix."""
    n = (2 * degree - 1) ** dim
    out = np.zeros((n, n))
    v = (C.c_int * dim)(*vertex)
    _check(load_library().c0ip_host_patch_inverse(dim, degree, n_cells, gamma, v, out.ctypes.data))
    return out


def host_patch_inverse_exact(dim, degree, n_cells, vertex, gamma=0.0):
    """Library's dense inverse of one exact patch matrix A_v = R_v A R_v^T."""
    n = (2 * degree - 1) ** dim
    out = np.zeros((n, n))
    v = (C.c_int * dim)(*vertex)
    _check(load_library().c0ip_host_patch_inverse_exact(dim, degree, n_cells, gamma, v, out.ctypes.data))
    return out
