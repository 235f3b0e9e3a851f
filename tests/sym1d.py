"""Exact (SymPy) 1D matrices of the C0IP form on a uniform mesh of [0,1].

Test-only helper, independent of both the oracle and the library: it
integrates the 1D factors that appear in the paper's tensor representation
of the patch/global matrix (Sec. 4, eqs. ``bulk1``-``bulk3``, ``ev``,
``matrix1d``) symbolically, on exact Gauss-Lobatto nodes (k = 2, 3, 4).
"""
import functools

import numpy as np
import sympy as S

X = S.Symbol("x")


def gll_exact(k):
    if k == 2:
        return [S.Integer(0), S.Rational(1, 2), S.Integer(1)]
    if k == 3:
        r = 1 / S.sqrt(5)
        return [S.Integer(0), (1 - r) / 2, (1 + r) / 2, S.Integer(1)]
    if k == 4:
        r = S.sqrt(S.Rational(3, 7))
        return [S.Integer(0), (1 - r) / 2, S.Rational(1, 2), (1 + r) / 2, S.Integer(1)]
    raise ValueError(k)


@functools.lru_cache(maxsize=None)
def matrices_1d(k, N, gamma=None):
    """Return float arrays (M, L, B) of size kN+1: mass, stiffness and the
    bi-Laplace factor (cellwise int phi'' phi'' plus, at every grid point,
    gamma/h [phi'][phi'] - {phi''}[phi'] - [phi']{phi''}; interior points
    use jump = left minus right derivative and the average of the second
    derivatives, the two end points use the one-sided outward values)."""
    gam = S.Integer(k * (k + 1)) if gamma is None else S.nsimplify(gamma)
    h = S.Rational(1, N)
    z = gll_exact(k)
    n1 = k * N + 1
    M = np.zeros((n1, n1))
    L = np.zeros((n1, n1))
    B = np.zeros((n1, n1))
    polys = []
    for c in range(N):
        t = (X - c * h) / h
        ps = []
        for j in range(k + 1):
            p = S.Integer(1)
            for m in range(k + 1):
                if m != j:
                    p = p * (t - z[m]) / (z[j] - z[m])
            ps.append(S.expand(p))
        polys.append(ps)
        a, b = c * h, (c + 1) * h
        for i in range(k + 1):
            for j in range(k + 1):
                gi, gj = c * k + i, c * k + j
                M[gi, gj] += float(S.integrate(ps[i] * ps[j], (X, a, b)))
                L[gi, gj] += float(S.integrate(S.diff(ps[i], X) * S.diff(ps[j], X), (X, a, b)))
                B[gi, gj] += float(S.integrate(S.diff(ps[i], X, 2) * S.diff(ps[j], X, 2), (X, a, b)))
    for f in range(N + 1):
        xf = f * h
        jump = {}
        mean = {}
        if f > 0:  # left cell, outward normal +x
            for j in range(k + 1):
                g = (f - 1) * k + j
                d1 = S.diff(polys[f - 1][j], X).subs(X, xf)
                d2 = S.diff(polys[f - 1][j], X, 2).subs(X, xf)
                jump[g] = jump.get(g, 0) + d1
                mean[g] = mean.get(g, 0) + (d2 / 2 if f < N else d2)
        if f < N:  # right cell, outward normal -x
            for j in range(k + 1):
                g = f * k + j
                d1 = S.diff(polys[f][j], X).subs(X, xf)
                d2 = S.diff(polys[f][j], X, 2).subs(X, xf)
                jump[g] = jump.get(g, 0) - d1
                mean[g] = mean.get(g, 0) + (d2 / 2 if f > 0 else d2)
        keys = sorted(set(jump) | set(mean))
        for i in keys:
            for j in keys:
                ji, jj = jump.get(i, 0), jump.get(j, 0)
                mi, mj = mean.get(i, 0), mean.get(j, 0)
                B[i, j] += float(S.N(gam / h * ji * jj - mj * ji - jj * mi, 30))
    return M, L, B


def kron_sum(dim, k, N, separable=False):
    """Kronecker representation (eqs. ``c0iptensorvp``/``c0iptensorvp3D``;
    separable: eq. ``localsolverbila``) with dimension 0 fastest, boundary
    rows and columns zeroed."""
    M, L, B = matrices_1d(k, N)
    kr = lambda *fs: functools.reduce(lambda acc, f: np.kron(f, acc), fs[1:], fs[0])  # noqa: E731
    if dim == 2:
        A = kr(B, M) + kr(M, B)
        if not separable:
            A = A + 2 * kr(L, L)
    else:
        A = kr(B, M, M) + kr(M, B, M) + kr(M, M, B)
        if not separable:
            A = A + 2 * (kr(L, L, M) + kr(M, L, L) + kr(L, M, L))
    n1 = k * N + 1
    g = np.arange(n1 ** dim)
    bd = np.zeros(n1 ** dim, dtype=bool)
    for m in range(dim):
        im = (g // n1 ** m) % n1
        bd |= (im == 0) | (im == n1 - 1)
    A[bd, :] = 0
    A[:, bd] = 0
    return A
