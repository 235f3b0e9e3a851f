"""Pins of the oracle's smoother, transfers, V-cycle and FGMRES (not GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle as O
from paper_2412_05082_amd.inputs import seeded_vector
from tests import sym1d


def _rand(n, seed, mask=None):
    v = np.random.default_rng(seed).uniform(-1, 1, n)
    if mask is not None:
        v[mask] = 0
    return v


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (2, 5), (3, 2)])
def test_single_patch_exact_avs_is_direct_solve(dim, k):
    """2^dim cells = one vertex patch whose space is all of V_0: one AVS step
    from x = 0 with the exact local solver and omega = 1 is A_0^{-1} b.
    Pins the sign of the correction and the patch DoF set."""
    N = 2
    A = O.assemble(dim, k, N)
    bd = O.boundary_mask(dim, k, N)
    pidx = O.patch_indices(dim, k, N)
    assert pidx.shape == (1, (2 * k - 1) ** dim)
    assert set(pidx.ravel()) == set(np.where(~bd)[0])
    b = _rand(A.shape[0], 0, bd)
    x = O.avs_apply(A, O.patch_blocks(A, pidx), pidx, None, b, 1.0, 1, x_is_zero=True)
    xd = np.zeros_like(b)
    xd[~bd] = np.linalg.solve(A[~bd][:, ~bd].toarray(), b[~bd])
    assert np.allclose(x, xd, rtol=1e-12, atol=1e-14 * np.abs(xd).max())
    # the printed minus sign would give -A^{-1} b
    assert np.linalg.norm(x + xd) > np.linalg.norm(xd)


@pytest.mark.parametrize("dim,k,N", [(2, 2, 4), (2, 3, 4), (3, 2, 4)])
def test_patch_blocks_are_kronecker_separable(dim, k, N):
    """Patch matrices of the separable local solver equal B_v x M_v + M_v x B_v
    (eq. ``localsolverbila``) from the exact 1D factors restricted to the
    patch, and eig(A~_v^{-1} A_v) >= 1 (the dropped 2 L x L term is PSD)."""
    A = O.assemble(dim, k, N)
    At = O.assemble(dim, k, N, bulk="diag")
    pidx = O.patch_indices(dim, k, N)
    Bt = O.patch_blocks(At, pidx)
    Ba = O.patch_blocks(A, pidx)
    M, L, B = sym1d.matrices_1d(k, N)
    n = 2 * k - 1
    verts = O.patch_vertices(dim, N)
    for p, v in enumerate(verts):
        I = [np.arange((vm - 1) * k + 1, (vm + 1) * k) for vm in v]
        Bs = [B[np.ix_(i, i)] for i in I]
        Ms = [M[np.ix_(i, i)] for i in I]
        if dim == 2:
            K = np.kron(Ms[1], Bs[0]) + np.kron(Bs[1], Ms[0])
        else:
            K = (np.kron(Ms[2], np.kron(Ms[1], Bs[0])) + np.kron(Ms[2], np.kron(Bs[1], Ms[0]))
                 + np.kron(Bs[2], np.kron(Ms[1], Ms[0])))
        assert np.abs(Bt[p] - K).max() <= 1e-12 * np.abs(K).max()
        ev = sla.eigh(Ba[p], Bt[p], eigvals_only=True)
        assert ev.min() >= 1 - 1e-9
        assert ev.max() <= 3.0
    assert Bt.shape[1] == n ** dim


@pytest.mark.parametrize("dim,k,Nc", [(2, 2, 2), (2, 3, 4), (2, 7, 2), (3, 2, 2)])
def test_prolongation_reproduces_polynomials(dim, k, Nc):
    """The embedding maps coarse nodal values of a function in V_{l-1} to its
    exact fine nodal values: checked with a global polynomial of degree k
    per variable vanishing on the boundary."""
    P = O.prolongation(dim, k, Nc)
    z = O.gll_nodes(k)

    def coords(N):
        x1 = np.concatenate([c / N + z[:-1] / N for c in range(N)] + [[1.0]])
        mi = O.node_multi_index(dim, k * N + 1)
        return x1[mi]

    def g(X):
        v = np.ones(X.shape[0])
        for m in range(dim):
            x = X[:, m]
            v *= x * (1 - x) * (1 + 0.3 * x ** (k - 2)) if k > 2 else x * (1 - x)
        return v
    uc = g(coords(Nc))
    uf = g(coords(2 * Nc))
    assert np.allclose(P @ uc, uf, atol=1e-13)
    # a function in V_l but not in V_{l-1} is not reproduced (P is not trivial)
    assert P.shape == (O.num_dofs(dim, k, 2 * Nc), O.num_dofs(dim, k, Nc))


def test_vcycle_symmetric_and_two_level_limit():
    dim, k, N = 2, 2, 8
    H = O.Hierarchy(dim, k, N, omega=0.25)
    bd = O.boundary_mask(dim, k, N)
    b1, b2 = _rand(bd.size, 1, bd), _rand(bd.size, 2, bd)
    m1, m2 = H.vcycle(b1), H.vcycle(b2)
    assert abs(m1 @ b2 - b1 @ m2) <= 1e-12 * abs(m1 @ b2)
    # no smoothing, two levels: MG = P A_0^{-1} P^T
    H2 = O.Hierarchy(dim, k, 4, pre=0, post=0)
    bd4 = O.boundary_mask(dim, k, 4)
    b = _rand(bd4.size, 3, bd4)
    P = H2.P[1]
    bc = P.T @ b
    bd2 = O.boundary_mask(dim, k, 2)
    e = np.zeros(bc.size)
    e[~bd2] = np.linalg.solve(H2.A[0][~bd2][:, ~bd2].toarray(), bc[~bd2])
    assert np.allclose(H2.vcycle(b), P @ e, rtol=1e-12, atol=1e-14)


def test_fgmres_identity_preconditioner_matches_direct_solve():
    dim, k, N = 2, 2, 4
    A = O.assemble(dim, k, N)
    bd = O.boundary_mask(dim, k, N)
    b = _rand(bd.size, 0, bd)
    x, info = O.fgmres(A, b, rtol=1e-12, restart=20, maxiter=400)
    xd = np.zeros_like(b)
    xd[~bd] = spla.spsolve(A[~bd][:, ~bd].tocsc(), b[~bd])
    assert info["converged"]
    assert np.allclose(x, xd, rtol=1e-8, atol=1e-10 * np.abs(xd).max())
    h = np.array(info["history"])
    assert np.all(np.diff(h) <= 1e-12 * h[0])


@pytest.mark.parametrize("k", [2, 3])
def test_mg_fgmres_converges_and_mixed_precision_matches(k):
    dim, N = 2, 16
    A = O.assemble(dim, k, N)
    bd = O.boundary_mask(dim, k, N)
    b = _rand(bd.size, 0, bd)
    H = O.Hierarchy(dim, k, N, omega=0.25)
    x, info = O.fgmres(A, b, H.vcycle, rtol=1e-8)
    assert info["converged"] and info["rel_res_true"] <= 1.05e-8
    assert 10 <= info["iterations"] <= 40
    Hf = O.Hierarchy(dim, k, N, omega=0.25, dtype=np.float32)
    x32, info32 = O.fgmres(A, b, Hf.vcycle, rtol=1e-8)
    assert info32["converged"] and info32["rel_res_true"] <= 1.05e-8
    assert abs(info32["iterations"] - info["iterations"]) <= 2
    nu = O.fractional_iterations(info["iterations"], info["history"][-1], info["history"][0])
    assert 0.5 * info["iterations"] < nu <= info["iterations"] + 1e-9


def test_literal_damping_07_does_not_converge():
    """omega = 0.7 exceeds the additive smoother's stability bound (the
    overlap count bounds omega by 1/4 in 2D, Sec. 3): FGMRES(50) does not
    reach 1e-8 within 100 iterations (damping reading G12)."""
    dim, k, N = 2, 2, 16
    A = O.assemble(dim, k, N)
    bd = O.boundary_mask(dim, k, N)
    b = _rand(bd.size, 0, bd)
    H = O.Hierarchy(dim, k, N, omega=0.7)
    x, info = O.fgmres(A, b, H.vcycle, rtol=1e-8, maxiter=100)
    assert not info["converged"]


def test_fcg_identity_terminates_and_matches_direct_solve():
    """Flexible CG with the identity preconditioner is plain CG: on the
    9-unknown level-0 system it terminates (to rounding) within 9 steps, and
    on a small mesh it reaches the sparse direct solution."""
    for k, N, nmax in [(2, 2, 9), (3, 4, None)]:
        A = O.assemble(2, k, N)
        b = np.random.default_rng(3).uniform(-1, 1, A.shape[0])
        free = ~O.boundary_mask(2, k, N)
        b[~free] = 0.0
        x, info = O.fcg(A, b, rtol=1e-13, maxiter=5000)
        xd = np.zeros_like(b)
        xd[free] = spla.spsolve(A[free][:, free].tocsc(), b[free])
        assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
        if nmax is not None:
            assert info["iterations"] <= nmax


def test_fcg_with_vcycle_converges_like_fgmres():
    """With the symmetric additive V-cycle, flexible CG converges to 1e-8 in a
    number of iterations close to FGMRES (the paper uses CG for AVS)."""
    dim, k, N = 2, 3, 16
    A = O.assemble(dim, k, N)
    b = seeded_vector(dim, k, N, 0)
    H = O.Hierarchy(dim, k, N, omega=0.25)
    _, ig = O.fgmres(A, b, H.vcycle, rtol=1e-8, restart=50)
    x, ic = O.fcg(A, b, H.vcycle, rtol=1e-8)
    assert ic["converged"] and ic["rel_res_true"] <= 1.05e-8
    assert abs(ic["iterations"] - ig["iterations"]) <= 3
