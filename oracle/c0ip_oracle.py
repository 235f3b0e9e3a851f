"""Plain float64 CPU oracle for the C0IP biharmonic problem and its solver.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the HIP path.

What it computes, each function naming the passage it follows:

* Q_k Lagrange elements on uniform Cartesian meshes of [0,1]^d (Sec. 2,
  eq. ``fespace``), nodes = Gauss-Lobatto-Legendre points (the paper does
  not name the node set; reading G10).
* The C0IP matrix by explicit quadrature of eq. ``bfc0ip``: full Hessian
  contraction on every cell, and on every face the penalty, consistency and
  adjoint-consistency terms built from the jump/mean definitions of Sec. 2
  (interior faces: jump = sum of outward normal derivatives, mean = 1/2 sum
  of second normal derivatives; boundary faces: one-sided, full weight).
  Penalty gamma/h_e with gamma = k(k+1) (the value is not given in the
  paper), h_e = h on uniform meshes.
* The separable local-solver matrix of eq. ``localsolverbila`` by the same
  quadrature with the mixed second derivatives dropped from the bulk term.
* Vertex patches, the additive vertex-patch smoother (Sec. 3) with dense LU
  local solves; the damped correction is *added* (the printed minus sign
  is read as a typo: reading G4).
* Grid transfers = FE embedding and its transpose (Sec. 3), the V-cycle of
  Algorithm 1 (returning after the coarse solve), flexible GMRES
  (Sec. 5.1), the mixed-precision V-cycle (Sec. 5.2).
* The clamped manufactured solution prod sin^2(pi x_i) and the energy
  error of eq. ``hnorm`` (estimate eq. ``energyerror``).

Windows: ``assemble(..., window=...)`` assembles only the cells of a box of
the mesh (and the faces whose cells are all in the box), numbered locally;
rows whose stencil lies inside the box are exact rows of the global matrix.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg

__all__ = [
    "gll_nodes", "gauss_legendre", "lagrange_eval", "num_dofs", "node_multi_index",
    "boundary_mask", "assemble", "Window", "patch_vertices", "patch_indices",
    "patch_blocks", "avs_apply", "prolongation_1d", "prolongation", "Hierarchy",
    "fgmres", "fractional_iterations", "load_vector", "manufactured_rhs", "energy_error",
    "exact_solution_nodal", "window_around", "apply_rows_windowed", "avs_nodes_windowed", "apply_blocked",
    "mvs_colors", "mvs_apply", "mvs_sequential", "fcg",
]


# --------------------------------------------------------------------------
# 1D ingredients (Sec. 2: tensor-product Lagrange elements Q_k)
# --------------------------------------------------------------------------

def gll_nodes(k: int) -> np.ndarray:
    """k+1 Gauss-Lobatto-Legendre points on [0,1]: the endpoints and the roots
    of P_k' (node set reading G10; the FE space of eq. ``fespace`` does not
    depend on it)."""
    if k < 1:
        raise ValueError("k >= 1")
    c = np.zeros(k + 1)
    c[k] = 1.0
    dc = npleg.legder(c)
    ddc = npleg.legder(dc)
    r = np.sort(npleg.legroots(dc).real) if k > 1 else np.zeros(0)
    for _ in range(4):  # Newton polish on P_k'
        if r.size:
            r = r - npleg.legval(r, dc) / npleg.legval(r, ddc)
    x = np.concatenate(([-1.0], r, [1.0]))
    x = 0.5 * (x - x[::-1])
    return 0.5 * (x + 1.0)


def gauss_legendre(q: int):
    """q-point Gauss-Legendre rule on [0,1] (quadrature reading G16)."""
    x, w = npleg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_eval(z, t, nder: int = 2) -> np.ndarray:
    """out[d, q, j] = d-th derivative of the Lagrange polynomial of node z_j at t_q."""
    z = np.asarray(z, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = z.size
    out = np.zeros((nder + 1, t.size, n))
    # product form l_j(t) = prod_{m != j} (t - z_m) / (z_j - z_m) and its
    # derivatives by the product rule (sums over the dropped factors)
    for j in range(n):
        others = [m for m in range(n) if m != j]
        den = np.prod([z[j] - z[m] for m in others])

        def prod_except(skip):
            p = np.ones(t.size)
            for m in others:
                if m not in skip:
                    p = p * (t - z[m])
            return p

        out[0, :, j] = prod_except(()) / den
        if nder >= 1:
            out[1, :, j] = sum(prod_except((a,)) for a in others) / den
        if nder >= 2:
            out[2, :, j] = sum(prod_except((a, b)) for a in others for b in others if b != a) / den
    return out


def _kron_list(mats):
    """kron of per-dimension factors with dimension 0 fastest: mats[0] acts on x."""
    out = np.asarray(mats[0])
    for m in mats[1:]:
        out = np.kron(np.asarray(m), out)
    return out


# --------------------------------------------------------------------------
# Mesh and numbering (Sec. 2; table DoF counts (kN+1)^d include boundary nodes)
# --------------------------------------------------------------------------

def num_dofs(dim: int, k: int, N: int) -> int:
    return (k * N + 1) ** dim


def node_multi_index(dim: int, n1: int) -> np.ndarray:
    """(n1^dim, dim) array of node multi-indices, dimension 0 fastest."""
    g = np.arange(n1 ** dim)
    return np.stack([(g // n1 ** m) % n1 for m in range(dim)], axis=1)


def boundary_mask(dim: int, k: int, N: int) -> np.ndarray:
    """True on nodes of the domain boundary (held at 0: V_l is a subset of H^1_0)."""
    n1 = k * N + 1
    mi = node_multi_index(dim, n1)
    return np.any((mi == 0) | (mi == n1 - 1), axis=1)


class Window:
    """A box of cells [lo_m, hi_m) of the N^dim mesh, with local node numbering.

    Local nodes are the nodes of the box's cells, dimension 0 fastest.
    ``gidx`` maps local to global node numbers, ``free`` is False on domain
    boundary nodes."""

    def __init__(self, dim, k, N, lo=None, hi=None):
        self.dim, self.k, self.N = dim, k, N
        self.lo = np.array([0] * dim if lo is None else lo, dtype=np.int64)
        self.hi = np.array([N] * dim if hi is None else hi, dtype=np.int64)
        if np.any(self.lo < 0) or np.any(self.hi > N) or np.any(self.hi <= self.lo):
            raise ValueError("bad window")
        self.n1 = k * N + 1
        self.shape = tuple(int((self.hi[m] - self.lo[m]) * k + 1) for m in range(dim))
        self.size = int(np.prod(self.shape))
        loc = np.stack([(np.arange(self.size) // int(np.prod(self.shape[:m]))) % self.shape[m]
                        for m in range(dim)], axis=1)
        gmi = loc + self.lo[None, :] * k
        self.gmulti = gmi
        self.gidx = sum(gmi[:, m] * self.n1 ** m for m in range(dim))
        self.free = ~np.any((gmi == 0) | (gmi == self.n1 - 1), axis=1)
        self.strides = np.array([int(np.prod(self.shape[:m])) for m in range(dim)], dtype=np.int64)

    def exact_rows(self, margin: int = 1) -> np.ndarray:
        """Mask of local nodes whose row of the window matrix equals the
        global row: every cell containing the node, and every cell within
        ``margin`` cells of those (face neighbours: margin 1), lies in the
        window or outside the domain."""
        k, N = self.k, self.N
        ok = np.ones(self.size, dtype=bool)
        for m in range(self.dim):
            i = self.gmulti[:, m]
            cmax = np.minimum(i // k, N - 1)
            cmin = np.where(i % k == 0, np.maximum(i // k - 1, 0), i // k)
            lo_req = np.maximum(cmin - margin, 0)
            hi_req = np.minimum(cmax + margin, N - 1)
            ok &= (lo_req >= self.lo[m]) & (hi_req < self.hi[m])
        return ok

    def local_of_global_multi(self, gm):
        """Local indices of nodes given by global multi-indices (..., dim)."""
        lm = np.asarray(gm) - self.lo * self.k
        if np.any(lm < 0) or np.any(lm >= np.array(self.shape)):
            raise IndexError("node outside window")
        return (lm * self.strides).sum(axis=-1)


# --------------------------------------------------------------------------
# Assembly of eq. bfc0ip by explicit quadrature
# --------------------------------------------------------------------------

def _cell_matrix(dim, k, h, bulk):
    """Cell integral of the Hessian contraction (bulk term of eq. ``bfc0ip``).
    bulk='full': sum_{i,j} d_ij u d_ij v; bulk='diag': sum_i d_ii u d_ii v
    (the separable approximation of eq. ``localsolverbila``)."""
    z = gll_nodes(k)
    tq, wq = gauss_legendre(k + 1)
    E = lagrange_eval(z, tq)  # [der, q, a]
    W = _kron_list([wq * h] * dim).ravel()
    if bulk == "full":
        pairs = [(i, j) for i in range(dim) for j in range(dim)]
    elif bulk == "diag":
        pairs = [(i, i) for i in range(dim)]
    else:
        raise ValueError(bulk)
    nloc = (k + 1) ** dim
    K = np.zeros((nloc, nloc))
    for (i, j) in pairs:
        c = [0] * dim
        c[i] += 1
        c[j] += 1
        H = _kron_list([E[c[m]] / h ** c[m] for m in range(dim)])  # (nq, nloc)
        K += H.T @ (W[:, None] * H)
    return K


def _face_traces(dim, k, h, m, t_face):
    """Normal first/second derivative (along axis m) of the cell's basis at
    the face x_m = t_face (reference coordinate 0 or 1), at the face's
    tensor Gauss points: arrays (nq_face, nloc) and face weights."""
    z = gll_nodes(k)
    tq, wq = gauss_legendre(k + 1)
    E = lagrange_eval(z, tq)
    Ef = lagrange_eval(z, [t_face])  # [der, 1, a]
    G = _kron_list([(Ef[1] / h) if o == m else E[0] for o in range(dim)])
    S = _kron_list([(Ef[2] / h ** 2) if o == m else E[0] for o in range(dim)])
    W = _kron_list([np.ones(1) if o == m else wq * h for o in range(dim)]).ravel()
    return G, S, W


def _face_matrix(J, Mn, W, pen):
    """Face integral of eq. ``bfc0ip``: penalty, consistency, adjoint
    consistency.  Row = test function, column = trial function."""
    JW = J.T * W[None, :]
    return pen * (JW @ J) - JW @ Mn - (Mn.T * W[None, :]) @ J


def _local_offsets(dim, k, strides):
    a = node_multi_index(dim, k + 1)
    return (a * strides[None, :]).sum(axis=1)


def assemble(dim: int, k: int, N: int, gamma: float | None = None, bulk: str = "full",
             window: Window | None = None, faces: bool = True) -> sp.csr_matrix:
    """Matrix of the C0IP form (eq. ``bfc0ip``), or of its separable
    approximation (bulk='diag'), over the nodes of ``window`` (whole mesh by
    default), by explicit quadrature over cells and faces.  Rows and
    columns of domain boundary nodes are zero (Dirichlet part of the clamped
    condition is built into V_l; the Neumann part is imposed weakly by the
    boundary face terms)."""
    win = Window(dim, k, N) if window is None else window
    h = 1.0 / N
    gam = float(k * (k + 1) if gamma is None else gamma)
    pen = gam / h  # h_e = harmonic mean of orthogonal extents = h (uniform mesh)
    strides = win.strides
    off = _local_offsets(dim, k, strides)
    ncell = win.hi - win.lo
    cells = np.stack(np.meshgrid(*[np.arange(int(n)) for n in ncell], indexing="ij"), -1).reshape(-1, dim)
    rows, cols, vals = [], [], []

    def add(base, loc_off, mat):
        g = base[:, None] + loc_off[None, :]
        rows.append(np.repeat(g, mat.shape[1], axis=1).ravel())
        cols.append(np.tile(g, (1, mat.shape[0])).ravel())
        vals.append(np.broadcast_to(mat.ravel()[None, :], (g.shape[0], mat.size)).ravel())

    # cells
    Kc = _cell_matrix(dim, k, h, bulk)
    base = (cells * k * strides[None, :]).sum(axis=1)
    add(base, off, Kc)

    # faces, per normal axis m
    for m in range(dim if faces else 0):
        GL, SL, W = _face_traces(dim, k, h, m, 1.0)  # left cell, face at its right end
        GR, SR, _ = _face_traces(dim, k, h, m, 0.0)  # right cell, face at its left end
        # interior face between left cell (outward normal +e_m) and right cell (-e_m)
        J = np.concatenate([GL, -GR], axis=1)
        Mn = 0.5 * np.concatenate([SL, SR], axis=1)
        Fint = _face_matrix(J, Mn, W, pen)
        off2 = np.concatenate([off, off + k * strides[m]])
        lc = cells[cells[:, m] + 1 < ncell[m]]  # left cells whose right neighbour is in the window
        if lc.size:
            add((lc * k * strides[None, :]).sum(axis=1), off2, Fint)
        # boundary faces (one-sided, full weight)
        if win.lo[m] == 0:
            F0 = _face_matrix(-GR, SR, W, pen)  # outward normal -e_m
            bc = cells[cells[:, m] == 0]
            add((bc * k * strides[None, :]).sum(axis=1), off, F0)
        if win.hi[m] == N:
            F1 = _face_matrix(GL, SL, W, pen)  # outward normal +e_m
            bc = cells[cells[:, m] == ncell[m] - 1]
            add((bc * k * strides[None, :]).sum(axis=1), off, F1)

    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(win.size, win.size)).tocsr()
    A.sum_duplicates()
    D = sp.diags(win.free.astype(np.float64))
    return (D @ A @ D).tocsr()


# --------------------------------------------------------------------------
# Vertex patches (Sec. 3) and the additive smoother
# --------------------------------------------------------------------------

def patch_vertices(dim: int, N: int) -> np.ndarray:
    """Interior vertices (multi-indices in [1, N-1]^dim), dimension 0 fastest."""
    g = node_multi_index(dim, N - 1) + 1
    return g


def patch_indices(dim: int, k: int, N: int, vertices=None, window: Window | None = None) -> np.ndarray:
    """For each vertex v, the nodes strictly inside the 2^dim cells around v
    (the DoFs of V_v, localisation R_v), as global indices (or local indices
    of ``window``), (2k-1)^dim per patch, dimension 0 fastest."""
    if vertices is None:
        vertices = patch_vertices(dim, N)
    vertices = np.atleast_2d(vertices)
    n = 2 * k - 1
    loc = node_multi_index(dim, n)  # (n^dim, dim)
    gm = (vertices[:, None, :] - 1) * k + 1 + loc[None, :, :]
    if window is None:
        n1 = k * N + 1
        return (gm * (n1 ** np.arange(dim))[None, None, :]).sum(axis=-1)
    return window.local_of_global_multi(gm)


def patch_blocks(A: sp.csr_matrix, pidx: np.ndarray) -> np.ndarray:
    """Dense blocks A[I_v, I_v] for every patch: A_v = R_v A R_v^T."""
    P, m = pidx.shape
    out = np.empty((P, m, m))
    if m > 256:  # large blocks (3D, high degree): row then column slices of the CSR matrix
        for p in range(P):
            out[p] = A[pidx[p]][:, pidx[p]].toarray()
        return out
    chunk = max(1, 2_000_000 // (m * m))
    for s in range(0, P, chunk):
        idx = pidx[s:s + chunk]
        r = np.repeat(idx, m, axis=1).ravel()
        c = np.tile(idx, (1, m)).ravel()
        out[s:s + chunk] = np.asarray(A[r, c]).reshape(-1, m, m)
    return out


def avs_apply(A, blocks, pidx, x, b, omega, steps=1, x_is_zero=False):
    """Additive vertex-patch Schwarz: repeated ``steps`` times,
    x <- x + omega * sum_v R_v^T A_v^{-1} R_v (b - A x)   (Sec. 3; sign reading G4),
    with each A_v^{-1} applied by dense LU (``numpy.linalg.solve``).  The
    arithmetic type is that of ``blocks``."""
    dt = blocks.dtype
    x = np.zeros_like(b, dtype=dt) if x_is_zero else np.array(x, dtype=dt)
    b = np.asarray(b, dtype=dt)
    w = dt.type(omega)
    for s in range(steps):
        r = b if (x_is_zero and s == 0) else b - (A @ x).astype(dt)
        u = np.linalg.solve(blocks, r[pidx][..., None])[..., 0]
        corr = np.zeros_like(x)
        np.add.at(corr, pidx.ravel(), u.ravel())
        x = x + w * corr
    return x


def mvs_colors(dim: int, N: int, vertices=None) -> np.ndarray:
    """Colour of each interior vertex for the coloured multiplicative smoother
    (Sec. 3, Fig. 2): first the 2^dim classes of vertex parity, whose patches
    do not overlap, then a red-black split of each class by the parity of
    sum_m floor(v_m / 2), so that two patches of one colour never touch
    across a face (their DoF sets are then A-orthogonal).  Colour =
    sum_m (v_m mod 2) 2^m + 2^dim (sum_m floor(v_m / 2) mod 2): 8 colours in
    two and 16 in three dimensions; the colours are swept in this order
    (reading: the paper fixes the colouring, not the order)."""
    v = patch_vertices(dim, N) if vertices is None else np.atleast_2d(vertices)
    base = sum((v[:, m] % 2) << m for m in range(dim))
    rb = (v // 2).sum(axis=1) % 2
    return base + (rb << dim)


def mvs_apply(A, blocks, pidx, colors, x, b, omega, steps=1, x_is_zero=False):
    """Coloured multiplicative vertex-patch smoother (Sec. 3): per step, for
    each colour c = 0, 1, ... in turn,
    x <- x + omega * sum_{v of colour c} R_v^T A_v^{-1} R_v (b - A x)
    (sign reading G4), the residual taken after the previous colour.  Patch
    solves by dense LU; the arithmetic type is that of ``blocks``."""
    dt = blocks.dtype
    x = np.zeros_like(b, dtype=dt) if x_is_zero else np.array(x, dtype=dt)
    b = np.asarray(b, dtype=dt)
    w = dt.type(omega)
    ncol = int(colors.max()) + 1 if colors.size else 0
    for s in range(steps):
        for c in range(ncol):
            sel = np.where(colors == c)[0]
            if sel.size == 0:
                continue
            r = b - (A @ x).astype(dt)
            u = np.linalg.solve(blocks[sel], r[pidx[sel]][..., None])[..., 0]
            corr = np.zeros_like(x)
            np.add.at(corr, pidx[sel].ravel(), u.ravel())
            x = x + w * corr
    return x


def mvs_sequential(A, blocks, pidx, order, x, b, omega, steps=1, x_is_zero=False):
    """The multiplicative vertex-patch smoother as defined before colouring
    (Sec. 3): one patch at a time in the given vertex order,
    x <- x + omega R_v^T A_v^{-1} R_v (b - A x).  Plain definition, for small
    meshes only."""
    x = np.zeros_like(b, dtype=np.float64) if x_is_zero else np.array(x, dtype=np.float64)
    for s in range(steps):
        for v in order:
            r = b - A @ x
            x[pidx[v]] += omega * np.linalg.solve(blocks[v], r[pidx[v]])
    return x


# --------------------------------------------------------------------------
# Transfers (Sec. 3: prolongation = embedding, restriction = transpose)
# --------------------------------------------------------------------------

def prolongation_1d(k: int, Nc: int) -> np.ndarray:
    """1D embedding: value of each coarse basis function (Nc cells) at each
    fine node (2 Nc cells).  Shape (2 k Nc + 1, k Nc + 1)."""
    z = gll_nodes(k)
    hc, hf = 1.0 / Nc, 1.0 / (2 * Nc)
    xf = np.concatenate([c * hf + z[:-1] * hf for c in range(2 * Nc)] + [[1.0]])
    P = np.zeros((2 * k * Nc + 1, k * Nc + 1))
    for i, xv in enumerate(xf):
        c = min(int(math.floor(xv / hc + 1e-12)), Nc - 1)
        t = (xv - c * hc) / hc
        vals = lagrange_eval(z, [t], nder=0)[0, 0]
        P[i, c * k:(c + 1) * k + 1] = vals
    return P


def prolongation(dim: int, k: int, Nc: int) -> sp.csr_matrix:
    """Embedding V_{l-1} -> V_l on free nodes (tensor-product basis), as a
    sparse matrix in full-length numbering with boundary rows/cols zero."""
    P1 = sp.csr_matrix(prolongation_1d(k, Nc))
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P).tocsr()
    ff = (~boundary_mask(dim, k, 2 * Nc)).astype(np.float64)
    fc = (~boundary_mask(dim, k, Nc)).astype(np.float64)
    return (sp.diags(ff) @ P @ sp.diags(fc)).tocsr()


# --------------------------------------------------------------------------
# Sampled outputs at full size (windows of the mesh)
# --------------------------------------------------------------------------

def window_around(dim, k, N, node_multi, margin):
    """Window of cells within ``margin`` cells of the cells containing the
    node (clipped to the mesh)."""
    lo, hi = [], []
    for m in range(dim):
        i = int(node_multi[m])
        cmax = min(i // k, N - 1)
        cmin = max(i // k - 1, 0) if i % k == 0 else i // k
        lo.append(max(cmin - margin, 0))
        hi.append(min(cmax + margin + 1, N))
    return Window(dim, k, N, lo, hi)


def _global_multi(dim, n1, g):
    return np.array([(g // n1 ** m) % n1 for m in range(dim)])


def apply_rows_windowed(dim, k, N, x, rows, gamma=None):
    """(A x)[rows] for the full-size mesh, each row from the matrix assembled
    on a window around it (rows of windows are exact, see Window.exact_rows)."""
    n1 = k * N + 1
    out = np.empty(len(rows))
    for t, g in enumerate(rows):
        gm = _global_multi(dim, n1, int(g))
        win = window_around(dim, k, N, gm, 1)
        A = assemble(dim, k, N, gamma, window=win)
        li = int(win.local_of_global_multi(gm))
        out[t] = float((A.getrow(li) @ x[win.gidx])[0])
    return out


def apply_blocked(dim, k, N, X, block=64, gamma=None, absolute=False):
    """A X (or |A| X with ``absolute``) for a full-size mesh without holding A:
    the mesh is cut into boxes of ``block`` cells per direction; each box,
    widened by two cells (every row of a node owned by the box then lies in
    the widened window, see Window.exact_rows), is assembled on its own and
    gives the rows of the nodes it owns.  A node is owned by the box holding
    cell min(i // k, N - 1) in every direction.  X: (n,) or (n, m)."""
    X = np.asarray(X, dtype=np.float64)
    n1 = k * N + 1
    Y = np.zeros_like(X)
    own_cell = np.minimum(np.arange(n1) // k, N - 1)
    starts = list(range(0, N, block))
    for corner in np.stack(np.meshgrid(*[starts] * dim, indexing="ij"), -1).reshape(-1, dim):
        lo = [max(int(c) - 2, 0) for c in corner]
        hi = [min(int(c) + block + 2, N) for c in corner]
        win = Window(dim, k, N, lo, hi)
        owned = np.ones(win.size, dtype=bool)
        for m in range(dim):
            oc = own_cell[win.gmulti[:, m]]
            owned &= (oc >= corner[m]) & (oc < min(corner[m] + block, N))
        if not np.all(win.exact_rows(1)[owned]):
            raise AssertionError("block window too small")
        A = assemble(dim, k, N, gamma, window=win)
        if absolute:
            A = abs(A)
        Y[win.gidx[owned]] = (A @ X[win.gidx])[owned]
    return Y


def avs_nodes_windowed(dim, k, N, x, b, omega, nodes, gamma=None, x_is_zero=False):
    """One additive smoothing step S(x, b) (or S(0, b)) evaluated at selected
    nodes of the full-size mesh: residual, patch solves by dense LU and the
    sum over the patches covering the node, on a window of cells around it."""
    n1 = k * N + 1
    out = np.empty(len(nodes))
    for t, g in enumerate(nodes):
        gm = _global_multi(dim, n1, int(g))
        if np.any(gm == 0) or np.any(gm == n1 - 1):
            out[t] = 0.0
            continue
        win = window_around(dim, k, N, gm, 3)
        A = assemble(dim, k, N, gamma, window=win)
        At = assemble(dim, k, N, gamma, bulk="diag", window=win)
        xl = np.zeros(win.size) if x_is_zero else x[win.gidx] * win.free
        r = b[win.gidx] * win.free - (A @ xl)
        # vertices whose patch contains the node
        cand = []
        for m in range(dim):
            i = int(gm[m])
            cand.append([i // k] if i % k == 0 else [i // k, i // k + 1])
        verts = np.array(np.meshgrid(*cand, indexing="ij")).reshape(dim, -1).T
        verts = verts[np.all((verts >= 1) & (verts <= N - 1), axis=1)]
        pidx = patch_indices(dim, k, N, verts, window=win)
        blocks = patch_blocks(At, pidx)
        li = int(win.local_of_global_multi(gm))
        corr = 0.0
        for p in range(len(verts)):
            u = np.linalg.solve(blocks[p], r[pidx[p]])
            corr += u[np.where(pidx[p] == li)[0][0]]
        out[t] = (0.0 if x_is_zero else x[g]) + omega * corr
    return out


# --------------------------------------------------------------------------
# Multigrid (Algorithm 1) and flexible GMRES
# --------------------------------------------------------------------------

class Hierarchy:
    """Levels l = 0..L with N_l = 2^(l+1) cells per direction (coarsest grid:
    2^dim cells, one vertex patch; Sec. 5.1).  Each level re-assembles A_l
    from the bilinear form.  ``local`` = 'inexact' uses the separable patch
    matrices, 'exact' the restriction of A_l.  ``dtype`` float32 runs the
    whole V-cycle in single precision except the coarse solve (Sec. 5.2).
    ``smoother`` = 'avs' (additive) or 'mvs' (coloured multiplicative, the
    same colour order before and after the coarse correction)."""

    def __init__(self, dim, k, N, gamma=None, omega=0.25, pre=1, post=1,
                 local="inexact", dtype=np.float64, coarse="cholesky", smoother="avs"):
        L = int(round(math.log2(N))) - 1
        if 2 ** (L + 1) != N or L < 0:
            raise ValueError("N must be a power of two >= 2")
        self.dim, self.k, self.N, self.L = dim, k, N, L
        self.omega, self.pre, self.post = omega, pre, post
        if smoother not in ("avs", "mvs"):
            raise ValueError(smoother)
        self.smoother = smoother
        self.dtype = np.dtype(dtype)
        self.coarse_mode = coarse
        self.A, self.Alow, self.blocks, self.pidx, self.P, self.colors = [], [], [], [], [None], []
        for l in range(L + 1):
            Nl = 2 ** (l + 1)
            A = assemble(dim, k, Nl, gamma)
            At = A if local == "exact" else assemble(dim, k, Nl, gamma, bulk="diag")
            pidx = patch_indices(dim, k, Nl)
            self.A.append(A)
            self.Alow.append(A.astype(self.dtype))
            self.blocks.append(patch_blocks(At, pidx).astype(self.dtype))
            self.pidx.append(pidx)
            self.colors.append(mvs_colors(dim, Nl))
            if l > 0:
                self.P.append(prolongation(dim, k, Nl // 2).astype(self.dtype))
        free0 = ~boundary_mask(dim, k, 2)
        self.free0 = free0
        A0 = self.A[0][free0][:, free0].toarray()
        self.chol0 = sla.cho_factor(A0, lower=True)

    def coarse_solve(self, b0):
        """x_0 = A_0^{-1} b_0 in float64 (dense Cholesky; coarse solver reading G9)."""
        x = np.zeros(b0.shape, dtype=np.float64)
        if self.coarse_mode == "cholesky":
            x[self.free0] = sla.cho_solve(self.chol0, np.asarray(b0, np.float64)[self.free0])
            return x.astype(self.dtype)
        return avs_apply(self.Alow[0], self.blocks[0], self.pidx[0], None, b0, 1.0, 1, x_is_zero=True)

    def smooth(self, l, x, b, steps, x_is_zero=False):
        if self.smoother == "mvs":
            return mvs_apply(self.Alow[l], self.blocks[l], self.pidx[l], self.colors[l], x, b, self.omega, steps,
                             x_is_zero)
        return avs_apply(self.Alow[l], self.blocks[l], self.pidx[l], x, b, self.omega, steps, x_is_zero)

    def mg(self, l, b):
        """MG_l(0, b) of Algorithm 1 (with a return right after the coarse
        solve: reading G6)."""
        if l == 0:
            return self.coarse_solve(b)
        if self.pre > 0:
            x = self.smooth(l, None, b, self.pre, x_is_zero=True)
        else:
            x = np.zeros_like(b)
        r = b - self.Alow[l] @ x
        bc = (self.P[l].T @ r).astype(self.dtype)
        e = self.mg(l - 1, bc)
        x = x + (self.P[l] @ e).astype(self.dtype)
        if self.post > 0:
            x = self.smooth(l, x, b, self.post)
        return x

    def vcycle(self, b):
        """z = MG_L(0, b); in float32 mode b is rounded on entry and z returned in float64."""
        return self.mg(self.L, np.asarray(b).astype(self.dtype)).astype(np.float64)


def fgmres(A, b, precond=None, rtol=1e-8, restart=50, maxiter=1000, x0=None):
    """Right-preconditioned flexible GMRES(m) in float64 with classical
    Gram-Schmidt applied twice and Givens rotations; stops when the Arnoldi
    residual estimate |g_{j+1}| <= rtol * ||b|| (Sec. 5.1: relative residual
    reduction 1e-8; restart, orthogonalisation and x0 are readings G15).
    Returns (x, info)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if precond is None:
        precond = lambda v: v  # noqa: E731
    r = b - A @ x
    beta = np.linalg.norm(r)
    hist = [beta]
    its = 0
    converged = beta <= rtol * bnorm
    while not converged and its < maxiter:
        m = restart
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(m):
            Z[:, j] = precond(V[:, j])
            w = A @ Z[:, j]
            h = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h
            h2 = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= rtol * bnorm or hn == 0.0 or its >= maxiter:
                break
            V[:, j + 1] = w / hn
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done])
        x = x + Z[:, :j_done] @ y
        r = b - A @ x
        beta = np.linalg.norm(r)
        converged = hist[-1] <= rtol * bnorm
    return x, {"iterations": its, "converged": bool(converged), "history": hist,
               "rel_res_est": hist[-1] / bnorm if bnorm else 0.0,
               "rel_res_true": beta / bnorm if bnorm else 0.0}


def fcg(A, b, precond=None, rtol=1e-8, maxiter=1000, x0=None):
    """Flexible conjugate gradients in float64 with one retained direction
    (the paper's Krylov method for the symmetric additive smoother, Sec.
    5.1; the flexible form tolerates a preconditioner that is only nearly
    symmetric, such as a float32 V-cycle):
        z = M(r);  p = z - (z.q_old / p_old.q_old) p_old  (p = z at first);
        q = A p;  alpha = (r.p) / (p.q);  x += alpha p;  r -= alpha q,
    stopping when the recursive residual |r| <= rtol |b| (x0 = 0 unless
    given).  Returns (x, info) with the true residual of x."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if precond is None:
        precond = lambda v: v  # noqa: E731
    r = b - A @ x
    hist = [np.linalg.norm(r)]
    p = q = None
    pq = None
    its = 0
    while hist[-1] > rtol * bnorm and its < maxiter:
        z = precond(r)
        p = z.copy() if p is None else z - (z @ q) / pq * p
        q = A @ p
        pq = p @ q
        alpha = (r @ p) / pq
        x = x + alpha * p
        r = r - alpha * q
        its += 1
        hist.append(np.linalg.norm(r))
    rt = np.linalg.norm(b - A @ x)
    return x, {"iterations": its, "converged": bool(hist[-1] <= rtol * bnorm), "history": hist,
               "rel_res_est": hist[-1] / bnorm if bnorm else 0.0, "rel_res_true": rt / bnorm if bnorm else 0.0}


def fractional_iterations(n: int, rn: float, r0: float) -> float:
    """nu_frac = 8 n / (-log10(|r_n| / |r_0|)): steps needed for a 1e-8
    reduction at the average rate (Sec. 5.1; the printed formula is read as
    having its log inverted: reading G7)."""
    return 8.0 * n / (-math.log10(rn / r0))


# --------------------------------------------------------------------------
# Manufactured clamped solution u = prod sin^2(pi x_i) (eq. hnorm, eq. energyerror)
# --------------------------------------------------------------------------

def _s(x, d):
    """d-th derivative of sin^2(pi x) = (1 - cos 2 pi x) / 2."""
    p = math.pi
    if d == 0:
        return 0.5 - 0.5 * np.cos(2 * p * x)
    if d == 1:
        return p * np.sin(2 * p * x)
    if d == 2:
        return 2 * p ** 2 * np.cos(2 * p * x)
    if d == 3:
        return -4 * p ** 3 * np.sin(2 * p * x)
    if d == 4:
        return -8 * p ** 4 * np.cos(2 * p * x)
    raise ValueError(d)


def _u_deriv(X, orders):
    """Partial derivative of u = prod sin^2(pi x_m) with orders[m] in axis m."""
    out = np.ones(X.shape[:-1])
    for m, o in enumerate(orders):
        out = out * _s(X[..., m], o)
    return out


def _f_bilaplace(X):
    """f = Delta^2 u (closed form) for the model problem (reading G1: +Delta^2)."""
    dim = X.shape[-1]
    f = np.zeros(X.shape[:-1])
    for i in range(dim):
        o = [0] * dim
        o[i] = 4
        f += _u_deriv(X, o)
    for i in range(dim):
        for j in range(i + 1, dim):
            o = [0] * dim
            o[i] = 2
            o[j] = 2
            f += 2 * _u_deriv(X, o)
    return f


def _cell_points(dim, k, N, q):
    """Physical quadrature points (ncell, nq, dim), weights (nq,), basis (nq, nloc)."""
    h = 1.0 / N
    tq, wq = gauss_legendre(q)
    z = gll_nodes(k)
    E = lagrange_eval(z, tq)
    ref = node_multi_index(dim, q)  # (nq, dim) indices into tq
    cells = node_multi_index(dim, N)
    X = (cells[:, None, :] + tq[ref][None, :, :]) * h
    W = _kron_list([wq * h] * dim).ravel()
    return X, W, E, cells


def load_vector(dim: int, k: int, N: int, f, q: int | None = None) -> np.ndarray:
    """F(phi_i) = int f phi_i (eq. ``bfandrhs``) with q-point Gauss quadrature
    per direction (default k+4); zero on boundary nodes.  ``f`` maps an
    array of points (..., dim) to values (...)."""
    X, W, E, cells = _cell_points(dim, k, N, k + 4 if q is None else q)
    Bv = _kron_list([E[0]] * dim)  # (nq, nloc)
    f = f(X)  # (ncell, nq)
    loc = (f * W[None, :]) @ Bv
    n1 = k * N + 1
    strides = n1 ** np.arange(dim)
    off = _local_offsets(dim, k, strides)
    base = (cells * k * strides[None, :]).sum(axis=1)
    F = np.zeros(n1 ** dim)
    np.add.at(F, (base[:, None] + off[None, :]).ravel(), loc.ravel())
    F[boundary_mask(dim, k, N)] = 0.0
    return F


def manufactured_rhs(dim: int, k: int, N: int) -> np.ndarray:
    """Load vector of f = Delta^2 u for u = prod sin^2(pi x_m)."""
    return load_vector(dim, k, N, _f_bilaplace)


def exact_solution_nodal(dim: int, k: int, N: int) -> np.ndarray:
    """Nodal interpolant of u = prod sin^2(pi x_m)."""
    h = 1.0 / N
    z = gll_nodes(k)
    n1 = k * N + 1
    x1 = np.concatenate([c * h + z[:-1] * h for c in range(N)] + [[1.0]])
    mi = node_multi_index(dim, n1)
    return _u_deriv(x1[mi], [0] * dim)


def energy_error(dim: int, k: int, N: int, uh: np.ndarray, gamma=None) -> float:
    """||u - u_h||_h of eq. ``hnorm``: broken H^2 seminorm over cells plus
    gamma/h ||[d_n u_h]||^2 over faces (the exact solution has no jumps)."""
    h = 1.0 / N
    gam = float(k * (k + 1) if gamma is None else gamma)
    q = k + 3
    X, W, E, cells = _cell_points(dim, k, N, q)
    n1 = k * N + 1
    strides = n1 ** np.arange(dim)
    off = _local_offsets(dim, k, strides)
    base = (cells * k * strides[None, :]).sum(axis=1)
    U = uh[base[:, None] + off[None, :]]  # (ncell, nloc)
    err2 = 0.0
    for i in range(dim):
        for j in range(dim):
            c = [0] * dim
            c[i] += 1
            c[j] += 1
            H = _kron_list([E[c[m]] / h ** c[m] for m in range(dim)])
            d = U @ H.T - _u_deriv(X, c)
            err2 += float(((d ** 2) * W[None, :]).sum())
    # faces: jumps of the discrete normal derivative
    for m in range(dim):
        GL, _, Wf = _face_traces(dim, k, h, m, 1.0)
        GR, _, _ = _face_traces(dim, k, h, m, 0.0)
        for f in range(N + 1):
            jmp = 0.0
            if f > 0:
                sel = cells[:, m] == f - 1
                jmp = jmp + U[sel] @ GL.T
            if f < N:
                sel = cells[:, m] == f
                jmp = jmp - U[sel] @ GR.T
            err2 += gam / h * float(((jmp ** 2) * Wf[None, :]).sum())
    return math.sqrt(err2)
