"""Pins of the oracle's 1D ingredients against closed forms (not GPU)."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle as O


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7])
def test_gll_nodes_closed_form_and_exactness(k):
    z = O.gll_nodes(k)
    assert z[0] == 0.0 and z[-1] == 1.0
    assert np.allclose(z + z[::-1], 1.0, atol=1e-15)
    # Lobatto weights from the textbook closed form 2/(k(k+1) P_k(x)^2) on [-1,1]
    x = 2 * z - 1
    Pk = npleg.legval(x, [0] * k + [1])
    w = 1.0 / (k * (k + 1) * Pk ** 2)  # mapped to [0,1]
    assert abs(w.sum() - 1.0) < 1e-14
    for m in range(2 * k):  # exact up to degree 2k-1
        assert abs((w * z ** m).sum() - 1.0 / (m + 1)) < 1e-14
    if k == 2:
        assert np.allclose(z, [0, 0.5, 1])
    if k == 3:
        assert np.allclose(z, [0, 0.5 - 0.5 / math.sqrt(5), 0.5 + 0.5 / math.sqrt(5), 1], atol=1e-15)
    if k == 4:
        r = math.sqrt(3 / 7)
        assert np.allclose(z, [0, 0.5 - r / 2, 0.5, 0.5 + r / 2, 1], atol=1e-15)


@pytest.mark.parametrize("q", [1, 2, 4, 8])
def test_gauss_legendre_exactness(q):
    t, w = O.gauss_legendre(q)
    for m in range(2 * q):
        assert abs((w * t ** m).sum() - 1.0 / (m + 1)) < 1e-14
    assert abs((w * t ** (2 * q)).sum() - 1.0 / (2 * q + 1)) > 1e-12


@pytest.mark.parametrize("k", [2, 3, 5, 7])
def test_lagrange_partition_interpolation_reproduction(k):
    z = O.gll_nodes(k)
    t = np.linspace(0, 1, 23)
    E = O.lagrange_eval(z, t)
    assert np.allclose(E[0].sum(1), 1, atol=1e-12)
    assert np.allclose(E[1].sum(1), 0, atol=1e-9)
    assert np.allclose(E[2].sum(1), 0, atol=1e-8)
    assert np.allclose(O.lagrange_eval(z, z)[0], np.eye(k + 1), atol=1e-13)
    for m in range(k + 1):  # reproduces t^m and its derivatives
        assert np.allclose(E[0] @ z ** m, t ** m, atol=1e-12)
        assert np.allclose(E[1] @ z ** m, m * t ** max(m - 1, 0) if m else 0 * t, atol=1e-9)
        d2 = m * (m - 1) * t ** max(m - 2, 0) if m > 1 else 0 * t
        assert np.allclose(E[2] @ z ** m, d2, atol=1e-7)


def test_dof_counts_match_paper_tables():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "dof_counts.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        assert O.num_dofs(r["dim"], r["k"], r["N"]) == r["dofs"], r
