"""Oracle pins: quadrature rules, Lagrange tables and the periodic mesh
(paper Sec. III.A, eqn:FEWfns, eqn:cellIntegrals; Sec. III.B.2 for M_D)."""
import math

import numpy as np
import pytest

from oracle import fe


def test_gll_closed_forms():
    x, w = fe.gauss_lobatto(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = fe.gauss_lobatto(4)
    s = math.sqrt(3 / 7)
    assert np.allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


def test_gl_closed_forms():
    x, w = fe.gauss_legendre(2)
    assert np.allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)
    assert np.allclose(w, [1, 1], atol=1e-15)
    x, w = fe.gauss_legendre(3)
    assert np.allclose(x, [-math.sqrt(0.6), 0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


def _mono_int(k):
    return 0.0 if k % 2 else 2.0 / (k + 1)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_exactness_degree(p):
    x, w = fe.gauss_lobatto(p)
    assert abs(w.sum() - 2) < 1e-14
    for k in range(2 * p):
        assert abs(w @ x ** k - _mono_int(k)) < 1e-13
    # not exact one degree higher (identifies the rule)
    assert abs(w @ x ** (2 * p) - _mono_int(2 * p)) > 1e-6


@pytest.mark.parametrize("n", range(1, 10))
def test_gl_exactness_degree(n):
    x, w = fe.gauss_legendre(n)
    for k in range(2 * n):
        assert abs(w @ x ** k - _mono_int(k)) < 1e-13
    assert abs(w @ x ** (2 * n) - _mono_int(2 * n)) > 1e-6


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
def test_lagrange_tables(p):
    xi, _ = fe.gauss_lobatto(p)
    B, D = fe.lagrange_tables(xi, xi)
    assert np.allclose(B, np.eye(p + 1), atol=1e-14)
    t = np.linspace(-1, 1, 17)
    B, D = fe.lagrange_tables(xi, t)
    # reproduces polynomials up to degree p, and their derivatives
    for k in range(p + 1):
        assert np.allclose(xi ** k @ B, t ** k, atol=1e-12)
        dk = k * t ** (k - 1) if k else np.zeros_like(t)
        assert np.allclose(xi ** k @ D, dk, atol=1e-10)
    # derivative table against central differences of the value table
    h = 1e-6
    Bp, _ = fe.lagrange_tables(xi, t + h)
    Bm, _ = fe.lagrange_tables(xi, t - h)
    assert np.allclose((Bp - Bm) / (2 * h), D, atol=1e-6)


def test_mesh_numbering_and_mass():
    m = fe.Mesh((3, 2, 4), (6.0, 5.0, 7.0), 3, "gl", 4)
    assert m.n_nodes == 9 * 6 * 12
    counts = np.zeros(m.n_nodes, dtype=int)
    for e in range(m.n_cell_total):
        g = m.cell_nodes(e)
        assert len(set(g.tolist())) == g.size
        counts[g] += 1
    # interior nodes of a cell: 1 cell; face: 2; edge: 4; vertex: 8
    assert set(np.unique(counts).tolist()) == {1, 2, 4, 8}
    assert np.sum(counts == 8) == 3 * 2 * 4
    M = m.lumped_mass()
    assert abs(M.sum() - 6.0 * 5.0 * 7.0) < 1e-12
    # node coordinates of a cell's nodes equal its GLL-mode quadrature points
    mg = fe.Mesh((3, 2, 4), (6.0, 5.0, 7.0), 3, "gll")
    X = mg.node_coords()
    for e in [0, 5, 23]:
        assert np.allclose(X[mg.cell_nodes(e)], np.mod(mg.quad_points(e), mg.box), atol=1e-14)
