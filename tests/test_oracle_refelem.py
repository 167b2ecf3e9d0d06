"""Pins of the oracle reference element against closed forms (nodal P_k, k=1..4)."""
import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_triangle_quadrature_monomials(k):
    # int_T r^a s^b = a! b! / (a+b+2)!  for a+b <= 2k+1
    pts, w = O.tri_quad(k + 2)
    for a in range(2 * k + 2):
        for b in range(2 * k + 2 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(got - exact) < 1e-15, (a, b, got, exact)


def test_p1_mass_closed_form():
    r = O.refelem(1)
    assert np.allclose(r["M"], np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]]) / 24.0, atol=1e-15, rtol=0)
    # facet mass on [0,1]: 1/6 [[2,1],[1,2]]
    assert np.allclose(r["M1"], np.array([[2, 1], [1, 2]]) / 6.0, atol=1e-15, rtol=0)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_mass_properties(k):
    r = O.refelem(k)
    npk = (k + 1) * (k + 2) // 2
    assert abs(r["M"].sum() - 0.5) < 1e-14            # partition of unity: sum M = |T| = 1/2
    assert np.allclose(r["M"], r["M"].T, atol=1e-16)
    assert np.all(np.linalg.eigvalsh(r["M"]) > 0)
    assert np.abs(r["M"] @ r["Minv"] - np.eye(npk)).max() < 1e-12
    assert abs(r["M1"].sum() - 1.0) < 1e-14


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_nodal_basis_and_derivatives_exact(k):
    r = O.refelem(k)
    nodes = r["nodes"]
    npk = nodes.shape[0]
    # Lagrange property at the nodes
    for i in range(npk):
        phi = O.basis(k, nodes[i, 0], nodes[i, 1])
        assert np.abs(phi - np.eye(npk)[i]).max() < 1e-12
    # Dr, Ds reproduce derivatives of every monomial of degree <= k
    for a in range(k + 1):
        for b in range(k + 1 - a):
            p = nodes[:, 0] ** a * nodes[:, 1] ** b
            dr = a * nodes[:, 0] ** max(a - 1, 0) * nodes[:, 1] ** b if a else 0 * p
            ds = b * nodes[:, 0] ** a * nodes[:, 1] ** max(b - 1, 0) if b else 0 * p
            assert np.abs(r["Dr"] @ p - dr).max() < 1e-11
            assert np.abs(r["Ds"] @ p - ds).max() < 1e-11


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_facet_nodes(k):
    r = O.refelem(k)
    nodes, fn = r["nodes"], r["fnodes"]
    verts = np.array([[0, 0], [1, 0], [0, 1]], float)
    for f in range(3):
        a, b = verts[f], verts[(f + 1) % 3]
        for m in range(k + 1):
            assert np.allclose(nodes[fn[f, m]], a + (b - a) * m / k)


def _exact_tables(k):
    """The element's tables in exact rational arithmetic (Python fractions):
    Lagrange basis from the monomial Vandermonde matrix, mass matrices from the
    exact monomial moments int r^a s^b = a! b! / (a+b+2)! and int_0^1 t^e = 1/(e+1)."""
    from fractions import Fraction as F

    def inv(A):
        n = len(A)
        a = [list(row) + [F(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
        for c in range(n):
            p = next(r for r in range(c, n) if a[r][c] != 0)
            a[c], a[p] = a[p], a[c]
            d = a[c][c]
            a[c] = [x / d for x in a[c]]
            for r in range(n):
                if r != c and a[r][c] != 0:
                    f = a[r][c]
                    a[r] = [x - f * y for x, y in zip(a[r], a[c])]
        return [row[n:] for row in a]

    nodes = [(F(i, k), F(j, k)) for j in range(k + 1) for i in range(k + 1 - j)]
    ex = [(d - b, b) for d in range(k + 1) for b in range(d + 1)]
    n = len(nodes)
    C = inv([[r ** a * s ** b for (a, b) in ex] for (r, s) in nodes])

    def der(a, b, r, s, wrt_r):
        if wrt_r:
            return a * r ** (a - 1) * s ** b if a else F(0)
        return b * r ** a * s ** (b - 1) if b else F(0)

    Dr = [[sum(der(*ex[m], *nodes[i], True) * C[m][j] for m in range(n)) for j in range(n)] for i in range(n)]
    Ds = [[sum(der(*ex[m], *nodes[i], False) * C[m][j] for m in range(n)) for j in range(n)] for i in range(n)]
    mom = lambda a, b: F(math.factorial(a) * math.factorial(b), math.factorial(a + b + 2))
    M = [[sum(C[p][i] * C[q][j] * mom(ex[p][0] + ex[q][0], ex[p][1] + ex[q][1]) for p in range(n) for q in range(n))
          for j in range(n)] for i in range(n)]
    C1 = inv([[F(a, k) ** e for e in range(k + 1)] for a in range(k + 1)])
    M1 = [[sum(C1[e1][a] * C1[e2][b] * F(1, e1 + e2 + 1) for e1 in range(k + 1) for e2 in range(k + 1))
           for b in range(k + 1)] for a in range(k + 1)]
    return dict(Dr=Dr, Ds=Ds, M=M, Minv=inv(M), M1=M1)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_tables_are_the_exact_rationals_rounded_once(k):
    """Every table equals the exact rational value rounded to the nearest double
    (up to one unit in the last place: the tables are computed in binary128 and
    rounded once, so double rounding may move a tie by one ulp); entries that are
    exactly zero come out below 1e-30."""
    r = O.refelem(k)
    ex = _exact_tables(k)
    for name, exact in ex.items():
        got = r[name]
        for i, row in enumerate(exact):
            for j, e in enumerate(row):
                g = got[i, j]
                if e == 0:
                    assert abs(g) < 1e-30, (name, i, j, g)
                else:
                    assert abs(g - float(e)) <= np.spacing(abs(float(e))), (name, i, j, g, float(e))
