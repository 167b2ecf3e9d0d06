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
