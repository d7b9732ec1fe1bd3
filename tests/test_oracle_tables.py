"""Pins of the oracle's reference tables against values the paper prints and
closed-form facts of the rules and tableaux."""
import math
import os

import numpy as np
import pytest

from oracle import (basis_nodes, eq_rule, gl_rule, gll_rule, lagrange_derivs,
                    lagrange_values, tableau, tensor_basis)
from oracle.swdg import Oracle, Mesh, Params

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_table2_positivity_cfl():
    """Table 2: CFL = w1(GLL_{r+2}) / a21(RK32) prints as 0.28, 0.14, 0.085."""
    rows = np.loadtxt(os.path.join(GOLD, "table2_positivity_cfl.txt"))
    A, _, _ = tableau("rk32")
    a21 = A[1][0]
    for r, printed, lin in rows:
        r = int(r)
        _, w = gll_rule(r + 2)
        cfl = w[0] / a21
        # the paper prints two significant digits
        assert float(f"{cfl:.2g}") == pytest.approx(printed, abs=1e-12), (r, cfl)
        assert 1.0 / (2 * r + 1) == pytest.approx(lin)
        assert cfl < lin       # positivity is the binding restriction


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 16])
def test_gll_exactness_and_endpoint_weight(n):
    x, w = gll_rule(n)
    assert x[0] == 0.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    # exact for degree 2n-3 (closed form int_0^1 x^k = 1/(k+1)), not for 2n-2
    for k in range(2 * n - 2):
        assert np.dot(w, x ** k) == pytest.approx(1.0 / (k + 1), rel=1e-13, abs=1e-15)
    if n <= 8:
        k = 2 * n - 2
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) > 1e-11
    # end-point weight of the n-point Lobatto rule on [0,1]: 1/(n(n-1))
    assert w[0] == pytest.approx(1.0 / (n * (n - 1)), rel=1e-13)


@pytest.mark.parametrize("n", [3, 8, 16, 32])
def test_equispaced_rule(n):
    x, w = eq_rule(n)
    assert w.sum() == pytest.approx(1.0, rel=1e-15)
    assert np.dot(w, x) == pytest.approx(0.5, rel=1e-15)
    assert w[0] == pytest.approx(0.5 / (n - 1))


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_gauss_legendre_exactness(n):
    x, w = gl_rule(n)
    for k in range(2 * n):
        assert np.dot(w, x ** k) == pytest.approx(1.0 / (k + 1), rel=1e-13)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_lagrange_basis(r):
    nodes = basis_nodes(r)
    # interpolation property and partition of unity (used in Prop. 3.2's proof)
    assert np.allclose(lagrange_values(nodes, nodes), np.eye(r + 1), atol=1e-14)
    xs = np.linspace(0, 1, 17)
    assert np.allclose(lagrange_values(nodes, xs).sum(1), 1.0, atol=1e-14)
    # derivative reproduces d/dx of x^k for k <= r (closed form k x^(k-1))
    for k in range(r + 1):
        coef = nodes ** k
        d = lagrange_derivs(nodes, xs) @ coef
        assert np.allclose(d, k * xs ** max(k - 1, 0) if k else 0.0, atol=1e-12)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_tensor_basis_gradient_matches_difference(r):
    rng = np.random.default_rng(1)
    X, Y = rng.uniform(0.1, 0.9, 5), rng.uniform(0.1, 0.9, 5)
    v, gx, gy = tensor_basis(r, X, Y)
    e = 1e-6
    vxp, _, _ = tensor_basis(r, X + e, Y)
    vxm, _, _ = tensor_basis(r, X - e, Y)
    vyp, _, _ = tensor_basis(r, X, Y + e)
    vym, _, _ = tensor_basis(r, X, Y - e)
    assert np.allclose((vxp - vxm) / (2 * e), gx, atol=1e-8)
    assert np.allclose((vyp - vym) / (2 * e), gy, atol=1e-8)


@pytest.mark.parametrize("name,order", [("fe", 1), ("ssp3", 3), ("rk32", 2), ("rk44", 4)])
def test_tableau_order_conditions(name, order):
    A, b, c = tableau(name)
    A, b, c = np.array(A), np.array(b), np.array(c)
    assert np.allclose(A.sum(1), c)                 # row-sum condition (Appendix A)
    assert b.sum() == pytest.approx(1.0)            # first order
    if order >= 2:
        assert b @ c == pytest.approx(0.5)          # second order (Appendix A)
    if order >= 3:
        assert b @ c ** 2 == pytest.approx(1 / 3)
        assert b @ A @ c == pytest.approx(1 / 6)
    if order >= 4:
        assert b @ c ** 3 == pytest.approx(1 / 4)
        assert b @ (c * (A @ c)) == pytest.approx(1 / 8)
        assert b @ A @ c ** 2 == pytest.approx(1 / 12)
        assert b @ A @ A @ c == pytest.approx(1 / 24)


def test_rk32_free_parameter_and_ratio():
    """Appendix A: chi = 1 - sqrt(2)/2, a32 = 1/2; Sec. 3.4: 1/a21 is about 1.7."""
    A, b, c = tableau("rk32")
    chi = 1 - math.sqrt(2) / 2
    assert A[1][0] == pytest.approx(2 * chi)
    assert A[2][1] == pytest.approx(0.5)
    assert b[2] == pytest.approx(chi)
    assert 1 / A[1][0] == pytest.approx(1.7, abs=0.05)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_discharge_mass_matrix_is_exact(r):
    """Table 1: GL (r+1)^2 integrates psi_i psi_j exactly; compare with a 12-point rule."""
    m = Mesh.uniform(1, 1, 0.0, 0.0, 1.0)
    o = Oracle(m, Params(r=r, S=(r + 2,)))
    x, w = gl_rule(12)
    v, _, _ = tensor_basis(r, np.tile(x, 12), np.repeat(x, 12))
    ref = v.T @ (np.outer(w, w).ravel()[:, None] * v)
    assert np.allclose(o.Mq_ref.numpy(), ref, atol=1e-15)
    assert o.mean_w.numpy().sum() == pytest.approx(1.0)
