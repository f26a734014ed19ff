"""Pins of the oracle's velocity set, Hermite tensors and equilibrium.

Each check compares against something other than the oracle's own formulas:
numpy's Gauss-Hermite rule and Hermite polynomials, closed-form Gaussian
moments, and the numbers printed in Table I.
"""
import math
import os

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

from oracle.equilibrium import f_eq, g_eq
from oracle.velocity import d1q3, d1q5, d2q9, d2q25, hermite_tensor, index_tuples
from tests.conftest import GOLDEN


def test_d1q5_matches_table1_fixture():
    """Table I as printed (golden fixture) against the oracle's arrays."""
    xi, w = d1q5()
    rows = [l.split() for l in open(os.path.join(GOLDEN, "d1q5_table1.txt"))
            if l.strip() and not l.startswith("#")]
    env = {"sqrt": math.sqrt}
    for k, (idx, xe, we) in enumerate(rows):
        assert int(idx) == k
        assert xi[k] == pytest.approx(eval(xe, env), abs=1e-15)
        assert w[k] == pytest.approx(eval(we, env), abs=1e-15)


def test_d1q5_is_gauss_hermite_rule():
    """Nodes = roots of He_5 and weights = numpy's probabilists' Gauss-Hermite
    weights normalised by sqrt(2 pi)."""
    xi, w = d1q5()
    ref_x, ref_w = He.hermegauss(5)
    ref_w = ref_w / np.sqrt(2.0 * np.pi)
    order = np.argsort(xi)
    np.testing.assert_allclose(xi[order], ref_x, atol=1e-14)
    np.testing.assert_allclose(w[order], ref_w, atol=1e-15)
    # He_5(x) = x^5 - 10 x^3 + 15 x vanishes at every node
    np.testing.assert_allclose(xi ** 5 - 10 * xi ** 3 + 15 * xi, 0.0, atol=1e-12)


def test_quadrature_order_nine():
    """sum_a w_a He_k He_m = k! delta_km for k + m <= 9 (Sec. II.B: Q = 9), and the
    rule is not exact at degree 10."""
    xi, w = d1q5()
    for k in range(10):
        for m in range(10 - k):
            ck = np.zeros(k + 1)
            ck[k] = 1
            cm = np.zeros(m + 1)
            cm[m] = 1
            s = np.sum(w * He.hermeval(xi, ck) * He.hermeval(xi, cm))
            assert s == pytest.approx(math.factorial(k) if k == m else 0.0, abs=1e-11)
    assert abs(np.sum(w * xi ** 10) - 945.0) > 1.0


def _he(n, x):
    c = np.zeros(n + 1)
    c[n] = 1
    return He.hermeval(x, c)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4])
def test_hermite_tensors_factorise(n):
    """A 2-D Hermite tensor component with k x-indices and m y-indices equals
    He_k(xi_x) He_m(xi_y) (numpy's Hermite polynomials); a dropped or wrong
    symmetrisation term breaks this for some index tuple."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 7))
    for idx in index_tuples(n):
        k = idx.count(0)
        m = idx.count(1)
        np.testing.assert_allclose(hermite_tensor(n, idx, x), _he(k, x[0]) * _he(m, x[1]),
                                   rtol=1e-13, atol=1e-12)


def _gauss_moment(u, t, k):
    """E[X^k] for X ~ N(u, t), closed form."""
    return [1.0, u, u * u + t, u ** 3 + 3 * u * t, u ** 4 + 6 * u * u * t + 3 * t * t][k]


@pytest.mark.parametrize("rho,ux,uy,theta", [(1.3, 0.7, -0.4, 1.7), (0.2, -1.1, 0.3, 0.6),
                                             (1.0, 0.0, 0.0, 1.0), (2.5, 0.05, 1.4, 0.9)])
def test_equilibrium_moments_are_maxwellian(rho, ux, uy, theta):
    """All moments of total order <= 4 of the discrete equilibrium equal those of
    rho N(u_x, theta) N(u_y, theta) (Sec. II.A: the coefficients are the
    Maxwellian's Hermite moments; Sec. II.B: Q = 9 quadrature)."""
    xi, w = d2q25()
    f = f_eq(xi, w, np.array([rho]), np.array([ux]), np.array([uy]), np.array([theta]))[:, 0]
    for a in range(5):
        for b in range(5 - a):
            num = np.sum(f * xi[:, 0] ** a * xi[:, 1] ** b)
            ex = rho * _gauss_moment(ux, theta, a) * _gauss_moment(uy, theta, b)
            assert num == pytest.approx(ex, rel=1e-13, abs=1e-13)


def test_equilibrium_at_rest_is_weights():
    xi, w = d2q25()
    f = f_eq(xi, w, np.array([1.7]), np.array([0.0]), np.array([0.0]), np.array([1.0]))[:, 0]
    np.testing.assert_allclose(f, 1.7 * w, rtol=1e-15)


def test_equilibrium_factorises_per_axis():
    """The 4th-order truncation equals rho w_a w_b sum_{k+m<=4} A_k(u_x)He_k(xi_a)/k!
    * A_m(u_y)He_m(xi_b)/m! with A_k the Hermite moments of N(u, theta): an
    independent form built from numpy's Hermite polynomials."""
    xi1, w1 = d1q5()
    xi, w = d2q25()
    rho, ux, uy, th = 0.8, 0.45, -0.9, 1.3

    def A(u, k):
        t = th - 1.0
        return [1.0, u, u * u + t, u ** 3 + 3 * u * t, u ** 4 + 6 * u * u * t + 3 * t * t][k]

    ref = np.zeros(25)
    for b in range(5):
        for a in range(5):
            s = 0.0
            for k in range(5):
                for m in range(5 - k):
                    s += (A(ux, k) * _he(k, xi1[a]) / math.factorial(k)
                          * A(uy, m) * _he(m, xi1[b]) / math.factorial(m))
            ref[a + 5 * b] = rho * w1[a] * w1[b] * s
    f = f_eq(xi, w, np.array([rho]), np.array([ux]), np.array([uy]), np.array([th]))[:, 0]
    np.testing.assert_allclose(f, ref, rtol=1e-13, atol=1e-16)


def test_g_equilibrium_carries_internal_energy():
    """sum_i g_eq_i = (2 C_v - D) theta rho, so that 2 rho E = rho |u|^2 + 2 C_v rho theta
    (Sec. II, eq. for E, and Sec. II.D)."""
    xi, w = d2q25()
    rho, ux, uy, th, gamma = 1.2, 0.3, -0.2, 0.9, 1.4
    f = f_eq(xi, w, np.array([rho]), np.array([ux]), np.array([uy]), np.array([th]))
    g = g_eq(f, th, gamma)
    cv = 1.0 / (gamma - 1.0)
    two_rho_e = np.sum((xi[:, 0] ** 2 + xi[:, 1] ** 2) * f[:, 0]) + g.sum()
    assert two_rho_e == pytest.approx(rho * (ux * ux + uy * uy) + 2 * cv * rho * th, rel=1e-14)


# ---- D2Q9 (the on-lattice set Sec. III.A compares against) --------------------------
def test_d1q3_is_gauss_hermite_rule_exact_to_degree_five():
    """Nodes = roots of He_3 = x^3 - 3x, weights = numpy's Gauss-Hermite
    weights over sqrt(2 pi) (2/3, 1/6, 1/6); the rule integrates the unit
    Gaussian's moments exactly to degree 5 and not at degree 6 (9 vs 15)."""
    xi, w = d1q3()
    assert xi[0] == 0.0 and xi[1] > 0 > xi[2]
    ref_x, ref_w = He.hermegauss(3)
    order = np.argsort(xi)
    np.testing.assert_allclose(xi[order], ref_x, atol=1e-15)
    np.testing.assert_allclose(w[order], ref_w / np.sqrt(2.0 * np.pi), atol=1e-15)
    gauss = [1, 0, 1, 0, 3, 0, 15]
    for n in range(6):
        assert np.sum(w * xi ** n) == pytest.approx(gauss[n], abs=1e-14)
    assert np.sum(w * xi ** 6) == pytest.approx(9.0, abs=1e-13)


def test_d2q9_second_order_equilibrium_is_the_textbook_one():
    """Truncated at second order, the Hermite equilibrium on D2Q9 is the
    textbook f_eq = w rho (1 + xi.u + ((xi.u)^2 - |u|^2)/2) (c_s = 1)."""
    xi, w = d2q9()
    rho = np.array([1.0, 0.7, 1.3])
    ux = np.array([0.0, 0.05, -0.12])
    uy = np.array([0.0, -0.08, 0.03])
    got = f_eq(xi, w, rho, ux, uy, np.ones(3), order=2)
    xu = xi[:, 0, None] * ux + xi[:, 1, None] * uy
    want = w[:, None] * rho * (1 + xu + 0.5 * (xu ** 2 - (ux ** 2 + uy ** 2)))
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-16)


def test_d2q9_fourth_order_equilibrium_moments():
    """The 4th-order equilibrium at theta = 1 on D2Q9 (the paper's D2Q9 runs,
    Sec. III.A): mass and momentum exact; per axis, the quadrature of
    He_4(xi) xi^2 gives -6 instead of 0 and He_3 vanishes at the nodes, so
    sum f_eq xi_x^2 = rho (1 + u_x^2 - u_x^4 / 4) (Gaussian: rho (1 + u_x^2))
    and sum f_eq xi_x^3 = 3 rho u_x (Gaussian: rho (3 u_x + u_x^3)) -- the
    missing u^3 of the on-lattice set's Galilean error."""
    xi, w = d2q9()
    rho, ux, uy = 1.1, 0.21, -0.13
    f = f_eq(xi, w, rho, ux, uy, 1.0)[:, 0]
    X, Y = xi[:, 0], xi[:, 1]
    assert np.sum(f) == pytest.approx(rho, rel=1e-14)
    assert np.sum(f * X) == pytest.approx(rho * ux, rel=1e-14)
    assert np.sum(f * Y) == pytest.approx(rho * uy, rel=1e-14)
    assert np.sum(f * X * X) == pytest.approx(rho * (1 + ux ** 2 - ux ** 4 / 4), rel=1e-14)
    assert np.sum(f * Y * Y) == pytest.approx(rho * (1 + uy ** 2 - uy ** 4 / 4), rel=1e-14)
    assert np.sum(f * X ** 3) == pytest.approx(3 * rho * ux, rel=1e-14)
    # the mixed second moment keeps the Gaussian's rho u_x u_y: the terms
    # He_k(xi_x) He_m(xi_y) with k + m <= 4 and k, m <= 3 integrate exactly
    assert np.sum(f * X * Y) == pytest.approx(rho * ux * uy, rel=1e-13)


def test_d2q9_equilibrium_factorises_per_axis():
    """The factorised form the kernels evaluate,
    f_eq_{a+3b} = rho w_a w_b sum_{k+m<=4} A_k(u_x) He_k(xi_a)/k! A_m(u_y) He_m(xi_b)/m!
    with A_k = u^k at theta = 1, equals the literal contraction on D2Q9."""
    x1, w1 = d1q3()
    xi, w = d2q9()
    rho, ux, uy = 0.9, -0.3, 0.17
    lit = f_eq(xi, w, rho, ux, uy, 1.0)[:, 0]
    fac = np.zeros(9)
    for b in range(3):
        for a in range(3):
            s = 0.0
            for k in range(5):
                for m in range(5 - k):
                    s += (ux ** k * _he(k, x1[a]) / math.factorial(k)
                          * uy ** m * _he(m, x1[b]) / math.factorial(m))
            fac[a + 3 * b] = rho * w1[a] * w1[b] * s
    np.testing.assert_allclose(fac, lit, rtol=1e-14, atol=1e-16)
