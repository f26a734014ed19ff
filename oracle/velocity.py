"""Velocity set and scaled Hermite tensors (oracle; test infrastructure only).

Sec. II.B, Table I: the D1Q5 abscissae are 0, +-sqrt(5 - sqrt(10)),
+-sqrt(5 + sqrt(10)) with weights 8/15, (7 + 2 sqrt(10))/60 and
(7 - 2 sqrt(10))/60; D2Q25 is their tensor product.  Reading of the table's
"1,3: +-" and "2,4: +-" labels: indices 1 and 2 carry the positive values,
3 and 4 the negative ones.  The 2-D index is i = a + 5 b with a the x- and b the
y-component index.  The lattice speed of sound is 1 (Sec. II.B: c_s = 1 unless
scaled), so normalised and physical velocities coincide.

The D1Q3 rule (roots of He_3) and its tensor product D2Q9 are the on-lattice
set that Sec. III.A compares D2Q25 against, streamed by the same
semi-Lagrangian step and with the same 4th-order equilibrium at theta = 1.

Sec. II.A: the scaled Hermite tensors up to 4th order, with the symmetrising
"overbrace" operator written out as the explicit sum over the distinct index
permutations (3 terms for xi I at 3rd order, 6 terms for xi^2 I and 3 terms
for I delta at 4th order).
"""
import itertools

import numpy as np

D = 2  # spatial dimension


def d1q5():
    """1-D abscissae and weights of Table I, in the index order 0, +s, +l, -s, -l."""
    s10 = np.sqrt(10.0)
    small = np.sqrt(5.0 - s10)
    large = np.sqrt(5.0 + s10)
    xi = np.array([0.0, small, large, -small, -large])
    w = np.array([8.0 / 15.0, (7.0 + 2.0 * s10) / 60.0, (7.0 - 2.0 * s10) / 60.0,
                  (7.0 + 2.0 * s10) / 60.0, (7.0 - 2.0 * s10) / 60.0])
    return xi, w


def d1q3():
    """The three-point Gauss-Hermite rule (roots of He_3, x^3 - 3x): abscissae
    0, +sqrt(3), -sqrt(3) and weights 2/3, 1/6, 1/6, in the index order of
    Table I (zero first, then the positive and the negative value).  Its tensor
    product is the D2Q9 set with which Sec. III.A compares D2Q25 (c_s = 1)."""
    r3 = np.sqrt(3.0)
    return np.array([0.0, r3, -r3]), np.array([2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0])


def tensor_product(xi1, w1):
    """2-D velocity set from a 1-D one: xi_i = (xi_a, xi_b), w_i = w_a w_b, i = a + q b."""
    q = len(xi1)
    xi = np.zeros((q * q, D))
    w = np.zeros(q * q)
    for b in range(q):
        for a in range(q):
            i = a + q * b
            xi[i, 0] = xi1[a]
            xi[i, 1] = xi1[b]
            w[i] = w1[a] * w1[b]
    return xi, w


def d2q25():
    return tensor_product(*d1q5())


def d2q9():
    return tensor_product(*d1q3())


def delta(a, b):
    return 1.0 if a == b else 0.0


def hermite_tensor(n, idx, x):
    """Component ``idx`` (tuple of n axis indices) of H^(n) evaluated at velocity ``x``.

    ``x`` may be a 2-vector or an array of shape (2, ...).  Written term by term
    from the list of scaled Hermite tensors in Sec. II.A with c_s = 1.
    """
    if n == 0:
        return np.ones_like(x[0])
    if n == 1:
        (a,) = idx
        return x[a]
    if n == 2:
        a, b = idx
        return x[a] * x[b] - delta(a, b)
    if n == 3:
        a, b, c = idx
        return (x[a] * x[b] * x[c]
                - (x[a] * delta(b, c) + x[b] * delta(a, c) + x[c] * delta(a, b)))
    if n == 4:
        a, b, c, d = idx
        six = (x[a] * x[b] * delta(c, d) + x[a] * x[c] * delta(b, d)
               + x[a] * x[d] * delta(b, c) + x[b] * x[c] * delta(a, d)
               + x[b] * x[d] * delta(a, c) + x[c] * x[d] * delta(a, b))
        three = (delta(a, b) * delta(c, d) + delta(a, c) * delta(b, d)
                 + delta(a, d) * delta(b, c))
        return x[a] * x[b] * x[c] * x[d] - six + three
    raise ValueError("Hermite tensors are only needed up to 4th order")


def index_tuples(n):
    """All 2^n index tuples (alpha_1, ..., alpha_n) in {0, 1}^n."""
    return list(itertools.product(range(D), repeat=n))
