"""Fourth-order Hermite equilibrium (oracle; test infrastructure only).

Sec. II.A, eq. (10): the equilibrium Hermite coefficients are the Hermite
moments of the Maxwellian,

    a0 = rho
    a1_a = rho u_a
    a2_ab = rho (u_a u_b + T0 (theta - 1) d_ab)
    a3_abc = rho [u_a u_b u_c + T0 (theta - 1)(d_ab u_c + d_ac u_b + d_bc u_a)]
    a4_abcd = rho [u_a u_b u_c u_d
                   + T0 (theta - 1)(d_ab u_c u_d + d_ac u_b u_d + d_ad u_b u_c
                                    + d_bc u_a u_d + d_bd u_a u_c + d_cd u_a u_b)
                   + T0^2 (theta - 1)^2 (d_ab d_cd + d_ac d_bd + d_ad d_bc)]

(the printed 4th-order line is garbled; this is the reading in which the
bracket carries one factor T0 (theta - 1) on the six u u delta terms and two
factors on the three delta delta terms, i.e. the 4th Hermite moment of a
Gaussian with mean u and variance theta).  T0 = 1 and c_s = 1 (code units).

The discrete equilibrium (Sec. II.A eq. (9) with the quadrature weights of
Sec. II.B) is

    f_eq_i = w_i sum_{n=0}^{4} (1/n!) a_eq^(n) : H^(n)(xi_i),

evaluated here as the literal full contraction over all 2^n index tuples.

Sec. II.D, eq. (15): g_eq_i = (2 C_v - D) theta f_eq_i with C_v = R/(gamma-1)
and R = 1.
"""
import math

import numpy as np

from .velocity import D, delta, hermite_tensor, index_tuples


def eq_coefficient(n, idx, rho, ux, uy, theta):
    """Component ``idx`` of a_eq^(n) (eq. (10)); arrays broadcast over nodes."""
    u = (ux, uy)
    t = theta - 1.0
    if n == 0:
        return rho
    if n == 1:
        (a,) = idx
        return rho * u[a]
    if n == 2:
        a, b = idx
        return rho * (u[a] * u[b] + t * delta(a, b))
    if n == 3:
        a, b, c = idx
        return rho * (u[a] * u[b] * u[c]
                      + t * (delta(a, b) * u[c] + delta(a, c) * u[b] + delta(b, c) * u[a]))
    if n == 4:
        a, b, c, d = idx
        uu = (delta(a, b) * u[c] * u[d] + delta(a, c) * u[b] * u[d]
              + delta(a, d) * u[b] * u[c] + delta(b, c) * u[a] * u[d]
              + delta(b, d) * u[a] * u[c] + delta(c, d) * u[a] * u[b])
        dd = (delta(a, b) * delta(c, d) + delta(a, c) * delta(b, d)
              + delta(a, d) * delta(b, c))
        return rho * (u[a] * u[b] * u[c] * u[d] + t * uu + t * t * dd)
    raise ValueError("the equilibrium is truncated at 4th order")


def f_eq(xi, w, rho, ux, uy, theta, order=4):
    """Discrete Hermite equilibrium for every velocity.

    xi: (Q, 2), w: (Q,); rho, ux, uy, theta: arrays of shape (n,) (or scalars).
    Returns an array of shape (Q, n): for each order n and each index tuple the
    product a_eq^(n)[idx] * H^(n)[idx](xi_i) / n! is added, then the sum is
    multiplied by w_i.
    """
    rho = np.atleast_1d(np.asarray(rho))
    ux = np.atleast_1d(np.asarray(ux))
    uy = np.atleast_1d(np.asarray(uy))
    theta = np.asarray(theta) * np.ones_like(rho)
    dtype = np.result_type(rho, ux, uy, theta, float)
    xT = np.asarray(xi, dtype=float).T  # (2, Q)
    total = np.zeros((len(w),) + rho.shape, dtype=dtype)
    for n in range(order + 1):
        for idx in index_tuples(n):
            h = hermite_tensor(n, idx, xT)  # (Q,)
            a = eq_coefficient(n, idx, rho, ux, uy, theta)  # (n_nodes,)
            total = total + np.multiply.outer(h, a) / math.factorial(n)
    return np.asarray(w, dtype=float)[:, None] * total


def cv_of_gamma(gamma):
    """Heat capacity at constant volume with R = 1 (Sec. II.D: gamma = R/C_v + 1)."""
    return 1.0 / (gamma - 1.0)


def g_eq(feq, theta, gamma):
    """Second-population equilibrium g_eq_i = (2 C_v - D) theta f_eq_i (Sec. II.D)."""
    return (2.0 * cv_of_gamma(gamma) - D) * theta * feq
