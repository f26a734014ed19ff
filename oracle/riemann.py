"""Exact solution of the 1-D Riemann problem for an ideal gas (oracle; test infrastructure only).

Reference solution for the Sod shock tube (Sec. III.C compares with Sod's
exact solution).  Written from the Euler equations: the star pressure p* makes
the velocity jumps across the left and right waves add up,

    f_L(p*) + f_R(p*) + (u_R - u_L) = 0,

where a wave into a state K = (rho_K, u_K, p_K) with sound speed c_K is

    a shock (p > p_K):        f_K = (p - p_K) sqrt(A_K / (p + B_K)),
                              A_K = 2 / ((gamma + 1) rho_K),
                              B_K = p_K (gamma - 1) / (gamma + 1);
    a rarefaction (p <= p_K): f_K = 2 c_K / (gamma - 1) [(p / p_K)^((gamma - 1)/(2 gamma)) - 1].

p* is found by bisection (f_L + f_R is monotone in p), u* = (u_L + u_R)/2 +
(f_R(p*) - f_L(p*))/2, and the self-similar solution is sampled at x/t.
"""
import numpy as np


def _wave_function(p, rho, pk, ck, gamma):
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = pk * (gamma - 1.0) / (gamma + 1.0)
        return (p - pk) * np.sqrt(A / (p + B))
    return 2.0 * ck / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma):
    """(p*, u*) for primitive states left = (rho, u, p), right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = np.sqrt(gamma * pl / rl)
    cr = np.sqrt(gamma * pr / rr)

    def residual(p):
        return (_wave_function(p, rl, pl, cl, gamma) + _wave_function(p, rr, pr, cr, gamma)
                + (ur - ul))

    lo, hi = 1e-14, 10.0 * max(pl, pr)
    while residual(hi) < 0.0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if residual(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    u = 0.5 * (ul + ur) + 0.5 * (_wave_function(p, rr, pr, cr, gamma)
                                 - _wave_function(p, rl, pl, cl, gamma))
    return p, u


def sample(left, right, gamma, s):
    """Primitive state (rho, u, p) of the exact solution at similarity coordinate s = x/t."""
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    if s <= us:
        rk, uk, pk = left
        ck = np.sqrt(gamma * pk / rk)
        if ps > pk:  # left shock
            speed = uk - ck * np.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pk
                                      + (gamma - 1.0) / (2.0 * gamma))
            if s < speed:
                return rk, uk, pk
            return rk * (ps / pk + g1) / (g1 * ps / pk + 1.0), us, ps
        # left rarefaction
        cs = ck * (ps / pk) ** ((gamma - 1.0) / (2.0 * gamma))
        head, tail = uk - ck, us - cs
        if s < head:
            return rk, uk, pk
        if s > tail:
            return rk * (ps / pk) ** (1.0 / gamma), us, ps
        u = 2.0 / (gamma + 1.0) * (ck + 0.5 * (gamma - 1.0) * uk + s)
        c = 2.0 / (gamma + 1.0) * (ck + 0.5 * (gamma - 1.0) * (uk - s))
        return rk * (c / ck) ** (2.0 / (gamma - 1.0)), u, pk * (c / ck) ** (2.0 * gamma / (gamma - 1.0))
    rk, uk, pk = right
    ck = np.sqrt(gamma * pk / rk)
    if ps > pk:  # right shock
        speed = uk + ck * np.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pk
                                  + (gamma - 1.0) / (2.0 * gamma))
        if s > speed:
            return rk, uk, pk
        return rk * (ps / pk + g1) / (g1 * ps / pk + 1.0), us, ps
    cs = ck * (ps / pk) ** ((gamma - 1.0) / (2.0 * gamma))
    head, tail = uk + ck, us + cs
    if s > head:
        return rk, uk, pk
    if s < tail:
        return rk * (ps / pk) ** (1.0 / gamma), us, ps
    u = 2.0 / (gamma + 1.0) * (-ck + 0.5 * (gamma - 1.0) * uk + s)
    c = 2.0 / (gamma + 1.0) * (ck - 0.5 * (gamma - 1.0) * (uk - s))
    return rk * (c / ck) ** (2.0 / (gamma - 1.0)), u, pk * (c / ck) ** (2.0 * gamma / (gamma - 1.0))


def solution(left, right, gamma, x, x0, t):
    """Arrays rho, u, p of the exact solution at positions x and time t > 0."""
    out = np.array([sample(left, right, gamma, (xx - x0) / t) for xx in np.asarray(x)])
    return out[:, 0], out[:, 1], out[:, 2]
