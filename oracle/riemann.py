"""Exact solution of the Riemann problem of the 1-D Euler equations (ideal gas).

The reference of the classical Riemann tests of Sec. 2.2 (Table 9), which the
paper compares against exact solutions.  Written from the mathematics of the
problem: across the two non-linear waves the star pressure p* satisfies
f_L(p*) + f_R(p*) + (u_R - u_L) = 0, where for side K

  shock (p > p_K):        f_K(p) = (p - p_K) sqrt(A_K / (p + B_K)),
                          A_K = 2 / ((gamma+1) rho_K),  B_K = (gamma-1)/(gamma+1) p_K
  rarefaction (p <= p_K): f_K(p) = 2 c_K / (gamma-1) ((p / p_K)^((gamma-1)/(2 gamma)) - 1)

(Rankine-Hugoniot conditions across a shock, Riemann invariants across a
rarefaction); u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.  The solution is
self-similar in x/t; it is sampled wave by wave.  Test infrastructure only.
"""

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * np.sqrt(A / (p + B)), (1.0 - 0.5 * (p - pk) / (B + p)) * np.sqrt(A / (B + p))
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rho * ck)


def star_state(left, right, gamma=1.4, tol=1e-15):
    """(p*, u*) of the Riemann problem with primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
    if 2.0 * (cl + cr) / (gamma - 1.0) <= ur - ul:
        raise ValueError("the data create vacuum")
    p = max(tol, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, gamma)
        fr, dr = _f(p, rr, pr, cr, gamma)
        p_new = max(tol, p - (fl + fr + ur - ul) / (dl + dr))
        if abs(p_new - p) <= 1e-15 * max(p_new, p):
            p = p_new
            break
        p = p_new
    fl, _ = _f(p, rl, pl, cl, gamma)
    fr, _ = _f(p, rr, pr, cr, gamma)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, s, gamma=1.4):
    """Primitive state (rho, u, p) at the self-similar coordinate s = (x - x_c) / t."""
    g = gamma
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    if s <= us:                                         # left of the contact
        if ps > pl:                                     # left shock
            sl = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if s <= sl:
                return rl, ul, pl
            r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
            return r, us, ps
        cs = cl * (ps / pl) ** ((g - 1) / (2 * g))     # left rarefaction
        if s <= ul - cl:
            return rl, ul, pl
        if s >= us - cs:
            return rl * (ps / pl) ** (1 / g), us, ps
        u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
        c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
        return rl * (c / cl) ** (2 / (g - 1)), u, pl * (c / cl) ** (2 * g / (g - 1))
    if ps > pr:                                         # right shock
        sr = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if s >= sr:
            return rr, ur, pr
        r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
        return r, us, ps
    cs = cr * (ps / pr) ** ((g - 1) / (2 * g))         # right rarefaction
    if s >= ur + cr:
        return rr, ur, pr
    if s <= us + cs:
        return rr * (ps / pr) ** (1 / g), us, ps
    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
    return rr * (c / cr) ** (2 / (g - 1)), u, pr * (c / cr) ** (2 * g / (g - 1))


def density(left, right, x, t, xc=0.5, gamma=1.4):
    """Exact density at the points x (array) and time t > 0."""
    return np.array([sample(left, right, (xi - xc) / t, gamma)[0] for xi in np.ravel(x)]).reshape(np.shape(x))
