"""Exact solution of the Riemann problem for one stiffened gas -- TEST ONLY.

Follows the textbook construction of Toro (1997), the paper's reference for
its Riemann solvers (Sec. 3.2.2): solve f_L(p*) + f_R(p*) + (u_R - u_L) = 0
for the star pressure by Newton's method, then sample the self-similar
solution at x/t.  A stiffened gas with parameters (gamma, pi_inf) behaves as
an ideal gas in the shifted pressure p + pi_inf, so the ideal-gas formulas are
applied to p + pi_inf throughout.
"""
from __future__ import annotations

import math

import numpy as np


def _pressure_function(p, rho_k, p_k, c_k, g):
    """f_K(p) and its derivative (shifted pressures)."""
    if p > p_k:  # shock
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        f = (p - p_k) * s
        df = s * (1.0 - 0.5 * (p - p_k) / (B + p))
    else:  # rarefaction
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * c_k / (g - 1.0) * ((p / p_k) ** e - 1.0)
        df = 1.0 / (rho_k * c_k) * (p / p_k) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, gamma=1.4, pi_inf=0.0, tol=1e-14, maxit=200):
    """Return (p*, u*) for primitive states left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    plt, prt = pl + pi_inf, pr + pi_inf
    cl = math.sqrt(g * plt / rl)
    cr = math.sqrt(g * prt / rr)
    du = ur - ul
    if 2.0 * (cl + cr) / (g - 1.0) <= du:
        raise ValueError("vacuum is generated")
    # two-rarefaction initial guess (Toro eq. 4.46), shifted pressure
    e = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * du) / (cl / plt ** e + cr / prt ** e)) ** (1.0 / e)
    p = max(p, 1e-12 * min(plt, prt))
    for _ in range(maxit):
        fl, dfl = _pressure_function(p, rl, plt, cl, g)
        fr, dfr = _pressure_function(p, rr, prt, cr, g)
        pn = p - (fl + fr + du) / (dfl + dfr)
        if pn <= 0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _pressure_function(p, rl, plt, cl, g)
    fr, _ = _pressure_function(p, rr, prt, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p - pi_inf, u


def sample(left, right, xi, gamma=1.4, pi_inf=0.0):
    """Sample (rho, u, p) of the exact solution at xi = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    ps, us = star_state(left, right, gamma, pi_inf)
    plt, prt, pst = pl + pi_inf, pr + pi_inf, ps + pi_inf
    cl = math.sqrt(g * plt / rl)
    cr = math.sqrt(g * prt / rr)
    gm = (g - 1.0) / (g + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if pst > plt:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * pst / plt + (g - 1) / (2 * g))
                if s < sl:
                    w = (rl, ul, plt)
                else:
                    w = (rl * (pst / plt + gm) / (gm * pst / plt + 1.0), us, pst)
            else:  # left rarefaction
                shl = ul - cl
                cml = cl * (pst / plt) ** ((g - 1) / (2 * g))
                stl = us - cml
                if s < shl:
                    w = (rl, ul, plt)
                elif s > stl:
                    w = (rl * (pst / plt) ** (1.0 / g), us, pst)
                else:
                    b = 2.0 / (g + 1) + (g - 1) / ((g + 1) * cl) * (ul - s)
                    w = (rl * b ** (2.0 / (g - 1)), 2.0 / (g + 1) * (cl + 0.5 * (g - 1) * ul + s),
                         plt * b ** (2.0 * g / (g - 1)))
        else:  # right of the contact
            if pst > prt:  # right shock
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * pst / prt + (g - 1) / (2 * g))
                if s > sr:
                    w = (rr, ur, prt)
                else:
                    w = (rr * (pst / prt + gm) / (gm * pst / prt + 1.0), us, pst)
            else:  # right rarefaction
                shr = ur + cr
                cmr = cr * (pst / prt) ** ((g - 1) / (2 * g))
                str_ = us + cmr
                if s > shr:
                    w = (rr, ur, prt)
                elif s < str_:
                    w = (rr * (pst / prt) ** (1.0 / g), us, pst)
                else:
                    b = 2.0 / (g + 1) - (g - 1) / ((g + 1) * cr) * (ur - s)
                    w = (rr * b ** (2.0 / (g - 1)), 2.0 / (g + 1) * (-cr + 0.5 * (g - 1) * ur + s),
                         prt * b ** (2.0 * g / (g - 1)))
        rho[n], u[n], p[n] = w[0], w[1], w[2] - pi_inf
    return rho, u, p


def wave_speeds(left, right, gamma=1.4, pi_inf=0.0):
    """Head/tail/contact/shock speeds for a left rarefaction + right shock."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    ps, us = star_state(left, right, gamma, pi_inf)
    plt, prt, pst = pl + pi_inf, pr + pi_inf, ps + pi_inf
    cl = math.sqrt(g * plt / rl)
    cr = math.sqrt(g * prt / rr)
    head = ul - cl
    tail = us - cl * (pst / plt) ** ((g - 1) / (2 * g))
    shock = ur + cr * math.sqrt((g + 1) / (2 * g) * pst / prt + (g - 1) / (2 * g))
    return dict(head=head, tail=tail, contact=us, shock=shock)
