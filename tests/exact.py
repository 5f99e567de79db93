"""Closed-form and exact solutions used to pin the oracle (test side only).

These are textbook results written independently of the oracle:

* the exact Riemann solution of the 1D shallow-water equations (two
  rarefaction/shock branches joined at the middle state found by a root solve);
* Rankine-Hugoniot shock speeds (from the conserved jumps).
"""

from __future__ import annotations

import math

import numpy as np


def _phi(h, hk, g):
    """Velocity change across a wave connecting depth hk to depth h."""
    if h <= hk:
        return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hk))
    return (h - hk) * math.sqrt(0.5 * g * (h + hk) / (h * hk))


def sw_middle_state(hl, ul, hr, ur, g=1.0):
    """Middle state (h_m, u_m) of the shallow-water Riemann problem (bisection)."""
    f = lambda h: _phi(h, hl, g) + _phi(h, hr, g) + ur - ul
    lo, hi = 1e-12, max(hl, hr) * 10.0 + (ul - ur) ** 2 / g
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    hm = 0.5 * (lo + hi)
    um = ul - _phi(hm, hl, g)
    return hm, um


def sw_exact(hl, ul, hr, ur, xi, g=1.0):
    """Exact (h, u) at similarity coordinate xi = x/t (array)."""
    hm, um = sw_middle_state(hl, ul, hr, ur, g)
    cl, cr, cm = math.sqrt(g * hl), math.sqrt(g * hr), math.sqrt(g * hm)
    xi = np.asarray(xi, float)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    # left wave
    if hm > hl:   # 1-shock
        s1 = (hm * um - hl * ul) / (hm - hl)
        left = xi < s1
        h[left], u[left] = hl, ul
        mid_l = ~left
    else:         # 1-rarefaction
        head, tail = ul - cl, um - cm
        left = xi < head
        fan = (xi >= head) & (xi < tail)
        h[left], u[left] = hl, ul
        c = (ul + 2.0 * cl - xi[fan]) / 3.0
        h[fan], u[fan] = c * c / g, xi[fan] + c
        mid_l = xi >= tail
    # right wave
    if hm > hr:   # 2-shock
        s2 = (hm * um - hr * ur) / (hm - hr)
        right = xi > s2
        mid_r = ~right
        h[right], u[right] = hr, ur
    else:         # 2-rarefaction
        head, tail = ur + cr, um + cm
        right = xi > head
        fan = (xi <= head) & (xi > tail)
        h[right], u[right] = hr, ur
        c = (xi[fan] - ur + 2.0 * cr) / 3.0
        h[fan], u[fan] = c * c / g, xi[fan] - c
        mid_r = xi <= tail
    mid = mid_l & mid_r
    h[mid], u[mid] = hm, um
    return h, u


# ---------------------------------------------------------------------------
# Exact Riemann solution of the 1D Euler equations for an ideal gas (Toro,
# "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4): the star
# pressure from f_L(p) + f_R(p) + (u_R - u_L) = 0 (bisection), then sampling
# of the self-similar solution at xi = x / t.
# ---------------------------------------------------------------------------
def _euler_f(p, rho, pk, gam):
    c = math.sqrt(gam * pk / rho)
    if p > pk:   # shock
        A = 2.0 / ((gam + 1.0) * rho)
        B = (gam - 1.0) / (gam + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gam - 1.0) * ((p / pk) ** ((gam - 1.0) / (2.0 * gam)) - 1.0)


def euler_star(rl, ul, pl, rr, ur, pr, gam=1.4):
    """Star-region pressure and velocity."""
    g = lambda p: _euler_f(p, rl, pl, gam) + _euler_f(p, rr, pr, gam) + ur - ul
    lo, hi = 1e-12, 10.0 * max(pl, pr) + 10.0
    while g(hi) < 0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (_euler_f(ps, rr, pr, gam) - _euler_f(ps, rl, pl, gam))
    return ps, us


def euler_exact(rl, ul, pl, rr, ur, pr, xi, gam=1.4):
    """(rho, u, p) of the exact solution at xi = x/t (array)."""
    ps, us = euler_star(rl, ul, pl, rr, ur, pr, gam)
    gm, gp = gam - 1.0, gam + 1.0
    cl, cr = math.sqrt(gam * pl / rl), math.sqrt(gam * pr / rr)
    out = np.zeros((3, len(xi)))
    for n, x in enumerate(np.asarray(xi, float)):
        if x <= us:   # left of the contact
            if ps > pl:   # left shock
                rs = rl * ((ps / pl + gm / gp) / (gm / gp * ps / pl + 1.0))
                S = ul - cl * math.sqrt(gp / (2 * gam) * ps / pl + gm / (2 * gam))
                out[:, n] = (rl, ul, pl) if x < S else (rs, us, ps)
            else:         # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / gam)
                cs = cl * (ps / pl) ** (gm / (2 * gam))
                if x < ul - cl:
                    out[:, n] = (rl, ul, pl)
                elif x > us - cs:
                    out[:, n] = (rs, us, ps)
                else:
                    u = 2.0 / gp * (cl + gm / 2.0 * ul + x)
                    c = 2.0 / gp * (cl + gm / 2.0 * (ul - x))
                    r = rl * (c / cl) ** (2.0 / gm)
                    out[:, n] = (r, u, pl * (c / cl) ** (2.0 * gam / gm))
        else:
            if ps > pr:   # right shock
                rs = rr * ((ps / pr + gm / gp) / (gm / gp * ps / pr + 1.0))
                S = ur + cr * math.sqrt(gp / (2 * gam) * ps / pr + gm / (2 * gam))
                out[:, n] = (rr, ur, pr) if x > S else (rs, us, ps)
            else:         # right rarefaction
                rs = rr * (ps / pr) ** (1.0 / gam)
                cs = cr * (ps / pr) ** (gm / (2 * gam))
                if x > ur + cr:
                    out[:, n] = (rr, ur, pr)
                elif x < us + cs:
                    out[:, n] = (rs, us, ps)
                else:
                    u = 2.0 / gp * (-cr + gm / 2.0 * ur + x)
                    c = 2.0 / gp * (cr - gm / 2.0 * (ur - x))
                    r = rr * (c / cr) ** (2.0 / gm)
                    out[:, n] = (r, u, pr * (c / cr) ** (2.0 * gam / gm))
    return out
