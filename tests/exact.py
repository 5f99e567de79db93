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
