"""Exact solutions used to pin the oracle (test infrastructure only).

* Burgers (Examples 3.1, 3.2): characteristics, u = u0(x - u t), solved by
  Newton iteration before the breaking time.
* Euler with gamma = 3 (Examples 3.3, 3.4; the cited exact solution exists for
  this gamma): with p = rho^3 the sound speed is c = sqrt(3) rho, the
  initial velocity makes the Riemann invariant mu - c vanish, so the flow is a
  simple wave and w = mu + c = 2 sqrt(3) rho obeys w_t + w w_x = 0.  In 2D the
  same holds along s = (x + y)/sqrt(2).
* The exact Riemann solver for the Euler equations (two-shock/two-rarefaction
  pressure iteration from the textbook literature), for the Lax problem.
"""
from __future__ import annotations

import math

import numpy as np


def burgers_char(u0, x, t, speed: float = 1.0, iters: int = 60):
    """Solve u = u0(x - speed*u*t) by Newton; u0 must be vectorised and
    supply its derivative as u0.d."""
    u = u0(x)
    for _ in range(iters):
        g = u - u0(x - speed * u * t)
        dg = 1.0 + u0.d(x - speed * u * t) * speed * t
        u = u - g / dg
    return u


class _Fn:
    def __init__(self, f, d):
        self.f, self.d = f, d

    def __call__(self, x):
        return self.f(x)


def burgers1d_example(x, t):
    """Example 3.1: u0 = 0.5 + sin(pi x)."""
    u0 = _Fn(lambda s: 0.5 + np.sin(np.pi * s), lambda s: np.pi * np.cos(np.pi * s))
    return burgers_char(u0, x, t)


def burgers2d_example(x, y, t):
    """Example 3.2: u0 = 0.5 + sin(pi (x+y)/2); u = U(x+y, t), U_t + 2 U U_s = 0."""
    u0 = _Fn(lambda s: 0.5 + np.sin(np.pi * s / 2.0), lambda s: 0.5 * np.pi * np.cos(np.pi * s / 2.0))
    return burgers_char(u0, x + y, t, speed=2.0)


def euler1d_gamma3(x, t):
    """Example 3.3 with gamma = 3: returns (rho, mu, p)."""
    w0 = _Fn(lambda s: 1.0 + 0.2 * np.sin(s), lambda s: 0.2 * np.cos(s))
    w = burgers_char(w0, x, t)
    rho = w / (2.0 * math.sqrt(3.0))
    return rho, w / 2.0, rho ** 3


def euler2d_gamma3(x, y, t):
    """Example 3.4 with gamma = 3: returns (rho, mu, nu, p)."""
    s = (x + y) / math.sqrt(2.0)
    w0 = _Fn(lambda q: math.sqrt(2.0) * (1.0 + 0.2 * np.sin(q / math.sqrt(2.0))),
             lambda q: 0.2 * np.cos(q / math.sqrt(2.0)))
    w = burgers_char(w0, s, t)
    rho = w / (2.0 * math.sqrt(3.0))
    un = w / 2.0
    return rho, un / math.sqrt(2.0), un / math.sqrt(2.0), rho ** 3


# --------------------------------------------------------------------------
# Exact Riemann solver (ideal gas)
# --------------------------------------------------------------------------
def _fk(p, rk, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rk)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - (p - pk) / (2.0 * (B + p)))
    else:       # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rk * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def riemann_star(left, right, g):
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-12)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(left, right, g, xi):
    """(rho, u, p) of the self-similar solution at xi = x/t (vectorised)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = riemann_star(left, right, g)
    xi = np.asarray(xi, dtype=float)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for k, s in np.ndenumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:
                sh = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sh:
                    r, v, q = rl, ul, pl
                else:
                    r = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                    v, q = us, ps
            else:
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                if s <= ul - cl:
                    r, v, q = rl, ul, pl
                elif s >= us - csl:
                    r, v, q = rl * (ps / pl) ** (1 / g), us, ps
                else:
                    v = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2 / (g - 1))
                    q = pl * (c / cl) ** (2 * g / (g - 1))
        else:
            if ps > pr:
                sh = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sh:
                    r, v, q = rr, ur, pr
                else:
                    r = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
                    v, q = us, ps
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                if s >= ur + cr:
                    r, v, q = rr, ur, pr
                elif s <= us + csr:
                    r, v, q = rr * (ps / pr) ** (1 / g), us, ps
                else:
                    v = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2 / (g - 1))
                    q = pr * (c / cr) ** (2 * g / (g - 1))
        rho[k], u[k], p[k] = r, v, q
    return rho, u, p
