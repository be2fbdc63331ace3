"""Exact solution of the 1D Riemann problem between two stiffened gases
(or a stiffened gas and a Tait liquid).

Independent check of the oracle: Toro's exact solver (Riemann Solvers and
Numerical Methods for Fluid Dynamics, ch. 4) with each side's pressure
shifted by its own p_inf, which is exact for the stiffened-gas EOS
p = (gamma - 1) rho e - gamma p_inf.  Each side keeps its own (gamma, p_inf),
so the contact separates two materials, as at the interfaces of the
multi-material shock tube (Sec. 3, Case I).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


class Side:
    def __init__(self, rho, u, p, gamma, pinf=0.0):
        self.rho, self.u, self.p, self.g, self.pinf = rho, u, p, gamma, pinf
        self.c = math.sqrt(gamma * (p + pinf) / rho)

    def f(self, ps):
        """Velocity jump across the left/right wave for star pressure ps."""
        g, pb, psb = self.g, self.p + self.pinf, ps + self.pinf
        if ps > self.p:  # shock
            A = 2.0 / ((g + 1.0) * self.rho)
            B = (g - 1.0) / (g + 1.0) * pb
            return (ps - self.p) * math.sqrt(A / (psb + B))
        return 2.0 * self.c / (g - 1.0) * ((psb / pb) ** ((g - 1.0) / (2.0 * g)) - 1.0)


class TaitSide:
    """A barotropic Tait liquid, p = B (rho/rho0)^gamma - B + p0: across a
    shock only mass and momentum jump conditions apply, (u_* - u)^2 =
    (p_* - p)(1/rho - 1/rho_*); a rarefaction keeps u -+ 2c/(gamma-1)
    constant, with c^2 = dp/drho = gamma (p + B - p0)/rho proportional to
    rho^(gamma-1)."""

    def __init__(self, rho, u, p_unused, gamma, B, rho0, p0):
        self.g, self.B, self.rho0, self.p0 = gamma, B, rho0, p0
        self.rho, self.u = rho, u
        self.p = self.pressure(rho)
        self.pinf = B - p0
        self.c = self.sound(rho)

    def pressure(self, rho):
        return self.B * (rho / self.rho0) ** self.g - self.B + self.p0

    def density(self, p):
        return self.rho0 * ((p - self.p0 + self.B) / self.B) ** (1.0 / self.g)

    def sound(self, rho):
        return math.sqrt(self.g * self.B / self.rho0 * (rho / self.rho0) ** (self.g - 1.0))

    def f(self, ps):
        rs = self.density(ps)
        if ps > self.p:
            return math.sqrt((ps - self.p) * (1.0 / self.rho - 1.0 / rs))
        return 2.0 / (self.g - 1.0) * (self.sound(rs) - self.c)

    def edges(self, ps, us, sgn):
        rs = self.density(ps)
        if ps > self.p:
            m = math.sqrt((ps - self.p) / (1.0 / self.rho - 1.0 / rs))
            sh = self.u + sgn * m / self.rho
            return sh, sh
        return self.u + sgn * self.c, us + sgn * self.sound(rs)

    def state(self, s, ps, us, sgn):
        head, tail = self.edges(ps, us, sgn)
        if (s - head) * sgn >= 0.0:
            return self.rho, self.u, self.p
        if ps > self.p or (s - tail) * sgn <= 0.0:
            rs = self.density(ps)
            return rs, us, ps
        g = self.g
        if sgn > 0:
            c = (g - 1.0) / (g + 1.0) * (s - self.u) + 2.0 * self.c / (g + 1.0)
            uu = s - c
        else:
            c = (g - 1.0) / (g + 1.0) * (self.u - s) + 2.0 * self.c / (g + 1.0)
            uu = s + c
        c0 = math.sqrt(g * self.B / self.rho0)
        rr = self.rho0 * (c / c0) ** (2.0 / (g - 1.0))
        return rr, uu, self.pressure(rr)


def star_state(L: Side, R: Side):
    """Star pressure and contact velocity."""
    fn = lambda p: L.f(p) + R.f(p) + (R.u - L.u)
    lo = -min(L.pinf, R.pinf) + 1e-14 * (1.0 + max(L.p, R.p))
    hi = max(L.p, R.p) * 10.0 + 1.0
    while fn(hi) < 0.0:
        hi *= 10.0
    ps = brentq(fn, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (L.u + R.u) + 0.5 * (R.f(ps) - L.f(ps))
    return ps, us


def wave_speeds(L: Side, R: Side):
    """Speeds of the left wave (head, tail), contact, right wave (tail,
    head).  For a shock head == tail == shock speed."""
    ps, us = star_state(L, R)
    out = {}
    for S, sgn, key in ((L, -1.0, "left"), (R, 1.0, "right")):
        if hasattr(S, "edges"):
            a, b = S.edges(ps, us, sgn)
            out[key] = (a, b)
            continue
        g, pb, psb = S.g, S.p + S.pinf, ps + S.pinf
        if ps > S.p:
            sh = S.u + sgn * S.c * math.sqrt((g + 1.0) / (2.0 * g) * psb / pb
                                             + (g - 1.0) / (2.0 * g))
            out[key] = (sh, sh)
        else:
            cs = S.c * (psb / pb) ** ((g - 1.0) / (2.0 * g))
            out[key] = (S.u + sgn * S.c, us + sgn * cs)
    return ps, us, out


def sample(L: Side, R: Side, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t."""
    ps, us = star_state(L, R)
    xi = np.asarray(xi, dtype=float)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi.ravel()):
        if s <= us:
            S, sgn = L, -1.0
        else:
            S, sgn = R, 1.0
        if hasattr(S, "state"):
            rho.flat[n], u.flat[n], p.flat[n] = S.state(s, ps, us, sgn)
            continue
        g, pinf, pb, psb = S.g, S.pinf, S.p + S.pinf, ps + S.pinf
        if ps > S.p:  # shock
            sh = S.u + sgn * S.c * math.sqrt((g + 1.0) / (2.0 * g) * psb / pb
                                             + (g - 1.0) / (2.0 * g))
            behind = (s - sh) * sgn < 0.0
            if behind:
                q = psb / pb
                gg = (g - 1.0) / (g + 1.0)
                r = S.rho * (q + gg) / (gg * q + 1.0)
                val = (r, us, ps)
            else:
                val = (S.rho, S.u, S.p)
        else:  # rarefaction
            head = S.u + sgn * S.c
            cs = S.c * (psb / pb) ** ((g - 1.0) / (2.0 * g))
            tail = us + sgn * cs
            if (s - head) * sgn >= 0.0:
                val = (S.rho, S.u, S.p)
            elif (s - tail) * sgn <= 0.0:
                val = (S.rho * (psb / pb) ** (1.0 / g), us, ps)
            else:
                # inside the fan: Riemann invariant and isentrope
                if sgn > 0:
                    uu = 2.0 / (g + 1.0) * (-S.c + (g - 1.0) / 2.0 * S.u + s)
                    cc = 2.0 / (g + 1.0) * (S.c - (g - 1.0) / 2.0 * (S.u - s))
                else:
                    uu = 2.0 / (g + 1.0) * (S.c + (g - 1.0) / 2.0 * S.u + s)
                    cc = 2.0 / (g + 1.0) * (S.c + (g - 1.0) / 2.0 * (S.u - s))
                rr = S.rho * (cc / S.c) ** (2.0 / (g - 1.0))
                pp = (pb) * (cc / S.c) ** (2.0 * g / (g - 1.0)) - pinf
                val = (rr, uu, pp)
        rho.flat[n], u.flat[n], p.flat[n] = val
    return rho, u, p
