"""Analytic reference solutions used to pin the oracle (test-only).

* Exact solution of the 1D Riemann problem for the ideal-gas Euler equations
  (Toro 2009, ch. 4: pressure function, Newton iteration for p*, sampling of
  the self-similar solution).
* Sedov-Taylor blast wave radius R(t) = xi0 (E t^2 / rho0)^(1/5) (Taylor 1950;
  Sedov 1959) with the dimensionless constant supplied by the caller.
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, cK, g):
    """Toro's pressure function f_K and its derivative (Sec. 4.2)."""
    if p > pK:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        return (p - pK) * s, s * (1.0 - 0.5 * (p - pK) / (B + p))
    e = (g - 1.0) / (2.0 * g)
    f = 2.0 * cK / (g - 1.0) * ((p / pK) ** e - 1.0)
    df = 1.0 / (rho * cK) * (p / pK) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def riemann_star(rhoL, uL, pL, rhoR, uR, pR, g):
    """Star-region pressure and velocity by Newton iteration (Toro Sec. 4.3)."""
    cL = math.sqrt(g * pL / rhoL)
    cR = math.sqrt(g * pR / rhoR)
    p = max(1e-12, 0.5 * (pL + pR) - 0.125 * (uR - uL) * (rhoL + rhoR) * (cL + cR))
    for _ in range(100):
        fL, dL = _fK(p, rhoL, pL, cL, g)
        fR, dR = _fK(p, rhoR, pR, cR, g)
        pn = p - (fL + fR + (uR - uL)) / (dL + dR)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rhoL, pL, cL, g)
    fR, _ = _fK(p, rhoR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def riemann_sample(rhoL, uL, pL, rhoR, uR, pR, g, xi):
    """(rho, u, p) of the exact solution at similarity coordinates xi = x/t.

    Also returns a dict of the wave structure."""
    cL = math.sqrt(g * pL / rhoL)
    cR = math.sqrt(g * pR / rhoR)
    ps, us = riemann_star(rhoL, uL, pL, rhoR, uR, pR, g)
    gm = (g - 1.0) / (g + 1.0)
    info = {"p_star": ps, "u_star": us}
    # left wave
    if ps > pL:
        rsL = rhoL * ((ps / pL + gm) / (gm * ps / pL + 1.0))
        SL = uL - cL * math.sqrt((g + 1.0) / (2.0 * g) * ps / pL + (g - 1.0) / (2.0 * g))
        info.update(rho_starL=rsL, left_shock=SL)
    else:
        rsL = rhoL * (ps / pL) ** (1.0 / g)
        csL = cL * (ps / pL) ** ((g - 1.0) / (2.0 * g))
        info.update(rho_starL=rsL, rare_head=uL - cL, rare_tail=us - csL)
    if ps > pR:
        rsR = rhoR * ((ps / pR + gm) / (gm * ps / pR + 1.0))
        SR = uR + cR * math.sqrt((g + 1.0) / (2.0 * g) * ps / pR + (g - 1.0) / (2.0 * g))
        info.update(rho_starR=rsR, right_shock=SR)
    else:
        rsR = rhoR * (ps / pR) ** (1.0 / g)
        info.update(rho_starR=rsR, right_head=uR + cR,
                    right_tail=us + cR * (ps / pR) ** ((g - 1.0) / (2.0 * g)))
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi.flat):
        if s <= us:   # left of contact
            if ps > pL:
                r, v, q = (rhoL, uL, pL) if s <= info["left_shock"] else (rsL, us, ps)
            else:
                if s <= info["rare_head"]:
                    r, v, q = rhoL, uL, pL
                elif s >= info["rare_tail"]:
                    r, v, q = rsL, us, ps
                else:   # inside the left fan (Toro eq. 4.56)
                    f = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cL) * (uL - s)
                    r = rhoL * f ** (2.0 / (g - 1.0))
                    v = 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * uL + s)
                    q = pL * f ** (2.0 * g / (g - 1.0))
        else:
            if ps > pR:
                r, v, q = (rhoR, uR, pR) if s >= info["right_shock"] else (rsR, us, ps)
            else:
                if s >= info["right_head"]:
                    r, v, q = rhoR, uR, pR
                elif s <= info["right_tail"]:
                    r, v, q = rsR, us, ps
                else:
                    f = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cR) * (uR - s)
                    r = rhoR * f ** (2.0 / (g - 1.0))
                    v = 2.0 / (g + 1.0) * (-cR + (g - 1.0) / 2.0 * uR + s)
                    q = pR * f ** (2.0 * g / (g - 1.0))
        rho.flat[n], u.flat[n], p.flat[n] = r, v, q
    return rho, u, p, info


def sedov_radius(E, t, rho0, xi0):
    return xi0 * (E * t * t / rho0) ** 0.2
