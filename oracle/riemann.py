"""TEST INFRASTRUCTURE ONLY -- exact solution of the Riemann problem of an ideal
polytropic gas, used to pin the ideal-gas limit (a = b = 0) of the scheme.

Ideal gas: p = rho R T and e = C_v T with C_v = R/delta, so the ratio of specific
heats is gamma = 1 + delta (Reyhanian et al., arXiv:2002.09217, main text: the
ideal gas is the special limit of the van der Waals fluid).

The solver is the textbook one (two nonlinear waves separated by a contact;
the star pressure is the root of f_L(p) + f_R(p) + u_R - u_L = 0 with the shock
branch from the Rankine-Hugoniot relations and the rarefaction branch from the
isentropic Riemann invariants), written out here from those relations.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _fK(p, rK, pK, cK, g):
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rK)
        B = (g - 1.0) / (g + 1.0) * pK
        return (p - pK) * math.sqrt(A / (p + B))
    return 2.0 * cK / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)  # rarefaction


def star_state(left, right, gamma):
    rL, uL, pL = left
    rR, uR, pR = right
    cL, cR = math.sqrt(gamma * pL / rL), math.sqrt(gamma * pR / rR)
    f = lambda p: _fK(p, rL, pL, cL, gamma) + _fK(p, rR, pR, cR, gamma) + uR - uL
    hi = max(pL, pR)
    while f(hi) < 0.0:
        hi *= 2.0
    ps = brentq(f, 1e-14 * min(pL, pR), hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (uL + uR) + 0.5 * (_fK(ps, rR, pR, cR, gamma) - _fK(ps, rL, pL, cL, gamma))
    return ps, us


def sample(left, right, gamma, xi):
    """(rho, u, p) of the self-similar solution at xi = (x - x_interface)/t."""
    g = gamma
    rL, uL, pL = left
    rR, uR, pR = right
    cL, cR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    ps, us = star_state(left, right, gamma)
    gm = (g - 1.0) / (g + 1.0)
    out = np.zeros((len(xi), 3))
    for n, S in enumerate(np.atleast_1d(xi)):
        if S <= us:
            if ps > pL:
                SL = uL - cL * math.sqrt((g + 1.0) / (2.0 * g) * ps / pL + (g - 1.0) / (2.0 * g))
                if S <= SL:
                    out[n] = (rL, uL, pL)
                else:
                    out[n] = (rL * (ps / pL + gm) / (gm * ps / pL + 1.0), us, ps)
            else:
                SHL = uL - cL
                csL = cL * (ps / pL) ** ((g - 1.0) / (2.0 * g))
                STL = us - csL
                if S <= SHL:
                    out[n] = (rL, uL, pL)
                elif S > STL:
                    out[n] = (rL * (ps / pL) ** (1.0 / g), us, ps)
                else:
                    br = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cL) * (uL - S)
                    out[n] = (rL * br ** (2.0 / (g - 1.0)),
                              2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * uL + S),
                              pL * br ** (2.0 * g / (g - 1.0)))
        else:
            if ps > pR:
                SR = uR + cR * math.sqrt((g + 1.0) / (2.0 * g) * ps / pR + (g - 1.0) / (2.0 * g))
                if S >= SR:
                    out[n] = (rR, uR, pR)
                else:
                    out[n] = (rR * (ps / pR + gm) / (gm * ps / pR + 1.0), us, ps)
            else:
                SHR = uR + cR
                csR = cR * (ps / pR) ** ((g - 1.0) / (2.0 * g))
                STR = us + csR
                if S >= SHR:
                    out[n] = (rR, uR, pR)
                elif S <= STR:
                    out[n] = (rR * (ps / pR) ** (1.0 / g), us, ps)
                else:
                    br = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cR) * (uR - S)
                    out[n] = (rR * br ** (2.0 / (g - 1.0)),
                              2.0 / (g + 1.0) * (-cR + 0.5 * (g - 1.0) * uR + S),
                              pR * br ** (2.0 * g / (g - 1.0)))
    return out
