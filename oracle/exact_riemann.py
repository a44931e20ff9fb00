"""Exact solution of the Riemann problem of the 1-D Euler equations.

TEST INFRASTRUCTURE ONLY (part of the oracle).

For a one-dimensional flow of a collisionless fluid the moment equations reduce
to the classical 1-D hydrodynamic equations with rho sigma_xx^2 playing the
pressure and gamma = 3 (Sec. 4 of the paper, eqs. (33)-(38)); the paper obtains
its Sod reference from the standard solution procedure (Sod 1978).  This
module implements that procedure for any gamma, written from the textbook
mathematics (the two-shock/two-rarefaction pressure function of the star
region, root-finding for p*, then sampling of the self-similar solution in
xi = (x - x0) / t; e.g. Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4).

The transverse stress of the moment equations is carried along: for a 1-D
flow in x with v = Pxy = 0 the Pyy equation reduces to D(Pyy/rho)/Dt = 0, so
Pyy/rho is constant on particle paths and jumps only at the contact.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.optimize import brentq


@dataclass
class State:
    rho: float
    u: float
    p: float


def _f_and_speed(p: float, s: State, g: float) -> float:
    """Velocity change across the left or right wave as a function of p*."""
    a = math.sqrt(g * s.p / s.rho)
    if p > s.p:  # shock
        A = 2.0 / ((g + 1.0) * s.rho)
        B = (g - 1.0) / (g + 1.0) * s.p
        return (p - s.p) * math.sqrt(A / (p + B))
    # rarefaction
    return 2.0 * a / (g - 1.0) * ((p / s.p) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(L: State, R: State, g: float):
    """(p*, u*) of the star region."""
    du = R.u - L.u
    aL = math.sqrt(g * L.p / L.rho)
    aR = math.sqrt(g * R.p / R.rho)
    if 2.0 * (aL + aR) / (g - 1.0) <= du:
        raise ValueError("vacuum is generated")

    def phi(p):
        return _f_and_speed(p, L, g) + _f_and_speed(p, R, g) + du

    lo, hi = 1e-14, max(L.p, R.p)
    while phi(hi) < 0.0:
        hi *= 2.0
    p = brentq(phi, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    u = 0.5 * (L.u + R.u) + 0.5 * (_f_and_speed(p, R, g) - _f_and_speed(p, L, g))
    return p, u


def star_densities(L: State, R: State, g: float):
    p, u = star_state(L, R, g)
    gm = (g - 1.0) / (g + 1.0)

    def rho_star(s: State):
        if p > s.p:
            r = p / s.p
            return s.rho * (r + gm) / (gm * r + 1.0)
        return s.rho * (p / s.p) ** (1.0 / g)

    return rho_star(L), rho_star(R)


def wave_speeds(L: State, R: State, g: float) -> dict:
    """Speeds of the wave edges: left head/tail (or shock), contact, right."""
    p, u = star_state(L, R, g)
    out = {"contact": u}
    for side, s, sign in (("left", L, -1.0), ("right", R, 1.0)):
        a = math.sqrt(g * s.p / s.rho)
        if p > s.p:
            sp = s.u + sign * a * math.sqrt((g + 1.0) / (2.0 * g) * p / s.p + (g - 1.0) / (2.0 * g))
            out[side + "_shock"] = sp
        else:
            a_star = a * (p / s.p) ** ((g - 1.0) / (2.0 * g))
            out[side + "_head"] = s.u + sign * a
            out[side + "_tail"] = u + sign * a_star
    return out


def sample(L: State, R: State, g: float, xi: np.ndarray):
    """(rho, u, p, side) at xi = (x - x0)/t; side = -1 left of the contact, +1 right."""
    p_s, u_s = star_state(L, R, g)
    rL, rR = star_densities(L, R, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi); u = np.empty_like(xi); p = np.empty_like(xi)
    side = np.where(xi < u_s, -1, 1)
    for n, x in enumerate(xi.ravel()):
        if x < u_s:
            s, sign, r_star = L, -1.0, rL
        else:
            s, sign, r_star = R, 1.0, rR
        a = math.sqrt(g * s.p / s.rho)
        if p_s > s.p:  # shock on this side
            sp = s.u + sign * a * math.sqrt((g + 1.0) / (2.0 * g) * p_s / s.p + (g - 1.0) / (2.0 * g))
            outside = (x < sp) if sign < 0 else (x > sp)
            vals = (s.rho, s.u, s.p) if outside else (r_star, u_s, p_s)
        else:  # rarefaction
            head = s.u + sign * a
            a_star = a * (p_s / s.p) ** ((g - 1.0) / (2.0 * g))
            tail = u_s + sign * a_star
            if (x < head) if sign < 0 else (x > head):
                vals = (s.rho, s.u, s.p)
            elif (x > tail) if sign < 0 else (x < tail):
                vals = (r_star, u_s, p_s)
            else:  # inside the fan
                c = 2.0 / (g + 1.0) - sign * (g - 1.0) / ((g + 1.0) * a) * (s.u - x)
                vals = (s.rho * c ** (2.0 / (g - 1.0)),
                        2.0 / (g + 1.0) * (-sign * a + (g - 1.0) / 2.0 * s.u + x),
                        s.p * c ** (2.0 * g / (g - 1.0)))
        rho.ravel()[n], u.ravel()[n], p.ravel()[n] = vals
    return rho, u, p, side


def sod_bme_solution(x: np.ndarray, t: float, x0: float = 0.5,
                     left=(1.0, 0.0, 1.0, 1.0), right=(0.125, 0.0, 0.1, 0.1)):
    """Exact primitive fields (rho, u, v, Pxx, Pxy, Pyy) of the 1-D BME Riemann
    problem with states (rho, u, Pxx, Pyy), v = Pxy = 0 on both sides: gamma = 3
    for (rho, u, Pxx); Pyy = rho * (Pyy/rho of the side of the contact)."""
    L = State(left[0], left[1], left[2])
    R = State(right[0], right[1], right[2])
    rho, u, p, side = sample(L, R, 3.0, (np.asarray(x) - x0) / t)
    ratio = np.where(side < 0, left[3] / left[0], right[3] / right[0])
    z = np.zeros_like(rho)
    return np.stack([rho, u, z, p, z, rho * ratio])
