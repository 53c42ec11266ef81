"""Exact Riemann solver for the 1D Euler equations of an ideal gas.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Follows Toro, "Riemann
Solvers and Numerical Methods for Fluid Dynamics", chapter 4: the pressure
functions f_L, f_R (eqs. 4.6-4.7), the Newton iteration for the star
pressure p* (section 4.3.2), the star velocity u* (eq. 4.9) and the sampling
of the self-similar solution at speed x/t (section 4.5).  It pins the FP64
oracle through closed-form wave structure (star values, wave speeds) and
through convergence of the discrete solution to the exact one.
"""
import math

import numpy as np

GAMMA = 1.4


def _f_and_df(p, rho, pk, ck, g=GAMMA):
    """Toro eq. 4.6/4.7: f_K(p) and its derivative for side K."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        sq = math.sqrt(A / (p + B))
        f = (p - pk) * sq
        df = sq * (1.0 - 0.5 * (p - pk) / (B + p))
    else:  # rarefaction
        pr = p / pk
        f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rhoL, uL, pL, rhoR, uR, pR, g=GAMMA, tol=1e-14, maxit=100):
    """Return (p*, u*) for the Riemann problem with the given primitive states."""
    cL = math.sqrt(g * pL / rhoL)
    cR = math.sqrt(g * pR / rhoR)
    du = uR - uL
    if 2.0 * (cL + cR) / (g - 1.0) <= du:
        raise ValueError("vacuum is generated; no star region")
    # initial guess: two-rarefaction approximation (Toro eq. 4.46)
    z = (g - 1.0) / (2.0 * g)
    p = ((cL + cR - 0.5 * (g - 1.0) * du) /
         (cL / pL ** z + cR / pR ** z)) ** (1.0 / z)
    p = max(p, 1e-12)
    for _ in range(maxit):
        fL, dfL = _f_and_df(p, rhoL, pL, cL, g)
        fR, dfR = _f_and_df(p, rhoR, pR, cR, g)
        p_new = p - (fL + fR + du) / (dfL + dfR)
        if p_new < 0.0:
            p_new = tol
        change = 2.0 * abs(p_new - p) / (p_new + p)
        p = p_new
        if change < tol:
            break
    fL, _ = _f_and_df(p, rhoL, pL, cL, g)
    fR, _ = _f_and_df(p, rhoR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def wave_structure(rhoL, uL, pL, rhoR, uR, pR, g=GAMMA):
    """Star densities and wave speeds for the solution.

    Returns a dict with p_star, u_star, rho_star_L, rho_star_R and, per side,
    either the shock speed or the rarefaction head and tail speeds."""
    ps, us = star_state(rhoL, uL, pL, rhoR, uR, pR, g)
    cL = math.sqrt(g * pL / rhoL)
    cR = math.sqrt(g * pR / rhoR)
    gm = (g - 1.0) / (g + 1.0)
    out = {"p_star": ps, "u_star": us}
    if ps > pL:
        r = ps / pL
        out["rho_star_L"] = rhoL * (r + gm) / (gm * r + 1.0)
        out["shock_L"] = uL - cL * math.sqrt((g + 1.0) / (2.0 * g) * r + (g - 1.0) / (2.0 * g))
    else:
        out["rho_star_L"] = rhoL * (ps / pL) ** (1.0 / g)
        cs = cL * (ps / pL) ** ((g - 1.0) / (2.0 * g))
        out["head_L"] = uL - cL
        out["tail_L"] = us - cs
    if ps > pR:
        r = ps / pR
        out["rho_star_R"] = rhoR * (r + gm) / (gm * r + 1.0)
        out["shock_R"] = uR + cR * math.sqrt((g + 1.0) / (2.0 * g) * r + (g - 1.0) / (2.0 * g))
    else:
        out["rho_star_R"] = rhoR * (ps / pR) ** (1.0 / g)
        cs = cR * (ps / pR) ** ((g - 1.0) / (2.0 * g))
        out["head_R"] = uR + cR
        out["tail_R"] = us + cs
    return out


def sample(xi, rhoL, uL, pL, rhoR, uR, pR, g=GAMMA):
    """Primitive solution (rho, u, p) at similarity coordinate xi = x / t.

    xi may be a scalar or a numpy array (Toro section 4.5)."""
    ps, us = star_state(rhoL, uL, pL, rhoR, uR, pR, g)
    cL = math.sqrt(g * pL / rhoL)
    cR = math.sqrt(g * pR / rhoR)
    gm = (g - 1.0) / (g + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if ps > pL:
                SL = uL - cL * math.sqrt((g + 1.0) / (2.0 * g) * ps / pL + (g - 1.0) / (2.0 * g))
                if s <= SL:
                    r, v, q = rhoL, uL, pL
                else:
                    r = rhoL * (ps / pL + gm) / (gm * ps / pL + 1.0)
                    v, q = us, ps
            else:
                head = uL - cL
                tail = us - cL * (ps / pL) ** ((g - 1.0) / (2.0 * g))
                if s <= head:
                    r, v, q = rhoL, uL, pL
                elif s >= tail:
                    r = rhoL * (ps / pL) ** (1.0 / g)
                    v, q = us, ps
                else:  # inside the left fan (Toro eq. 4.56)
                    c = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * (uL - s))
                    v = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * uL + s)
                    r = rhoL * (c / cL) ** (2.0 / (g - 1.0))
                    q = pL * (c / cL) ** (2.0 * g / (g - 1.0))
        else:  # right of the contact
            if ps > pR:
                SR = uR + cR * math.sqrt((g + 1.0) / (2.0 * g) * ps / pR + (g - 1.0) / (2.0 * g))
                if s >= SR:
                    r, v, q = rhoR, uR, pR
                else:
                    r = rhoR * (ps / pR + gm) / (gm * ps / pR + 1.0)
                    v, q = us, ps
            else:
                head = uR + cR
                tail = us + cR * (ps / pR) ** ((g - 1.0) / (2.0 * g))
                if s >= head:
                    r, v, q = rhoR, uR, pR
                elif s <= tail:
                    r = rhoR * (ps / pR) ** (1.0 / g)
                    v, q = us, ps
                else:  # inside the right fan (Toro eq. 4.63)
                    c = 2.0 / (g + 1.0) * (cR - 0.5 * (g - 1.0) * (uR - s))
                    v = 2.0 / (g + 1.0) * (-cR + 0.5 * (g - 1.0) * uR + s)
                    r = rhoR * (c / cR) ** (2.0 / (g - 1.0))
                    q = pR * (c / cR) ** (2.0 * g / (g - 1.0))
        rho[idx], u[idx], p[idx] = r, v, q
    return rho, u, p


def cell_averages(n, t, x0, left, right, g=GAMMA, sub=16):
    """Cell averages of the exact primitive solution on n cells of [0, 1].

    The initial jump sits at x0; left/right are (rho, u, p).  Each cell is
    averaged over `sub` midpoint sub-samples (enough for an L1 reference)."""
    xs = (np.arange(n * sub) + 0.5) / (n * sub)
    xi = (xs - x0) / t
    rho, u, p = sample(xi, *left, *right, g=g)
    return (rho.reshape(n, sub).mean(1), u.reshape(n, sub).mean(1),
            p.reshape(n, sub).mean(1))
