"""Independent reference solutions used to pin the oracle.

* ``riemann_exact``: the exact solution of the 1-D Riemann problem for an ideal
  gas (textbook construction: pressure function, Newton iteration for the star
  pressure, then sampling of the self-similar wave pattern).
* ``lax_friedrichs_step``: the 2-D Lax-Friedrichs scheme on the conserved
  variables, written directly from its textbook formula. With beta = 1/2 the
  VLBM relaxation returns the equilibrium, and one VLBM step reduces exactly to
  this scheme with dt/dx = 1/c (paper eqs. num-equilibrium and num-relaxation).
* ``euler_flux``: the Euler flux of an ideal gas.
"""
from __future__ import annotations

import math

import numpy as np


def euler_flux(U, gamma=1.4):
    rho, mx, my, E = U
    u = mx / rho
    v = my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    Fx = np.stack([mx, mx * u + p, my * u, (E + p) * u])
    Fy = np.stack([my, mx * v, my * v + p, (E + p) * v])
    return Fx, Fy


def lax_friedrichs_step(U, c, gamma=1.4):
    """W_ij^{n+1} = (W_{i-1} + W_{i+1} + W_{j-1} + W_{j+1})/4
                  - (1/(2c)) [Fx_{i+1} - Fx_{i-1} + Fy_{j+1} - Fy_{j-1}], periodic."""
    Fx, Fy = euler_flux(U, gamma)
    roll = np.roll
    avg = 0.25 * (roll(U, 1, axis=2) + roll(U, -1, axis=2) + roll(U, 1, axis=1) + roll(U, -1, axis=1))
    div = (roll(Fx, -1, axis=2) - roll(Fx, 1, axis=2)) + (roll(Fy, -1, axis=1) - roll(Fy, 1, axis=1))
    return avg - div / (2.0 * c)


# ------------------------------------------------------------ exact Riemann
def _pressure_fn(p, rho, pk, ck, gamma):
    """f_K(p) and its derivative: shock branch (p > p_K) or rarefaction branch."""
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        sq = math.sqrt(A / (p + B))
        f = (p - pk) * sq
        df = sq * (1.0 - 0.5 * (p - pk) / (B + p))
    else:
        e = (gamma - 1.0) / (2.0 * gamma)
        f = 2.0 * ck / (gamma - 1.0) * ((p / pk) ** e - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma=1.4):
    """Star pressure and velocity of the Riemann problem (rho, u, p)_L / _R."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _pressure_fn(p, rl, pl, cl, gamma)
        fr, dfr = _pressure_fn(p, rr, pr, cr, gamma)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        if pn < 0:
            pn = 1e-10
        if abs(pn - p) / (0.5 * (pn + p)) < 1e-15:
            p = pn
            break
        p = pn
    fl, _ = _pressure_fn(p, rl, pl, cl, gamma)
    fr, _ = _pressure_fn(p, rr, pr, cr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_exact(left, right, xi, gamma=1.4):
    """Sample (rho, u, p) at similarity coordinates xi = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = np.empty((3, len(xi)))
    for i, s in enumerate(np.asarray(xi, dtype=np.float64)):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rho_s = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                S = ul - cl * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                val = (rl, ul, pl) if s <= S else (rho_s, us, ps)
            else:  # left rarefaction
                rho_s = rl * (ps / pl) ** (1.0 / gamma)
                cs = cl * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                head, tail = ul - cl, us - cs
                if s <= head:
                    val = (rl, ul, pl)
                elif s >= tail:
                    val = (rho_s, us, ps)
                else:
                    u = 2.0 / (gamma + 1) * (cl + (gamma - 1) / 2 * ul + s)
                    c = 2.0 / (gamma + 1) * (cl + (gamma - 1) / 2 * (ul - s))
                    rho = rl * (c / cl) ** (2.0 / (gamma - 1))
                    p = pl * (c / cl) ** (2 * gamma / (gamma - 1))
                    val = (rho, u, p)
        else:  # right of contact
            if ps > pr:  # right shock
                rho_s = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                S = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                val = (rr, ur, pr) if s >= S else (rho_s, us, ps)
            else:  # right rarefaction
                rho_s = rr * (ps / pr) ** (1.0 / gamma)
                cs = cr * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                head, tail = ur + cr, us + cs
                if s >= head:
                    val = (rr, ur, pr)
                elif s <= tail:
                    val = (rho_s, us, ps)
                else:
                    u = 2.0 / (gamma + 1) * (-cr + (gamma - 1) / 2 * ur + s)
                    c = 2.0 / (gamma + 1) * (cr - (gamma - 1) / 2 * (ur - s))
                    rho = rr * (c / cr) ** (2.0 / (gamma - 1))
                    p = pr * (c / cr) ** (2 * gamma / (gamma - 1))
                    val = (rho, u, p)
        out[:, i] = val
    return out


# ------------------------------------------------------------ helpers
def composite_1d_rho(orc, case):
    """Density along x on the finest data available (y-averaged), with centres."""
    xs, rhos = [], []
    for l in range(case.nlev):
        U = orc.get_state(l)
        act = orc.active_mask(l)
        NY, NX = U.shape[1:]
        dx = case.dx0 / case.r ** l
        cols = act.any(axis=0)
        rho = np.where(act, U[0], 0.0).sum(axis=0)
        cnt = act.sum(axis=0)
        for i in np.nonzero(cols)[0]:
            xs.append(case.x0 + (i + 0.5) * dx)
            rhos.append(rho[i] / cnt[i])
    order = np.argsort(xs)
    return np.asarray(xs)[order], np.asarray(rhos)[order]


def run_oracle(case, steps=None, oracle_cls=None, **kw):
    from oracle.oracle import Oracle
    if getattr(case, "eos", None) is not None and "eos" not in kw:
        kw = dict(kw, eos=case.eos[0], eos_a=case.eos[1], eos_b=case.eos[2])
    o = Oracle(case.nx0, case.ny0, case.dx0, case.r, case.nlev, case.gamma, case.c, case.beta,
               case.bc, case.w_inflow, **kw)
    o.set_boxes(case.boxes)
    for l in range(case.nlev):
        if case.states[l] is not None:
            o.set_state(l, case.states[l])
    if steps is None:
        steps = case.steps
    if steps:
        o.advance(steps)
    return o
