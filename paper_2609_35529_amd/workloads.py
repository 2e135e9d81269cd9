"""Seeded synthetic inputs shaped like the paper's 2-D test cases.

This module holds initial conditions, grid hierarchies and run parameters only:
no part of the VLBM update (equilibrium, relaxation, streaming, coupling) lives
here. Both the GPU path and the CPU oracle take their inputs from it.

Every generator returns conserved fields ``U[4][ny][nx] = (rho, rho u, rho v,
rho E)`` in float64 for an ideal gas, ``E = p/(gamma-1) + rho |u|^2 / 2``.
Random draws use NumPy's PCG64 (``numpy.random.default_rng(seed)``) in the order
documented on each function.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

PERIODIC, OUTFLOW, REFLECT, INFLOW = 0, 1, 2, 3

Box = Tuple[int, int, int, int, int]  # (level, i0, j0, nx, ny) in level-l cells


def conserved(rho, u, v, p, gamma=1.4):
    """Primitive (rho, u, v, p) -> conserved (rho, rho u, rho v, rho E)."""
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, u, v, p)))
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E]).astype(np.float64)


def cell_centres(n, dx, x0=0.0):
    return x0 + (np.arange(n) + 0.5) * dx


def level_grid(nx0, ny0, dx0, r, level, box=None, x0=0.0, y0=0.0):
    """Cell-centre coordinates (X, Y) of a level-l rectangle (default: whole level)."""
    s = r ** level
    dx = dx0 / s
    if box is None:
        i0, j0, nx, ny = 0, 0, nx0 * s, ny0 * s
    else:
        i0, j0, nx, ny = box
    xs = x0 + (i0 + np.arange(nx) + 0.5) * dx
    ys = y0 + (j0 + np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(xs, ys)
    return X, Y


def max_signal_speed(U, gamma=1.4):
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    cs = np.sqrt(gamma * np.maximum(p, 0.0) / rho)
    return float(max(np.max(np.abs(u) + cs), np.max(np.abs(v) + cs)))


def link_speed(U, gamma=1.4, kappa=1.5, D=2):
    """Link speed c = kappa * D * max(|u_alpha| + c_s) over the initial data."""
    return kappa * D * max_signal_speed(U, gamma)


@dataclasses.dataclass
class Case:
    """A full problem: base grid, hierarchy, parameters and per-level initial state."""
    name: str
    nx0: int
    ny0: int
    dx0: float
    r: int
    nlev: int
    gamma: float
    c: float
    beta: float
    bc: Tuple[int, int, int, int]
    boxes: List[Box]
    states: List[np.ndarray]          # states[l] = U over the whole level-l domain (None: unset)
    steps: int
    w_inflow: Optional[np.ndarray] = None  # [4 sides][4] conserved inflow states
    x0: float = 0.0
    y0: float = 0.0
    eos: Optional[Tuple[int, float, float]] = None  # (kind, a, b); None: ideal gas

    def level_shape(self, level):
        s = self.r ** level
        return self.ny0 * s, self.nx0 * s

    def fine_equivalent_per_coarse_step(self):
        s = self.r ** (self.nlev - 1)
        return self.nx0 * s * self.ny0 * s * s

    def coverage(self):
        """Per level, the boolean mask of covered cells (level 0: everything)."""
        cov = []
        for l in range(self.nlev):
            NY, NX = self.level_shape(l)
            m = np.zeros((NY, NX), dtype=bool)
            if l == 0:
                m[:] = True
            for (lv, i0, j0, nx, ny) in self.boxes:
                if lv == l:
                    m[j0:j0 + ny, i0:i0 + nx] = True
            cov.append(m)
        return cov

    def actual_updates_per_coarse_step(self):
        """sum_l (active cells of level l) * r^l."""
        cov = self.coverage()
        total = 0
        for l in range(self.nlev):
            act = cov[l].copy()
            if l + 1 < self.nlev:
                act &= ~cov[l + 1][::self.r, ::self.r]
            total += int(act.sum()) * self.r ** l
        return total

    def launches_per_coarse_step(self):
        present = [l for l in range(self.nlev) if l == 0 or any(b[0] == l for b in self.boxes)]
        return sum(self.r ** l for l in present)


def _states_for(nx0, ny0, dx0, r, nlev, fn, x0=0.0, y0=0.0):
    out = []
    for l in range(nlev):
        X, Y = level_grid(nx0, ny0, dx0, r, l, x0=x0, y0=y0)
        out.append(fn(X, Y))
    return out


# ------------------------------------------------------------ Sod (Sec. 4.1.2)
def sod_2d(nx0=128, ny0=8, steps=200, refine=True, r=2, beta=0.9, c=7.8125):
    """Sod shock tube on a y-periodic strip [0,1] x [0, ny0/nx0].

    Left (rho,u,p) = (1,0,1), right (0.125,0,0.1), diaphragm at x = 0.5, one
    static patch at ratio r over x in [0.375, 0.625] spanning y. With the
    default c = 7.8125 and dx0 = 1/128, 200 coarse steps reach t = 0.2.
    """
    dx0 = 1.0 / nx0
    gamma = 1.4

    def ic(X, Y):
        left = X < 0.5
        rho = np.where(left, 1.0, 0.125)
        p = np.where(left, 1.0, 0.1)
        return conserved(rho, 0.0 * X, 0.0 * X, p, gamma)

    nlev = 2 if refine else 1
    boxes = []
    if refine:
        i0 = int(round(0.375 * nx0)) * r
        i1 = int(round(0.625 * nx0)) * r
        boxes = [(1, i0, 0, i1 - i0, ny0 * r)]
    return Case("sod_2d", nx0, ny0, dx0, r, nlev, gamma, c, beta,
                (OUTFLOW, OUTFLOW, PERIODIC, PERIODIC), boxes,
                _states_for(nx0, ny0, dx0, r, nlev, ic), steps)


# ------------------------------------------- random four-quadrant Riemann problem
def quadrant_states(seed):
    """Four quadrant states drawn in the order NE, NW, SW, SE; per quadrant
    rho ~ U[0.1,1.5], p ~ U[0.02,1.5], u ~ U[-1.2,1.2], v ~ U[-1.2,1.2]."""
    rng = np.random.default_rng(seed)
    st = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        p = rng.uniform(0.02, 1.5)
        u = rng.uniform(-1.2, 1.2)
        v = rng.uniform(-1.2, 1.2)
        st.append((rho, u, v, p))
    return st  # NE, NW, SW, SE


def _quadrant_ic(states, gamma, xs=0.5, ys=0.5):
    ne, nw, sw, se = states

    def ic(X, Y):
        east = X >= xs
        north = Y >= ys
        out = np.empty((4,) + X.shape)
        for (cond, s) in ((east & north, ne), (~east & north, nw), (~east & ~north, sw),
                          (east & ~north, se)):
            rho, u, v, p = s
            U = conserved(rho, u, v, p, gamma)
            for k in range(4):
                out[k][cond] = U[k]
        return out
    return ic


def quadrant(n0=512, seed=0, steps=1000, refine=True, r=2, beta=0.6, kappa=1.5,
             patch=(0.25, 0.75), bc=OUTFLOW, states=None):
    """Four-quadrant Riemann problem on [0,1]^2 with one centred static patch.

    Quadrant states come from ``quadrant_states(seed)`` unless given; the link
    speed is ``link_speed`` of the initial data.
    """
    gamma = 1.4
    dx0 = 1.0 / n0
    st = quadrant_states(seed) if states is None else states
    ic = _quadrant_ic(st, gamma)
    nlev = 2 if refine else 1
    boxes = []
    if refine:
        a = int(round(patch[0] * n0)) * r
        b = int(round(patch[1] * n0)) * r
        boxes = [(1, a, a, b - a, b - a)]
    states_l = _states_for(n0, n0, dx0, r, nlev, ic)
    c = link_speed(states_l[0], gamma, kappa)
    return Case("quadrant", n0, n0, dx0, r, nlev, gamma, c, beta, (bc,) * 4, boxes, states_l,
                steps)


def lax_liu_12(n0=64, steps=100, boxes=None, r=2, nlev=2, beta=0.6, kappa=1.5):
    """Lax-Liu configuration 12 (paper eq. case12-ic), outflow sides."""
    st = [(0.5313, 0.0, 0.0, 0.4), (1.0, 0.7276, 0.0, 1.0), (0.8, 0.0, 0.0, 1.0),
          (1.0, 0.0, 0.7276, 1.0)]
    gamma = 1.4
    dx0 = 1.0 / n0
    ic = _quadrant_ic(st, gamma)
    states_l = _states_for(n0, n0, dx0, r, nlev, ic)
    c = link_speed(states_l[0], gamma, kappa)
    return Case("lax_liu_12", n0, n0, dx0, r, nlev, gamma, c, beta, (OUTFLOW,) * 4,
                list(boxes or []), states_l, steps)


# ------------------------------------------ isentropic vortex (Sec. 4.1.3)
def vortex_U(X, Y, gamma=1.4, beta_v=2.0, Rc=0.05, xc=(0.5, 0.5), rho_inf=1.0, p_inf=1.0):
    """Stationary isentropic vortex, paper eq. (vortex-exact)."""
    dx = X - xc[0]
    dy = Y - xc[1]
    r2 = dx * dx + dy * dy
    T_inf = p_inf / rho_inf
    dT = -(gamma - 1.0) * beta_v ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2 / Rc ** 2)
    T = T_inf + dT
    rho = rho_inf * (T / T_inf) ** (1.0 / (gamma - 1.0))
    p = rho * T
    # u_phi(r) = beta_v / (2 pi Rc) r exp((1 - r^2/Rc^2)/2);  (u, v) = u_phi (-dy, dx)/r
    amp = beta_v / (2.0 * math.pi * Rc) * np.exp(0.5 * (1.0 - r2 / Rc ** 2))
    u = -amp * dy
    v = amp * dx
    return conserved(rho, u, v, p, gamma)


def vortex(n0=64, t_end=0.5, refine=True, r=2, beta=1.0, kappa=1.5):
    gamma = 1.4
    dx0 = 1.0 / n0
    nlev = 2 if refine else 1
    boxes = []
    if refine:
        a = (n0 // 4) * r
        b = (3 * n0 // 4) * r
        boxes = [(1, a, a, b - a, b - a)]
    states_l = _states_for(n0, n0, dx0, r, nlev, lambda X, Y: vortex_U(X, Y, gamma))
    c = link_speed(states_l[0], gamma, kappa)
    steps = int(round(t_end * c / dx0))
    c = steps * dx0 / t_end  # land exactly on t_end
    return Case("vortex", n0, n0, dx0, r, nlev, gamma, c, beta, (PERIODIC,) * 4, boxes,
                states_l, steps)


# ---------------------------------------------- explosion in a box (Sec. 4.2)
def explosion(n0=64, steps=50, refine=True, r=2, beta=0.7, kappa=1.5):
    gamma = 1.4
    dx0 = 1.0 / n0

    def ic(X, Y):
        inside = (X - 0.4) ** 2 + (Y - 0.4) ** 2 < 0.3 ** 2
        rho = np.where(inside, 5.0, 1.0)
        p = np.where(inside, 5.0, 1.0)
        return conserved(rho, 0 * X, 0 * X, p, gamma)

    nlev = 2 if refine else 1
    boxes = []
    if refine:
        a = (n0 // 4) * r
        b = (3 * n0 // 4) * r
        boxes = [(1, a, a, b - a, b - a)]
    states_l = _states_for(n0, n0, dx0, r, nlev, ic)
    c = link_speed(states_l[0], gamma, kappa)
    return Case("explosion", n0, n0, dx0, r, nlev, gamma, c, beta, (REFLECT,) * 4, boxes,
                states_l, steps)


# ------------------------------------- 1-D acoustic pulse (Sec. 4.1.1)
def acoustic_pulse(dx1=0.01, r=2, beta=0.99, c=3.0, ny0=1, t_end=1.2, A=0.01, sigma=0.05,
                   x0=-0.6):
    """Coarse x in [-1,0] (dx1), fine x in [0,1.5] (dx1/r), y-periodic strip.

    Ambient rho0 = 1, u0 = 0, p0 = 1/gamma so that c_s0 = 1; right-moving
    linear pulse of paper eq. (val-acoustic-ic).
    """
    gamma = 1.4
    nx0 = int(round(2.5 / dx1))
    p0 = 1.0 / gamma
    rho0, cs0 = 1.0, 1.0

    def ic(X, Y):
        rho = rho0 + A * np.exp(-(X - x0) ** 2 / (2 * sigma ** 2))
        u = cs0 / rho0 * (rho - rho0)
        p = p0 + cs0 ** 2 * (rho - rho0)
        return conserved(rho, u, 0 * X, p, gamma)

    i0 = int(round(1.0 / dx1))
    boxes = [(1, i0 * r, 0, (nx0 - i0) * r, ny0 * r)]
    states_l = _states_for(nx0, ny0, dx1, r, 2, ic, x0=-1.0)
    steps = int(round(t_end * c / dx1))
    return Case("acoustic_pulse", nx0, ny0, dx1, r, 2, gamma, c, beta,
                (OUTFLOW, OUTFLOW, PERIODIC, PERIODIC), boxes, states_l, steps, x0=-1.0)


# --------------------------------------------------------- generic helpers
def uniform_flow(n0=32, rho=1.3, u=0.4, v=-0.3, p=0.9, gamma=1.4, nlev=3, r=2, beta=0.8,
                 c=4.0, bc=PERIODIC):
    boxes = nested_centre_boxes(n0, n0, r, nlev)
    states_l = _states_for(n0, n0, 1.0 / n0, r, nlev,
                           lambda X, Y: conserved(rho + 0 * X, u, v, p, gamma))
    return Case("uniform_flow", n0, n0, 1.0 / n0, r, nlev, gamma, c, beta, (bc,) * 4, boxes,
                states_l, 50)


def nested_centre_boxes(nx0, ny0, r, nlev, frac=0.5):
    """Centred nested boxes, each level covering ``frac`` of its parent's box."""
    boxes = []
    lo_x, hi_x, lo_y, hi_y = 0, nx0, 0, ny0
    for l in range(1, nlev):
        wx = hi_x - lo_x
        wy = hi_y - lo_y
        a_x = lo_x + int(round(wx * (1 - frac) / 2))
        b_x = hi_x - int(round(wx * (1 - frac) / 2))
        a_y = lo_y + int(round(wy * (1 - frac) / 2))
        b_y = hi_y - int(round(wy * (1 - frac) / 2))
        lo_x, hi_x, lo_y, hi_y = a_x * r, b_x * r, a_y * r, b_y * r
        boxes.append((l, lo_x, lo_y, hi_x - lo_x, hi_y - lo_y))
    return boxes


def random_smooth_U(nx, ny, seed, gamma=1.4, modes=3, amp=0.2):
    """Random smooth periodic field (sum of low Fourier modes) on an nx x ny grid."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)

    def field(base, a):
        f = np.full_like(X, base)
        for _ in range(modes):
            kx, ky = rng.integers(1, 4, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            f += a * rng.uniform(-1, 1) * np.sin(2 * np.pi * (kx * X + ky * Y) + ph)
        return f

    rho = field(1.0, amp)
    u = field(0.2, amp)
    v = field(-0.1, amp)
    p = field(1.0, amp)
    return conserved(rho, u, v, p, gamma)


def random_state_U(nx, ny, seed, gamma=1.4):
    """Cell-by-cell random valid states (rough data for conservation pins):
    rho ~ U[0.5,1.5], u,v ~ U[-0.5,0.5], p ~ U[0.5,1.5], drawn as four arrays."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, (ny, nx))
    u = rng.uniform(-0.5, 0.5, (ny, nx))
    v = rng.uniform(-0.5, 0.5, (ny, nx))
    p = rng.uniform(0.5, 1.5, (ny, nx))
    return conserved(rho, u, v, p, gamma)


def prolong_piecewise(U, r):
    """Copy each coarse value to its r x r children (used to seed finer levels)."""
    return np.repeat(np.repeat(U, r, axis=1), r, axis=2)


# --------------------------------------------------- Kelvin-Helmholtz shear layer
def kelvin_helmholtz(n0=4096, seed=0, nlev=4, r=2, beta=0.8, kappa=1.5, steps=5000,
                     band=0.25, dynamic=False):
    """Shear layer on [0,1]^2, periodic: |y - 0.5| < band has rho = 2, u = +0.5,
    outside rho = 1, u = -0.5; p = 2.5, gamma = 1.4. Perturbation drawn as two
    arrays in order: U1 for v (v = 0.01 sin(4 pi x) + 0.01 (U1 - 1/2)), then U2
    for u (u += 0.01 (U2 - 1/2)). Levels refine nested bands around the two
    interfaces at y = 0.25 and 0.75; with dynamic=True there are no static
    boxes and no finer-level states: the hierarchy comes from tagging and
    clustering, and splitting fills the finer levels (the 4096^2 problem's
    finest level alone would be a 32768^2 array on the host)."""
    gamma = 1.4
    dx0 = 1.0 / n0
    rng = np.random.default_rng(seed)
    U1 = rng.uniform(0, 1, (n0, n0))
    U2 = rng.uniform(0, 1, (n0, n0))

    def ic0(X, Y):
        inner = np.abs(Y - 0.5) < band
        rho = np.where(inner, 2.0, 1.0)
        u = np.where(inner, 0.5, -0.5) + 0.01 * (U2 - 0.5)
        v = 0.01 * np.sin(4 * np.pi * X) + 0.01 * (U1 - 0.5)
        return conserved(rho, u, v, 2.5 + 0 * X, gamma)

    X, Y = level_grid(n0, n0, dx0, r, 0)
    U0 = ic0(X, Y)
    if dynamic:
        return Case("kelvin_helmholtz", n0, n0, dx0, r, nlev, gamma, link_speed(U0, gamma, kappa), beta,
                    (PERIODIC,) * 4, [], [U0] + [None] * (nlev - 1), steps)
    states = [U0]
    for l in range(1, nlev):
        states.append(prolong_piecewise(states[-1], r))
    boxes = []
    widths = [0.125, 0.0625, 0.03125, 0.015625]
    for l in range(1, nlev):
        s = r ** l
        h = widths[min(l - 1, len(widths) - 1)]
        for yc in (0.5 - band, 0.5 + band):
            j0 = int(round((yc - h) * n0)) * s
            j1 = int(round((yc + h) * n0)) * s
            boxes.append((l, 0, j0, n0 * s, j1 - j0))
    c = link_speed(U0, gamma, kappa)
    return Case("kelvin_helmholtz", n0, n0, dx0, r, nlev, gamma, c, beta, (PERIODIC,) * 4,
                boxes, states, steps)


def kelvin_helmholtz_strip(n0=4096, ny0=512, yc=0.25, seed=0, nlev=4, r=2, beta=0.8, kappa=1.5,
                           steps=5000, band=0.25):
    """One horizontal strip of the Kelvin-Helmholtz problem above: n0 x ny0
    coarse cells of the n0 x n0 domain, centred on the shear layer at y = yc.
    The perturbation is drawn for the whole n0 x n0 domain exactly as in
    kelvin_helmholtz (same generator, same order) and the strip's rows are
    taken, so the strip's data equal those rows of the full problem. Periodic
    in x; the strip's two cut sides are outflow, standing in for the rows that
    neighbouring strips would exchange. No static boxes: the hierarchy comes
    from tagging and clustering."""
    gamma = 1.4
    dx0 = 1.0 / n0
    rng = np.random.default_rng(seed)
    U1 = rng.uniform(0, 1, (n0, n0))
    U2 = rng.uniform(0, 1, (n0, n0))
    j0 = int(round(yc * n0)) - ny0 // 2
    if j0 < 0 or j0 + ny0 > n0:
        raise ValueError("strip outside the domain")
    y0 = j0 * dx0
    U1s, U2s = U1[j0:j0 + ny0], U2[j0:j0 + ny0]

    def ic0(X, Y):
        inner = np.abs(Y - 0.5) < band
        rho = np.where(inner, 2.0, 1.0)
        u = np.where(inner, 0.5, -0.5) + 0.01 * (U2s - 0.5)
        v = 0.01 * np.sin(4 * np.pi * X) + 0.01 * (U1s - 0.5)
        return conserved(rho, u, v, 2.5 + 0 * X, gamma)

    X, Y = level_grid(n0, ny0, dx0, r, 0, y0=y0)
    U0 = ic0(X, Y)
    c = link_speed(U0, gamma, kappa)
    # finer levels start empty and are filled by splitting at the first regrids
    return Case("kh_strip", n0, ny0, dx0, r, nlev, gamma, c, beta,
                (PERIODIC, PERIODIC, OUTFLOW, OUTFLOW), [], [U0] + [None] * (nlev - 1), steps)


# --------------------------------------------------- shock - bubble interaction
def shock_bubble(nx0=1024, ny0=256, steps=500, nlev=3, r=2, beta=0.8, kappa=1.5):
    """Mach 1.22 shock (x = 0.5, moving +x) into a circular bubble of density
    0.138 (centre (1.0, 0.5), radius 0.25) on [0,4] x [0,1]. Pre-shock
    (1, 0, 0, 1); post-shock state from the Rankine-Hugoniot relations. Inflow
    west, outflow east, reflective south/north."""
    gamma = 1.4
    dx0 = 4.0 / nx0
    Ms = 1.22
    rho1, p1 = 1.0, 1.0
    c1 = math.sqrt(gamma * p1 / rho1)
    p2 = p1 * (1 + 2 * gamma / (gamma + 1) * (Ms ** 2 - 1))
    rho2 = rho1 * (gamma + 1) * Ms ** 2 / ((gamma - 1) * Ms ** 2 + 2)
    u2 = Ms * c1 * (1 - rho1 / rho2)

    def ic(X, Y):
        post = X < 0.5
        bub = (X - 1.0) ** 2 + (Y - 0.5) ** 2 < 0.25 ** 2
        rho = np.where(post, rho2, np.where(bub, 0.138, rho1))
        u = np.where(post, u2, 0.0)
        p = np.where(post, p2, p1)
        return conserved(rho, u, 0 * X, p, gamma)

    states = _states_for(nx0, ny0, dx0, r, nlev, ic)
    win = np.zeros((4, 4))
    win[0] = conserved(rho2, u2, 0.0, p2, gamma).reshape(4)
    c = link_speed(states[0], gamma, kappa)
    return Case("shock_bubble", nx0, ny0, dx0, r, nlev, gamma, c, beta,
                (INFLOW, OUTFLOW, REFLECT, REFLECT), [], states, steps, w_inflow=win)


def patch_set(seed=0, nx0=1024, ny0=256, np_range=(100, 400), size_range=(16, 128), steps=100,
              beta=0.8, kappa=1.5, max_tries=200):
    """Batched uneven patches on the shock-bubble problem (its base grid,
    state and sides): a seeded, static set of N_p ~ U{np_range} boxes, levels
    1 and 2 in a 3:1 ratio (N_p // 4 on level 2), sides ~ U{size_range}
    level-l cells made even (whole parent cells). Draws in order: N_p; per
    level-1 box its width, height and position until it overlaps no earlier
    level-1 box (at most max_tries draws per box); per level-2 box its width,
    height, host level-1 box and position, its parent footprint one level-1
    cell inside the host on every side and overlapping no earlier level-2
    box. Boxes whose draws all fail are left out (the Case name states the
    counts placed)."""
    base = shock_bubble(nx0=nx0, ny0=ny0, steps=steps, nlev=3, beta=beta, kappa=kappa)
    rng = np.random.default_rng(seed)
    n = int(rng.integers(np_range[0], np_range[1] + 1))
    n2 = n // 4
    n1 = n - n2
    lo, hi = size_range

    def side():
        v = int(rng.integers(lo, hi + 1))
        return v + (v % 2)

    W1, H1 = 2 * nx0, 2 * ny0
    occ1 = np.zeros((H1, W1), dtype=bool)
    b1 = []
    for _ in range(n1):
        for _ in range(max_tries):
            w, h = min(side(), W1), min(side(), H1)
            x = 2 * int(rng.integers(0, (W1 - w) // 2 + 1))
            y = 2 * int(rng.integers(0, (H1 - h) // 2 + 1))
            if not occ1[y:y + h, x:x + w].any():
                occ1[y:y + h, x:x + w] = True
                b1.append((1, x, y, w, h))
                break
    occ2 = np.zeros((2 * H1, 2 * W1), dtype=bool)
    b2 = []
    for _ in range(n2):
        for _ in range(max_tries):
            w, h = side(), side()
            _, hx, hy, hw, hh = b1[int(rng.integers(0, len(b1)))]
            fw, fh = w // 2, h // 2  # parent footprint in level-1 cells
            if fw > hw - 2 or fh > hh - 2:
                continue
            fx = hx + 1 + int(rng.integers(0, hw - 2 - fw + 1))
            fy = hy + 1 + int(rng.integers(0, hh - 2 - fh + 1))
            x, y = 2 * fx, 2 * fy
            if not occ2[y:y + h, x:x + w].any():
                occ2[y:y + h, x:x + w] = True
                b2.append((2, x, y, w, h))
                break
    name = f"patch_set(seed {seed}: {len(b1)} level-1 and {len(b2)} level-2 boxes of {n} drawn)"
    return dataclasses.replace(base, name=name, boxes=b1 + b2)


def request_stream(n_requests, rate, seed=0, sizes=(64, 128, 256, 512, 1024),
                   steps_range=(200, 2000)):
    """Poisson arrivals of quadrant Riemann solves: per request draw in order
    inter-arrival ~ Exp(rate), size index, number of levels in {1,2,3}, steps in
    steps_range, and the quadrant seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n0 = int(sizes[rng.integers(0, len(sizes))])
        nlev = int(rng.integers(1, 4))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        qseed = int(rng.integers(0, 2 ** 31 - 1))
        reqs.append(dict(id=i, arrival=t, n0=n0, nlev=nlev, steps=steps, seed=qseed))
    return reqs


def request_case(req, beta=0.6, kappa=1.5, r=2):
    """The Case of one served request: level 1 over the central half box,
    level 2 over the central quarter box."""
    n0 = req["n0"]
    nlev = req["nlev"]
    case = quadrant(n0=n0, seed=req["seed"], steps=req["steps"], refine=False, r=r, beta=beta,
                    kappa=kappa)
    boxes = nested_centre_boxes(n0, n0, r, nlev)
    states = list(case.states)
    for l in range(1, nlev):
        X, Y = level_grid(n0, n0, 1.0 / n0, r, l)
        states.append(_quadrant_ic(quadrant_states(req["seed"]), 1.4)(X, Y))
    if req.get("poison"):  # a faulty request: negative density in one level-0 cell
        U = np.array(states[0], copy=True)
        U[0, 1, 1] = -abs(U[0, 1, 1])
        states[0] = U
    return dataclasses.replace(case, nlev=nlev, boxes=boxes, states=states, name="request")


# ------------------------------------------------ three dimensions (D3Q6)
Box3 = Tuple[int, int, int, int, int, int, int]  # (level, i0, j0, k0, nx, ny, nz)


@dataclasses.dataclass
class Case3:
    """A 3-D problem: base grid, static hierarchy, parameters and per-level
    initial state U[5][Nz][Ny][Nx] (rho, rho u, rho v, rho w, E)."""
    name: str
    nx0: int
    ny0: int
    nz0: int
    dx0: float
    r: int
    nlev: int
    gamma: float
    c: float
    beta: float
    bc: Tuple[int, int, int, int, int, int]
    boxes: List[Box3]
    states: List[Optional[np.ndarray]]  # states[l]: U of a block of level-l cells (None: unset)
    steps: int
    origins: Optional[List[Tuple[int, int, int]]] = None  # (i0, j0, k0) of states[l]; None: 0

    def level_shape(self, level):
        s = self.r ** level
        return self.nz0 * s, self.ny0 * s, self.nx0 * s

    def origin(self, level):
        return tuple(self.origins[level]) if self.origins else (0, 0, 0)

    def full_state(self, level):
        """states[level] placed in a zero array over the whole level."""
        U = np.zeros((5,) + self.level_shape(level))
        i0, j0, k0 = self.origin(level)
        S = self.states[level]
        U[:, k0:k0 + S.shape[1], j0:j0 + S.shape[2], i0:i0 + S.shape[3]] = S
        return U

    def fine_equivalent_per_coarse_step(self):
        """Cells of the finest level's resolution over the whole domain, times
        the finest level's sub-steps per coarse step."""
        s = self.r ** (self.nlev - 1)
        return self.nx0 * self.ny0 * self.nz0 * s ** 3 * s

    def actual_updates_per_coarse_step(self):
        """sum_l (active cells of level l) * r^l, from the box volumes (boxes of a
        level do not overlap)."""
        vol = [self.nx0 * self.ny0 * self.nz0] + [0] * (self.nlev - 1)
        for (lv, i0, j0, k0, nx, ny, nz) in self.boxes:
            vol[lv] += nx * ny * nz
        total = 0
        for l in range(self.nlev):
            act = vol[l] - (vol[l + 1] // self.r ** 3 if l + 1 < self.nlev else 0)
            total += act * self.r ** l
        return total


def conserved3(rho, u, v, w, p, gamma=1.4):
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def level_grid3(nx0, ny0, nz0, dx0, r, level):
    """Cell-centre coordinates (Z, Y, X) of the whole level-l domain."""
    s = r ** level
    dx = dx0 / s
    z = (np.arange(nz0 * s) + 0.5) * dx
    y = (np.arange(ny0 * s) + 0.5) * dx
    x = (np.arange(nx0 * s) + 0.5) * dx
    return np.meshgrid(z, y, x, indexing="ij")


def link_speed3(U, gamma=1.4, kappa=1.5):
    rho = U[0]
    vel = [U[1] / rho, U[2] / rho, U[3] / rho]
    p = (gamma - 1.0) * (U[4] - 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2))
    cs = np.sqrt(gamma * np.maximum(p, 0.0) / rho)
    return kappa * 3 * float(max(np.max(np.abs(a) + cs) for a in vel))


def prolong3(U, r):
    return U.repeat(r, axis=1).repeat(r, axis=2).repeat(r, axis=3)


def random_state3(nx, ny, nz, seed, gamma=1.4, amp=0.25):
    """Seeded smooth random 3-D state: a uniform base, three low Fourier modes
    per field and small cellwise noise."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")

    def field(base, a):
        f = np.full(x.shape, base)
        for _ in range(3):
            kx, ky, kz = rng.integers(0, 3, 3)
            f = f + a * rng.uniform(-1, 1) * np.sin(2 * np.pi * (kx * x + ky * y + kz * z)
                                                   + rng.uniform(0, 6.3))
        return f + 0.02 * a * rng.normal(size=x.shape)

    rho = np.maximum(field(1.0, amp), 0.3)
    p = np.maximum(field(1.0, amp), 0.3)
    return conserved3(rho, field(0.0, 0.3), field(0.0, 0.3), field(0.0, 0.3), p, gamma)


def blast3d(n0=256, steps=100, refine=True, r=2, beta=0.8, kappa=1.5, bc=REFLECT):
    """Spherical blast in the unit cube with reflecting walls (the 3-D
    counterpart of the explosion in a box, Sec. 4.2): rho = p = 5 inside a
    sphere of radius 0.2 centred at (0.45, 0.45, 0.45), 1 outside, at rest;
    one r = 2 patch over the central half of the domain along every axis."""
    gamma = 1.4
    dx0 = 1.0 / n0

    def ic(Z, Y, X):
        inside = (X - 0.45) ** 2 + (Y - 0.45) ** 2 + (Z - 0.45) ** 2 < 0.2 ** 2
        rho = np.where(inside, 5.0, 1.0)
        p = np.where(inside, 5.0, 1.0)
        return conserved3(rho, 0 * X, 0 * X, 0 * X, p, gamma)

    nlev = 2 if refine else 1
    boxes = []
    origins = [(0, 0, 0)]
    if refine:
        a, b = (n0 // 4) * r, (3 * n0 // 4) * r
        boxes = [(1, a, a, a, b - a, b - a, b - a)]
        origins.append((a, a, a))
    states = [ic(*level_grid3(n0, n0, n0, dx0, r, 0))]
    for l in range(1, nlev):
        # the patch's own cells only (a level-l array over the whole domain
        # would be r^3 times the level-0 array)
        (_, i0, j0, k0, nx, ny, nz) = boxes[l - 1]
        dx = dx0 / r ** l
        zc = (k0 + np.arange(nz) + 0.5) * dx
        yc = (j0 + np.arange(ny) + 0.5) * dx
        xc = (i0 + np.arange(nx) + 0.5) * dx
        states.append(ic(*np.meshgrid(zc, yc, xc, indexing="ij")))
    c = link_speed3(states[0], gamma, kappa)
    return Case3("blast3d", n0, n0, n0, dx0, r, nlev, gamma, c, beta, (bc,) * 6, boxes, states, steps,
                 origins)
