"""Pins of oracle parts that the closed forms and invariants elsewhere leave
loose: the non-ideal equations of state, the specular wall, the magnitude of
the adaptive-relaxation sensor, the density-gradient tag and the temporal
history across a regrid. Each is checked against something other than the
oracle's own formula (a textbook relation, the method of images, analytic
derivatives, numpy differences of the held state, runs without the regrid),
and a planted mistake shows that the check can fail. CPU only.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_35529_amd import workloads as wl
from tests import exact

GAMMA = 1.4


# ------------------------------------------------ equations of state (Sec. 2.1)
def _textbook_rho_e(eos, a, b, rho, p, gamma=GAMMA):
    """Internal energy per volume from the textbook caloric relations.

    - ideal gas: rho e = p / (gamma - 1);
    - stiffened gas with reference pressure p_inf = a: rho e = (p + gamma p_inf) / (gamma - 1);
    - van der Waals gas with constant c_v (here 1) and R = (gamma - 1) c_v:
      p = rho R T / (1 - b rho) - a rho^2 and e = c_v T - a rho, so T is solved
      from p and e follows from T.
    """
    if eos == O.EOS_IDEAL:
        return p / (gamma - 1.0)
    if eos == O.EOS_STIFFENED:
        return (p + gamma * a) / (gamma - 1.0)
    cv = 1.0
    R = (gamma - 1.0) * cv
    T = (p + a * rho * rho) * (1.0 - b * rho) / (rho * R)
    return rho * (cv * T - a * rho)


@pytest.mark.parametrize("eos,a,b", [(O.EOS_IDEAL, 0.0, 0.0), (O.EOS_STIFFENED, 0.3, 0.0),
                                     (O.EOS_STIFFENED, 2.0, 0.0), (O.EOS_VDW, 0.2, 0.05),
                                     (O.EOS_VDW, 0.9, 0.3)])
def test_pressure_inverts_the_textbook_energy(eos, a, b):
    """The oracle's flux carries p(rho, rho e) (Sec. 2.1 leaves the EOS
    generic). Built from states whose energy comes from the textbook caloric
    relation, its pressure is the pressure the state was built with."""
    rng = np.random.default_rng(31)
    for _ in range(200):
        rho = rng.uniform(0.2, 2.0)
        u, v = rng.uniform(-0.6, 0.6, 2)
        p = rng.uniform(0.2, 3.0)
        E = _textbook_rho_e(eos, a, b, rho, p) + 0.5 * rho * (u * u + v * v)
        W = np.array([rho, rho * u, rho * v, E])
        qx, qy = O.flux(W, GAMMA, eos, a, b)
        assert qx[1] - rho * u * u == pytest.approx(p, rel=1e-12, abs=1e-12)
        assert qy[2] - rho * v * v == pytest.approx(p, rel=1e-12, abs=1e-12)


def test_planted_van_der_waals_sign_slip_fails_the_energy_pin():
    O.set_function_mutation(O.FMUT_VDW_SIGN)
    try:
        with pytest.raises(AssertionError):
            test_pressure_inverts_the_textbook_energy(O.EOS_VDW, 0.2, 0.05)
    finally:
        O.set_function_mutation(O.FMUT_NONE)
    test_pressure_inverts_the_textbook_energy(O.EOS_VDW, 0.2, 0.05)


# ------------------------------------------------ specular wall (method of images)
def _mirror(U, axis):
    """Mirror image of a state across the high side of `axis` (2: x, 1: y):
    the order of the cells reverses and the normal momentum changes sign."""
    M = np.flip(U, axis=axis).copy()
    M[1 if axis == 2 else 2] *= -1.0
    return M


def _mirror_box(box, N, axis):
    l, i0, j0, nx, ny = box
    if axis == 2:
        return (l, N - i0 - nx, j0, nx, ny)
    return (l, i0, N - j0 - ny, nx, ny)


def _wall_vs_images(axis, mut=O.MUT_NONE, steps=6):
    """Run a box with reflecting sides normal to `axis` and, separately, the
    periodic box of twice the length holding the state and its mirror image.
    Returns the largest difference over the original half, every level."""
    nx0, ny0, r = (12, 8, 2) if axis == 2 else (8, 12, 2)
    if axis == 2:   # patches touching both walls span the periodic direction
        boxes = [(1, 0, 0, 6, 16), (1, 18, 0, 6, 16), (1, 10, 4, 4, 6)]
        bc = (O.REFLECT, O.REFLECT, O.PERIODIC, O.PERIODIC)
    else:
        boxes = [(1, 0, 0, 16, 6), (1, 0, 18, 16, 6), (1, 4, 10, 6, 4)]
        bc = (O.PERIODIC, O.PERIODIC, O.REFLECT, O.REFLECT)
    U0 = wl.random_state_U(nx0, ny0, seed=3)
    U1 = wl.random_smooth_U(nx0 * r, ny0 * r, seed=4)
    c, beta = 4.0, 0.8

    wall = O.Oracle(nx0, ny0, 1.0 / 16, r, 2, GAMMA, c, beta, bc)
    wall.set_mutation(mut)
    wall.set_boxes(boxes)
    wall.set_state(0, U0)
    wall.set_state(1, U1)
    wall.advance(steps)

    big = (2 * nx0, ny0) if axis == 2 else (nx0, 2 * ny0)
    N1 = (big[0] if axis == 2 else big[1]) * r
    img_boxes = list(boxes) + [_mirror_box(b, N1, axis) for b in boxes]
    per = O.Oracle(big[0], big[1], 1.0 / 16, r, 2, GAMMA, c, beta, (O.PERIODIC,) * 4)
    per.set_boxes(img_boxes)
    per.set_state(0, np.concatenate([U0, _mirror(U0, axis)], axis=axis))
    per.set_state(1, np.concatenate([U1, _mirror(U1, axis)], axis=axis))
    per.advance(steps)

    worst = 0.0
    for l in range(2):
        Fw = wall.get_pop(l)
        n = Fw.shape[axis]
        Fp = per.get_pop(l)
        Fp = Fp[:, :, :n] if axis == 2 else Fp[:, :n, :]
        both = np.isnan(Fw) & np.isnan(Fp)
        assert np.array_equal(np.isnan(Fw), np.isnan(Fp))
        d = np.where(both, 0.0, np.abs(Fw - Fp))
        worst = max(worst, float(d.max()))
    return worst


@pytest.mark.parametrize("axis", [2, 1])
def test_reflecting_sides_equal_the_mirrored_periodic_run(axis):
    """Method of images: a box with specular walls (reflecting sides as in
    Sec. 4.2) evolves exactly like its half of a periodic box twice as long
    that holds the state and its mirror image (normal momentum negated), with
    refinement patches touching both walls. Across x the mirror swaps f_+x and
    f_-x, the first pair of the density sum ((f_+x + f_-x) + f_+y) + f_-y, so
    the two runs agree bit for bit; across y it swaps the last two terms,
    which reorders the rounding (agreement to round-off)."""
    worst = _wall_vs_images(axis)
    if axis == 2:
        assert worst == 0.0
    else:
        assert worst < 1e-13, worst


@pytest.mark.parametrize("axis", [2, 1])
def test_planted_wall_without_momentum_flip_fails_the_images(axis):
    assert _wall_vs_images(axis, O.MUT_WALL_NO_FLIP) > 1e-3


# ------------------------------------------------ adaptive relaxation (eq. sensor-B)
TWO_PI = 2.0 * np.pi


def _field(x, y):
    """Smooth periodic primitive field on [0,1]^2 (numpy, real or complex)."""
    rho = 1.0 + 0.3 * np.sin(TWO_PI * x) * np.sin(TWO_PI * y)
    u = 0.4 * np.sin(TWO_PI * x) * np.cos(TWO_PI * y) + 0.1
    v = 0.2 * np.cos(TWO_PI * x) * np.sin(TWO_PI * y) + 0.1 * np.sin(TWO_PI * x)
    p = 1.0 + 0.2 * np.cos(TWO_PI * (x + y))
    return rho, u, v, p


def _flux_of(x, y):
    rho, u, v, p = _field(x, y)
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)
    Qx = [rho * u, rho * u * u + p, rho * u * v, (E + p) * u]
    Qy = [rho * v, rho * u * v, rho * v * v + p, (E + p) * v]
    return Qx, Qy, u, v


def _d(f, x, y, axis, h=1e-30):
    """Complex-step derivative of the analytic field function f along axis."""
    if axis == 0:
        return np.imag(f(x + 1j * h, y)) / h
    return np.imag(f(x, y + 1j * h)) / h


def _analytic_sensor(n, C):
    """s_k = dx (div Q)_k / max|Q_k| with exact derivatives, the RMS over the
    four components, its mean over the 3 x 3 block (box filter), and the
    Ducros-type ratio theta = dil^2 / (dil^2 + vort^2) under compression.
    Returns z = clip(C sbar theta, 0, 1) per cell."""
    dx = 1.0 / n
    xc = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(xc, xc)
    Qx, Qy, u, v = _flux_of(X, Y)
    s = []
    for k in range(4):
        qmax = max(np.abs(Qx[k]).max(), np.abs(Qy[k]).max())
        div = _d(lambda a, b: _flux_of(a, b)[0][k], X, Y, 0) + _d(lambda a, b: _flux_of(a, b)[1][k], X, Y, 1)
        s.append(dx * div / qmax)
    a = np.sqrt(0.25 * sum(sk * sk for sk in s))
    sbar = sum(np.roll(np.roll(a, dy, 0), dxx, 1) for dy in (-1, 0, 1) for dxx in (-1, 0, 1)) / 9.0
    ux = _d(lambda a_, b_: _field(a_, b_)[1], X, Y, 0)
    uy = _d(lambda a_, b_: _field(a_, b_)[1], X, Y, 1)
    vx = _d(lambda a_, b_: _field(a_, b_)[2], X, Y, 0)
    vy = _d(lambda a_, b_: _field(a_, b_)[2], X, Y, 1)
    dil, vort = dx * (ux + vy), dx * (vx - uy)
    theta = np.where(dil < 0.0, dil * dil / (dil * dil + vort * vort), 0.0)
    return np.clip(C * sbar * theta, 0.0, 1.0)


def _oracle_sensor_z(n, C, bmin, bmax, mut=O.MUT_NONE):
    dx = 1.0 / n
    xc = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(xc, xc)
    rho, u, v, p = _field(X, Y)
    U = wl.conserved(rho, u, v, p, GAMMA)
    o = O.Oracle(n, n, dx, 2, 1, GAMMA, 5.0, 0.8, (O.PERIODIC,) * 4)
    o.set_mutation(mut)
    o.set_boxes([])
    o.set_state(0, U)
    o.set_sensor(True, C, bmin, bmax)
    o.advance(1)
    beta = o.get_beta(0)
    return (bmax - beta) / (bmax - bmin)


def _sensor_error(mut=O.MUT_NONE, n=128, C=6.0):
    z_ref = _analytic_sensor(n, C)
    assert 0.2 < z_ref.max() < 0.9 and (z_ref == 0).any()  # unsaturated, gated somewhere
    z = _oracle_sensor_z(n, C, 0.4, 0.9, mut)
    return float(np.abs(z - z_ref).max()), float(z_ref.max())


def test_sensor_matches_analytic_derivatives():
    """eq. sensor-B on a smooth analytic field: the oracle's beta, from its
    central differences, matches beta built from exact derivatives (complex
    step) to the O(dx^2) truncation error of the differences (n = 128:
    relative error about (2 pi / n)^2 / 6 = 4e-4)."""
    err, zmax = _sensor_error()
    assert err < 3e-3 * zmax, err


@pytest.mark.parametrize("mut", [O.MUT_SENSOR_BOX_SUM, O.MUT_SENSOR_MAX_NORM])
def test_planted_sensor_mistakes_fail_the_analytic_pin(mut):
    err, zmax = _sensor_error(mut)
    assert err > 3e-2 * zmax, (mut, err)


# ------------------------------------------------ density-gradient tags (2-D)
def _tag_reference_2d(rho, act, bc):
    """max over axes of |rho(+1) - rho(-1)| / (2 rho), a missing or inactive
    neighbour replaced by the cell itself (numpy, from the held density)."""
    g = np.zeros_like(rho)
    for axis, (lo, hi) in ((1, (bc[0], bc[1])), (0, (bc[2], bc[3]))):
        per = lo == O.PERIODIC
        plus, minus = np.roll(rho, -1, axis), np.roll(rho, 1, axis)
        ap, am = np.roll(act, -1, axis), np.roll(act, 1, axis)
        if not per:
            idx = [slice(None)] * 2
            idx[axis] = -1
            ap[tuple(idx)] = False
            idx[axis] = 0
            am[tuple(idx)] = False
        plus = np.where(ap, plus, rho)
        minus = np.where(am, minus, rho)
        g = np.maximum(g, np.abs(plus - minus) / (2.0 * rho))
    return np.where(act, g, 0.0)


def _tag_case(bc, mut=O.MUT_NONE):
    nx0, ny0 = 20, 14
    U0 = wl.random_smooth_U(nx0, ny0, seed=11, amp=0.3)
    o = O.Oracle(nx0, ny0, 1.0 / 20, 2, 2, GAMMA, 4.0, 0.8, bc)
    o.set_mutation(mut)
    o.set_boxes([(1, 10, 6, 12, 10)])
    o.set_state(0, U0)
    o.set_state(1, wl.random_smooth_U(2 * nx0, 2 * ny0, seed=12, amp=0.3))
    o.advance(2)
    ok = True
    for l in range(2):
        act = o.active_mask(l)
        rho = o.get_state(l)[0]
        g = _tag_reference_2d(np.where(act, rho, 1.0), act, bc)
        vals = np.unique(np.round(g[act], 12))
        for qq in (0.3, 0.6, 0.85):
            k = int(qq * (len(vals) - 1))
            thr = 0.5 * (vals[k] + vals[k + 1])
            t = o.tag(l, thr).astype(bool)
            assert not t[~act].any()
            ok &= np.array_equal(t, act & (g > thr))
    return ok


@pytest.mark.parametrize("bc", [(O.PERIODIC,) * 4, (O.OUTFLOW, O.REFLECT, O.PERIODIC, O.PERIODIC),
                                (O.REFLECT, O.REFLECT, O.OUTFLOW, O.INFLOW)])
def test_2d_tags_match_central_differences(bc):
    """The refinement tag (density-gradient reading of eq. amr-sigma) equals
    numpy's central differences of the density the oracle holds, thresholded,
    on both levels: holes carry no tag, and a neighbour that is inactive, in
    the other level or outside a non-periodic side, is replaced by the cell."""
    assert _tag_case(bc)


def test_planted_one_sided_tag_fails_the_numpy_pin():
    assert not _tag_case((O.PERIODIC,) * 4, O.MUT_TAG_ONE_SIDED)


# ------------------------------------------------ temporal history across a regrid
def _same_boxes_regrid(mut=O.MUT_NONE):
    n = 16
    U = wl.random_smooth_U(n, n, seed=5)
    case = wl.Case("t", n, n, 1.0 / n, 2, 3, GAMMA, 4.0, 0.8, (1, 1, 2, 2),
                   [(1, 8, 8, 12, 12), (2, 20, 20, 8, 8)],
                   [U, wl.prolong_piecewise(U, 2), wl.prolong_piecewise(U, 4)], 0)
    a = exact.run_oracle(case, 4)
    a.set_mutation(mut)
    a.regrid(case.boxes)
    a.advance(3)
    c = exact.run_oracle(case, 7)
    return all(np.array_equal(a.get_pop(l), c.get_pop(l), equal_nan=True) for l in range(3))


def test_planted_restart_of_every_interface_fails_the_same_box_pin():
    """The former reading (a regrid restarts the temporal reconstruction of
    every interface) modifies eq. 1d-recon at interfaces the regrid keeps."""
    assert _same_boxes_regrid()
    assert not _same_boxes_regrid(O.MUT_REGRID_RESTART_ALL)


def _new_patch_matches_restart(mut=O.MUT_NONE):
    n = 32
    U = wl.random_smooth_U(n, n, seed=9)
    B1, B2 = (1, 4, 4, 12, 12), (1, 40, 40, 12, 12)
    case = wl.Case("t", n, n, 1.0 / n, 2, 2, GAMMA, 4.0, 0.8, (0,) * 4, [B1],
                   [U, wl.prolong_piecewise(U, 2)], 0)
    a = exact.run_oracle(case, 4)
    a.set_mutation(mut)
    a.regrid([B1, B2])
    post = [np.nan_to_num(a.get_pop(l)) for l in range(2)]
    a.advance(1)
    case2 = wl.Case("t", n, n, 1.0 / n, 2, 2, GAMMA, 4.0, 0.8, (0,) * 4, [B1, B2],
                    [U, wl.prolong_piecewise(U, 2)], 0)
    ref = exact.run_oracle(case2, 0)
    for l in range(2):
        ref.set_pop(l, post[l])
    ref.advance(1)
    s2 = np.s_[:, 40:52, 40:52]
    return np.array_equal(a.get_pop(1)[s2], ref.get_pop(1)[s2])


def test_planted_history_on_new_interfaces_fails_the_new_patch_pin():
    """An interface the regrid creates has no older sample on its face: using
    the ring cell's own previous value there changes the new patch's first
    coarse step (the unmutated rule matches a restart there, bit for bit)."""
    assert _new_patch_matches_restart()
    assert not _new_patch_matches_restart(O.MUT_REGRID_NEW_FACE_HISTORY)


# ------------------------------------------------ refinement sensor (eq. amr-sigma)
def _analytic_flux_sensor(n):
    """max_k |dx (div Q)_k / max|Q_k|| with exact derivatives (complex step)."""
    dx = 1.0 / n
    xc = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(xc, xc)
    Qx, Qy, _, _ = _flux_of(X, Y)
    s = []
    for k in range(4):
        qmax = max(np.abs(Qx[k]).max(), np.abs(Qy[k]).max())
        div = _d(lambda a, b: _flux_of(a, b)[0][k], X, Y, 0) + _d(lambda a, b: _flux_of(a, b)[1][k], X, Y, 1)
        s.append(np.abs(dx * div / qmax))
    return np.max(s, axis=0)


def _oracle_flux_sensor(n, mut=O.MUT_NONE):
    dx = 1.0 / n
    xc = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(xc, xc)
    o = O.Oracle(n, n, dx, 2, 1, GAMMA, 5.0, 0.8, (O.PERIODIC,) * 4)
    o.set_mutation(mut)
    o.set_boxes([])
    o.set_state(0, wl.conserved(*_field(X, Y), GAMMA))
    return o.flux_sensor(0)


def test_flux_sensor_matches_analytic_derivatives():
    """eq. amr-sigma on a smooth analytic field: the oracle's s (central
    differences, the domain-wide max of |Q_k|, the max norm over k) matches s
    from exact derivatives to the differences' O(dx^2) truncation."""
    s_ref = _analytic_flux_sensor(128)
    s = _oracle_flux_sensor(128)
    assert np.max(np.abs(s - s_ref)) < 3e-3 * s_ref.max()


def test_planted_rms_flux_sensor_fails_the_analytic_pin():
    s_ref = _analytic_flux_sensor(128)
    s = _oracle_flux_sensor(128, O.MUT_FLUX_SENSOR_RMS)
    assert np.max(np.abs(s - s_ref)) > 5e-2 * s_ref.max()


def test_flux_sensor_and_tags_match_numpy_on_two_levels():
    """Two levels with a wall and an outflow side: s on each level equals numpy's
    central differences of the Euler flux of the held state, with the max of
    |Q_k| over the active cells of both levels, inactive neighbours replaced by
    the cell; tags are s above the threshold on active cells only."""
    nx0, ny0 = 24, 18
    bc = (O.REFLECT, O.OUTFLOW, O.PERIODIC, O.PERIODIC)
    o = O.Oracle(nx0, ny0, 1.0 / 24, 2, 2, GAMMA, 4.0, 0.8, bc)
    o.set_boxes([(1, 12, 8, 16, 20)])
    o.set_state(0, wl.random_smooth_U(nx0, ny0, seed=13, amp=0.3))
    o.set_state(1, wl.random_smooth_U(2 * nx0, 2 * ny0, seed=14, amp=0.3))
    o.advance(2)
    acts = [o.active_mask(l) for l in range(2)]
    Us = [o.get_state(l) for l in range(2)]
    qmax = np.zeros(4)
    for U, act in zip(Us, acts):
        Fx, Fy = exact.euler_flux(np.where(act, U, 1.0), GAMMA)
        qmax = np.maximum(qmax, np.max(np.where(act, np.maximum(np.abs(Fx), np.abs(Fy)), 0.0), axis=(1, 2)))
    for l in range(2):
        act, U = acts[l], np.where(acts[l], Us[l], 1.0)
        Fx, Fy = exact.euler_flux(U, GAMMA)

        def nb(F, axis, shift, per):
            G = np.roll(F, shift, axis=axis + 1)
            a = np.roll(act, shift, axis=axis)
            if not per:
                idx = [slice(None)] * 2
                idx[axis] = 0 if shift == 1 else -1
                a[tuple(idx)] = False
            return np.where(a, G, F)

        div = (nb(Fx, 1, -1, False) - nb(Fx, 1, 1, False)) + (nb(Fy, 0, -1, True) - nb(Fy, 0, 1, True))
        s_np = np.where(act, np.max(np.abs(0.5 * div / qmax[:, None, None]), axis=0), 0.0)
        s = o.flux_sensor(l)
        assert np.allclose(s, s_np, rtol=1e-11, atol=1e-14), l
        thr = np.quantile(s[act], 0.7)
        assert np.array_equal(o.tag_flux(l, thr).astype(bool), act & (s > thr))
