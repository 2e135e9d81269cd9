"""Pins of the three-dimensional (D3Q6) FP64 oracle against what the paper and
the mathematics fix. CPU only; each test names the passage it follows."""
import numpy as np
import pytest

from oracle import oracle3 as O3
from tests import exact

RNG = np.random.default_rng(2026)


def _random_W(n, rng):
    rho = rng.uniform(0.3, 2.5, n)
    u, v, w = (rng.uniform(-1.2, 1.2, n) for _ in range(3))
    p = rng.uniform(0.2, 2.5, n)
    return _cons(rho, u, v, w, p).T


def _cons(rho, u, v, w, p, gamma=1.4):
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def _random_state(nz, ny, nx, rng, amp=0.15):
    """A smooth-ish random state: a uniform base plus low modes and noise."""
    z, y, x = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")
    f = lambda a, b, c: np.sin(2 * np.pi * (a * x + b * y + c * z) + rng.uniform(0, 6.3))
    rho = 1.0 + amp * f(1, 0, 1) + 0.02 * rng.normal(size=x.shape)
    u = 0.3 * f(0, 1, 1)
    v = -0.2 * f(1, 1, 0)
    w = 0.25 * f(1, 0, 0)
    p = 1.0 + amp * f(0, 1, 0)
    return _cons(rho, u, v, w, p)


def _prolong(U, r):
    return U.repeat(r, axis=1).repeat(r, axis=2).repeat(r, axis=3)


def _oracle(U0, nlev=1, boxes=(), r=2, c=4.0, beta=0.8, bc=(0,) * 6, fine=None, mut=O3.MUT_NONE):
    nz, ny, nx = U0.shape[1:]
    o = O3.Oracle3(nx, ny, nz, 1.0 / nx, r=r, nlev=nlev, c=c, beta=beta, bc=bc)
    o.set_mutation(mut)
    o.set_boxes(boxes)
    o.set_state(0, U0)
    for l in range(1, nlev):
        o.set_state(l, fine[l - 1] if fine else _prolong(U0, r ** l))
    return o


# ----------------------------------------------------------- single cell (Sec. 2.2)
def test_equilibrium_moments_and_flux():
    """sum_i f_i^eq = W and sum_i c_i f_i^eq = Q(W) with W/(2D), D = 3
    (eq. num-equilibrium); Q is the textbook 3-D Euler flux."""
    c = 2.7
    for W in _random_W(40, RNG):
        f = O3.feq(W, 1.4, c)
        assert np.allclose(f.sum(axis=0), W, rtol=0, atol=8e-16 * np.abs(W).max())
        Q = O3.flux(W)
        for a in range(3):
            assert np.allclose(c * (f[2 * a] - f[2 * a + 1]), Q[a], rtol=0,
                               atol=8e-16 * c * np.abs(Q).max())
        rho, mx, my, mz, E = W
        u, v, w = mx / rho, my / rho, mz / rho
        p = 0.4 * (E - 0.5 * rho * (u * u + v * v + w * w))
        want = np.array([[mx, mx * u + p, my * u, mz * u, (E + p) * u],
                         [my, mx * v, my * v + p, mz * v, (E + p) * v],
                         [mz, mx * w, my * w, mz * w + p, (E + p) * w]])
        assert np.allclose(Q, want, rtol=1e-14, atol=1e-14)


def test_collision_conserves_and_special_betas():
    """Relaxation conserves W for any beta; beta = 1/2 gives f^eq, 0 the identity
    (eq. num-relaxation)."""
    for _ in range(50):
        W = _random_W(1, RNG)[0]
        g = O3.feq(W, 1.4, 3.0) + RNG.normal(0, 0.03, (6, 5))
        Wg = g.sum(axis=0)
        b = RNG.uniform(0.0, 1.0)
        assert np.allclose(O3.collide(g, 1.4, 3.0, b).sum(axis=0), Wg, rtol=0,
                           atol=4e-15 * (np.abs(g).sum(axis=0) + 1))
    assert np.array_equal(O3.collide(g, 1.4, 3.0, 0.0), g)
    assert np.allclose(O3.collide(g, 1.4, 3.0, 0.5), O3.feq(g.sum(axis=0), 1.4, 3.0), atol=1e-15)


# ----------------------------------------------------------- streaming (Sec. 2.2)
def test_streaming_is_an_exact_shift():
    """beta = 0: one step shifts each population one cell along its axis; N
    steps on a periodic N^3 grid return every value bitwise."""
    n = 6
    o = O3.Oracle3(n, n, n, 1.0 / n, nlev=1, c=2.0, beta=0.0)
    F0 = RNG.normal(1.0, 0.1, (30, n, n, n))
    o.set_pop(0, F0)
    o.advance(1)
    F1 = o.get_pop(0)
    for q, (axis, s) in enumerate([(3, 1), (3, -1), (2, 1), (2, -1), (1, 1), (1, -1)]):
        for k in range(5):
            assert np.array_equal(F1[q * 5 + k], np.roll(F0[q * 5 + k], s, axis=axis - 1))
    o.advance(n - 1)
    assert np.array_equal(o.get_pop(0), F0)


def _lax_friedrichs_3d(U, c, gamma=1.4):
    rho, mx, my, mz, E = U
    u, v, w = mx / rho, my / rho, mz / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w))
    F = [np.stack([mx, mx * u + p, my * u, mz * u, (E + p) * u]),
         np.stack([my, mx * v, my * v + p, mz * v, (E + p) * v]),
         np.stack([mz, mx * w, my * w, mz * w + p, (E + p) * w])]
    avg = sum(np.roll(U, s, axis=ax) for ax in (1, 2, 3) for s in (1, -1)) / 6.0
    div = sum(np.roll(F[a], -1, axis=3 - a) - np.roll(F[a], 1, axis=3 - a) for a in range(3))
    return avg - div / (2.0 * c)


def test_beta_half_is_lax_friedrichs_3d():
    """beta = 1/2: f* = f^eq(W) and one step is the 3-D Lax-Friedrichs scheme
    with dt/dx = 1/c (eqs. num-equilibrium, num-relaxation)."""
    n, c = 8, 3.0
    U = _random_state(n, n, n, RNG)
    o = _oracle(U, c=c, beta=0.5)
    W = U.copy()
    for _ in range(5):
        o.advance(1)
        W = _lax_friedrichs_3d(W, c)
    assert np.allclose(o.get_state(0), W, rtol=0, atol=2e-13)


# ----------------------------------------------------------- refinement (Sec. 3)
BOX = [(1, 4, 4, 2, 8, 6, 8)]  # level-1 cells x 4..11, y 4..9, z 2..9 of 16 x 16 x 12


def test_uniform_flow_is_preserved_through_a_patch():
    n = (6, 8, 8)  # nz, ny, nx
    U = _cons(*(np.full(n, v) for v in (1.3, 0.4, -0.3, 0.2, 0.9)))
    o = _oracle(U, nlev=2, boxes=BOX, c=4.0, beta=0.9)
    o.advance(6)
    for l in range(2):
        S = o.get_state(l)
        m = o.active_mask(l)
        assert np.allclose(S[:, m], U[:, :1, :1, :1].reshape(5, 1), rtol=0, atol=2e-14)


def _conservation_drift(beta, c, mut=O3.MUT_NONE):
    U = _random_state(6, 8, 8, np.random.default_rng(77), amp=0.3)
    o = _oracle(U, nlev=2, boxes=BOX, c=c, beta=beta, mut=mut)
    T0, _ = o.totals()
    o.advance(8)
    T1, _ = o.totals()
    scale = np.abs(T0) + 1e-3 * np.abs(T0).max()
    return float(np.max(np.abs(T1 - T0) / scale))


@pytest.mark.parametrize("beta,c", [(0.6, 4.0), (0.95, 6.0)])
def test_conservation_periodic_two_interfaces(beta, c):
    """Totals stay constant to round-off across a refined patch for any beta and c
    (Sec. 3.3, exact conservation of the coupling, one face at a time)."""
    assert _conservation_drift(beta, c) < 2e-14


def test_planted_r2_reflux_weight_breaks_conservation():
    """The reflux averages r^2 face cells over r sub-steps (weight 1 / r^3);
    the 2-D weight 1 / r^2 does not conserve in 3-D."""
    assert _conservation_drift(0.6, 4.0, O3.MUT_REFLUX_R2) > 1e-6


@pytest.mark.parametrize("bc", [(1,) * 6, (2,) * 6, (0, 0, 1, 1, 2, 2)])
def test_boundary_ledger_balances(bc):
    """Non-periodic sides: T(t) - T(0) equals the ledger of what crossed them."""
    U = _random_state(6, 8, 8, RNG, amp=0.3)
    o = _oracle(U, nlev=2, boxes=[(1, 0, 4, 2, 8, 6, 8)], c=4.0, beta=0.8, bc=bc)
    T0, L0 = o.totals()
    o.advance(6)
    T1, L1 = o.totals()
    scale = np.abs(T0).max()
    assert np.all(np.abs((T1 - T0) - (L1 - L0)) <= 1e-14 * scale)


def test_ratio_one_patch_is_the_uniform_grid_bitwise():
    """r = 1: the hand-off returns the coarse value (a_k = b_j = 0) and the
    reflux the fine value itself, so a partial patch changes nothing, bit for bit."""
    U = _random_state(6, 8, 8, RNG, amp=0.3)
    a = _oracle(U, nlev=1, r=1, c=4.0, beta=0.8)
    b = _oracle(U, nlev=2, r=1, boxes=[(1, 2, 1, 1, 4, 5, 3)], c=4.0, beta=0.8, fine=[U])
    a.advance(5)
    b.advance(5)
    Fa = a.get_pop(0)
    Fb0, Fb1 = b.get_pop(0), b.get_pop(1)
    m1 = b.active_mask(1)
    assert m1.sum() == 4 * 5 * 3
    assert np.array_equal(Fa[:, ~m1], Fb0[:, ~m1])
    assert np.array_equal(Fa[:, m1], Fb1[:, m1])


@pytest.mark.parametrize("shift", [3, 5])
def test_periodic_translation_equivariance(shift):
    """Translating state and boxes by whole coarse cells along x (periodic)
    translates the result bit for bit: the patch wraps across the seam."""
    U = _random_state(6, 8, 8, RNG, amp=0.3)
    boxes = [(1, 10, 4, 2, 6, 6, 8)]
    a = _oracle(U, nlev=2, boxes=boxes, c=4.0, beta=0.8)
    Us = np.roll(U, shift, axis=3)
    b = _oracle(Us, nlev=2, boxes=[(1, (10 + 2 * shift) % 16, 4, 2, 6, 6, 8)], c=4.0, beta=0.8)
    if (10 + 2 * shift) % 16 + 6 > 16:
        pytest.skip("shifted box would cross the seam")
    a.advance(4)
    b.advance(4)
    for l, s in ((0, shift), (1, 2 * shift)):
        assert np.array_equal(np.roll(a.get_pop(l), s, axis=3), b.get_pop(l), equal_nan=True), l


def test_axis_permutation_equivariance():
    """Relabelling the axes (x, y, z) -> (y, z, x), with momenta and boxes,
    relabels the result (to round-off: the sums over populations run in
    another order)."""
    U = _random_state(8, 8, 8, RNG, amp=0.3)
    box = (1, 4, 6, 2, 8, 6, 10)  # (level, i0, j0, k0, nx, ny, nz)
    a = _oracle(U, nlev=2, boxes=[box], c=4.0, beta=0.8)
    # new axes: x' = y, y' = z, z' = x; arrays are [k][z][y][x]
    Up = np.transpose(U, (0, 3, 1, 2))[[0, 2, 3, 1, 4]]
    boxp = (1, box[2], box[3], box[1], box[5], box[6], box[4])
    b = _oracle(Up, nlev=2, boxes=[boxp], c=4.0, beta=0.8)
    a.advance(4)
    b.advance(4)
    for l in range(2):
        Sa = a.get_state(l)
        Sb = b.get_state(l)
        Sa_p = np.transpose(Sa, (0, 3, 1, 2))[[0, 2, 3, 1, 4]]
        assert np.array_equal(np.isnan(Sa_p), np.isnan(Sb))
        m = ~np.isnan(Sb)
        assert np.allclose(Sa_p[m], Sb[m], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_tangentially_linear_handoff_is_exact(axis):
    """beta = 0 (pure transport), the populations along `axis` linear in the two
    tangential coordinates and constant along `axis`, the others constant: the
    fine level keeps the linear field exactly, so both tangential slopes of the
    hand-off (eqs. 2d-recon-tanslope, 2d-recon, one per tangential axis) enter
    with the right sign and offset on both faces normal to `axis`."""
    assert _linear_handoff_error(axis) <= 2e-15


@pytest.mark.parametrize("mut", [O3.MUT_TAN_SLOPE_SIGN, O3.MUT_TAN_OFFSETS_SWAPPED])
def test_planted_handoff_mistakes_break_the_linear_field(mut):
    assert _linear_handoff_error(0, mut) > 1e-3


def _linear_handoff_error(axis, mut=O3.MUT_NONE):
    n = 8
    r = 2
    co = (np.arange(n) + 0.5) / n
    cf = (np.arange(n * r) + 0.5) / (n * r)
    t = [a for a in range(3) if a != axis]
    slope = {t[0]: 0.7, t[1]: -0.4}

    def field(coords):  # coords: (z, y, x) meshes
        val = 1.0
        for a in t:
            val = val + slope[a] * coords[2 - a]
        return val

    Zc, Yc, Xc = np.meshgrid(co, co, co, indexing="ij")
    Zf, Yf, Xf = np.meshgrid(cf, cf, cf, indexing="ij")
    F0 = np.full((30, n, n, n), 0.5)
    F1 = np.full((30, n * r, n * r, n * r), 0.5)
    for q in (2 * axis, 2 * axis + 1):
        for k in range(5):
            F0[q * 5 + k] = field((Zc, Yc, Xc)) * (1 + 0.1 * k)
            F1[q * 5 + k] = field((Zf, Yf, Xf)) * (1 + 0.1 * k)
    o = O3.Oracle3(n, n, n, 1.0 / n, r=r, nlev=2, c=2.0, beta=0.0, bc=(1,) * 6)
    o.set_mutation(mut)
    o.set_boxes([(1, 4, 4, 4, 8, 8, 8)])
    o.set_pop(0, F0)
    o.set_pop(1, F1)
    o.advance(2)
    G = o.get_pop(1)
    m = o.active_mask(1)
    err = 0.0
    for q in (2 * axis, 2 * axis + 1):
        for k in range(5):
            err = max(err, float(np.abs(G[q * 5 + k][m] - F1[q * 5 + k][m]).max()))
    return err


def _sod_l1(n, axis):
    """Sod along `axis` on n x 4 x 4 cells, c = 7.8125 (t = 0.2 after 0.2 c n
    steps); returns the L1 density error and the profile."""
    shape = [4, 4, 4]
    shape[2 - axis] = n
    coord = (np.arange(n) + 0.5) / n
    x = coord.reshape([-1 if i == 2 - axis else 1 for i in range(3)]) * np.ones(shape)
    z0 = np.zeros(shape)
    U = _cons(np.where(x < 0.5, 1.0, 0.125), z0, z0, z0, np.where(x < 0.5, 1.0, 0.1))
    bc = [0] * 6
    bc[2 * axis] = bc[2 * axis + 1] = 1
    c = 7.8125
    o = O3.Oracle3(shape[2], shape[1], shape[0], 1.0 / n, nlev=1, c=c, beta=0.9, bc=tuple(bc))
    o.set_state(0, U)
    steps = int(round(0.2 * c * n))
    o.advance(steps)
    t = steps / (c * n)
    line = np.moveaxis(o.get_state(0)[0], 2 - axis, 0).reshape(n, -1)
    assert np.allclose(line, line[:, :1])  # uniform across the other two axes
    rho_ex = exact.riemann_exact(np.array([1.0, 0.0, 1.0]), np.array([0.125, 0.0, 0.1]),
                                 (coord - 0.5) / t)[0]
    return float(np.mean(np.abs(line[:, 0] - rho_ex))), line[:, 0]


def test_sod_along_each_axis_converges_and_agrees():
    """The 1-D Sod problem carried along x, y or z: the L1 density error
    against the exact Riemann solution falls with resolution, and the three
    orientations give the same profile (to round-off)."""
    e64, l64 = _sod_l1(64, 0)
    e128, _ = _sod_l1(128, 0)
    assert e128 < 0.75 * e64
    for axis in (1, 2):
        e, l = _sod_l1(64, axis)
        assert np.allclose(l, l64, rtol=0, atol=1e-12)


# ----------------------------------------------------------- regrid (Sec. 3.4)
def test_regrid_conserves_through_moves_and_removal():
    """Merges (eq. amr-merge, r^3 children) and splits (eqs. amr-slope,
    amr-split, one slope per axis) conserve the totals exactly, through a
    moved level-1 box, a new level-2 box and its removal."""
    U = _random_state(6, 8, 8, RNG, amp=0.3)
    o = _oracle(U, nlev=3, boxes=[(1, 4, 4, 2, 8, 6, 8)], c=4.0, beta=0.8)
    o.advance(2)
    seq = [[(1, 6, 4, 4, 8, 8, 6)],
           [(1, 4, 2, 2, 10, 10, 8), (2, 12, 8, 8, 8, 8, 8)],
           [(1, 0, 0, 0, 6, 6, 6)]]
    T, _ = o.totals()
    for boxes in seq:
        o.regrid(boxes)
        T1, _ = o.totals()
        assert np.allclose(T1, T, rtol=1e-14, atol=1e-14 * np.abs(T).max()), boxes
        o.advance(2)
        T, _ = o.totals()


def _merge_of_split_error(mut=O3.MUT_NONE):
    U = _random_state(6, 8, 8, np.random.default_rng(78), amp=0.3)
    o = _oracle(U, nlev=2, boxes=[], c=4.0, beta=0.8, mut=mut)
    F0 = o.get_pop(0)
    o.regrid([(1, 4, 4, 2, 8, 6, 8)])
    o.regrid([])
    F1 = o.get_pop(0)
    return float(np.abs(F1 - F0).max() / np.abs(F0).max())


def test_merge_of_split_returns_the_parent():
    """Splitting a block into r^3 children and merging them back returns the
    parent to round-off (the offsets sum to zero along every axis)."""
    assert _merge_of_split_error() <= 8e-16


def test_planted_r2_merge_weight_fails_the_round_trip():
    assert _merge_of_split_error(O3.MUT_MERGE_R2) > 0.1


def _same_box_regrid(mut=O3.MUT_NONE):
    """(regrid-then-run equals run-on, a restart from the same populations differs)"""
    U = _random_state(6, 8, 8, np.random.default_rng(79), amp=0.3)
    boxes = [(1, 4, 4, 2, 8, 6, 8)]
    a = _oracle(U, nlev=2, boxes=boxes, c=4.0, beta=0.8, mut=mut)
    b = _oracle(U, nlev=2, boxes=boxes, c=4.0, beta=0.8)
    a.advance(3)
    b.advance(3)
    F = [a.get_pop(l) for l in range(2)]
    fresh = O3.Oracle3(8, 8, 6, 1.0 / 8, r=2, nlev=2, c=4.0, beta=0.8)
    fresh.set_boxes(boxes)
    for l in range(2):
        fresh.set_pop(l, np.nan_to_num(F[l]))
    a.regrid(boxes)
    a.advance(3)
    b.advance(3)
    fresh.advance(3)
    same = all(np.array_equal(a.get_pop(l), b.get_pop(l), equal_nan=True) for l in range(2))
    restart_differs = not np.array_equal(fresh.get_pop(1), b.get_pop(1), equal_nan=True)
    return same, restart_differs


def test_regrid_to_same_boxes_changes_nothing():
    """A regrid that changes no box keeps every interface, whose reconstruction
    runs unmodified (Sec. 3.4): running on after it equals running on without
    it, bit for bit. The history matters here: a restart from the same
    populations gives another result."""
    assert _same_box_regrid() == (True, True)


def test_planted_restart_of_every_interface_fails_the_same_box_pin():
    assert _same_box_regrid(O3.MUT_REGRID_RESTART_ALL)[0] is False


def _regrid_adds_a_far_patch(mut=O3.MUT_NONE):
    """A patch added 5 coarse cells from an existing one (periodic x). After one
    coarse step the old patch's fine cells equal the run without the regrid
    (its interfaces kept their history) and the new patch's fine cells equal a
    run restarted from the regridded populations (new interfaces start flat)."""
    U = _random_state(8, 8, 16, np.random.default_rng(80), amp=0.3)
    B1, B2 = (1, 2, 4, 4, 6, 8, 8), (1, 18, 4, 4, 6, 8, 8)
    a = _oracle(U, nlev=2, boxes=[B1], c=4.0, beta=0.8, mut=mut)
    a.advance(3)
    a.regrid([B1, B2])
    post = [np.nan_to_num(a.get_pop(l)) for l in range(2)]
    a.advance(1)
    old = _oracle(U, nlev=2, boxes=[B1], c=4.0, beta=0.8)
    old.advance(4)
    new = O3.Oracle3(16, 8, 8, 1.0 / 16, r=2, nlev=2, c=4.0, beta=0.8)
    new.set_boxes([B1, B2])
    for l in range(2):
        new.set_pop(l, post[l])
    new.advance(1)
    s1, s2 = np.s_[:, 4:12, 4:12, 2:8], np.s_[:, 4:12, 4:12, 18:24]
    A = a.get_pop(1)
    return (np.array_equal(A[s1], old.get_pop(1)[s1]), np.array_equal(A[s2], new.get_pop(1)[s2]),
            not np.array_equal(A[s1], new.get_pop(1)[s1]))


def test_regrid_keeps_surviving_interfaces_and_starts_new_ones_flat():
    assert _regrid_adds_a_far_patch() == (True, True, True)


def test_planted_history_on_new_interfaces_fails_the_new_patch_pin():
    assert _regrid_adds_a_far_patch(O3.MUT_REGRID_NEW_FACE_HISTORY)[1] is False


def test_split_of_linear_populations_is_exact():
    """Populations linear in x, y and z split into children that sample the
    same linear function at their own centres (to round-off)."""
    assert _linear_split_error() <= 2e-15


def test_planted_split_slope_sign_fails_the_linear_split():
    assert _linear_split_error(O3.MUT_SPLIT_SLOPE_SIGN) > 1e-3


def _linear_split_error(mut=O3.MUT_NONE):
    n, r = 8, 2
    co = (np.arange(n) + 0.5) / n
    cf = (np.arange(n * r) + 0.5) / (n * r)
    lin = lambda Z, Y, X, i: 1.0 + 0.3 * X - 0.2 * Y + 0.1 * Z + 0.01 * i
    Zc, Yc, Xc = np.meshgrid(co, co, co, indexing="ij")
    Zf, Yf, Xf = np.meshgrid(cf, cf, cf, indexing="ij")
    F0 = np.stack([lin(Zc, Yc, Xc, i) for i in range(30)])
    o = O3.Oracle3(n, n, n, 1.0 / n, r=r, nlev=2, c=2.0, beta=0.0, bc=(1,) * 6)
    o.set_mutation(mut)
    o.set_boxes([])
    o.set_pop(0, F0)
    o.regrid([(1, 4, 4, 4, 8, 8, 8)])
    G = o.get_pop(1)
    m = o.active_mask(1)
    want = np.stack([lin(Zf, Yf, Xf, i) for i in range(30)])
    return float(np.abs(G[:, m] - want[:, m]).max())


# ------------------------------------------------ refinement tags (Sec. 3.4)
def _tag_reference(rho, active, bc):
    """Central density differences per axis with numpy: a neighbour across a
    non-periodic side or inactive stands in as the cell itself."""
    g = np.zeros_like(rho)
    for ax, (a0, a1) in zip((2, 1, 0), ((bc[0], bc[1]), (bc[2], bc[3]), (bc[4], bc[5]))):
        n = rho.shape[ax]
        side = []
        for s in (1, -1):
            nb = np.roll(rho, -s, axis=ax)
            ok = np.roll(active, -s, axis=ax)
            if a0 != 0:  # non-periodic: the wrapped neighbour does not exist
                idx = [slice(None)] * 3
                idx[ax] = n - 1 if s == 1 else 0
                ok = ok.copy()
                ok[tuple(idx)] = False
            side.append(np.where(ok, nb, rho))
        g = np.maximum(g, np.abs(side[0] - side[1]) / (2 * rho))
    return g


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bc", [(0,) * 6, (1, 1, 2, 2, 1, 2)])
def test_tags_match_central_differences(axis, bc):
    """A density wave along one axis: the oracle's tags equal numpy's central
    differences of the density it holds, thresholded; a uniform state has no
    tag."""
    nz, ny, nx = 10, 12, 14
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coord, n = [(x, nx), (y, ny), (z, nz)][axis]
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * coord / n) ** 3
    one = np.ones_like(rho)
    o = _oracle(_cons(rho, 0.1 * one, -0.2 * one, 0.05 * one, one), bc=bc)
    held = o.get_state(0)[0]
    g = _tag_reference(held, np.ones(held.shape, bool), bc)
    vals = np.unique(np.round(g, 12))
    for q in (0.3, 0.6, 0.85):  # thresholds halfway between distinct values
        k = int(q * (len(vals) - 1))
        thr = 0.5 * (vals[k] + vals[k + 1])
        assert np.min(np.abs(g - thr)) > 1e-9
        t = o.tag(0, thr)
        assert np.array_equal(t.astype(bool), g > thr), thr
        assert t.any() and not t.all()
    flat = _oracle(_cons(one, 0 * one, 0 * one, 0 * one, one), bc=bc)
    assert not flat.tag(0, 1e-12).any()


def test_tags_skip_holes_and_use_the_cell_for_inactive_neighbours():
    """Two levels: cells under the patch carry no tag at level 0, and a level-0
    cell next to the patch uses itself for the neighbour inside it; the fine
    level is tagged from its own cells only."""
    U0 = _random_state(8, 10, 12, RNG)
    box = (1, 8, 6, 4, 8, 8, 8)
    o = _oracle(U0, nlev=2, boxes=[box])
    act0 = o.active_mask(0)
    rho0 = o.get_state(0)[0]
    g = _tag_reference(np.where(act0, rho0, 1.0), act0, (0,) * 6)
    thr = np.quantile(g[act0], 0.6)
    t = o.tag(0, thr)
    assert not t[~act0].any()
    assert np.array_equal(t.astype(bool), act0 & (g > thr))
    act1 = o.active_mask(1)
    rho1 = o.get_state(1)[0]
    g1 = _tag_reference(np.where(act1, rho1, 1.0), act1, (0,) * 6)
    thr1 = np.quantile(g1[act1], 0.5)
    assert np.array_equal(o.tag(1, thr1).astype(bool), act1 & (g1 > thr1))


# ------------------------------------------------ specular wall (method of images)
def _wall_vs_images3(mut=O3.MUT_NONE, steps=5):
    """Reflecting x sides against the periodic box of twice the length holding
    the state and its mirror image (x reversed, x momentum negated), with
    patches touching both walls (spanning the periodic y and z)."""
    nx, ny, nz = 8, 6, 4
    U = _random_state(nz, ny, nx, np.random.default_rng(81), amp=0.3)
    boxes = [(1, 0, 0, 0, 4, 12, 8), (1, 12, 0, 0, 4, 12, 8)]
    bc = (2, 2, 0, 0, 0, 0)
    wall = _oracle(U, nlev=2, boxes=boxes, c=4.0, beta=0.8, bc=bc, mut=mut)
    M = np.flip(U, axis=3).copy()
    M[1] *= -1.0
    mirror = [(l, 2 * nx * 2 - i0 - w, j0, k0, w, h, d) for (l, i0, j0, k0, w, h, d) in boxes]
    per = _oracle(np.concatenate([U, M], axis=3), nlev=2, boxes=boxes + mirror, c=4.0, beta=0.8)
    wall.advance(steps)
    per.advance(steps)
    worst = 0.0
    for l in range(2):
        A = wall.get_pop(l)
        B = per.get_pop(l)[..., :A.shape[3]]
        assert np.array_equal(np.isnan(A), np.isnan(B))
        worst = max(worst, float(np.nanmax(np.abs(A - B))))
    return worst


def test_reflecting_sides_equal_the_mirrored_periodic_run():
    """Method of images in 3-D: specular x walls equal the mirrored periodic
    run bit for bit (the mirror swaps f_+x and f_-x, the first pair of every
    population sum)."""
    assert _wall_vs_images3() == 0.0


def test_planted_wall_without_momentum_flip_fails_the_images():
    assert _wall_vs_images3(O3.MUT_WALL_NO_FLIP) > 1e-3
