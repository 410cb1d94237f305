"""Pins of the oracle's time discretisation (Crank-Nicolson, section 2) and of
its wall ghost cells (section 3.1) against facts the paper and mathematics fix.

* Crank-Nicolson is the trapezoidal rule: it integrates exactly a state whose
  momentum grows linearly and whose energy grows quadratically in time (a
  uniform gas under uniform gravity), and its error falls as dt^2.  An
  off-centred weighting or backward Euler gets the closed form wrong and
  converges at first order or not at all.
* Section 3.1: at a reflecting wall the ghost temperature is extrapolated
  linearly and the ghost density follows from hydrostatic balance.  On a
  discretely hydrostatic layer with a linear temperature the ghost cell is
  therefore the next row of the same layer: the upwind face flux next to a
  wall must equal the one of a grid that holds that row as a real cell.  And
  with smooth fields the residual converges to eqs. (1)-(3) at second order
  in the rows next to the walls as it does inside.

None of these compares the oracle with itself under the same arithmetic: the
closed forms and the convergence orders come from the equations; the
extension test builds the ghost row from the discrete hydrostatic balance of
the momentum equation (pinned separately by the hydrostatic-preservation
test) and reads the flux through the residual of a larger grid.
"""
import math

import numpy as np
import pytest

from _helpers import desc2d, opts, rel_l2, state_from_primitive
from oracle import Oracle
from test_oracle_pins import exact_rhs
from workloads import BC_PERIODIC, BC_WALL, make_config, mirror_x, split_state

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------- Crank-Nicolson (section 2)

@pytest.mark.parametrize("dt", [0.4, 1.3])
def test_cn_uniform_gravity_closed_form(dt):
    """Uniform gas moving with velocity v0 under uniform gravity g on a
    periodic box: rho stays, m(t) = m0 + rho g t, E(t) = E0 + t g.m0 +
    rho |g|^2 t^2 / 2.  The trapezoidal rule integrates a linear m and a
    quadratic E exactly, so one step of any length reproduces them to
    roundoff; a weighting theta != 1/2 adds (theta - 1/2) rho |g|^2 dt^2
    to E."""
    desc = desc2d(8, 8, g=(0.3, -0.7), gamma=1.4)
    N = 64
    rho, p, vx, vy = 1.3, 2.0, 0.2, -0.1
    E0 = p / (desc["gamma"] - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    u = np.concatenate([np.full(N, rho), np.full(N, E0), np.full(N, rho * vx), np.full(N, rho * vy)])
    orc = Oracle(desc, opts(newton_rtol=1e-13), u)
    rc, st = orc.newton_solve(dt)
    assert rc == 0, st
    f = split_state(orc.get_state(), desc)
    gx, gy = desc["g"][0], desc["g"][1]
    g2 = gx * gx + gy * gy
    assert np.max(np.abs(f["rho"] - rho)) <= 1e-15
    assert np.max(np.abs(f["mx"] - (rho * vx + rho * gx * dt))) <= 1e-13
    assert np.max(np.abs(f["my"] - (rho * vy + rho * gy * dt))) <= 1e-13
    E1 = E0 + dt * (gx * rho * vx + gy * rho * vy) + 0.5 * rho * g2 * dt * dt
    # the t^2 term is what distinguishes the weighting: check it to 1e-10 of itself
    assert np.max(np.abs(f["E"] - E1)) <= 1e-10 * (0.5 * rho * g2 * dt * dt)
    # pressure stays uniform and unchanged (the gained kinetic energy is the work of gravity)
    mx, my = f["mx"] / f["rho"], f["my"] / f["rho"]
    p1 = (desc["gamma"] - 1.0) * (f["E"] - 0.5 * f["rho"] * (mx * mx + my * my))
    assert np.max(np.abs(p1 - p)) <= 1e-12


def test_cn_second_order_in_dt():
    """Self-convergence in time at a fixed grid: a smooth, subsonic wave on a
    uniform flow (velocities of one sign, so the upwind side never changes)
    integrated to t = 0.4 with 4, 8, ..., 64 steps, each Newton solve
    converged to 1e-12.  Successive differences fall by 4 per halving of dt
    (second order; the limiter's kinks, which the trajectory crosses a fixed
    number of times, only delay the asymptotic regime)."""
    n = 16
    desc = desc2d(n, n, gamma=1.4)
    rho = lambda x, y, z: 1.0 + 0.05 * np.sin(TWO_PI * x) * np.cos(TWO_PI * y)
    ux = lambda x, y, z: 0.5 + 0.05 * np.cos(TWO_PI * y)
    uy = lambda x, y, z: 0.4 + 0.05 * np.sin(TWO_PI * x)
    p = lambda x, y, z: 1.0 + 0.1 * np.cos(TWO_PI * (x + y))
    u0 = state_from_primitive(desc, rho, (ux, uy), p)
    o = opts(newton_rtol=1e-12, newton_atol=1e-16, gmres_eta=1e-6, newton_corr_tol=0.0)
    sols = []
    for k in (4, 8, 16, 32, 64):
        orc = Oracle(desc, o, u0)
        for _ in range(k):
            rc, st = orc.newton_solve(0.4 / k)
            assert rc == 0, (k, st)
        sols.append(orc.get_state())
    diffs = np.array([np.linalg.norm(sols[i] - sols[i + 1]) for i in range(len(sols) - 1)])
    orders = np.log2(diffs[:-1] / diffs[1:])
    assert orders[-1] > 1.85 and orders[-2] > 1.7, (orders, diffs)


# ---------------------------------------------------------------- wall ghost cells (section 3.1)

def _layer(nrows, g, T0=1.5, dT=-0.02, rho0=1.0):
    """A discretely hydrostatic layer with a linear temperature T_j = T0 +
    j dT: p_{j+1} - p_j = dy g (rho_j + rho_{j+1}) / 2 with p = rho T (the
    balance the staggered momentum equation holds exactly), dy = 1/nrows
    before any extension.  Returned as functions of the row index j, valid
    for j outside [0, nrows) too."""
    dy = 1.0 / nrows
    hg = 0.5 * g * dy

    def T(j):
        return T0 + j * dT

    def rho(j):
        r = rho0
        if j >= 0:
            for i in range(j):
                r = r * (T(i) + hg) / (T(i + 1) - hg)
        else:
            for i in range(0, j, -1):
                r = r * (T(i) - hg) / (T(i - 1) + hg)
        return r
    return T, rho, dy


def _layer_state(desc, rows, T, rho, vy_faces, gamma):
    """Conserved state of a 2D wall problem whose row r holds layer row
    rows[r]; the y-velocity on lower face r is vy_faces[r] (face 0 is the
    wall), x-velocity 0."""
    nx, ny = desc["n"][0], desc["n"][1]
    rr = np.array([rho(j) for j in rows])
    TT = np.array([T(j) for j in rows])
    v = np.asarray(vy_faces, dtype=float)
    v_up = np.append(v[1:], 0.0)
    q = 0.5 * (v * v + v_up * v_up)  # mean over the axis of the two squared face speeds
    E = rr * TT / (gamma - 1.0) + 0.5 * rr * q
    rf = 0.5 * (rr + np.roll(rr, 1))
    my = rf * v
    my[0] = 0.0
    col = lambda a: np.repeat(a[:, None], nx, axis=1).ravel()
    return np.concatenate([col(rr), col(E), np.zeros(nx * ny), col(my)])


def _face_fluxes_from_rhs(R, desc, g, rows_sum, m_faces):
    """Mass and energy flux through the upper face of the rows summed:
    with zero flux through the wall below row 0 (or above the top row),
    dy times the summed residual gives the flux; the energy residual first
    loses its gravitational work g (m_lo + m_hi)/2."""
    nx, ny = desc["n"][0], desc["n"][1]
    N = nx * ny
    dy = (desc["hi"][1] - desc["lo"][1]) / ny
    Rr = R[:N].reshape(ny, nx)[:, 0]
    RE = R[N:2 * N].reshape(ny, nx)[:, 0]
    m_up = np.append(m_faces[1:], 0.0)
    RE = RE - g * 0.5 * (m_faces + m_up)
    return sum(Rr[r] for r in rows_sum) * dy, sum(RE[r] for r in rows_sum) * dy


@pytest.mark.parametrize("side", ["bottom", "top"])
def test_wall_ghost_is_next_row_of_hydrostatic_layer(side):
    """Grid A holds rows 0..n-1 of a discretely hydrostatic, linear-T layer
    between walls; grid B holds rows -1..n of the same layer (the rows A's
    ghost cells stand for), with the same y-velocity c on the faces that A
    and B share and on the faces next to B's extra rows.  The flow goes
    into the wall cell's side (c > 0 at the bottom: upwind is A's row 0,
    whose limited slopes read the ghost; c < 0 at the top).  The mass and
    energy fluxes through the first interior face of A must equal those
    through the corresponding face of B.  A ghost density without the
    hydrostatic term or with its sign flipped, or a ghost temperature that
    is not extrapolated linearly, changes A's fluxes at first order in the
    slopes."""
    n, nx, gamma, g = 16, 4, 1.4, -0.8
    T, rho, dy = _layer(n, g)
    c = 1e-7 if side == "bottom" else -1e-7
    dA = desc2d(nx, n, L=(nx * dy, 1.0), bc=(BC_PERIODIC, BC_WALL), g=(0.0, g), gamma=gamma)
    dB = desc2d(nx, n + 2, L=(nx * dy, (n + 2) * dy), bc=(BC_PERIODIC, BC_WALL), g=(0.0, g), gamma=gamma)
    vA = np.full(n, c)
    vA[0] = 0.0
    vB = np.full(n + 2, c)
    vB[0] = 0.0
    uA = _layer_state(dA, range(0, n), T, rho, vA, gamma)
    uB = _layer_state(dB, range(-1, n + 1), T, rho, vB, gamma)
    RA = Oracle(dA, opts(), uA).rhs(uA)
    RB = Oracle(dB, opts(), uB).rhs(uB)
    mA = split_state(uA, dA)["my"][0, :, 0]
    mB = split_state(uB, dB)["my"][0, :, 0]
    if side == "bottom":
        # face 1 of A is face 2 of B
        fA = _face_fluxes_from_rhs(RA, dA, g, [0], mA)
        fB = _face_fluxes_from_rhs(RB, dB, g, [0, 1], mB)
        sgn = 1.0
    else:
        # face n-1 of A is face n of B; fluxes from the rows above it, with
        # zero flux through the top wall: flux = -dy * sum
        fA = _face_fluxes_from_rhs(RA, dA, g, [n - 1], mA)
        fB = _face_fluxes_from_rhs(RB, dB, g, [n, n + 1], mB)
        sgn = -1.0
    # the two grids' residuals differ only by rounding
    for a, b in zip(fA, fB):
        assert abs(a - b) <= 1e-13 * abs(b), (side, fA, fB)
    # and the flux is what goes into the wall cell's side: sign of c
    assert -sgn * fA[0] * np.sign(c) > 0


def _wall_layer_fields(g, a=-0.3, T0=1.5, p0=2.0):
    """Smooth fields between walls at y = 0 and 1: a hydrostatic layer with
    a linear temperature (dp/dy = rho g, p = rho T), a y-velocity odd and
    an x-velocity even about both walls (stress-free), flowing into the
    wall cells' sides (upward near y = 0, downward near y = 1)."""
    T = lambda x, y, z: T0 + a * y + 0.0 * x
    p = lambda x, y, z: p0 * (T(x, y, z) / T0) ** (g / a)
    rho = lambda x, y, z: p(x, y, z) / T(x, y, z)
    ux = lambda x, y, z: 0.3 + 0.1 * np.cos(TWO_PI * y) * np.cos(TWO_PI * x)
    uy = lambda x, y, z: 0.1 * np.sin(TWO_PI * y) * (1.0 + 0.5 * np.cos(TWO_PI * x))
    return rho, (ux, uy), p


def test_residual_second_order_in_wall_rows():
    """R(u) against eqs. (1)-(3) in the rows next to the walls only (mean
    absolute error over the first and last row of cells, and over the
    first interior faces for m_y): mass and energy converge at second order
    there, as inside.  The ghost cells beyond the walls are second-order
    extensions of this layer, so a ghost density or temperature off by a
    term of O(dy) drops the mass and energy orders towards one."""
    g = -0.5
    rho, vel, p = _wall_layer_fields(g)
    errs = []
    for n in (32, 64, 128):
        desc = desc2d(n, n, bc=(BC_PERIODIC, BC_WALL), g=(0.0, g))
        u = state_from_primitive(desc, rho, vel, p)
        R = Oracle(desc, opts(), u).rhs(u)
        ex = exact_rhs(desc, rho, vel, p)
        N = n * n
        row = np.arange(N) // n
        e = []
        for k, ref in enumerate(ex):
            got = R[k * N:(k + 1) * N]
            sel = (row == 0) | (row == n - 1) if k != 3 else (row == 1) | (row == n - 1)
            e.append(np.mean(np.abs(got - ref)[sel]))
        errs.append(e)
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    # rho, E: second order; momenta: at least first (the tangential velocity
    # has its extremum on the wall, where the limiter clips the slope)
    assert np.all(orders[-1, :2] > 1.85), (orders, errs)
    assert np.all(orders[-1, 2:] > 0.9), (orders, errs)


# ---------------------------------------------------------------- mirror symmetry with the preconditioner (section 3.3)

@pytest.mark.parametrize("rtol,bound", [(1e-8, 1e-10), (1e-12, 1e-13)])
def test_rt_mirror_symmetry_preconditioned_scales_with_tolerance(rtol, bound):
    """Red-black smoothing is not mirror-symmetric, so with the
    preconditioner on the left-right symmetry of the Rayleigh-Taylor run
    holds to the accuracy of the Newton solve rather than bit for bit:
    ~4e-12 after three steps at rtol 1e-8 (the relative change of a step,
    ~1e-2, times the residual tolerance bounds it by 1e-10), and at
    roundoff (~6e-15) when Newton is converged to 1e-12."""
    desc, o, u = make_config("rt", n=16, newton_rtol=rtol)
    orc = Oracle(desc, o, u)
    for _ in range(3):
        assert orc.implicit_step()[0] == 0
    s = orc.get_state()
    assert rel_l2(mirror_x(s, desc), s) < bound
