"""Pins of the oracle's internal-energy form: the energy variable rho e of
eq. (2) as written (advective flux rho e u, -p div u at cell centres, no
gravitational work), against facts fixed by the equation and by the pinned
total-energy form.

None of these compares the oracle with itself in the same form or with the
GPU library.
"""
import math

import numpy as np
import pytest

from _helpers import centres, desc2d, desc3d, exact_sum, opts, rel_l2, state_from_primitive
from oracle import Oracle
from workloads import (BC_PERIODIC, BC_WALL, ENERGY_INTERNAL, ENERGY_TOTAL, make_config,
                       split_state, unknown_mask)

TWO_PI = 2.0 * math.pi


def _d4(fn, X, Y, Z, d, h=1e-3):
    P = [X, Y, Z]

    def at(s):
        Q = list(P)
        Q[d] = P[d] + s * h
        return fn(*Q)
    return (-at(2) + 8 * at(1) - 8 * at(-1) + at(-2)) / (12 * h)


def exact_rhs_internal(desc, rho, vel, p, chi0=0.0):
    """Right-hand sides of eqs. (1)-(3) with the internal-energy equation (2)
    as written, from analytic primitive fields: cell centres for rho and
    rho e, lower faces for the momenta.  Derivatives by 4th-order differences
    (step 1e-3)."""
    ndim, gamma, g = desc["ndim"], desc["gamma"], desc["g"]
    X, Y, Z, c, f, dx = centres(desc)

    def u(d):
        return vel[d] if d < ndim else (lambda x, y, z: 0.0 * x)

    def rhoe(x, y, z):
        return p(x, y, z) / (gamma - 1)

    def T(x, y, z):
        return p(x, y, z) / rho(x, y, z)

    Rr = 0 * X
    for d in range(ndim):
        Rr = Rr - _d4(lambda x, y, z: rho(x, y, z) * u(d)(x, y, z), X, Y, Z, d)
    Re = 0 * X
    for d in range(ndim):
        def fe(x, y, z, d=d):
            adv = rhoe(x, y, z) * u(d)(x, y, z)
            if chi0:
                adv = adv - chi0 * T(x, y, z) ** 3 * _d4(T, x, y, z, d)
            return adv
        Re = Re - _d4(fe, X, Y, Z, d)
        Re = Re - p(X, Y, Z) * _d4(u(d), X, Y, Z, d)
    out = [Rr, Re]
    for cc in range(ndim):
        P = [X, Y, Z]
        P[cc] = P[cc] - 0.5 * dx[cc]
        Rm = 0 * X
        for d in range(ndim):
            def fm(x, y, z, d=d):
                v = rho(x, y, z) * u(cc)(x, y, z) * u(d)(x, y, z)
                return v + p(x, y, z) if d == cc else v
            Rm = Rm - _d4(fm, P[0], P[1], P[2], d)
        Rm = Rm + rho(*P) * g[cc]
        out.append(Rm)
    return [a.ravel() for a in out]


# the internal-energy equation reaches its asymptotic order later than the
# total-energy one (measured L1 orders of the rho e row on the 2D field:
# 1.78, 1.75, 1.91, 1.92 from 32 to 512 cells a side), hence 64..256
def _orders(make_desc, rho, vel, p, chi0=0.0, sizes=(64, 128, 256), skip_wall_rows=0):
    errs = []
    for n in sizes:
        desc = make_desc(n)
        desc["chi0"] = chi0
        u = state_from_primitive(desc, rho, vel, p)
        R = Oracle(desc, opts(), u).rhs(u)
        N = desc["n"][0] * desc["n"][1] * desc["n"][2]
        ex = exact_rhs_internal(desc, rho, vel, p, chi0)
        e = []
        for k, ref in enumerate(ex):
            got = R[k * N:(k + 1) * N]
            mask = np.ones(N, dtype=bool)
            if skip_wall_rows:
                ny = desc["n"][1]
                rows = np.arange(N) // desc["n"][0] % ny
                mask = (rows >= skip_wall_rows) & (rows < ny - skip_wall_rows)
            e.append(np.mean(np.abs(got - ref)[mask]) / (np.mean(np.abs(ref[mask])) + 1e-300))
        errs.append(e)
    errs = np.array(errs)
    return np.log2(errs[:-1] / errs[1:]), errs


def _smooth2d():
    rho = lambda x, y, z: 1.0 + 0.2 * np.sin(TWO_PI * (x + y))
    ux = lambda x, y, z: 0.3 + 0.1 * np.cos(TWO_PI * y) * np.sin(TWO_PI * x)
    uy = lambda x, y, z: -0.2 + 0.1 * np.sin(TWO_PI * x)
    p = lambda x, y, z: 1.0 + 0.1 * np.cos(TWO_PI * (x - y))
    return rho, (ux, uy), p


# ---------------------------------------------------------------- consistency with eq. (2)

def test_internal_residual_second_order_2d_periodic():
    """R(u) converges to eqs. (1)-(3) with eq. (2) as written, at second
    order in L1 for smooth flow."""
    rho, vel, p = _smooth2d()
    orders, errs = _orders(lambda n: desc2d(n, n, energy_form=ENERGY_INTERNAL), rho, vel, p)
    assert np.all(orders[-1] > 1.8), (orders, errs)


def test_internal_residual_second_order_with_gravity_and_conduction():
    """Gravity enters the momentum equation only: the internal-energy
    equation has no work term."""
    rho, vel, p = _smooth2d()
    mk = lambda n: desc2d(n, n, g=(0.3, -0.7), gamma=5.0 / 3.0, energy_form=ENERGY_INTERNAL)
    orders, errs = _orders(mk, rho, vel, p, chi0=0.05)
    assert np.all(orders[-1] > 1.8), (orders, errs)


def test_internal_residual_second_order_3d():
    rho = lambda x, y, z: 1.0 + 0.1 * np.sin(x + 2 * z) * np.cos(y)
    ux = lambda x, y, z: 0.4 + 0.2 * np.sin(x) * np.cos(y) * np.cos(z)
    uy = lambda x, y, z: -0.3 - 0.2 * np.cos(x) * np.sin(y) * np.cos(z)
    uz = lambda x, y, z: 0.25 + 0.1 * np.sin(y + z)
    p = lambda x, y, z: 2.0 + 0.1 * np.cos(x - y) * np.sin(z)
    orders, errs = _orders(lambda n: desc3d(n, energy_form=ENERGY_INTERNAL), rho, (ux, uy, uz), p,
                           sizes=(16, 32, 64))
    assert np.all(orders[-1] > 1.4) and np.all(orders[-1] > orders[0] - 0.05), (orders, errs)


def test_internal_residual_second_order_away_from_walls():
    rho = lambda x, y, z: 1.0 + 0.2 * np.sin(TWO_PI * x) * np.cos(math.pi * y)
    ux = lambda x, y, z: 0.3 + 0.1 * np.cos(math.pi * y)
    uy = lambda x, y, z: 0.1 * np.sin(math.pi * y) * (1 + 0.5 * np.cos(TWO_PI * x))
    p = lambda x, y, z: 1.0 + 0.1 * np.cos(TWO_PI * x) * np.cos(math.pi * y)
    mk = lambda n: desc2d(n, n, bc=(BC_PERIODIC, BC_WALL), g=(0.0, -0.5), energy_form=ENERGY_INTERNAL)
    orders, errs = _orders(mk, rho, (ux, uy), p, skip_wall_rows=3)
    assert np.all(orders[-1] > 1.8), (orders, errs)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_density_and_pressure_give_closed_form(ndim):
    """With uniform rho and p the limited reconstruction returns rho and e
    exactly, so the energy equation reduces to -(rho e + p) div u per cell
    and the mass equation to -rho div u, whatever the velocity field."""
    n = 8
    desc = desc2d(n, n, gamma=5.0 / 3.0, energy_form=ENERGY_INTERNAL) if ndim == 2 else \
        desc3d(n, energy_form=ENERGY_INTERNAL)
    N = n ** ndim
    rho0, p0 = 1.3, 0.9
    rhoe0 = p0 / (desc["gamma"] - 1.0)
    rng = np.random.default_rng(ndim)
    vel = [rng.uniform(-0.3, 0.3, N) for _ in range(ndim)]
    u = np.concatenate([np.full(N, rho0), np.full(N, rhoe0)] + [rho0 * v for v in vel])
    R = Oracle(desc, opts(), u).rhs(u)
    shape = (desc["n"][2], desc["n"][1], desc["n"][0])
    div = np.zeros(shape)
    for d in range(ndim):
        v = vel[d].reshape(shape)
        dx = (desc["hi"][d] - desc["lo"][d]) / desc["n"][d]
        div += (np.roll(v, -1, axis=2 - d) - v) / dx
    scale = (rhoe0 + p0) * np.max(np.abs(div))
    assert np.max(np.abs(R[:N] + rho0 * div.ravel())) <= 1e-13 * rho0 * np.max(np.abs(div))
    assert np.max(np.abs(R[N:2 * N] + (rhoe0 + p0) * div.ravel())) <= 1e-13 * scale


@pytest.mark.parametrize("ndim", [2, 3])
def test_internal_uniform_state_and_flow_give_zero_rhs(ndim):
    desc = desc2d(8, 8, energy_form=ENERGY_INTERNAL) if ndim == 2 else desc3d(8, energy_form=ENERGY_INTERNAL)
    N = 8 ** ndim
    for m in (0.0, 0.37):
        u = np.concatenate([np.full(N, 1.3), np.full(N, 2.9)] + [np.full(N, m)] * ndim)
        assert np.all(Oracle(desc, opts(), u).rhs(u) == 0.0)


# ---------------------------------------------------------------- against the total-energy form

def _pressure_from(u, desc):
    """p of a state in either form: (gamma-1)(E - K) with the discrete
    kinetic energy (mean of the squared face velocities), or (gamma-1) rho e."""
    f = split_state(u, desc)
    gm1 = desc["gamma"] - 1.0
    if desc.get("energy_form", 0) == ENERGY_INTERNAL:
        return gm1 * f["E"]
    q = np.zeros_like(f["rho"])
    for d, k in enumerate(["mx", "my", "mz"][: desc["ndim"]]):
        ax = 2 - d
        wall = desc["bc"][d] == BC_WALL
        rf = 0.5 * (np.roll(f["rho"], 1, axis=ax) + f["rho"])
        v = np.where(f[k] == 0.0, 0.0, f[k] / rf)
        vu = np.roll(v, -1, axis=ax)
        if wall:
            idx = [slice(None)] * 3
            idx[ax] = -1
            vu[tuple(idx)] = 0.0
        q += 0.5 * (v * v + vu * vu)
    return gm1 * (f["E"] - 0.5 * f["rho"] * q)


def test_forms_agree_on_small_amplitude_acoustics():
    """About a uniform state at rest both forms linearise to the same
    discrete system (the energies differ by the kinetic energy, second order
    in the amplitude), so one implicit step from the same rho, p and m moves
    rho, m and p alike to O(amplitude) relative."""
    A = 1e-6
    states = {}
    for form in (ENERGY_TOTAL, ENERGY_INTERNAL):
        desc = desc2d(32, 32, gamma=5.0 / 3.0, energy_form=form)
        vx = lambda x, y, z: A * np.sin(TWO_PI * x) * (1.0 + 0.5 * np.cos(TWO_PI * y))
        vy = lambda x, y, z: A * np.cos(TWO_PI * (x + 2 * y))
        u = state_from_primitive(desc, lambda x, y, z: 1.0 + 0 * x, (vx, vy), lambda x, y, z: 0.6 + 0 * x)
        o = Oracle(desc, opts(cfl_hydro=4.0, pc=1), u)
        states[form] = (desc, u, o)
    dt = states[ENERGY_TOTAL][2].time_step(states[ENERGY_TOTAL][1])["dt"]
    out = {}
    for form, (desc, u, o) in states.items():
        o.time_step(u)
        rc, st = o.newton_solve(dt)
        assert rc == 0, st
        u1 = o.get_state()
        fa, fb = split_state(u1, desc), split_state(u, desc)
        out[form] = {k: fa[k] - fb[k] for k in ("rho", "mx", "my")}
        out[form]["p"] = _pressure_from(u1, desc) - _pressure_from(u, desc)
    for k in ("rho", "mx", "my", "p"):
        a, b = out[ENERGY_INTERNAL][k], out[ENERGY_TOTAL][k]
        assert np.linalg.norm(b) > 0
        assert rel_l2(a, b) < 1e-4, (k, rel_l2(a, b))


def test_gravity_work_cancels_against_p_div_u_in_discrete_balance():
    """On a layer in discrete hydrostatic balance (two-cell balance with the
    face density the mean of its cells) the total-energy form's gravitational
    work equals, face by face, the pressure-work difference between the two
    forms, so for small velocities the energy right-hand sides agree to
    second order in the velocity."""
    A = 1e-6
    R = {}
    for form in (ENERGY_TOTAL, ENERGY_INTERNAL):
        desc, o_, u = make_config("rad", n=16, noise=False, energy_form=form)
        desc["chi0"] = 0.0
        desc["heat_balance"] = 0
        f = split_state(u, desc)
        rng = np.random.default_rng(11)
        shape = f["rho"].shape
        ux, uy = A * rng.uniform(-1, 1, shape), A * rng.uniform(-1, 1, shape)
        uy[:, 0, :] = 0.0
        rfx = 0.5 * (np.roll(f["rho"], 1, axis=2) + f["rho"])
        rfy = 0.5 * (np.roll(f["rho"], 1, axis=1) + f["rho"])
        rfy[:, 0, :] = 0.0
        p = _pressure_from(u, desc)
        mx, my = rfx * ux, rfy * uy
        # the same rho, p and m in both forms
        E = p / (desc["gamma"] - 1.0)
        uu = np.concatenate([f["rho"].ravel(), E.ravel(), mx.ravel(), my.ravel()])
        if form == ENERGY_TOTAL:
            uu[E.size:2 * E.size] = 0.0
            q = np.zeros(shape)
            for v, ax in ((ux, 2), (uy, 1)):
                vu = np.roll(v, -1, axis=ax)
                if ax == 1:
                    vu[:, -1, :] = 0.0
                q += 0.5 * (v * v + vu * vu)
            uu[E.size:2 * E.size] = (E + 0.5 * f["rho"] * q).ravel()
        o = Oracle(desc, opts(), uu)
        R[form] = split_state(o.rhs(uu), desc)
    Et, Ei = R[ENERGY_TOTAL]["E"], R[ENERGY_INTERNAL]["E"]
    assert np.max(np.abs(Et)) > 1e3 * A * A
    assert np.max(np.abs(Et - Ei)) <= 1e-6 * np.max(np.abs(Et))
    assert np.array_equal(R[ENERGY_TOTAL]["rho"], R[ENERGY_INTERNAL]["rho"])


# ---------------------------------------------------------------- invariants of a step

def test_internal_form_conserves_mass_to_roundoff():
    desc, o_, u = make_config("kh", n=32, energy_form=ENERGY_INTERNAL)
    o = Oracle(desc, o_, u)
    m0 = exact_sum(split_state(u, desc)["rho"])
    for _ in range(2):
        rc, st = o.implicit_step()
        assert rc == 0
    m1 = exact_sum(split_state(o.get_state(), desc)["rho"])
    assert abs(m1 - m0) <= 1e-13 * abs(m0)


def test_internal_form_preserves_hydrostatic_layer():
    """The radiative layer at rest (discrete hydrostatic balance, heat-balance
    source) is a steady state of the internal-energy form too."""
    desc, o_, u = make_config("rad", n=16, noise=False, energy_form=ENERGY_INTERNAL)
    o = Oracle(desc, o_, u)
    for _ in range(3):
        rc, st = o.implicit_step()
        assert rc == 0
    u1 = o.get_state()
    f0, f1 = split_state(u, desc), split_state(u1, desc)
    for k in ("rho", "E"):
        assert np.max(np.abs(f1[k] - f0[k])) <= 1e-12 * np.max(np.abs(f0[k])), k
    for k in ("mx", "my"):
        assert np.max(np.abs(f1[k])) <= 1e-12 * np.max(np.abs(f0["rho"])), k


def test_internal_form_state_layout_mask():
    """Wall faces stay zero in the internal-energy form too."""
    desc, o_, u = make_config("rt", n=16, energy_form=ENERGY_INTERNAL)
    o = Oracle(desc, o_, u)
    rc, st = o.implicit_step()
    assert rc == 0
    u1 = o.get_state()
    assert np.all(u1[~unknown_mask(desc)] == 0.0)


def test_internal_rhs_galilean_along_the_walls():
    """For a layer between walls that is uniform along x, a uniform velocity
    along x changes neither the mass nor the internal-energy right-hand side:
    e, p and T, and with them the ghost cells beyond the walls (temperature
    extrapolated, e = T/(gamma-1)), do not see it."""
    desc, o_, u = make_config("rad", n=16, noise=False, energy_form=ENERGY_INTERNAL)
    f = split_state(u, desc)
    shape = f["rho"].shape
    rng = np.random.default_rng(12)
    vy = np.broadcast_to(1e-3 * rng.uniform(-1, 1, (1, shape[1], 1)), shape).copy()
    vy[:, 0, :] = 0.0
    rfy = 0.5 * (np.roll(f["rho"], 1, axis=1) + f["rho"])
    rfy[:, 0, :] = 0.0
    R = []
    for U in (0.0, 0.3):
        rfx = 0.5 * (np.roll(f["rho"], 1, axis=2) + f["rho"])
        uu = np.concatenate([f["rho"].ravel(), f["E"].ravel(), (rfx * U).ravel(), (rfy * vy).ravel()])
        R.append(split_state(Oracle(desc, opts(), uu).rhs(uu), desc))
    for k in ("rho", "E"):
        ref = np.max(np.abs(R[0][k]))
        assert ref > 0
        assert np.max(np.abs(R[1][k] - R[0][k])) <= 1e-12 * ref, k
