"""Pins of the oracle in 2D spherical geometry (axis 0 = radius r, axis 1 =
colatitude theta, azimuthal symmetry; the geometry of the paper's section 6
radiative test): consistency with the compressible Euler equations in
spherical coordinates, the planar limit, discrete hydrostatic balance,
conservation, and the preconditioner's block inverse.

None of these compares the oracle with itself in the same geometry or with
the GPU library.
"""
import math

import numpy as np
import pytest

from _helpers import centres, exact_sum, opts, rel_l2, state_from_primitive
from oracle import Oracle
from workloads import (BC_WALL, ENERGY_INTERNAL, GEOM_CARTESIAN, GEOM_SPHERICAL, PC_ACOUSTIC,
                       PC_ACOUSTIC_DIFFUSION, make_config, split_state, unknown_mask)


def sph_desc(nr, nt, r=(1.0, 2.0), th=(math.pi / 4, 3 * math.pi / 4), g=0.0, chi0=0.0, gamma=5.0 / 3.0,
             energy_form=0, geometry=GEOM_SPHERICAL, heat_balance=0):
    return dict(ndim=2, n=[nr, nt, 1], lo=[r[0], th[0], 0.0], hi=[r[1], th[1], 1.0],
                bc=[BC_WALL, BC_WALL, 0], gamma=gamma, g=[g, 0.0, 0.0], chi0=chi0,
                heat_balance=heat_balance, energy_form=energy_form, geometry=geometry)


def _d4(fn, R, TH, d, h=1e-4):
    def at(s):
        return fn(R + s * h, TH) if d == 0 else fn(R, TH + s * h)
    return (-at(2) + 8 * at(1) - 8 * at(-1) + at(-2)) / (12 * h)


def exact_rhs_spherical(desc, rho, ur, ut, p, internal=False):
    """Right-hand sides of eqs. (1)-(3) in spherical coordinates with
    azimuthal symmetry (u_phi = 0), radial gravity g and conduction
    chi0 T^3, from analytic fields f(r, theta): rho and the energy at cell
    centres, m_r on the lower r-faces, m_theta on the lower theta-faces.
    Divergence of a vector: (1/r^2) d_r(r^2 F_r) + (1/(r sin)) d_th(sin F_th);
    momentum: the divergence of rho u u with the geometric terms
    +rho u_th^2 / r (radial) and -rho u_r u_th / r (polar), minus grad p,
    plus rho g (radial)."""
    g, gamma, chi0 = desc["g"][0], desc["gamma"], desc["chi0"]
    X, Y, Z, c, f, dx = centres(desc)
    R, TH = X[0], Y[0]

    def div(Fr, Ft, R, TH):
        return (_d4(lambda r, t: r * r * Fr(r, t), R, TH, 0) / (R * R)
                + _d4(lambda r, t: np.sin(t) * Ft(r, t), R, TH, 1) / (R * np.sin(TH)))

    T = lambda r, t: p(r, t) / rho(r, t)
    E = lambda r, t: p(r, t) / (gamma - 1) + 0.5 * rho(r, t) * (ur(r, t) ** 2 + ut(r, t) ** 2)
    Rr = -div(lambda r, t: rho(r, t) * ur(r, t), lambda r, t: rho(r, t) * ut(r, t), R, TH)
    if internal:
        ie = lambda r, t: p(r, t) / (gamma - 1)
        Re = -div(lambda r, t: ie(r, t) * ur(r, t), lambda r, t: ie(r, t) * ut(r, t), R, TH)
        Re = Re - p(R, TH) * div(ur, ut, R, TH)
    else:
        Re = -div(lambda r, t: (E(r, t) + p(r, t)) * ur(r, t), lambda r, t: (E(r, t) + p(r, t)) * ut(r, t), R, TH)
        Re = Re + rho(R, TH) * ur(R, TH) * g
    if chi0:
        kap = lambda r, t: chi0 * T(r, t) ** 3
        Re = Re + div(lambda r, t: kap(r, t) * _d4(T, r, t, 0), lambda r, t: kap(r, t) * _d4(T, r, t, 1) / r, R, TH)
    # radial momentum on the lower r-faces
    Rf, Tf = R - 0.5 * dx[0], TH
    Rmr = (-div(lambda r, t: rho(r, t) * ur(r, t) * ur(r, t), lambda r, t: rho(r, t) * ur(r, t) * ut(r, t), Rf, Tf)
           + rho(Rf, Tf) * ut(Rf, Tf) ** 2 / Rf - _d4(p, Rf, Tf, 0) + rho(Rf, Tf) * g)
    # polar momentum on the lower theta-faces
    Rc, Tc = R, TH - 0.5 * dx[1]
    Rmt = (-div(lambda r, t: rho(r, t) * ut(r, t) * ur(r, t), lambda r, t: rho(r, t) * ut(r, t) * ut(r, t), Rc, Tc)
           - rho(Rc, Tc) * ur(Rc, Tc) * ut(Rc, Tc) / Rc - _d4(p, Rc, Tc, 1) / Rc)
    return [a.ravel() for a in (Rr, Re, Rmr, Rmt)]


def _fields():
    rho = lambda r, t: 1.0 + 0.2 * np.sin(2.0 * r) * np.cos(2.0 * t)
    ur = lambda r, t: 0.2 + 0.1 * np.sin(3.0 * r) * np.cos(t)
    ut = lambda r, t: -0.15 + 0.1 * np.cos(2.0 * r) * np.sin(3.0 * t)
    p = lambda r, t: 1.0 + 0.1 * np.cos(2.0 * r - t)
    return rho, ur, ut, p


def _orders(chi0=0.0, g=0.0, internal=False, sizes=(32, 64, 128), skip=3):
    rho, ur, ut, p = _fields()
    errs = []
    for n in sizes:
        desc = sph_desc(n, n, g=g, chi0=chi0, energy_form=ENERGY_INTERNAL if internal else 0)
        u = state_from_primitive(desc, lambda x, y, z: rho(x, y), (lambda x, y, z: ur(x, y), lambda x, y, z: ut(x, y)),
                                 lambda x, y, z: p(x, y))
        R = Oracle(desc, opts(), u).rhs(u)
        N = n * n
        ex = exact_rhs_spherical(desc, rho, ur, ut, p, internal)
        ii = np.arange(N) % n
        jj = np.arange(N) // n
        mask = (ii >= skip) & (ii < n - skip) & (jj >= skip) & (jj < n - skip)
        e = []
        for k, ref in enumerate(ex):
            got = R[k * N:(k + 1) * N]
            e.append(np.mean(np.abs(got - ref)[mask]) / np.mean(np.abs(ref[mask])))
        errs.append(e)
    errs = np.array(errs)
    # limiter switches near extremal surfaces make the order between two
    # neighbouring sizes noisy (measured on the momenta: 1.61, 1.41, 2.47,
    # 1.92 from 16 to 256 cells a side); the order over the whole range is
    # the steady one
    return np.log2(errs[0] / errs[-1]) / math.log2(sizes[-1] / sizes[0]), errs


# ---------------------------------------------------------------- consistency with the equations

def test_spherical_residual_second_order():
    """R(u) converges at second order to eqs. (1)-(3) written in spherical
    coordinates (cell volumes, face areas and the geometric momentum terms)"""
    orders, errs = _orders()
    assert np.all(orders > 1.8), (orders, errs)


def test_spherical_residual_second_order_with_gravity_and_conduction():
    orders, errs = _orders(chi0=0.05, g=-0.7)
    assert np.all(orders > 1.8), (orders, errs)


def test_spherical_internal_energy_residual_second_order():
    orders, errs = _orders(g=-0.7, internal=True)
    assert np.all(orders > 1.8), (orders, errs)


def test_planar_limit_matches_cartesian():
    """A thin shell far from the centre is a box: with r0 = 1e4 and a polar
    width of 1/r0 the residual equals the Cartesian one (axis 0 vertical) up
    to O(1/r0)"""
    r0 = 1e4
    n = 16
    sph = sph_desc(n, n, r=(r0, r0 + 1.0), th=(0.5 * math.pi - 0.5 / r0, 0.5 * math.pi + 0.5 / r0), g=-0.5,
                   chi0=0.05)
    car = dict(sph, lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], geometry=GEOM_CARTESIAN)
    rng = np.random.default_rng(3)
    X, Y, Z, c, f, dx = centres(car)
    rho = 1.0 + 0.2 * np.sin(3 * X) * np.cos(2 * Y) + 0.01 * rng.uniform(-1, 1, X.shape)
    E = 2.5 + 0.2 * np.cos(2 * X + Y)
    mr = 0.1 * np.sin(4 * Y) * np.sin(math.pi * X)
    mt = 0.1 * np.cos(3 * X) * np.sin(math.pi * Y)
    u = np.concatenate([rho.ravel(), E.ravel(), mr.ravel(), mt.ravel()])
    u = np.where(unknown_mask(car), u, 0.0)
    Rs = split_state(Oracle(sph, opts(), u).rhs(u), sph)
    Rc = split_state(Oracle(car, opts(), u).rhs(u), car)
    for k in Rs:
        assert rel_l2(Rs[k], Rc[k]) < 1e-3, (k, rel_l2(Rs[k], Rc[k]))
        assert np.linalg.norm(Rc[k]) > 0


# ---------------------------------------------------------------- exact discrete properties

def test_uniform_state_at_rest_has_zero_rhs():
    desc = sph_desc(8, 8, chi0=0.1)
    N = 64
    u = np.concatenate([np.full(N, 1.3), np.full(N, 2.9), np.zeros(N), np.zeros(N)])
    assert np.all(Oracle(desc, opts(), u).rhs(u) == 0.0)


def test_spherical_layer_in_hydrostatic_balance_stays_at_rest():
    desc, o_, u = make_config("srad", n=8, noise=False)
    o = Oracle(desc, o_, u)
    for _ in range(3):
        rc, st = o.implicit_step()
        assert rc == 0, st
    f0, f1 = split_state(u, desc), split_state(o.get_state(), desc)
    for k in ("rho", "E"):
        assert np.max(np.abs(f1[k] - f0[k])) <= 1e-12 * np.max(np.abs(f0[k])), k
    for k in ("mx", "my"):
        assert np.max(np.abs(f1[k])) <= 1e-12, k


def _volumes(desc):
    nr, nt = desc["n"][0], desc["n"][1]
    rf = desc["lo"][0] + np.arange(nr + 1) * (desc["hi"][0] - desc["lo"][0]) / nr
    tf = desc["lo"][1] + np.arange(nt + 1) * (desc["hi"][1] - desc["lo"][1]) / nt
    Vr = (rf[1:] ** 3 - rf[:-1] ** 3) / 3.0
    Vt = np.cos(tf[:-1]) - np.cos(tf[1:])
    return (Vt[:, None] * Vr[None, :]).ravel()


@pytest.mark.parametrize("form", [0, ENERGY_INTERNAL])
def test_mass_and_energy_conserved_with_volumes(form):
    """walls everywhere: sum rho V is conserved to roundoff; without gravity
    and conduction so is sum E V in the total-energy form"""
    desc = sph_desc(16, 16, energy_form=form)
    rho, ur, ut, p = _fields()
    u = state_from_primitive(desc, lambda x, y, z: rho(x, y), (lambda x, y, z: ur(x, y), lambda x, y, z: ut(x, y)),
                             lambda x, y, z: p(x, y))
    u = np.where(unknown_mask(desc), u, 0.0)
    o = Oracle(desc, opts(cfl_hydro=2.0), u)
    V = _volumes(desc)
    f0 = split_state(u, desc)
    for _ in range(2):
        rc, st = o.implicit_step()
        assert rc == 0, st
    f1 = split_state(o.get_state(), desc)
    m0, m1 = exact_sum(f0["rho"].ravel() * V), exact_sum(f1["rho"].ravel() * V)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    e0, e1 = exact_sum(f0["E"].ravel() * V), exact_sum(f1["E"].ravel() * V)
    if form == 0:
        assert abs(e1 - e0) <= 1e-13 * abs(e0)
    else:
        assert abs(e1 - e0) > 1e-9 * abs(e0)  # -p div u exchanges with kinetic energy


# ---------------------------------------------------------------- preconditioner

def spherical_block_operator(desc, u, dt, diffusion):
    """The operator the physics-based preconditioner inverts, in spherical
    geometry, built densely at a state at rest: D F = (1/V) sum of +-A_f F_f,
    face gradient (x_c - x_l) / ds_f (ds = dr, or r_c dtheta), otherwise as in
    the Cartesian case (acoustic block on (drho, dE, dm), heat conduction on
    E first)."""
    nr, nt = desc["n"][0], desc["n"][1]
    N = nr * nt
    gm1, tau = desc["gamma"] - 1.0, 0.5 * dt
    dr = (desc["hi"][0] - desc["lo"][0]) / nr
    dth = (desc["hi"][1] - desc["lo"][1]) / nt
    rf = desc["lo"][0] + np.arange(nr + 1) * dr
    rc = desc["lo"][0] + (np.arange(nr) + 0.5) * dr
    tf = desc["lo"][1] + np.arange(nt + 1) * dth
    V = _volumes(desc)
    rho, E = u[:N], u[N:2 * N]
    h = (E + gm1 * E) / rho
    chi = desc["chi0"] * (gm1 * E / rho) ** 3

    def area(d, i, j):
        if d == 0:
            return rf[i] ** 2 * (math.cos(tf[j]) - math.cos(tf[j + 1]))
        return 0.5 * (rf[i + 1] ** 2 - rf[i] ** 2) * math.sin(tf[j])

    def ds(d, i):
        return dr if d == 0 else rc[i] * dth

    n = 4 * N
    Dv = np.zeros((N, n))
    Dh = np.zeros((N, n))
    G = np.zeros((n, N))
    B = np.eye(N)
    for j in range(nt):
        for i in range(nr):
            c = i + nr * j
            for d in range(2):
                base = (2 + d) * N
                up = (i + 1, j) if d == 0 else (i, j + 1)
                if (up[0] < nr) and (up[1] < nt):
                    cu = up[0] + nr * up[1]
                    A = area(d, *up)
                    Dv[c, base + cu] += A / V[c]
                    Dh[c, base + cu] += 0.5 * (h[c] + h[cu]) * A / V[c]
                lo = (i - 1, j) if d == 0 else (i, j - 1)
                if lo[0] >= 0 and lo[1] >= 0:
                    l = lo[0] + nr * lo[1]
                    A = area(d, i, j)
                    Dv[c, base + c] -= A / V[c]
                    Dh[c, base + c] -= 0.5 * (h[c] + h[l]) * A / V[c]
                    G[base + c, c] += 1.0 / ds(d, i)
                    G[base + c, l] -= 1.0 / ds(d, i)
                    if diffusion:
                        # flux -tau chi_f (W x_c - W x_l)/ds through the face of area A
                        cf = tau * 0.5 * (chi[c] + chi[l]) * A / ds(d, i)
                        B[c, c] += cf * gm1 / rho[c] / V[c]
                        B[c, l] -= cf * gm1 / rho[l] / V[c]
                        B[l, l] += cf * gm1 / rho[l] / V[l]
                        B[l, c] -= cf * gm1 / rho[c] / V[l]
    L = np.zeros((n, n))
    L[:N, :N] = np.eye(N)
    L[:N, :] += tau * Dv
    L[N:2 * N, N:2 * N] = np.eye(N)
    L[N:2 * N, :] += tau * Dh
    for d in range(2):
        base = (2 + d) * N
        for c in range(N):
            i, j = c % nr, c // nr
            if (i if d == 0 else j) > 0:
                L[base + c, base + c] = 1.0
    L[2 * N:, N:2 * N] += tau * gm1 * G[2 * N:, :]
    Dg = np.eye(n)
    Dg[N:2 * N, N:2 * N] = B
    return Dg @ L


@pytest.mark.parametrize("diffusion", [False, True])
def test_spherical_multigrid_converges_to_block_inverse(diffusion):
    desc = sph_desc(8, 8, chi0=0.4 if diffusion else 0.0)
    N = 64
    rng = np.random.default_rng(5)
    X, Y, Z, c, f, dx = centres(desc)
    rho = 1.0 + 0.3 * np.sin(3 * X) + 0.1 * rng.uniform(-1, 1, X.shape)
    E = 2.0 + 0.4 * np.cos(2 * Y) + 0.1 * rng.uniform(-1, 1, X.shape)
    u = np.concatenate([rho.ravel(), E.ravel(), np.zeros(N), np.zeros(N)])
    dt = 0.05
    L = spherical_block_operator(desc, u, dt, diffusion)
    mask = unknown_mask(desc)
    delta = np.where(mask, rng.uniform(-1, 1, u.size), 0.0)
    rhs = L @ delta
    pc = PC_ACOUSTIC_DIFFUSION if diffusion else PC_ACOUSTIC
    many = Oracle(desc, opts(pc=pc, mg_cycles=40), u)
    many.set_scales([1.0] * 5)
    assert rel_l2(many.precond(u, dt, rhs), delta) < 1e-10
    one = Oracle(desc, opts(pc=pc), u)
    one.set_scales([1.0] * 5)
    assert rel_l2(one.precond(u, dt, rhs), delta) < 0.3
