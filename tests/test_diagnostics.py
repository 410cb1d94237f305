"""Diagnostics: the oracle's definitions pinned to closed forms and limits
(CPU), and the device reductions against the oracle (GPU).

Pins: a uniform flow (kinetic energy, Mach number exact); the Taylor-Green
initial field, whose discrete kinetic energy per volume is rho0 u0^2 / 8; a
single moving face (both neighbouring cells see half of it); mixing width 0 for a sharp interface, exactly delta/2 for a
linear density ramp of thickness delta, and the layer average taken before
X_M (a checkerboard layer mixes fully)."""
import numpy as np
import pytest

from _helpers import desc2d, desc3d
from oracle import diagnostics as dg
from workloads import BC_PERIODIC, BC_WALL, make_config


def _state(desc, rho, vel, p):
    """conserved state from cell density, uniform-per-face velocity arrays
    (one per axis, shaped like rho, on the lower faces) and pressure"""
    nd = desc["ndim"]
    m = []
    q = np.zeros_like(rho)
    for d in range(nd):
        ax = 2 - d
        rho_f = 0.5 * (np.roll(rho, 1, axis=ax) + rho)
        m.append(rho_f * vel[d])
        up = np.roll(vel[d], -1, axis=ax)
        q = q + 0.5 * (vel[d] ** 2 + up ** 2)
    E = p / (desc["gamma"] - 1.0) + 0.5 * rho * q
    return np.concatenate([rho.ravel(), E.ravel()] + [a.ravel() for a in m])


def test_uniform_flow():
    desc = desc3d(8, gamma=1.4)
    desc["n"] = [8, 6, 4]
    shape = (4, 6, 8)
    rho = np.full(shape, 1.3)
    v = [np.full(shape, 0.3), np.full(shape, -0.2), np.full(shape, 0.1)]
    u = _state(desc, rho, v, np.full(shape, 2.0))
    vol = np.prod([desc["hi"][d] - desc["lo"][d] for d in range(3)])
    assert dg.kinetic_energy(u, desc) == pytest.approx(0.5 * 1.3 * 0.14 * vol, rel=1e-14)
    assert dg.max_mach(u, desc) == pytest.approx(np.sqrt(0.14) / np.sqrt(1.4 * 2.0 / 1.3), rel=1e-14)
    mass, energy = dg.totals(u, desc)
    assert mass == pytest.approx(1.3 * vol, rel=1e-14)
    assert energy == pytest.approx((2.0 / 0.4 + 0.5 * 1.3 * 0.14) * vol, rel=1e-14)


def test_taylor_green_kinetic_energy_is_one_eighth():
    """sampled on a uniform periodic grid, sin^2 and cos^2 sum to exactly half
    the points, so the staggered kinetic energy of the initial vortex is
    rho0 u0^2 / 8 per volume to rounding at every resolution"""
    for n in (8, 16, 32):
        desc, opts, u = make_config("tg", n=n, noise=False)
        assert abs(dg.kinetic_energy(u, desc) / (2 * np.pi) ** 3 - 0.125) < 1e-14


def test_single_moving_face():
    """one face with momentum m between cells of density r1 and r2: both
    cells see half its squared velocity, K = (1/2) m^2 / rho_f dV"""
    rng = np.random.default_rng(3)
    for bc in (BC_PERIODIC, BC_WALL):
        desc = desc2d(6, 5, bc=(BC_PERIODIC, bc), L=(1.2, 1.0))
        rho = rng.uniform(0.5, 2.0, (1, 5, 6))
        N = 30
        u = np.concatenate([rho.ravel(), np.full(N, 5.0), np.zeros(2 * N)])
        j, i, m = 3, 2, 0.7
        u[3 * N + j * 6 + i] = m               # m_y on the lower y-face of cell (i, j)
        rho_f = 0.5 * (rho[0, j - 1, i] + rho[0, j, i])
        dv = (1.2 / 6) * (1.0 / 5)
        assert dg.kinetic_energy(u, desc) == pytest.approx(0.5 * m * m / rho_f * dv, rel=1e-14)


def test_mixing_width_sharp_interface_is_zero():
    desc, opts, u = make_config("rt", noise=False, perturb=False)
    assert dg.mixing_width(u, desc, 1.0, 2.0, 1) == 0.0


def test_mixing_width_of_a_linear_ramp():
    # 16 x 32 cells over [0,1] x [0,2]; density ramps linearly from 1 to 2
    # across the 8 middle layers (thickness 0.5): h = 0.5 / 2 exactly
    desc = desc2d(16, 32, bc=(BC_PERIODIC, BC_WALL), L=(1.0, 2.0))
    ny, dy = 32, 2.0 / 32
    y = (np.arange(ny) + 0.5) * dy
    s = np.clip((y - 0.75) / 0.5, 0.0, 1.0)
    rho = np.broadcast_to((1.0 + s)[None, :, None], (1, ny, 16)).copy()
    u = _state(desc, rho, [np.zeros_like(rho), np.zeros_like(rho)], np.ones_like(rho))
    assert dg.mixing_width(u, desc, 1.0, 2.0, 1) == pytest.approx(0.25, rel=1e-14)


def test_mixing_width_averages_each_layer_before_mixing():
    desc = desc2d(16, 8, bc=(BC_PERIODIC, BC_WALL), L=(1.0, 1.0))
    i = np.arange(16)
    rho = np.broadcast_to((1.0 + (i % 2))[None, None, :], (1, 8, 16)).copy()  # checkerboard in x
    u = _state(desc, rho, [np.zeros_like(rho), np.zeros_like(rho)], np.ones_like(rho))
    assert dg.mixing_width(u, desc, 1.0, 2.0, 1) == pytest.approx(1.0, rel=1e-14)


def test_scalar_mixing_width_limits():
    desc = desc2d(8, 16, bc=(BC_PERIODIC, BC_WALL), L=(1.0, 2.0))
    N = 8 * 16
    rho = np.linspace(1.0, 2.0, N)
    u = np.concatenate([rho, np.full(N, 3.0), np.zeros(2 * N)])
    below = (np.arange(N) // 8 < 8).astype(float)
    sharp = np.concatenate([below * rho, (1.0 - below) * rho])
    assert dg.mixing_width_scalars(u, sharp, desc, 1) == 0.0
    mixed = np.concatenate([0.5 * rho, 0.5 * rho])
    assert dg.mixing_width_scalars(u, mixed, desc, 1) == pytest.approx(2.0, rel=1e-14)


# ---------------------------------------------------------------- GPU against the oracle
@pytest.mark.gpu
@pytest.mark.parametrize("name,n,steps,axis", [("rt", None, 5, 1), ("kh", 64, 3, 1), ("tg", 32, 2, -1),
                                               ("rad", 32, 2, 1)])
def test_gpu_diagnostics_match_oracle(name, n, steps, axis):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_10053_amd import jfnk
    jfnk.load()
    desc, opts, u = make_config(name, n=n)
    g = jfnk.Problem(desc, opts, u)
    for _ in range(steps):
        assert g.implicit_step()[0] == 0
    s = g.get_state()
    rl, rh = (1.0, 2.0) if name == "rt" else (float(s[:desc["n"][0]].min()), float(s[:desc["n"][0]].max()) + 1.0)
    d = g.eval_diagnostics(None, rl, rh, axis)
    dh = g.eval_diagnostics(s, rl, rh, axis)  # the same state passed in from the host
    assert d == dh
    assert d["kinetic"] == pytest.approx(dg.kinetic_energy(s, desc), rel=1e-12, abs=1e-300)
    mass, energy = dg.totals(s, desc)
    assert d["mass"] == pytest.approx(mass, rel=1e-13)
    assert d["energy"] == pytest.approx(energy, rel=1e-13)
    assert d["max_mach"] == dg.max_mach(s, desc)  # same operations per cell; max is order-free
    if axis >= 0:
        assert d["mix_width"] == pytest.approx(dg.mixing_width(s, desc, rl, rh, axis), rel=1e-12, abs=1e-15)
    else:
        assert d["mix_width"] == 0.0


# ---------------------------------------------------------------- eq. (17): error against a finer solution

def _shear_state(desc, vfun, axis):
    """uniform rho and p, velocity component `axis` = vfun(coordinate array
    of its faces), other components 0"""
    nx, ny, nz = desc["n"]
    shape = (nz, ny, nx)
    dx = [(desc["hi"][d] - desc["lo"][d]) / desc["n"][d] for d in range(3)]
    cz, cy, cx = [(np.arange(desc["n"][d]) + 0.5) * dx[d] for d in (2, 1, 0)]
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    P = [X, Y, Z]
    P[axis] = P[axis] - 0.5 * dx[axis]
    vel = [np.zeros(shape) for _ in range(desc["ndim"])]
    vel[axis] = vfun(*P)
    return _state(desc, np.full(shape, 1.3), vel, np.full(shape, 2.0))


def test_velocity_error_against_itself_and_uniform_fields():
    desc = desc2d(16, 8)
    u = _shear_state(desc, lambda x, y, z: np.sin(6.0 * y) + x, 0)
    assert dg.velocity_error(u, desc, u, desc, 0) == 0.0
    fine = desc2d(32, 16)
    one = _shear_state(fine, lambda x, y, z: 1.0 + 0 * x, 1)
    two = _shear_state(desc, lambda x, y, z: 2.0 + 0 * x, 1)
    assert dg.velocity_error(two, desc, one, fine, 1) == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("r", [2, 4, 8])
def test_velocity_error_of_a_sine_is_the_dirichlet_kernel(r):
    """v_x = sin(2 pi y): the mean of the r fine cell values over a coarse
    cell is sin(2 pi y_c) D, D = sin(pi r h)/(r sin(pi h)) with h the fine
    spacing, so eps = |1 - D| / D"""
    n = 16
    lo, hi = desc2d(n, n), desc2d(n * r, n * r)
    f = lambda x, y, z: np.sin(2.0 * np.pi * y)
    h = 1.0 / (n * r)
    D = np.sin(np.pi * r * h) / (r * np.sin(np.pi * h))
    eps = dg.velocity_error(_shear_state(lo, f, 0), lo, _shear_state(hi, f, 0), hi, 0)
    assert eps == pytest.approx(abs(1.0 - D) / D, rel=1e-10)


def test_velocity_error_dirichlet_kernel_3d():
    n, r = 8, 2
    lo, hi = desc3d(n, L=1.0), desc3d(n * r, L=1.0)
    f = lambda x, y, z: np.cos(2.0 * np.pi * x) + 0.25
    h = 1.0 / (n * r)
    D = np.sin(np.pi * r * h) / (r * np.sin(np.pi * h))
    xc = (np.arange(n) + 0.5) / n
    ref = np.sum(np.abs(np.cos(2 * np.pi * xc) * (1 - D))) / np.sum(np.abs(np.cos(2 * np.pi * xc) * D + 0.25))
    eps = dg.velocity_error(_shear_state(lo, f, 2), lo, _shear_state(hi, f, 2), hi, 2)
    assert eps == pytest.approx(ref, rel=1e-10)


def test_velocity_error_of_a_linear_profile_between_walls_is_zero():
    """the volume average of a linear field is its value at the centre"""
    lo = desc2d(8, 8, bc=(BC_PERIODIC, BC_WALL))
    hi = desc2d(32, 32, bc=(BC_PERIODIC, BC_WALL))
    f = lambda x, y, z: 0.5 + y
    eps = dg.velocity_error(_shear_state(lo, f, 0), lo, _shear_state(hi, f, 0), hi, 0)
    assert eps <= 1e-14


@pytest.mark.gpu
@pytest.mark.parametrize("name,n,axis,r", [("kh", 32, 1, 2), ("rt", 16, 1, 2), ("tg", 8, 0, 2), ("kh", 16, 0, 4),
                                           ("rad", 8, 1, 3)])
def test_gpu_velocity_error_matches_oracle(name, n, axis, r):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_10053_amd import jfnk
    jfnk.load()
    d_lo, o_lo, u_lo = make_config(name, n=n)
    d_hi, o_hi, u_hi = make_config(name, n=r * n)
    g_lo, g_hi = jfnk.Problem(d_lo, o_lo, u_lo), jfnk.Problem(d_hi, o_hi, u_hi)
    for _ in range(2):
        assert g_lo.implicit_step()[0] == 0
        assert g_hi.implicit_step()[0] == 0
    s_lo, s_hi = g_lo.get_state(), g_hi.get_state()
    ref = dg.velocity_error(s_lo, d_lo, s_hi, d_hi, axis)
    assert ref > 0
    e_host = g_lo.velocity_error(s_hi, r, axis)
    e_dev = g_lo.velocity_error(torch.from_numpy(s_hi).cuda(), r, axis)
    e_given = g_hi.velocity_error(s_hi, 1, axis, u_low=s_hi)
    print(name, n, axis, ref, e_host, e_dev, flush=True)
    assert e_host == pytest.approx(ref, rel=1e-12)
    assert e_dev == e_host
    assert e_given == 0.0
    g_lo.close()
    g_hi.close()


def test_max_mach_of_the_internal_energy_variable():
    """with the internal-energy variable p = (gamma - 1) rho e, whatever the
    velocity"""
    desc = desc2d(8, 8, gamma=1.4, energy_form=1)
    shape = (1, 8, 8)
    rho = np.full(shape, 1.3)
    v = [np.full(shape, 0.3), np.full(shape, -0.4)]
    m = [0.5 * (np.roll(rho, 1, axis=2 - d) + rho) * v[d] for d in range(2)]
    rhoe = np.full(shape, 2.0 / 0.4)
    u = np.concatenate([rho.ravel(), rhoe.ravel()] + [a.ravel() for a in m])
    assert dg.max_mach(u, desc) == pytest.approx(0.5 / np.sqrt(1.4 * 2.0 / 1.3), rel=1e-14)


@pytest.mark.gpu
def test_gpu_diagnostics_internal_energy_form():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_10053_amd import jfnk
    jfnk.load()
    desc, opts, u = make_config("kh", n=64, energy_form=1)
    g = jfnk.Problem(desc, opts, u)
    for _ in range(2):
        assert g.implicit_step()[0] == 0
    s = g.get_state()
    d = g.eval_diagnostics(None)
    assert d["max_mach"] == dg.max_mach(s, desc)
    assert d["kinetic"] == pytest.approx(dg.kinetic_energy(s, desc), rel=1e-12)
    g.close()
