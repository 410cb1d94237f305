"""Initial states for the four benchmark problems, in conserved variables.

State layout (shared by every consumer): one flat float64 array holding the
fields rho, E, m_x, m_y (and m_z in 3D) one after another, each of
n_x*n_y*n_z entries in C order (z slowest, x fastest).  Momentum component d
at flat index c is the value on the lower face of cell c along d (the face at
x_d = lo_d + i_d*dx_d).  Along a wall direction the face with i_d = 0 is the
wall itself: it always holds 0 and is not an unknown; the upper wall face is
not stored.

Problem set-ups follow the paper's test problems, shrunk or synthesised where
the paper relies on data that is not available:

* ``rt``  single-mode Rayleigh-Taylor instability (paper section 3: density
  jump, hydrostatic pressure with P0 = 2.5, velocity perturbation eq. 11),
  written in coordinates shifted to [0, 0.5] x [0, 1.5].
* ``kh``  subsonic shear layer with tanh-smoothed interfaces (paper section 4
  studies the McNally et al. set-up, whose exact data are not reproduced here).
* ``tg``  Taylor-Green vortex (paper section 5, eqs. 18-21) at Mach 0.1.
* ``rad`` a stratified layer in discrete hydrostatic equilibrium with a
  radiative conductivity chi = chi0 T^3 (a synthetic stand-in for the stellar
  envelope of paper section 6).
* ``srad`` the same layer as a spherical shell segment in 2D spherical
  geometry (r in [1, 2], a 0.25 rad wedge about the equator, walls on every
  side, constant radial gravity), the geometry of paper section 6.

Random numbers come from numpy's PCG64 generator with a fixed seed per
problem; every draw is uniform on [-1, 1).
"""
import math

import numpy as np

BC_PERIODIC = 0
BC_WALL = 1

PC_NONE = 0
PC_ACOUSTIC = 1
PC_ACOUSTIC_DIFFUSION = 2

PREC_FP64 = 0
PREC_MIXED = 1

PCS_MULTIGRID = 0
PCS_ADI = 1

# the linear tolerance of each Newton iteration: gmres_eta throughout, or
# Eisenstat-Walker choice 2 starting from (and capped at) gmres_eta
FORCING_FIXED = 0
FORCING_EW = 1

# energy variable of the state: total energy E, or internal energy rho e (eq. 2)
ENERGY_TOTAL = 0
ENERGY_INTERNAL = 1

# grid geometry: Cartesian, or 2D spherical (axis 0 = radius r, axis 1 =
# colatitude theta, azimuthal symmetry)
GEOM_CARTESIAN = 0
GEOM_SPHERICAL = 1

CONFIG_NAMES = ("rt", "kh", "tg", "rad")

# implicit steps each benchmark problem runs
DEFAULT_STEPS = {"rt": 10, "kh": 200, "tg": 100, "rad": 50}

# Relative GMRES tolerance per problem, picked from preliminary runs (as the
# paper picks CFL limits from preliminary calculations): the limited
# reconstruction makes Newton converge about linearly, so solving each linear
# system far below the Newton contraction is wasted work.  rt, kh and rad
# from low-resolution runs; tg from full 100-step runs at 128^3 (0.1, 0.15,
# 0.2 and 0.3 all converge every step; 0.2 and 0.3 take the least time).
LINEAR_TOL = {"rt": 1e-2, "kh": 3e-2, "tg": 2e-1, "rad": 5e-3}

# Multigrid V-cycles per preconditioner application, from the same kind of
# runs on the GPU: one cycle solves the stiff conduction block of the
# radiative layer too loosely (at 512 x 2048 GMRES stagnates and every step is
# halved; 128 x 512: 18.9 ms/step with one cycle, 12.7 with three; 512 x 2048:
# 811, 32 and 26 ms/step with one, two and three); two cycles take 3 % off the
# Taylor-Green step (GMRES 47 -> 35 iterations per step); one is best for
# the shear layer and the Rayleigh-Taylor problem.
MG_CYCLES = {"rt": 1, "kh": 1, "tg": 2, "rad": 3}

# Levels of at most this many cells take one pre- and one post-smoothing sweep
# instead of two (0: none), from GPU runs like the cycles: for TG 128^3 the
# 32^3 level and below (54.5 -> 52.6 ms/step, GMRES 34.8 -> 35.3 per step;
# including the 64^3 level: 53.5; V(1,0) there: 52.8).
MG_LIGHT_CELLS = {"rt": 0, "kh": 0, "tg": 32768, "rad": 0}

# The first Newton iterate extrapolated in time from the last two accepted
# states (used only when its residual is below F(u^n)'s), assessed like the
# linear tolerance on the full runs: on the Taylor-Green vortex at 128^3 it
# saves a Newton iteration in the early steps (36.8 -> 34.6 ms/step over
# steps 1-20) but little over the 100-step run (41.37 -> 41.32 ms/step; about
# 1 % in interleaved runs on one host, inside their spread; the internal-energy
# form 40.8 -> 41.3), because the extrapolated residual relative to F(u^n)
# rises from 0.16 early to 0.51 late in the run; on the shear layer and the
# radiative layer it is never taken, on Rayleigh-Taylor taken without saving
# an iteration.  So it is off everywhere.
EXTRAPOLATE = {"rt": 0, "kh": 0, "tg": 0, "rad": 0}


def default_opts(**over):
    """Solver options: Newton relative tolerance 1e-8, GMRES(30) to a
    relative linear tolerance of 1e-2, one multigrid V(2,2) cycle per
    elliptic solve in the preconditioner."""
    o = dict(newton_rtol=1e-8, newton_atol=1e-14, newton_max=20,
             gmres_restart=30, gmres_max_cycles=10, gmres_eta=1e-2,
             pc=PC_ACOUSTIC, prec=PREC_FP64, cfl_hydro=1.0,
             cfl_adv_max=0.0, cfl_rad_max=0.0, dt_max=0.0, max_halvings=5,
             pc_solver=PCS_MULTIGRID, mg_nu1=2, mg_nu2=2, mg_nuc=4, mg_cycles=1,
             newton_corr_tol=1e-12, mg_light_cells=0, newton_target=0, dt_grow=0.0, scalar_converge=1,
             gmres_forcing=0, newton_extrapolate=0)
    for k, v in over.items():
        if k not in o:
            raise KeyError(k)
        o[k] = v
    return o


def n_cells(desc):
    n = desc["n"]
    return n[0] * n[1] * n[2]


def n_vars(desc):
    return 2 + desc["ndim"]


def split_state(u, desc):
    """Return dict of field arrays shaped (nz, ny, nx)."""
    nx, ny, nz = desc["n"]
    N = nx * ny * nz
    u = np.asarray(u)
    names = ["rho", "E", "mx", "my", "mz"][: n_vars(desc)]
    return {k: u[i * N:(i + 1) * N].reshape(nz, ny, nx) for i, k in enumerate(names)}


def join_state(fields, desc):
    names = ["rho", "E", "mx", "my", "mz"][: n_vars(desc)]
    return np.concatenate([np.asarray(fields[k], dtype=np.float64).ravel() for k in names])


def unknown_mask(desc):
    """True where a state entry is an unknown (False on stored wall faces)."""
    nx, ny, nz = desc["n"]
    N = nx * ny * nz
    mask = np.ones(n_vars(desc) * N, dtype=bool)
    for d in range(desc["ndim"]):
        if desc["bc"][d] == BC_WALL:
            m = mask[(2 + d) * N:(3 + d) * N].reshape(nz, ny, nx)
            idx = [slice(None)] * 3
            idx[2 - d] = 0
            m[tuple(idx)] = False
    return mask


def mirror_x(u, desc):
    """Mirror a state about the mid-plane of x (x -> L - x), negating m_x."""
    f = split_state(np.array(u, dtype=np.float64), desc)
    out = {}
    for k, a in f.items():
        if k == "mx":
            # face i sits at lo + i*dx; its mirror image is face (nx - i) mod nx
            b = -np.roll(a[:, :, ::-1], 1, axis=2)
        else:
            b = a[:, :, ::-1]
        out[k] = b.copy()
    return join_state(out, desc)


def _desc(ndim, n, lo, hi, bc, gamma, g, chi0=0.0, heat_balance=0, energy_form=ENERGY_TOTAL,
          geometry=GEOM_CARTESIAN):
    n = list(n) + [1] * (3 - len(n))
    lo = list(lo) + [0.0] * (3 - len(lo))
    hi = list(hi) + [1.0] * (3 - len(hi))
    bc = list(bc) + [BC_PERIODIC] * (3 - len(bc))
    g = list(g) + [0.0] * (3 - len(g))
    return dict(ndim=ndim, n=[int(v) for v in n], lo=[float(v) for v in lo],
                hi=[float(v) for v in hi], bc=[int(v) for v in bc],
                gamma=float(gamma), g=[float(v) for v in g], chi0=float(chi0),
                heat_balance=int(heat_balance), energy_form=int(energy_form), geometry=int(geometry))


def _face_avg_rho(rho, axis, wall):
    """Arithmetic mean of the two cells adjacent to each lower face."""
    lower = np.roll(rho, 1, axis=axis)
    out = 0.5 * (lower + rho)
    if wall:
        idx = [slice(None)] * 3
        idx[axis] = 0
        out[tuple(idx)] = 0.0
    return out


def _upper(a, axis, wall):
    """Value on the upper face of each cell given lower-face values."""
    up = np.roll(a, -1, axis=axis)
    if wall:
        idx = [slice(None)] * 3
        idx[axis] = -1
        up[tuple(idx)] = 0.0
    return up


def _energy(p, rho, gamma, vel, bc, internal=False):
    """E = p/(gamma-1) + rho |v_c|^2 / 2 with v_c the mean of a cell's two
    faces, or rho e = p/(gamma-1) for the internal-energy variable."""
    if internal:
        return p / (gamma - 1.0)
    ke = np.zeros_like(p)
    for d, v in enumerate(vel):
        axis = 2 - d
        vc = 0.5 * (v + _upper(v, axis, bc[d] == BC_WALL))
        ke += vc * vc
    return p / (gamma - 1.0) + 0.5 * rho * ke


def _rt(n, seed, noise, perturb, internal):
    nx, ny = (32, 64) if n is None else (int(n), 2 * int(n))
    if nx % 2:
        raise ValueError("rt needs an even nx for the mirror-symmetric set-up")
    desc = _desc(2, (nx, ny), (0.0, 0.0), (0.5, 1.5), (BC_PERIODIC, BC_WALL),
                 1.4, (0.0, -0.1))
    dx, dy = 0.5 / nx, 1.5 / ny
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    yf = np.arange(ny) * dy
    rho = np.where(yc > 0.75, 2.0, 1.0)[:, None] * np.ones((1, nx))
    p = 2.5 - rho * 0.1 * (yc[:, None] - 0.75)
    half = nx // 2
    vy_l = np.zeros((ny, half))
    if perturb:
        # paper eq. (11) in coordinates centred on the box
        vy_l += 0.0025 * (1.0 + np.cos(4.0 * math.pi * (xc[:half] - 0.25)))[None, :] * \
            (1.0 + np.cos(4.0 * math.pi * (yf - 0.75) / 3.0))[:, None]
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        vy_l += 1e-6 * rng.uniform(-1.0, 1.0, size=(ny, half))
    vy_l[0, :] = 0.0
    vy = np.concatenate([vy_l, vy_l[:, ::-1]], axis=1)  # exact mirror copy
    rho3, p3, vy3 = rho[None], p[None], vy[None]
    vx3 = np.zeros_like(rho3)
    bc = desc["bc"]
    my = _face_avg_rho(rho3, 1, True) * vy3
    mx = np.zeros_like(rho3)
    E = _energy(p3, rho3, desc["gamma"], [vx3, vy3], bc, internal)
    u = join_state(dict(rho=rho3, E=E, mx=mx, my=my), desc)
    opts = default_opts(cfl_hydro=5.0, pc=PC_ACOUSTIC, gmres_eta=LINEAR_TOL["rt"], mg_cycles=MG_CYCLES["rt"])
    return desc, opts, u


def _kh(n, seed, noise, perturb, internal):
    nn = 256 if n is None else int(n)
    desc = _desc(2, (nn, nn), (0.0, 0.0), (1.0, 1.0), (BC_PERIODIC, BC_PERIODIC),
                 5.0 / 3.0, (0.0, 0.0))
    d = 1.0 / nn
    xc = (np.arange(nn) + 0.5) * d
    yc = (np.arange(nn) + 0.5) * d
    yf = np.arange(nn) * d

    def w(y):
        return np.tanh((y - 0.25) / 0.01) - np.tanh((y - 0.75) / 0.01)

    rho = (1.0 + 0.5 * w(yc))[:, None] * np.ones((1, nn))
    ux = (-0.05 + 0.05 * w(yc))[:, None] * np.ones((1, nn))
    vy = np.zeros((nn, nn))
    if perturb:
        s = 0.05
        vy = 1e-3 * np.sin(4.0 * math.pi * xc)[None, :] * \
            (np.exp(-(yf - 0.25) ** 2 / (2 * s * s)) + np.exp(-(yf - 0.75) ** 2 / (2 * s * s)))[:, None]
    p = np.full((nn, nn), 2.5)
    rho3, ux3, vy3, p3 = rho[None], ux[None], vy[None], p[None]
    bc = desc["bc"]
    mx = _face_avg_rho(rho3, 2, False) * ux3
    my = _face_avg_rho(rho3, 1, False) * vy3
    E = _energy(p3, rho3, desc["gamma"], [ux3, vy3], bc, internal)
    u = join_state(dict(rho=rho3, E=E, mx=mx, my=my), desc)
    opts = default_opts(cfl_hydro=10.0, pc=PC_ACOUSTIC, gmres_eta=LINEAR_TOL["kh"], mg_cycles=MG_CYCLES["kh"])
    return desc, opts, u


def _tg(n, seed, noise, perturb, internal):
    nn = 128 if n is None else int(n)
    L = 2.0 * math.pi
    desc = _desc(3, (nn, nn, nn), (0.0, 0.0, 0.0), (L, L, L),
                 (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC), 5.0 / 3.0, (0.0, 0.0, 0.0))
    d = L / nn
    c = (np.arange(nn) + 0.5) * d
    f = np.arange(nn) * d
    zc, yc, xc = np.meshgrid(c, c, c, indexing="ij")
    rho = np.ones((nn, nn, nn))
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        rho = rho + 1e-8 * rng.uniform(-1.0, 1.0, size=rho.shape)
    V0, M, gamma = 1.0, 0.1, desc["gamma"]
    p0 = 1.0 * V0 * V0 / (gamma * M * M)
    p = p0 + (1.0 * V0 * V0 / 16.0) * (np.cos(2 * xc) + np.cos(2 * yc)) * (np.cos(2 * zc) + 2.0)
    if perturb:
        zz, yy, xf = np.meshgrid(c, c, f, indexing="ij")
        ux = V0 * np.sin(xf) * np.cos(yy) * np.cos(zz)
        zz, yf, xx = np.meshgrid(c, f, c, indexing="ij")
        uy = -V0 * np.cos(xx) * np.sin(yf) * np.cos(zz)
    else:
        ux = np.zeros_like(rho)
        uy = np.zeros_like(rho)
    uz = np.zeros_like(rho)
    bc = desc["bc"]
    mx = _face_avg_rho(rho, 2, False) * ux
    my = _face_avg_rho(rho, 1, False) * uy
    mz = _face_avg_rho(rho, 0, False) * uz
    E = _energy(p, rho, gamma, [ux, uy, uz], bc, internal)
    u = join_state(dict(rho=rho, E=E, mx=mx, my=my, mz=mz), desc)
    opts = default_opts(cfl_hydro=20.0, pc=PC_ACOUSTIC, gmres_eta=LINEAR_TOL["tg"], mg_cycles=MG_CYCLES["tg"],
                        mg_light_cells=MG_LIGHT_CELLS["tg"], newton_extrapolate=EXTRAPOLATE["tg"])
    return desc, opts, u


RAD_CHI0 = 0.6304


def _rad(n, seed, noise, perturb, internal):
    nx = 128 if n is None else int(n)
    ny = 4 * nx
    d = 1.0 / ny
    T = 1.0 + (10.0 ** (-4.0 / 3.0) - 1.0) * np.arange(ny) / (ny - 1)
    g = -3.25 * (T[0] - T[-1]) / ((ny - 1) * d)  # polytrope of index 2.25
    desc = _desc(2, (nx, ny), (0.0, 0.0), (0.25, 1.0), (BC_PERIODIC, BC_WALL),
                 5.0 / 3.0, (0.0, g), chi0=RAD_CHI0, heat_balance=1)
    # density from the two-cell hydrostatic balance with p = rho T and a face
    # density equal to the mean of its two cells
    hg = 0.5 * abs(g) * d
    rho1 = np.empty(ny)
    rho1[0] = 1.0
    for j in range(ny - 1):
        rho1[j + 1] = rho1[j] * (T[j] - hg) / (T[j + 1] + hg)
    rho = rho1[:, None] * np.ones((1, nx))
    p = rho * T[:, None]
    vx = np.zeros((ny, nx))
    vy = np.zeros((ny, nx))
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        vx = 1e-10 * rng.uniform(-1.0, 1.0, size=(ny, nx))
        vy = 1e-10 * rng.uniform(-1.0, 1.0, size=(ny, nx))
    vy[0, :] = 0.0
    rho3, p3, vx3, vy3 = rho[None], p[None], vx[None], vy[None]
    bc = desc["bc"]
    mx = _face_avg_rho(rho3, 2, False) * vx3
    my = _face_avg_rho(rho3, 1, True) * vy3
    E = _energy(p3, rho3, desc["gamma"], [vx3, vy3], bc, internal)
    u = join_state(dict(rho=rho3, E=E, mx=mx, my=my), desc)
    opts = default_opts(cfl_hydro=10.0, cfl_rad_max=1000.0, pc=PC_ACOUSTIC_DIFFUSION,
                        gmres_eta=LINEAR_TOL["rad"], mg_cycles=MG_CYCLES["rad"])
    return desc, opts, u


def _srad(n, seed, noise, perturb, internal):
    nt = 128 if n is None else int(n)
    nr = 4 * nt
    r0, r1 = 1.0, 2.0
    dr = (r1 - r0) / nr
    th0, th1 = 0.5 * math.pi - 0.125, 0.5 * math.pi + 0.125
    T = 1.0 + (10.0 ** (-4.0 / 3.0) - 1.0) * np.arange(nr) / (nr - 1)
    g = -3.25 * (T[0] - T[-1]) / ((nr - 1) * dr)
    desc = _desc(2, (nr, nt), (r0, th0), (r1, th1), (BC_WALL, BC_WALL), 5.0 / 3.0, (g, 0.0),
                 chi0=RAD_CHI0, heat_balance=1, geometry=GEOM_SPHERICAL)
    # radial two-cell hydrostatic balance, face density the mean of its cells
    hg = 0.5 * abs(g) * dr
    rho1 = np.empty(nr)
    rho1[0] = 1.0
    for i in range(nr - 1):
        rho1[i + 1] = rho1[i] * (T[i] - hg) / (T[i + 1] + hg)
    rho = np.ones((nt, 1)) * rho1[None, :]          # (theta, r) = (axis 1, axis 0)
    p = rho * T[None, :]
    vr = np.zeros((nt, nr))
    vt = np.zeros((nt, nr))
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        vr = 1e-10 * rng.uniform(-1.0, 1.0, size=(nt, nr))
        vt = 1e-10 * rng.uniform(-1.0, 1.0, size=(nt, nr))
    vr[:, 0] = 0.0
    vt[0, :] = 0.0
    rho3, p3, vr3, vt3 = rho[None], p[None], vr[None], vt[None]
    bc = desc["bc"]
    mr = _face_avg_rho(rho3, 2, True) * vr3
    mt = _face_avg_rho(rho3, 1, True) * vt3
    E = _energy(p3, rho3, desc["gamma"], [vr3, vt3], bc, internal)
    u = join_state(dict(rho=rho3, E=E, mx=mr, my=mt), desc)
    opts = default_opts(cfl_hydro=10.0, cfl_rad_max=1000.0, pc=PC_ACOUSTIC_DIFFUSION,
                        gmres_eta=LINEAR_TOL["rad"], mg_cycles=MG_CYCLES["rad"])
    return desc, opts, u


_BUILDERS = {"rt": (_rt, 0), "kh": (_kh, 1), "tg": (_tg, 2), "rad": (_rad, 3), "srad": (_srad, 5)}


def make_config(name, n=None, seed=None, noise=True, perturb=True, energy_form=ENERGY_TOTAL, **opt_over):
    """Return (desc, opts, u0) for one of ``rt``, ``kh``, ``tg``, ``rad``.

    ``n`` rescales the grid keeping each problem's aspect ratio (rt: n x 2n,
    kh: n x n, tg: n^3, rad: n x 4n, srad: 4n radial x n polar cells).  ``noise``/``perturb`` switch off the
    seeded noise or the deterministic velocity perturbation.
    ``energy_form`` selects the energy variable (ENERGY_TOTAL or
    ENERGY_INTERNAL); the same pressure field gives the initial state.
    """
    fn, default_seed = _BUILDERS[name]
    internal = energy_form == ENERGY_INTERNAL
    desc, opts, u = fn(n, default_seed if seed is None else seed, noise, perturb, internal)
    desc["energy_form"] = int(energy_form)
    for k, v in opt_over.items():
        if k not in opts:
            raise KeyError(k)
        opts[k] = v
    return desc, opts, np.ascontiguousarray(u, dtype=np.float64)
