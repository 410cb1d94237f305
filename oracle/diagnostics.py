"""Diagnostics of a state, plain numpy (TEST INFRASTRUCTURE ONLY: imported by
tests/, the smoke check and the CPU-baseline leg of the benchmark).

Definitions, written out from the paper:
  - kinetic energy K = sum over cells of (1/2) rho |v|^2 dV (section 5.3, the
    kinetic energy whose rate of change the Taylor-Green study reports); on
    the staggered grid |v|^2 of a cell is the mean over each axis of the
    squared velocities of its two faces, v_f = m_f / rho_f with rho_f the
    mean of the two cells sharing face f (0 on wall faces);
  - mass and total energy: sum of rho dV and E dV;
  - maximum Mach number: max over cells of |v| / c_s, c_s^2 = gamma p / rho,
    p = (gamma - 1)(E - (1/2) rho |v|^2), or (gamma - 1) rho e when the energy
    variable is the internal energy of eq. (2) (section 3.1 quotes it);
  - mixing-region width, eqs. (12)-(14): X_H = (rho - rho_L)/(rho_H - rho_L)
    per cell, <X_H> its mean over each layer normal to the vertical axis,
    X_M = 2<X_H> if <X_H> <= 1/2 else 2(1 - <X_H>), and h = sum over layers
    of X_M dy (the integral of eq. 14 as a midpoint sum over the layers);
  - the same width from two passive scalars, eq. (16): X_M = 2 min(<c1>, <c2>)
    of the layer means of the concentrations c_k = s_k / rho;
  - the relative error of eq. (17) between a solution and a higher-resolution
    one: the velocity component of a cell is the mean of its two face
    velocities, the high-resolution field is volume averaged onto the coarse
    cells (section 4.3), and eps = sum |v_low - avg v_high| / sum |avg v_high|.
"""
import numpy as np


def _fields(u, desc):
    nx, ny, nz = desc["n"]
    N = nx * ny * nz
    nd = desc["ndim"]
    rho = u[:N].reshape(nz, ny, nx)
    E = u[N:2 * N].reshape(nz, ny, nx)
    m = [u[(2 + d) * N:(3 + d) * N].reshape(nz, ny, nx) for d in range(nd)]
    return rho, E, m


def _axis(d):
    """array axis of grid direction d for (nz, ny, nx) arrays"""
    return 2 - d


def face_velocities(u, desc):
    """v_f on the lower face of every cell, per direction (0 on wall faces)"""
    rho, E, m = _fields(u, desc)
    out = []
    for d in range(desc["ndim"]):
        ax = _axis(d)
        rho_lo = np.roll(rho, 1, axis=ax)          # the cell below along d
        v = m[d] / (0.5 * (rho_lo + rho))
        if desc["bc"][d] == 1:                      # wall: the face at index 0 is the wall
            idx = [slice(None)] * 3
            idx[ax] = 0
            v[tuple(idx)] = 0.0
        out.append(v)
    return out


def speed_squared(u, desc):
    """|v|^2 per cell: per axis the mean of the squared velocities of the
    cell's lower and upper faces (the upper face beyond a top wall is 0)"""
    vf = face_velocities(u, desc)
    q = np.zeros_like(vf[0])
    for d in range(desc["ndim"]):
        ax = _axis(d)
        up = np.roll(vf[d], -1, axis=ax)
        if desc["bc"][d] == 1:
            idx = [slice(None)] * 3
            idx[ax] = -1
            up[tuple(idx)] = 0.0
        q = q + 0.5 * (vf[d] ** 2 + up ** 2)
    return q


def cell_volume(desc):
    v = 1.0
    for d in range(desc["ndim"]):
        v *= (desc["hi"][d] - desc["lo"][d]) / desc["n"][d]
    return v


def kinetic_energy(u, desc):
    rho, E, m = _fields(u, desc)
    return float(np.sum(0.5 * rho * speed_squared(u, desc)) * cell_volume(desc))


def totals(u, desc):
    rho, E, m = _fields(u, desc)
    dv = cell_volume(desc)
    return float(np.sum(rho) * dv), float(np.sum(E) * dv)


def max_mach(u, desc):
    rho, E, m = _fields(u, desc)
    q = speed_squared(u, desc)
    g = desc["gamma"]
    p = (g - 1.0) * E if desc.get("energy_form", 0) == 1 else (g - 1.0) * (E - 0.5 * rho * q)
    return float(np.max(np.sqrt(q) / np.sqrt(g * p / rho)))


def mixing_width(u, desc, rho_light, rho_heavy, axis):
    """eqs. (12)-(14) along grid direction `axis`"""
    rho, E, m = _fields(u, desc)
    xh = (rho - rho_light) / (rho_heavy - rho_light)
    ax = _axis(axis)
    other = tuple(a for a in range(3) if a != ax)
    mean = xh.mean(axis=other)
    xm = np.where(mean <= 0.5, 2.0 * mean, 2.0 * (1.0 - mean))
    dy = (desc["hi"][axis] - desc["lo"][axis]) / desc["n"][axis]
    return float(np.sum(xm) * dy)


def mixing_width_scalars(u, s, desc, axis):
    """eq. (16) with eq. (14): layer means of c1 = s1/rho and c2 = s2/rho"""
    rho, E, m = _fields(u, desc)
    nx, ny, nz = desc["n"]
    N = nx * ny * nz
    c1 = s[:N].reshape(nz, ny, nx) / rho
    c2 = s[N:2 * N].reshape(nz, ny, nx) / rho
    ax = _axis(axis)
    other = tuple(a for a in range(3) if a != ax)
    xm = 2.0 * np.minimum(c1.mean(axis=other), c2.mean(axis=other))
    dy = (desc["hi"][axis] - desc["lo"][axis]) / desc["n"][axis]
    return float(np.sum(xm) * dy)


def cell_velocity(u, desc, axis):
    """component `axis` of the velocity per cell: the mean of its lower and
    upper face velocities (the face beyond a top wall is the wall, 0)"""
    v = face_velocities(u, desc)[axis]
    ax = _axis(axis)
    up = np.roll(v, -1, axis=ax)
    if desc["bc"][axis] == 1:
        idx = [slice(None)] * 3
        idx[ax] = -1
        up[tuple(idx)] = 0.0
    return 0.5 * (v + up)


def velocity_error(u_low, desc_low, u_high, desc_high, axis):
    """eq. (17): relative L1 error of velocity component `axis` of u_low
    against u_high volume averaged onto the low-resolution grid (every active
    axis of the high-resolution grid r times finer; equal cell volumes make
    the volume average the mean over the r^ndim fine cells)"""
    nd = desc_low["ndim"]
    r = desc_high["n"][0] // desc_low["n"][0]
    for d in range(nd):
        assert desc_high["n"][d] == r * desc_low["n"][d]
    vl = cell_velocity(u_low, desc_low, axis)
    vh = cell_velocity(u_high, desc_high, axis)
    nx, ny, nz = desc_low["n"]
    rz = r if nd == 3 else 1
    avg = vh.reshape(nz, rz, ny, r, nx, r).mean(axis=(1, 3, 5))
    return float(np.sum(np.abs(vl - avg)) / np.sum(np.abs(avg)))
