"""Shared helpers for the tests: independent re-statements of the paper's
equations (used only to pin the oracle), states, norms."""
import math

import numpy as np

from workloads import (BC_PERIODIC, BC_WALL, default_opts, join_state, n_vars,
                       split_state)


def desc2d(nx, ny, L=(1.0, 1.0), bc=(BC_PERIODIC, BC_PERIODIC), gamma=1.4, g=(0.0, 0.0),
           chi0=0.0, heat_balance=0, energy_form=0):
    return dict(ndim=2, n=[nx, ny, 1], lo=[0.0, 0.0, 0.0], hi=[L[0], L[1], 1.0],
                bc=[bc[0], bc[1], BC_PERIODIC], gamma=gamma, g=[g[0], g[1], 0.0],
                chi0=chi0, heat_balance=heat_balance, energy_form=energy_form)


def desc3d(n, L=2 * math.pi, gamma=5.0 / 3.0, energy_form=0):
    return dict(ndim=3, n=[n, n, n], lo=[0.0] * 3, hi=[L] * 3, bc=[BC_PERIODIC] * 3,
                gamma=gamma, g=[0.0] * 3, chi0=0.0, heat_balance=0, energy_form=energy_form)


def centres(desc):
    """cell-centre and lower-face coordinates, arrays shaped (nz, ny, nx)"""
    nx, ny, nz = desc["n"]
    dx = [(desc["hi"][d] - desc["lo"][d]) / desc["n"][d] for d in range(3)]
    c = [desc["lo"][d] + (np.arange(desc["n"][d]) + 0.5) * dx[d] for d in range(3)]
    f = [desc["lo"][d] + np.arange(desc["n"][d]) * dx[d] for d in range(3)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    return X, Y, Z, c, f, dx


def state_from_primitive(desc, rho_fn, vel_fns, p_fn):
    """Conserved state from smooth primitive fields sampled at the right
    positions; E = p/(gamma-1) + rho |v_c|^2/2 (v_c = mean of the face values),
    or rho e = p/(gamma-1) when desc selects the internal-energy variable.
    vel_fns[d](x, y, z) is sampled on the lower faces along d."""
    nx, ny, nz = desc["n"]
    X, Y, Z, c, f, dx = centres(desc)
    rho = rho_fn(X, Y, Z)
    p = p_fn(X, Y, Z)
    fields = dict(rho=rho)
    names = ["mx", "my", "mz"]
    ke = np.zeros_like(rho)
    for d in range(desc["ndim"]):
        P = [X, Y, Z]
        P[d] = P[d] - 0.5 * dx[d]
        v = vel_fns[d](*P)
        axis = 2 - d
        rf = 0.5 * (np.roll(rho, 1, axis=axis) + rho)
        if desc["bc"][d] == BC_WALL:
            idx = [slice(None)] * 3
            idx[axis] = 0
            v[tuple(idx)] = 0.0
        vu = np.roll(v, -1, axis=axis)
        if desc["bc"][d] == BC_WALL:
            idx = [slice(None)] * 3
            idx[axis] = -1
            vu[tuple(idx)] = 0.0
        ke += (0.5 * (v + vu)) ** 2
        fields[names[d]] = rf * v
    if desc.get("energy_form", 0) == 1:
        fields["E"] = p / (desc["gamma"] - 1.0)
    else:
        fields["E"] = p / (desc["gamma"] - 1.0) + 0.5 * rho * ke
    return join_state(fields, desc)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def exact_sum(a):
    return math.fsum(np.asarray(a, dtype=np.float64).ravel().tolist())


def field_sums(u, desc):
    f = split_state(u, desc)
    return {k: exact_sum(v) for k, v in f.items()}


def opts(**kw):
    return default_opts(**kw)


def nv(desc):
    return n_vars(desc)
