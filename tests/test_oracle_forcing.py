"""Pins of the oracle's optional Eisenstat-Walker forcing of the Newton
iterations' linear tolerance.

The forcing term is Eisenstat and Walker's choice 2 (SIAM J. Sci. Comput. 17,
1996) with gamma = 0.9 and exponent 2, safeguarded as in Kelley, Iterative
Methods for Linear and Nonlinear Equations (SIAM 1995), section 6.3.  The
first test checks values worked out by hand from that definition, one per
branch; the others check that the Newton loop applies it: the first
iteration takes gmres_eta, every later one the forcing term of the residual
norms of its own and the previous iterate, and every linear solve meets its
tolerance.
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from oracle.oracle import ew_forcing
from workloads import FORCING_EW, FORCING_FIXED, make_config, unknown_mask


@pytest.mark.parametrize("args,expected", [
    # choice 2 alone: 0.9 * (1e-2)^2
    ((1e-2, 1.0, 0.1, 0.9, 1e-12), 9e-5),
    # safeguard: 0.9 * 0.5^2 = 0.225 > 0.1 and above 9e-5
    ((1e-2, 1.0, 0.5, 0.9, 1e-12), 0.225),
    # the safeguard value 0.9 * 0.9^2 = 0.729 capped at eta_max 0.2
    ((0.5, 1.0, 0.9, 0.2, 1e-12), 0.2),
    # end game: 0.9 * (1e-3)^2 = 9e-7 raised to 0.5 * 1e-8 / 1e-7 = 0.05
    ((1e-7, 1e-4, 0.01, 0.2, 1e-8), 0.05),
    # end game above the cap: 0.5 * 1e-8 / 1e-9 = 5 capped at 0.2
    ((1e-9, 1e-4, 0.01, 0.2, 1e-8), 0.2),
    # safeguard not taken at 0.9 * 0.3^2 = 0.081 <= 0.1
    ((1e-1, 1.0, 0.3, 0.9, 1e-12), 0.009),
])
def test_forcing_term_worked_values(args, expected):
    assert ew_forcing(*args) == pytest.approx(expected, rel=1e-14)


def _tol(desc, opts, f0):
    nunk = int(np.count_nonzero(unknown_mask(desc)))
    return max(opts["newton_rtol"] * f0, opts["newton_atol"] * math.sqrt(nunk))


@pytest.mark.parametrize("name,n", [("kh", 16), ("kh", 32), ("rt", 16), ("tg", 8)])
def test_newton_applies_the_forcing_term(name, n):
    desc, opts, u = make_config(name, n=n, gmres_forcing=FORCING_EW)
    o = Oracle(desc, opts, u)
    rc, st = o.newton_solve(o.time_step(u)["dt"])
    assert rc == 0 and st["rel_res"] <= opts["newton_rtol"]
    f, eta, lin = o.newton_history()
    assert len(f) == int(st["newton_its"]) + 1 and len(eta) == len(f) - 1
    tol = _tol(desc, opts, f[0])
    assert eta[0] == opts["gmres_eta"]
    for k in range(1, len(eta)):
        assert eta[k] == ew_forcing(f[k], f[k - 1], eta[k - 1], opts["gmres_eta"], tol), k
        assert 0.0 < eta[k] <= opts["gmres_eta"]
    # every linear solve stopped at its own tolerance
    assert np.all(lin <= eta * (1 + 1e-12)), (lin, eta)
    # the forcing is active: some iteration solved tighter than gmres_eta
    assert np.any(eta[1:] < opts["gmres_eta"])


def test_fixed_forcing_keeps_gmres_eta():
    desc, opts, u = make_config("kh", n=16, gmres_forcing=FORCING_FIXED)
    o = Oracle(desc, opts, u)
    rc, _ = o.newton_solve(o.time_step(u)["dt"])
    assert rc == 0
    _, eta, lin = o.newton_history()
    assert np.all(eta == opts["gmres_eta"])
    assert np.all(lin <= eta * (1 + 1e-12))
