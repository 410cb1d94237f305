"""Pins of the oracle's optional extrapolated first Newton iterate,
u^n + (dt / dt_prev)(u^n - u^{n-1}) from the last two accepted states, kept
when its residual norm is below F(u^n)'s.

* A uniform gas moving under uniform gravity on a periodic box: Crank-
  Nicolson integrates m linearly and E quadratically in time (pinned in
  test_oracle_time_walls.py), so after steps dt_1 and then a step dt_2 the
  extrapolated iterate has the exact rho and m, and its energy misses the
  exact one by -rho |g|^2 dt_2 (dt_1 + dt_2) / 2 in every cell.  R is then
  the same at the iterate as at the solution (it depends on rho and m only),
  so F at the iterate is that energy error alone: its scaled norm is
  sqrt(N) rho |g|^2 dt_2 (dt_1 + dt_2) / (2 S_E).  A wrong time ratio, sign
  or pair of states fails this.
* When the extrapolated residual is not smaller the solve is exactly the one
  without extrapolation.
* Without an accepted previous step (a new problem, or a state set since)
  nothing is tried.
"""
import math

import numpy as np
import pytest

from _helpers import desc2d, opts
from oracle import Oracle
from workloads import make_config, split_state


def _uniform_box():
    desc = desc2d(8, 8, g=(0.3, -0.7), gamma=1.4)
    N = 64
    rho, p, vx, vy = 1.3, 2.0, 0.2, -0.1
    E0 = p / (desc["gamma"] - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    u = np.concatenate([np.full(N, rho), np.full(N, E0), np.full(N, rho * vx), np.full(N, rho * vy)])
    return desc, u, rho


@pytest.mark.parametrize("dt1,dt2", [(0.4, 0.4), (0.4, 0.7), (1.1, 0.3)])
def test_extrapolated_iterate_closed_form(dt1, dt2):
    desc, u, rho = _uniform_box()
    o = Oracle(desc, opts(newton_rtol=1e-13, newton_extrapolate=1), u)
    for dt in (dt1, dt1):
        rc, _ = o.newton_solve(dt)
        assert rc == 0
        assert o.extrap_info()[0] == -1.0 or dt == dt1
    un = o.get_state()
    S_E = o.time_step(un)["scales"][1]
    rc, _ = o.newton_solve(dt2)
    assert rc == 0
    fx, taken = o.extrap_info()
    gx, gy = desc["g"][0], desc["g"][1]
    g2 = gx * gx + gy * gy
    expected = math.sqrt(64) * 0.5 * rho * g2 * dt2 * (dt1 + dt2) / S_E
    assert fx == pytest.approx(expected, rel=1e-9), (fx, expected)
    assert taken
    # and the step still lands on the closed form of the trapezoidal rule
    # (to the Newton tolerance, relative to F(u^n))
    f = split_state(o.get_state(), desc)
    t = 2 * dt1 + dt2
    assert np.max(np.abs(f["mx"] - (rho * 0.2 + rho * gx * t))) <= 1e-10
    assert np.max(np.abs(f["my"] - (rho * -0.1 + rho * gy * t))) <= 1e-10


def test_first_step_and_set_state_try_nothing():
    desc, u, _ = _uniform_box()
    o = Oracle(desc, opts(newton_extrapolate=1), u)
    rc, _ = o.newton_solve(0.4)
    assert rc == 0 and o.extrap_info() == (-1.0, False)
    rc, _ = o.newton_solve(0.4)
    assert rc == 0 and o.extrap_info()[0] >= 0.0
    o.set_state(u)
    rc, _ = o.newton_solve(0.4)
    assert rc == 0 and o.extrap_info() == (-1.0, False)


def test_rejected_iterate_changes_nothing():
    """KH at CFL 10: the acoustic modes alternate in sign between steps, so
    the extrapolated residual is larger than F(u^n) and the solve is the one
    without extrapolation, bit for bit."""
    runs = {}
    for ex in (0, 1):
        desc, o_, u = make_config("kh", n=16, newton_extrapolate=ex)
        orc = Oracle(desc, o_, u)
        info = []
        for _ in range(3):
            rc, st = orc.implicit_step()
            assert rc == 0
            info.append(orc.extrap_info())
        runs[ex] = (orc.get_state(), info)
    info = runs[1][1]
    assert info[0] == (-1.0, False)
    assert all(fx >= 0.0 and not taken for fx, taken in info[1:]), info
    assert np.array_equal(runs[0][0], runs[1][0])
