"""The adaptive time-step controller (section 2.1: the step is adjusted for
efficiency within the user's CFL limits, the most restrictive applying).

Reading: a step takes the CFL time step of its state, but at most dt_ctrl;
after an accepted step at dt with k Newton iterations dt_ctrl = dt * f,
f = newton_target / k clamped to [0.5, dt_grow] (f = dt_grow without a
target); a failed attempt halves dt (up to max_halvings times).

The CPU tests check the oracle's step sequence against that rule written out
here (and against the CFL limit it may never exceed); the GPU test checks the
library against the oracle from identical states, bit for bit in dt.
"""
import pytest

from _helpers import rel_l2
from oracle import Oracle
from workloads import make_config

CASES = [dict(newton_max=4, newton_target=0), dict(newton_max=5, newton_target=0),
         dict(newton_max=4, newton_target=4, cfl_hydro=20.0), dict(newton_max=20, newton_target=3),
         dict(newton_max=20, newton_target=1)]


def _expected_factor(opts, k):
    f = opts["dt_grow"]
    if opts["newton_target"] > 0 and k > 0:
        r = float(opts["newton_target"]) / float(k)
        f = 0.5 if r < 0.5 else (opts["dt_grow"] if r > opts["dt_grow"] else r)
    return f


@pytest.mark.parametrize("over", CASES)
def test_oracle_controller_follows_its_rule(over):
    desc, opts, u = make_config("kh", n=16, max_halvings=6, dt_grow=1.5, **over)
    orc = Oracle(desc, opts, u)
    ctrl = None
    bounded = False
    for _ in range(8):
        cfl = orc.time_step(orc.get_state())["dt"]
        base = cfl if ctrl is None or ctrl >= cfl else ctrl
        rc, st = orc.implicit_step()
        assert rc == 0
        # the accepted dt is the base halved once per rejected attempt, and
        # never above the CFL limit of the state
        assert st["dt"] == base * 0.5 ** int(st["rejections"])
        assert st["dt"] <= cfl
        bounded |= st["dt"] < cfl
        ctrl = st["dt"] * _expected_factor(opts, int(st["newton_its"]))
    assert bounded  # the controller, not the CFL limit, set some step


def test_controller_off_takes_the_cfl_step():
    desc, opts, u = make_config("kh", n=16)
    for grow in (0.0, 1.0):
        o2 = dict(opts, dt_grow=grow, newton_target=3)
        orc = Oracle(desc, o2, u)
        for _ in range(3):
            cfl = orc.time_step(orc.get_state())["dt"]
            rc, st = orc.implicit_step()
            assert rc == 0 and st["dt"] == cfl


def test_controller_regrows_after_a_rejection():
    """grow-only mode: after a halved step the next step is 1.5 times the
    accepted one (below the CFL limit), not the CFL step again"""
    desc, opts, u = make_config("kh", n=16, max_halvings=6, dt_grow=1.5, newton_max=5)
    orc = Oracle(desc, opts, u)
    rc, st0 = orc.implicit_step()
    assert rc == 0 and st0["rejections"] >= 1
    cfl = orc.time_step(orc.get_state())["dt"]
    rc, st1 = orc.implicit_step()
    assert rc == 0 and st1["rejections"] == 0
    assert st1["dt"] == st0["dt"] * 1.5 < cfl


@pytest.mark.gpu
@pytest.mark.parametrize("over", CASES)
def test_gpu_controller_matches_oracle(over):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_10053_amd import jfnk
    jfnk.load()
    desc, opts, u = make_config("kh", n=16, max_halvings=6, dt_grow=1.5, **over)
    print("case", over, flush=True)
    g, o = jfnk.Problem(desc, opts, u), Oracle(desc, opts, u)
    for k in range(6):
        o.set_state(g.get_state())  # the controllers keep their own memory
        rg, sg = g.implicit_step()
        ro, so = o.implicit_step()
        print("step", k, sg["dt"], so["dt"], sg["rejections"], sg["newton_its"], flush=True)
        assert rg == ro == 0
        assert sg["dt"] == so["dt"] and sg["rejections"] == so["rejections"]
        assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
        assert rel_l2(g.get_state(), o.get_state()) <= 1e-10
    g.close()
