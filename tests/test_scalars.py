"""Passive scalars (section 2.2): the oracle's scalar step pinned on the CPU,
and the GPU library against the oracle.

Pins: a uniform concentration c gives exactly c times the density
right-hand side (the reconstruction of a constant is the constant); a flow
at rest leaves the scalars unchanged bit for bit; without re-normalisation
every scalar's total is conserved to roundoff on a periodic domain; with it
the concentrations sum to one in every cell; a uniform concentration stays
uniform to within the flow's Newton tolerance."""
import numpy as np
import pytest

from _helpers import exact_sum
from oracle import Oracle
from workloads import make_config


def _two_scalars(desc, u, axis=1):
    """dye 1 below the middle of `axis`, dye 2 above (c1 + c2 = 1)"""
    nx, ny, nz = desc["n"]
    N = nx * ny * nz
    rho = u[:N].reshape(nz, ny, nx)
    idx = np.indices((nz, ny, nx))[2 - axis]
    c1 = (idx < desc["n"][axis] // 2).astype(float)
    return np.concatenate([(c1 * rho).ravel(), ((1.0 - c1) * rho).ravel()])


@pytest.mark.parametrize("name,n", [("kh", 16), ("rt", 8), ("tg", 8)])
def test_uniform_concentration_scales_the_density_rhs(name, n):
    desc, opts, u = make_config(name, n=n)
    o = Oracle(desc, opts, u)
    N = o.N
    rng = np.random.default_rng(1)
    u1 = u + 1e-3 * np.abs(u) * rng.uniform(-1, 1, u.size) * (np.arange(u.size) >= 2 * N)
    o.set_scalars(0.3 * u1[:N], 1, renormalize=False)
    r = o.scalar_rhs(u1, 0.3 * u1[:N])
    R = o.rhs(u1)[:N]
    assert np.max(np.abs(r - 0.3 * R)) <= 1e-13 * np.max(np.abs(R))


def test_flow_at_rest_leaves_scalars_unchanged():
    desc, opts, u = make_config("rt", noise=False, perturb=False)
    o = Oracle(desc, opts, u)
    s0 = _two_scalars(desc, u)
    o.set_scalars(s0, 2)
    for _ in range(3):
        assert o.implicit_step()[0] == 0
    assert np.array_equal(o.get_scalars(), s0)


@pytest.mark.parametrize("name,n", [("kh", 32), ("tg", 8)])
def test_scalar_totals_conserved_without_renormalisation(name, n):
    desc, opts, u = make_config(name, n=n)
    o = Oracle(desc, opts, u)
    N = o.N
    s0 = _two_scalars(desc, u)
    o.set_scalars(s0, 2, renormalize=False)
    for _ in range(3):
        assert o.implicit_step()[0] == 0
    s1 = o.get_scalars()
    for k in range(2):
        a0, a1 = s0[k * N:(k + 1) * N], s1[k * N:(k + 1) * N]
        assert abs(exact_sum(a1) - exact_sum(a0)) <= 1e-13 * np.abs(a0).sum()
    assert o.scalar_its()[0] >= 1


def test_renormalised_concentrations_sum_to_one():
    desc, opts, u = make_config("kh", n=32)
    o = Oracle(desc, opts, u)
    N = o.N
    o.set_scalars(_two_scalars(desc, u), 2)
    for _ in range(3):
        assert o.implicit_step()[0] == 0
    s = o.get_scalars()
    rho = o.get_state()[:N]
    assert np.max(np.abs((s[:N] + s[N:]) / rho - 1.0)) <= 1e-14


def test_uniform_concentration_stays_uniform():
    desc, opts, u = make_config("kh", n=32)
    o = Oracle(desc, opts, u)
    N = o.N
    o.set_scalars(0.3 * u[:N], 1, renormalize=False)
    for _ in range(3):
        assert o.implicit_step()[0] == 0
    rho = o.get_state()[:N]
    assert np.max(np.abs(o.get_scalars() / rho - 0.3)) <= 1e-7


def test_scalar_failure_restores_flow_and_scalars():
    desc, opts, u = make_config("kh", n=16, max_halvings=0)
    s0 = _two_scalars(desc, u)
    o2 = Oracle(desc, dict(opts, gmres_max_cycles=0), u)  # every linear solve fails at once
    o2.set_scalars(s0, 2)
    assert o2.implicit_step()[0] == 2
    assert np.array_equal(o2.get_state(), u) and np.array_equal(o2.get_scalars(), s0)


def test_scalars_relying_on_the_flow_take_its_newton_count():
    """scalar_converge = 0 (section 2.2's default: the non-linear iterations
    stop on the fluid's convergence alone): each step's scalar solve takes
    exactly as many Newton iterations as the flow's solve of that step, and
    the result stays within the flow's tolerance level of the converged
    scalars; the flow is untouched either way"""
    desc, opts, u = make_config("kh", n=32)
    s0 = _two_scalars(desc, u)
    runs = {}
    for conv in (1, 0):
        o = Oracle(desc, dict(opts, scalar_converge=conv), u)
        o.set_scalars(s0, 2, renormalize=False)
        its = []
        for _ in range(3):
            rc, st = o.implicit_step()
            assert rc == 0
            its.append((int(st["newton_its"]), o.scalar_its()[0]))
        runs[conv] = (o.get_state(), o.get_scalars(), its)
    assert all(sc == max(fl, 1) for fl, sc in runs[0][2]), runs[0][2]
    assert np.array_equal(runs[0][0], runs[1][0])
    e = np.linalg.norm(runs[0][1] - runs[1][1]) / np.linalg.norm(runs[1][1])
    assert e <= 1e-6, e


# ---------------------------------------------------------------- GPU against the oracle
@pytest.mark.gpu
@pytest.mark.parametrize("name,n,steps,renorm,conv", [("kh", 32, 3, True, 1), ("rt", None, 4, True, 1),
                                                      ("tg", 16, 2, False, 1), ("rad", 16, 2, True, 1),
                                                      ("kh", 32, 3, True, 0), ("rt", None, 4, False, 0)])
def test_gpu_scalars_match_oracle(name, n, steps, renorm, conv):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_10053_amd import jfnk
    jfnk.load()
    # each step from u^n on both sides (setting the oracle's state below
    # clears its extrapolation history)
    desc, opts, u = make_config(name, n=n, scalar_converge=conv, newton_extrapolate=0)
    s0 = _two_scalars(desc, u)
    g = jfnk.Problem(desc, opts, u)
    g.set_scalars(s0, 2, renorm)
    o = Oracle(desc, opts, u)
    o.set_scalars(s0, 2, renorm)
    plain = jfnk.Problem(desc, opts, u)  # the same flow without scalars
    for k in range(steps):
        o.set_state(g.get_state())
        o.set_scalars(g.get_scalars(), 2, renorm)
        rg, sg = g.implicit_step()
        ro, so = o.implicit_step()
        assert rg == 0 and ro == 0
        assert (sg["scalar_newton_its"], sg["scalar_gmres_its"]) == o.scalar_its()
        sgpu, sor = g.get_scalars(), o.get_scalars()
        e = np.linalg.norm(sgpu - sor) / np.linalg.norm(sor)
        print("step", k, sg["scalar_newton_its"], sg["scalar_gmres_its"], e, flush=True)
        assert e <= 1e-10
        assert plain.implicit_step()[0] == 0
    # the scalars do not touch the flow: bit for bit the run without them
    assert np.array_equal(g.get_state(), plain.get_state())
    # mixing width from the scalars, eq. (16), against the oracle's definition
    from oracle import diagnostics as dg
    d = g.eval_diagnostics(None, 1.0, 2.0, 1)
    ref = dg.mixing_width_scalars(g.get_state(), g.get_scalars(), desc, 1)
    assert d["mix_width_scalars"] == pytest.approx(ref, rel=1e-12, abs=1e-15)
