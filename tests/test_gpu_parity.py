"""GPU (MI355X) parity of the HIP library against the oracle, through the
C-ABI.  Same seeded inputs on both sides; tolerances stated per test.

FP64 residual, time step and preconditioner follow the same evaluation order
on both sides (no floating-point contraction), so they are compared bit for
bit.  So is the Jacobian-free product when both sides are given the same
difference step eps (jfnk_apply_jv_eps): then they difference F at the same
perturbed state, element by element.  With its automatic step the product
takes eps from two norms whose summation order differs, so the two sides
difference F at states that differ in the last bits; a roundoff change of F,
about 1e-16 of its largest terms, divided by eps ~ 1.5e-8 bounds that
product's relative difference by ~1e-8 in the worst case (measured: up to
3.4e-12), so the automatic product is compared to 1e-9 in relative L2 on
top of the bitwise check.  Newton steps are compared in relative L2, overall
and per field against each field's own norm (floored, see _fields_rel),
against the 1e-10 bar.
"""
import numpy as np
import pytest

from _helpers import exact_sum, rel_l2
from workloads import (ENERGY_INTERNAL, PC_ACOUSTIC, PC_ACOUSTIC_DIFFUSION, PC_NONE, PCS_ADI, PREC_MIXED,
                       make_config, mirror_x, split_state, unknown_mask)

pytestmark = pytest.mark.gpu

CASES = [("rt", 16), ("kh", 32), ("tg", 16), ("rad", 16)]
FULL = [("rt", None), ("kh", None), ("rad", None)]


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _lib():
    from paper_1610_10053_amd import jfnk
    jfnk.load()  # fails loudly if the HIP library is missing
    return jfnk


def _pair(name, n, **over):
    from oracle import Oracle
    jfnk = _lib()
    desc, opts, u = make_config(name, n=n, **over)
    print("case", name, n, over, flush=True)
    return desc, opts, u, jfnk.Problem(desc, opts, u), Oracle(desc, opts, u)


def _direction(desc, seed):
    rng = np.random.default_rng(seed)
    n = (2 + desc["ndim"]) * desc["n"][0] * desc["n"][1] * desc["n"][2]
    return np.where(unknown_mask(desc), rng.uniform(-1, 1, n), 0.0)


FIELD_FLOOR = 1e-6


def _fields_rel(a, b, desc, scales):
    """Per-field error in scaled variables, each relative to that field's
    own norm, floored at FIELD_FLOOR * sqrt(N): a field at noise level (the
    radiative layer's velocities sit at 1e-10 of their scale) is compared
    against 1e-6 of its scale per cell, so a noise field that is wrong by
    its own size still fails the 1e-10 bar by four orders of magnitude."""
    fa, fb = split_state(a, desc), split_state(b, desc)
    out = {}
    for i, k in enumerate(fa):
        ref = max(np.linalg.norm(fb[k] / scales[i]), FIELD_FLOOR * np.sqrt(fb[k].size))
        out[k] = np.linalg.norm((fa[k] - fb[k]) / scales[i]) / ref
    return out


def _perturbed_rad(n, amp=1e-3, seed=12):
    """The radiative layer with seeded velocities of amplitude amp times the
    sound speed at the bottom on every interior face, so that its momenta
    are well above noise and are checked as fields of their own."""
    desc, opts, u = make_config("rad", n=n)
    N = desc["n"][0] * desc["n"][1]
    rng = np.random.default_rng(seed)
    f = split_state(u, desc)
    rho = f["rho"]
    cs = np.sqrt(desc["gamma"] * (desc["gamma"] - 1.0) * np.max(f["E"] / rho))
    mask = unknown_mask(desc)
    for d, k in enumerate(("mx", "my")):
        rf = 0.5 * (rho + np.roll(rho, 1, axis=2 - d))
        v = amp * cs * rng.uniform(-1, 1, rho.shape)
        f[k][...] = rf * v
    u2 = np.concatenate([f["rho"].ravel(), f["E"].ravel(), f["mx"].ravel(), f["my"].ravel()])
    return desc, opts, np.where(mask, u2, 0.0)


# ---------------------------------------------------------------- components

@pytest.mark.parametrize("name,n", CASES + FULL)
def test_residual_components_bitwise(torch_cuda, name, n):
    desc, opts, u, g, o = _pair(name, n)
    assert np.array_equal(g.eval_rhs(u), o.rhs(u))
    tg, to = g.eval_time_step(u), o.time_step(u)
    assert tg["dt"] == to["dt"] and np.array_equal(tg["scales"], to["scales"])
    dt = to["dt"]
    b = o.cn_old(u, dt)
    assert np.array_equal(g.eval_cn_old(u, dt), b)
    u1 = u + 1e-3 * np.abs(u) * _direction(desc, 3)
    assert np.array_equal(g.eval_residual(u1, b, dt), o.residual(u1, b, dt))


@pytest.mark.parametrize("name,n", CASES + FULL)
def test_jv_parity(torch_cuda, name, n):
    desc, opts, u, g, o = _pair(name, n)
    ts = o.time_step(u)
    g.eval_time_step(u)  # same scales on both sides
    dt = ts["dt"]
    b = o.cn_old(u, dt)
    u1 = u + 1e-3 * np.abs(u) * _direction(desc, 4)
    v = _direction(desc, 5)
    wo = o.jv(u1, b, dt, v)
    assert rel_l2(g.apply_jv(u1, b, dt, v), wo) < 1e-9
    # same difference step on both sides: element by element, bit for bit
    for eps in (1.3e-8, 2.0e-6):
        assert np.array_equal(g.apply_jv_eps(u1, b, dt, v, eps), o.jv_eps(u1, b, dt, v, eps))


@pytest.mark.parametrize("name,n", [("tg", 16), ("rad", 16)])
def test_zero_direction_products(torch_cuda, name, n):
    """Degenerate direction v = 0: the product's step eps is 0 and the
    product is exactly 0 (no division by the zero step reaches the output);
    the preconditioner maps 0 to 0; both as the oracle."""
    desc, opts, u, g, o = _pair(name, n)
    ts = o.time_step(u)
    g.eval_time_step(u)
    dt = ts["dt"]
    b = o.cn_old(u, dt)
    v = np.zeros_like(u)
    w = g.apply_jv(u, b, dt, v)
    assert not np.any(w) and np.array_equal(w, o.jv(u, b, dt, v))
    z = g.apply_precond(u, dt, v)
    assert not np.any(z) and np.array_equal(z, o.precond(u, dt, v))


@pytest.mark.parametrize("solver", ["mg", "adi"])
@pytest.mark.parametrize("name,n", CASES + FULL)
def test_preconditioner_bitwise(torch_cuda, name, n, solver):
    over = {"pc_solver": PCS_ADI} if solver == "adi" else {}
    desc, opts, u, g, o = _pair(name, n, **over)
    dt = o.time_step(u)["dt"]
    g.eval_time_step(u)
    v = _direction(desc, 6)
    assert np.array_equal(g.apply_precond(u, dt, v), o.precond(u, dt, v))


@pytest.mark.parametrize("name,n", CASES + [("kh", 256)])
def test_newton_solve_parity_ew_forcing(torch_cuda, name, n):
    """Newton solves with the Eisenstat-Walker forcing of the linear
    tolerance: the same Newton and GMRES counts as the oracle's, states within
    1e-10 overall and per field."""
    from workloads import FORCING_EW
    desc, opts, u, g, o = _pair(name, n, gmres_forcing=FORCING_EW)
    ts = o.time_step(u)
    dt = ts["dt"]
    rg, sg = g.newton_solve(dt)
    ro, so = o.newton_solve(dt)
    print("gpu", sg["newton_its"], sg["gmres_its"], "oracle", so["newton_its"], so["gmres_its"], flush=True)
    assert rg == 0 and ro == 0
    assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
    ug, uo = g.get_state(), o.get_state()
    assert rel_l2(ug, uo) <= 1e-10
    for k, e in _fields_rel(ug, uo, desc, ts["scales"]).items():
        assert e <= 1e-10, (k, e)


@pytest.mark.parametrize("name,n", [("rt", 16), ("kh", 32), ("tg", 16), ("rad", 16), ("rt", None)])
def test_steps_parity_extrapolated_first_iterate(torch_cuda, name, n):
    """Implicit steps with the extrapolated first Newton iterate: per step the
    same choice (taken or not) as the oracle, the same Newton and GMRES
    counts, the extrapolated residual norm within 1e-8 relative (1e-12
    absolute where it is a cancellation-level residual of a near-static
    state), and the states within 1e-10 overall and per field."""
    desc, opts, u, g, o = _pair(name, n, newton_extrapolate=1)
    taken = 0
    for k in range(4):
        rg, sg = g.implicit_step()
        ro, so = o.implicit_step()
        fx, tk = o.extrap_info()
        print("step", k, "gpu", sg["newton_its"], sg["gmres_its"], sg["extrapolated"], sg["f_extrap"],
              "oracle", so["newton_its"], so["gmres_its"], tk, fx, flush=True)
        assert rg == 0 and ro == 0
        assert bool(sg["extrapolated"]) == tk
        assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
        if fx < 0.0:
            assert sg["f_extrap"] == -1.0
        else:
            assert sg["f_extrap"] == pytest.approx(fx, rel=1e-8, abs=1e-12)
        taken += tk
    ug, uo = g.get_state(), o.get_state()
    assert rel_l2(ug, uo) <= 1e-10
    for k, e in _fields_rel(ug, uo, desc, o.time_step(uo)["scales"]).items():
        assert e <= 1e-10, (k, e)


def test_extrapolated_iterate_uniform_gravity_gpu(torch_cuda):
    """A uniform gas under uniform gravity (m linear, E quadratic in time):
    the GPU's extrapolated iterate after steps 0.4, 0.4 and then 0.7 is taken
    and its residual norm is the closed form of the oracle's pin."""
    from _helpers import desc2d, opts
    from oracle import Oracle
    jfnk = _lib()
    desc = desc2d(8, 8, g=(0.3, -0.7), gamma=1.4)
    rho, p, vx, vy = 1.3, 2.0, 0.2, -0.1
    E0 = p / (desc["gamma"] - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    u = np.concatenate([np.full(64, rho), np.full(64, E0), np.full(64, rho * vx), np.full(64, rho * vy)])
    o_ = opts(newton_rtol=1e-13, newton_extrapolate=1)
    g, o = jfnk.Problem(desc, o_, u), Oracle(desc, o_, u)
    for dt in (0.4, 0.4):
        assert g.newton_solve(dt)[0] == 0 and o.newton_solve(dt)[0] == 0
    S_E = o.time_step(o.get_state())["scales"][1]
    rg, sg = g.newton_solve(0.7)
    assert rg == 0 and sg["extrapolated"] == 1
    g2 = 0.3 ** 2 + 0.7 ** 2
    assert sg["f_extrap"] == pytest.approx(8.0 * 0.5 * rho * g2 * 0.7 * (0.4 + 0.7) / S_E, rel=1e-9)


@pytest.mark.parametrize("name,n", [("kh", 1024), ("rt", 512)])
def test_large_2d_preconditioner_bitwise(torch_cuda, name, n):
    """2D hierarchies whose finest level exceeds 2^18 cells (KH 1024^2
    periodic, RT 512x1024 with walls along y), where the prolongation onto
    the finest level runs one thread per coarse cell, are bit for bit the
    oracle's multigrid preconditioner."""
    desc, opts, u, g, o = _pair(name, n)
    dt = o.time_step(u)["dt"]
    g.eval_time_step(u)
    v = _direction(desc, 6)
    assert np.array_equal(g.apply_precond(u, dt, v), o.precond(u, dt, v))


@pytest.mark.parametrize("name,n", [("kh", 32), ("tg", 16)])
def test_preconditioner_after_steps_bitwise(torch_cuda, name, n):
    """The preconditioner applied after implicit steps, whose GMRES solves
    form each basis vector's acoustic right-hand side as they store it, is bit
    for bit the oracle's on the stepped state (nothing of the solves' state
    leaks into a later application)."""
    desc, opts, u, g, o = _pair(name, n)
    for _ in range(2):
        rc, _ = g.implicit_step()
        assert rc == 0
    u1 = g.get_state()
    dt = o.time_step(u1)["dt"]
    g.eval_time_step(u1)
    v = _direction(desc, 7)
    assert np.array_equal(g.apply_precond(u1, dt, v), o.precond(u1, dt, v))


@pytest.mark.parametrize("name,n", [("kh", 66), ("rad", 68), ("kh", 54), ("kh", 108), ("rad", 60), ("kh", 40),
                                    ("tg", 24), ("rt", 20), ("kh", 48), ("rt", 24)])
def test_odd_and_large_coarsest_level_parity(torch_cuda, name, n):
    """Coarsest multigrid levels with an odd periodic axis, too large for the
    single-workgroup solve (33x33, 17x68: multi-block sweeps between two
    buffers) or inside it (27x27, 15x60, 5x5, 3x3x3, 5x10: two-phase sweeps in
    LDS, below a larger first level of the workgroup's for 54x54, 30x120,
    12^3, 48x48 and 24x48, the last two with 3x3 and 3x6 coarsest levels);
    preconditioner bitwise, Newton step to 1e-10."""
    desc, opts, u, g, o = _pair(name, n)
    dt = o.time_step(u)["dt"]
    g.eval_time_step(u)
    v = _direction(desc, 7)
    assert np.array_equal(g.apply_precond(u, dt, v), o.precond(u, dt, v))
    rg, sg = g.newton_solve(dt)
    ro, so = o.newton_solve(dt)
    assert rg == 0 and ro == 0 and sg["gmres_its"] == so["gmres_its"]
    assert rel_l2(g.get_state(), o.get_state()) <= 1e-10


# ---------------------------------------------------------------- ragged in-plane tiles

@pytest.mark.parametrize("shape,form", [((96, 10, 6), 0), ((4, 70, 12), 1)])
def test_periodic_3d_ragged_tiles_bitwise(torch_cuda, shape, form):
    """A periodic 3D grid of unequal axes whose x rows end in a partial
    64-cell tile or are narrower than one, and whose y extent ends in a
    partial 4-row tile (the sweeps that stage in-plane tiles in LDS), in the
    total- and internal-energy forms: residual and Jacobian-free product at a
    common difference step bit for bit against the oracle, on a random
    state."""
    from oracle import Oracle
    jfnk = _lib()
    desc, opts, _ = make_config("tg", n=16, energy_form=ENERGY_INTERNAL if form else 0)
    desc = dict(desc, n=list(shape))
    N = shape[0] * shape[1] * shape[2]
    rng = np.random.default_rng(11)
    rho = 1.0 + 0.3 * rng.uniform(-1, 1, N)
    E = 20.0 + rng.uniform(-1, 1, N)
    m = 0.5 * rng.uniform(-1, 1, 3 * N)
    u = np.concatenate([rho, E, m])
    print("case", shape, form, flush=True)
    g, o = jfnk.Problem(desc, opts, u), Oracle(desc, opts, u)
    assert np.array_equal(g.eval_rhs(u), o.rhs(u))
    ts = o.time_step(u)
    g.eval_time_step(u)
    dt = ts["dt"]
    b = o.cn_old(u, dt)
    assert np.array_equal(g.eval_cn_old(u, dt), b)
    u1 = u + 1e-3 * np.abs(u) * _direction(desc, 6)
    assert np.array_equal(g.eval_residual(u1, b, dt), o.residual(u1, b, dt))
    v = _direction(desc, 7)
    assert np.array_equal(g.apply_jv_eps(u1, b, dt, v, 1.3e-8), o.jv_eps(u1, b, dt, v, 1.3e-8))


# ---------------------------------------------------------------- the smallest grids

@pytest.mark.parametrize("name,n", [("rt", 4), ("kh", 4), ("tg", 4), ("rad", 4)])
def test_smallest_grids_parity(torch_cuda, name, n):
    """Four cells on the shortest axis (the least the library accepts; its
    multigrid stops at two): stencils whose halo wraps more than once around
    a periodic axis, tiles wider than the grid, the whole V-cycle in the
    coarse kernel.  Residual, time step and preconditioner bit for bit, one
    Newton solve with identical counts and the state within 1e-10."""
    desc, opts, u, g, o = _pair(name, n)
    assert np.array_equal(g.eval_rhs(u), o.rhs(u))
    ts = o.time_step(u)
    assert g.eval_time_step(u)["dt"] == ts["dt"]
    dt = ts["dt"]
    v = _direction(desc, 9)
    assert np.array_equal(g.apply_precond(u, dt, v), o.precond(u, dt, v))
    rg, sg = g.newton_solve(dt)
    ro, so = o.newton_solve(dt)
    assert rg == 0 and ro == 0
    assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
    assert rel_l2(g.get_state(), o.get_state()) <= 1e-10


# ---------------------------------------------------------------- Newton steps

@pytest.mark.parametrize("name,n", CASES + FULL + [("rad_perturbed", 16), ("rad_perturbed", 32)])
def test_newton_solve_parity(torch_cuda, name, n):
    if name == "rad_perturbed":
        from oracle import Oracle
        desc, opts, u = _perturbed_rad(n)
        print("case", name, n, flush=True)
        g, o = _lib().Problem(desc, opts, u), Oracle(desc, opts, u)
    else:
        desc, opts, u, g, o = _pair(name, n)
    ts = o.time_step(u)
    dt = ts["dt"]
    rg, sg = g.newton_solve(dt)
    ro, so = o.newton_solve(dt)
    assert rg == 0 and ro == 0
    assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
    assert sg["newton_exit"] == so["newton_exit"]
    ug, uo = g.get_state(), o.get_state()
    assert rel_l2(ug, uo) <= 1e-10
    fr = _fields_rel(ug, uo, desc, ts["scales"])
    print("per-field", {k: "%.2e" % e for k, e in fr.items()}, flush=True)
    for k, e in fr.items():
        assert e <= 1e-10, (k, e)
    if name == "rad_perturbed":
        # the momenta are fields of their own here, not noise
        f = split_state(uo, desc)
        for i, k in ((2, "mx"), (3, "my")):
            assert np.linalg.norm(f[k] / ts["scales"][i]) > 1e-5 * np.sqrt(f[k].size)


@pytest.mark.parametrize("name,n,steps", [("rt", None, 10), ("kh", 64, 5), ("tg", 16, 4), ("rad", 32, 5)])
def test_steps_from_identical_states(torch_cuda, name, n, steps):
    """Each step starts both sides from the same state (the GPU's).  Setting
    the oracle's state clears its extrapolation history, so both sides start
    each step from u^n."""
    desc, opts, u, g, o = _pair(name, n, newton_extrapolate=0)
    for k in range(steps):
        o.set_state(g.get_state())
        rg, sg = g.implicit_step()
        ro, so = o.implicit_step()
        assert rg == 0 and ro == 0
        assert sg["dt"] == so["dt"]
        e = rel_l2(g.get_state(), o.get_state())
        print("step", k, sg["newton_its"], sg["gmres_its"], e, flush=True)
        assert e <= 1e-10


@pytest.mark.parametrize("name,n", [("tg", 16), ("rad", 16)])
def test_adi_and_unpreconditioned_paths(torch_cuda, name, n):
    for over in ({"pc_solver": PCS_ADI, "gmres_max_cycles": 40}, {"pc": PC_NONE, "gmres_max_cycles": 40}):
        if name == "rad" and over.get("pc") == PC_NONE:
            continue
        desc, opts, u, g, o = _pair(name, n, **over)
        dt = o.time_step(u)["dt"] * (0.25 if name == "rad" else 1.0)
        rg, sg = g.newton_solve(dt)
        ro, so = o.newton_solve(dt)
        assert rg == ro
        if rg == 0:
            assert rel_l2(g.get_state(), o.get_state()) <= 1e-10


@pytest.mark.parametrize("name,n", [("tg", 16), ("rad", 16), ("kh", 32)])
def test_adi_mixed_precision_converges_to_fp64(torch_cuda, name, n):
    """ADI line solves in the mixed form (FP32 lines of the acoustic block,
    FP64 conduction lines): the same Newton tolerance reached, the state
    within 1e-8 of the FP64 ADI run after two steps"""
    jfnk = _lib()
    out = []
    for prec in (0, PREC_MIXED):
        desc, opts, u = make_config(name, n=n, pc_solver=PCS_ADI, gmres_max_cycles=40, prec=prec)
        print("case", name, n, prec, flush=True)
        p = jfnk.Problem(desc, opts, u)
        for _ in range(2):
            rc, st = p.implicit_step()
            assert rc == 0, st
            assert st["newton_exit"] == 0 or st["max_rel_corr"] <= 1e-12
        out.append(p.get_state())
        p.close()
    assert rel_l2(out[1], out[0]) <= 1e-8


# ---------------------------------------------------------------- internal-energy form (eq. 2 as written)

@pytest.mark.parametrize("name,n", CASES + [("rad", None), ("kh", 54), ("rt", 20)])
def test_internal_energy_form_components(torch_cuda, name, n):
    """residual, time step and preconditioner bit for bit, Jv to 1e-9"""
    desc, opts, u, g, o = _pair(name, n, energy_form=ENERGY_INTERNAL)
    assert np.array_equal(g.eval_rhs(u), o.rhs(u))
    tg, to = g.eval_time_step(u), o.time_step(u)
    assert tg["dt"] == to["dt"] and np.array_equal(tg["scales"], to["scales"])
    dt = to["dt"]
    b = o.cn_old(u, dt)
    assert np.array_equal(g.eval_cn_old(u, dt), b)
    u1 = u + 1e-3 * np.abs(u) * _direction(desc, 8)
    assert np.array_equal(g.eval_residual(u1, b, dt), o.residual(u1, b, dt))
    v = _direction(desc, 9)
    assert rel_l2(g.apply_jv(u1, b, dt, v), o.jv(u1, b, dt, v)) < 1e-9
    assert np.array_equal(g.apply_jv_eps(u1, b, dt, v, 1.3e-8), o.jv_eps(u1, b, dt, v, 1.3e-8))
    assert np.array_equal(g.apply_precond(u, dt, v), o.precond(u, dt, v))


@pytest.mark.parametrize("name,n,steps", [("rt", None, 4), ("kh", 32, 3), ("tg", 16, 3), ("rad", 32, 3)])
def test_internal_energy_form_steps(torch_cuda, name, n, steps):
    """implicit steps of the internal-energy form from identical states:
    same dt, same iteration counts, states within 1e-10 (each step from u^n:
    setting the oracle's state clears its extrapolation history)"""
    desc, opts, u, g, o = _pair(name, n, energy_form=ENERGY_INTERNAL, newton_extrapolate=0)
    for k in range(steps):
        o.set_state(g.get_state())
        rg, sg = g.implicit_step()
        ro, so = o.implicit_step()
        assert rg == 0 and ro == 0
        assert sg["dt"] == so["dt"]
        assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
        e = rel_l2(g.get_state(), o.get_state())
        print("step", k, sg["newton_its"], sg["gmres_its"], e, flush=True)
        assert e <= 1e-10


def test_internal_energy_form_mixed_precision(torch_cuda):
    """the mixed form of the internal-energy variable converges to the
    FP64 form's answer within the Newton tolerance"""
    jfnk = _lib()
    desc, opts, u = make_config("tg", n=32, energy_form=ENERGY_INTERNAL)
    out = []
    for prec in (0, PREC_MIXED):
        opts["prec"] = prec
        p = jfnk.Problem(desc, opts, u)
        for _ in range(2):
            rc, st = p.implicit_step()
            assert rc == 0
        out.append(p.get_state())
        p.close()
    assert rel_l2(out[1], out[0]) <= 1e-8


# ---------------------------------------------------------------- 2D spherical geometry

def _sph_flow(n, internal=False):
    """a spherical wedge (r in [1, 2], theta in [pi/4, 3pi/4], walls) with a
    smooth flow, radial gravity and conduction: every geometric term active"""
    import math
    from _helpers import state_from_primitive
    from workloads import default_opts
    desc = dict(ndim=2, n=[n, n, 1], lo=[1.0, math.pi / 4, 0.0], hi=[2.0, 3 * math.pi / 4, 1.0],
                bc=[1, 1, 0], gamma=5.0 / 3.0, g=[-0.7, 0.0, 0.0], chi0=0.05, heat_balance=0,
                energy_form=ENERGY_INTERNAL if internal else 0, geometry=1)
    rho = lambda x, y, z: 1.0 + 0.2 * np.sin(2.0 * x) * np.cos(2.0 * y)
    ur = lambda x, y, z: 0.02 + 0.01 * np.sin(3.0 * x) * np.cos(y)
    ut = lambda x, y, z: -0.015 + 0.01 * np.cos(2.0 * x) * np.sin(3.0 * y)
    p = lambda x, y, z: 1.0 + 0.1 * np.cos(2.0 * x - y)
    u = np.where(unknown_mask(desc), state_from_primitive(desc, rho, (ur, ut), p), 0.0)
    opts = default_opts(cfl_hydro=4.0, pc=PC_ACOUSTIC_DIFFUSION, gmres_eta=1e-2)
    return desc, opts, u


def _sph_pair(kind, n):
    from oracle import Oracle
    jfnk = _lib()
    if kind == "srad":
        desc, opts, u = make_config("srad", n=n)
    else:
        desc, opts, u = _sph_flow(n, internal=(kind == "flow_internal"))
    print("case", kind, n, flush=True)
    return desc, opts, u, jfnk.Problem(desc, opts, u), Oracle(desc, opts, u)


@pytest.mark.parametrize("kind,n", [("srad", 8), ("srad", 12), ("srad", 32), ("flow", 16), ("flow", 20), ("flow", 48),
                                    ("flow_internal", 16)])
def test_spherical_components(torch_cuda, kind, n):
    """residual, time step and preconditioner bit for bit, Jv to 1e-9"""
    desc, opts, u, g, o = _sph_pair(kind, n)
    assert np.array_equal(g.eval_rhs(u), o.rhs(u))
    tg, to = g.eval_time_step(u), o.time_step(u)
    assert tg["dt"] == to["dt"] and np.array_equal(tg["scales"], to["scales"])
    dt = to["dt"]
    b = o.cn_old(u, dt)
    assert np.array_equal(g.eval_cn_old(u, dt), b)
    u1 = u + 1e-3 * np.abs(u) * _direction(desc, 10)
    assert np.array_equal(g.eval_residual(u1, b, dt), o.residual(u1, b, dt))
    v = _direction(desc, 11)
    assert rel_l2(g.apply_jv(u1, b, dt, v), o.jv(u1, b, dt, v)) < 1e-9
    assert np.array_equal(g.apply_jv_eps(u1, b, dt, v, 1.3e-8), o.jv_eps(u1, b, dt, v, 1.3e-8))
    assert np.array_equal(g.apply_precond(u, dt, v), o.precond(u, dt, v))


@pytest.mark.parametrize("kind,n,steps", [("srad", 16, 3), ("flow", 32, 3), ("flow_internal", 16, 2)])
def test_spherical_steps(torch_cuda, kind, n, steps):
    """implicit steps from identical states: same dt and iteration counts,
    states within 1e-10"""
    desc, opts, u, g, o = _sph_pair(kind, n)
    for k in range(steps):
        o.set_state(g.get_state())
        rg, sg = g.implicit_step()
        ro, so = o.implicit_step()
        assert rg == 0 and ro == 0
        assert sg["dt"] == so["dt"]
        assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
        e = rel_l2(g.get_state(), o.get_state())
        print("step", k, sg["newton_its"], sg["gmres_its"], e, flush=True)
        assert e <= 1e-10


def test_spherical_mixed_precision_and_rejections(torch_cuda):
    """the mixed form converges to the FP64 answer; Cartesian-only calls
    refuse a spherical problem"""
    jfnk = _lib()
    desc, opts, u = make_config("srad", n=16)
    out = []
    for prec in (0, PREC_MIXED):
        opts["prec"] = prec
        p = jfnk.Problem(desc, opts, u)
        for _ in range(2):
            rc, st = p.implicit_step()
            assert rc == 0
        out.append(p.get_state())
        if prec == 0:
            with pytest.raises(jfnk.JfnkError):
                p.eval_diagnostics(None)
            with pytest.raises(jfnk.JfnkError):
                p.set_scalars(np.ones(p.N), 1)
        p.close()
    assert rel_l2(out[1], out[0]) <= 1e-8


# ---------------------------------------------------------------- invariants on the GPU path

@pytest.mark.parametrize("name,n", [("kh", 64), ("tg", 16)])
def test_gpu_conservation(torch_cuda, name, n):
    jfnk = _lib()
    desc, opts, u = make_config(name, n=n)
    g = jfnk.Problem(desc, opts, u)
    f0 = split_state(u, desc)
    s0 = {k: exact_sum(v) for k, v in f0.items()}
    mom = sum(np.abs(f0[k]).sum() for k in f0 if k.startswith("m"))
    for _ in range(3):
        assert g.implicit_step()[0] == 0
    f1 = split_state(g.get_state(), desc)
    for k in s0:
        scale = mom if k.startswith("m") else np.abs(f0[k]).sum()
        assert abs(exact_sum(f1[k]) - s0[k]) <= 1e-13 * scale, k


@pytest.mark.parametrize("name,n,steps", [("rt", None, 10), ("rad", 32, 10)])
def test_gpu_hydrostatic_state_preserved(torch_cuda, name, n, steps):
    jfnk = _lib()
    desc, opts, u = make_config(name, n=n, noise=False, perturb=False)
    g = jfnk.Problem(desc, opts, u)
    for _ in range(steps):
        rc, st = g.implicit_step()
        assert rc == 0 and st["newton_its"] == 0
    assert rel_l2(g.get_state(), u) <= 1e-14


def test_gpu_rt_mirror_symmetry_bitwise(torch_cuda):
    jfnk = _lib()
    desc, opts, u = make_config("rt", pc=PC_NONE)
    g = jfnk.Problem(desc, opts, u)
    for _ in range(5):
        assert g.implicit_step()[0] == 0
        s = g.get_state()
        assert np.array_equal(mirror_x(s, desc), s)


def test_device_buffers_and_determinism(torch_cuda):
    torch = torch_cuda
    jfnk = _lib()
    desc, opts, u = make_config("kh", n=64)
    outs = []
    for _ in range(2):
        g = jfnk.Problem(desc, opts, torch.from_numpy(u).cuda())
        for _ in range(2):
            assert g.implicit_step()[0] == 0
        d = torch.empty(u.size, dtype=torch.float64, device="cuda")
        g.get_state(d)
        outs.append(d.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


# ---------------------------------------------------------------- failure handling forced from the host

def test_gpu_failures_restore_state(torch_cuda):
    jfnk = _lib()
    desc, opts, u = make_config("kh", n=32, newton_max=1, max_halvings=0)
    g = jfnk.Problem(desc, opts, u)
    rc, st = g.implicit_step()
    assert rc == 1 and np.array_equal(g.get_state(), u)
    desc, opts, u = make_config("kh", n=32, gmres_max_cycles=0, max_halvings=0)
    g = jfnk.Problem(desc, opts, u)
    assert g.implicit_step()[0] == 2 and np.array_equal(g.get_state(), u)
    bad = u.copy()
    bad[7] = np.nan
    desc, opts, _ = make_config("kh", n=32, max_halvings=0)
    g = jfnk.Problem(desc, opts, bad)
    assert g.implicit_step()[0] == 3


def test_gpu_step_halving_recovers(torch_cuda):
    """The halve-and-retry branch of the adaptive step: with at most four
    Newton iterations the first attempts at the CFL time step fail, the state
    is restored and dt halved until a solve converges; the GPU rejects as
    many attempts as the oracle, lands on the same dt and the same state."""
    desc, opts, u, g, o = _pair("kh", 16, newton_max=4, max_halvings=6)
    rg, sg = g.implicit_step()
    ro, so = o.implicit_step()
    print("halving", sg["rejections"], so["rejections"], sg["dt"], so["dt"], flush=True)
    assert rg == 0 and ro == 0
    assert sg["rejections"] == so["rejections"] >= 1
    assert sg["dt"] == so["dt"]
    assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
    assert rel_l2(g.get_state(), o.get_state()) <= 1e-10
    # a second step from the same state on both sides
    o.set_state(g.get_state())
    rg, sg = g.implicit_step()
    ro, so = o.implicit_step()
    assert rg == ro == 0 and sg["rejections"] == so["rejections"] and sg["dt"] == so["dt"]
    assert rel_l2(g.get_state(), o.get_state()) <= 1e-10


# ---------------------------------------------------------------- full size, launch configuration of the benchmark

def test_tg128_components_against_oracle(torch_cuda):
    """Taylor-Green 128^3: residual, time step and preconditioner bitwise,
    Jacobian-free product to 1e-9, at the benchmark's full size."""
    desc, opts, u, g, o = _pair("tg", None)
    assert np.array_equal(g.eval_rhs(u), o.rhs(u))
    ts = o.time_step(u)
    assert g.eval_time_step(u)["dt"] == ts["dt"]
    dt = ts["dt"]
    b = o.cn_old(u, dt)
    v = _direction(desc, 8)
    assert np.array_equal(g.apply_precond(u, dt, v), o.precond(u, dt, v))
    assert rel_l2(g.apply_jv(u, b, dt, v), o.jv(u, b, dt, v)) < 1e-9
    assert np.array_equal(g.apply_jv_eps(u, b, dt, v, 1.3e-8), o.jv_eps(u, b, dt, v, 1.3e-8))


def test_tg128_newton_step_parity(torch_cuda):
    """The benchmark's workload itself: one Newton solve of Taylor-Green
    128^3 at the CFL time step from t = 0, on the GPU and in the oracle (its
    OpenMP build, bit for bit the serial one), with identical Newton and
    GMRES counts and the states within 1e-10 overall and per field."""
    from oracle import Oracle
    jfnk = _lib()
    desc, opts, u = make_config("tg")
    print("case tg 128^3 newton step", flush=True)
    g, o = jfnk.Problem(desc, opts, u), Oracle(desc, opts, u, threaded=True)
    ts = o.time_step(u)
    dt = ts["dt"]
    rg, sg = g.newton_solve(dt)
    ro, so = o.newton_solve(dt)
    print("gpu", sg["newton_its"], sg["gmres_its"], "oracle", so["newton_its"], so["gmres_its"], flush=True)
    assert rg == 0 and ro == 0
    assert (sg["newton_its"], sg["gmres_its"]) == (so["newton_its"], so["gmres_its"])
    assert sg["newton_exit"] == so["newton_exit"]
    ug, uo = g.get_state(), o.get_state()
    assert rel_l2(ug, uo) <= 1e-10
    fr = _fields_rel(ug, uo, desc, ts["scales"])
    print("per-field", {k: "%.2e" % e for k, e in fr.items()}, flush=True)
    for k, e in fr.items():
        assert e <= 1e-10, (k, e)
    g.close()


@pytest.mark.parametrize("prec,form", [(0, 0), (1, 0), (0, 1)])
def test_tg128_step_converges_by_oracle_residual(torch_cuda, prec, form):
    """One full-size step (FP64 and mixed, total-energy form; FP64 in the
    internal-energy form: the three forms the benchmark times): the oracle
    evaluates the Crank-Nicolson residual of the GPU's new state and confirms
    the Newton tolerance, and the conserved sums are unchanged (mass always;
    the total energy in the total-energy form, where it is a conserved
    variable)."""
    desc, opts, u, g, o = _pair("tg", None, prec=prec, energy_form=form)
    rc, st = g.implicit_step()
    assert rc == 0
    un = u
    o.time_step(un)
    b = o.cn_old(un, st["dt"])
    F0 = o.residual(un, b, st["dt"])
    unew = g.get_state()
    F1 = o.residual(unew, b, st["dt"])
    S = o.time_step(un)["scales"]
    N = desc["n"][0] ** 3

    def snorm(F):
        return np.sqrt(sum(np.sum((F[f * N:(f + 1) * N] / S[f]) ** 2) for f in range(5)))
    f0, f1 = snorm(F0), snorm(F1)
    print("tg128 prec", prec, "newton", st["newton_its"], "gmres", st["gmres_its"], "f1/f0", f1 / f0,
          "exit", st["newton_exit"], flush=True)
    # the step's own statistics agree with the oracle's evaluation of F
    assert abs(st["rel_res"] - f1 / f0) <= 1e-6 * (f1 / f0) + 1e-15
    if st["newton_exit"] == 0:
        assert f1 <= 1.05e-8 * f0
    else:
        # the density-correction exit: corrections at roundoff
        assert st["newton_exit"] == 1 and st["max_rel_corr"] <= 1e-12
    for k in (("rho", "E") if form == 0 else ("rho",)):
        a0, a1 = split_state(un, desc)[k], split_state(unew, desc)[k]
        assert abs(exact_sum(a1) - exact_sum(a0)) <= 1e-13 * np.abs(a0).sum()


def test_tg256_step_converges_by_oracle_residual(torch_cuda):
    """Eight times the benchmark's cells (256^3, 84 million unknowns, 56 GB of
    device memory): one FP64 step, the oracle confirms the Newton tolerance
    on the GPU's new state by its own residual, and mass and total energy
    are unchanged."""
    from oracle import Oracle
    jfnk = _lib()
    desc, opts, u = make_config("tg", n=256)
    print("case tg 256^3 step", flush=True)
    g = jfnk.Problem(desc, opts, u)
    rc, st = g.implicit_step()
    print("newton", st["newton_its"], "gmres", st["gmres_its"], "rel_res", st["rel_res"], flush=True)
    assert rc == 0 and st["newton_exit"] == 0
    unew = g.get_state()
    g.close()
    o = Oracle(desc, opts, u)
    S = o.time_step(u)["scales"]
    b = o.cn_old(u, st["dt"])
    F0 = o.residual(u, b, st["dt"])
    F1 = o.residual(unew, b, st["dt"])
    N = 256 ** 3

    def snorm(F):
        return np.sqrt(sum(np.sum((F[f * N:(f + 1) * N] / S[f]) ** 2) for f in range(5)))
    f0, f1 = snorm(F0), snorm(F1)
    print("oracle f1/f0", f1 / f0, flush=True)
    assert abs(st["rel_res"] - f1 / f0) <= 1e-6 * (f1 / f0) + 1e-15
    assert f1 <= 1.05e-8 * f0
    for k in ("rho", "E"):
        a0, a1 = split_state(u, desc)[k], split_state(unew, desc)[k]
        assert abs(exact_sum(a1) - exact_sum(a0)) <= 1e-13 * np.abs(a0).sum()


# ---------------------------------------------------------------- multigrid replayed as a HIP graph

@pytest.mark.parametrize("name,n,prec", [("rt", None, 0), ("kh", 64, 0), ("rad", 32, 0), ("tg", 16, 0),
                                         ("tg", 16, PREC_MIXED), ("srad", 16, 0)])
def test_graph_replayed_multigrid_is_bitwise_the_launches(torch_cuda, name, n, prec):
    """On a stream of its own the problem captures each multigrid solve once
    and replays it as a HIP graph (on the legacy default stream it launches
    the kernels one by one).  Every replay, with the solver's own work and
    synchronisations between replays, gives bit for bit the eager result:
    the preconditioner applied repeatedly, and whole implicit steps."""
    torch = torch_cuda
    jfnk = _lib()
    desc, opts, u = make_config(name, n=n, prec=prec)
    print("case", name, n, prec, flush=True)
    side = torch.cuda.Stream()
    eager = jfnk.Problem(desc, opts, u)  # created on the default stream
    with torch.cuda.stream(side):
        graph = jfnk.Problem(desc, opts, u)
        dt = eager.eval_time_step(u)["dt"]
        graph.eval_time_step(u)
        for k in range(3):
            v = _direction(desc, 20 + k)
            assert np.array_equal(graph.apply_precond(u, dt, v), eager.apply_precond(u, dt, v))
        for k in range(3):
            rg, sg = graph.implicit_step()
            re, se = eager.implicit_step()
            assert rg == re == 0 and sg["gmres_its"] == se["gmres_its"]
            assert np.array_equal(graph.get_state(), eager.get_state()), k
        graph.close()
    eager.close()
