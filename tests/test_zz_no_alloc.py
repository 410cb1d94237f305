"""The allocation-free entry point jfnk_velocity_error_noalloc against the
entry point it mirrors, jfnk_velocity_error, through the C-ABI on the GPU:
the same eq. (17) error bit for bit (same kernels, same summation order),
on two calls in a row of which the second has the smaller input, and
against the oracle's eq. (17) to 1e-12.  A grid whose partial sums do not fit
the fixed scratch is refused before anything is launched."""
import numpy as np
import pytest

from oracle import diagnostics as dg
from workloads import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_10053_amd import jfnk
    jfnk.load()
    return torch, jfnk


def _pair(jfnk, name, n, r):
    d_lo, o_lo, u_lo = make_config(name, n=n)
    d_hi, o_hi, u_hi = make_config(name, n=r * n)
    g_lo, g_hi = jfnk.Problem(d_lo, o_lo, u_lo), jfnk.Problem(d_hi, o_hi, u_hi)
    assert g_lo.implicit_step()[0] == 0
    assert g_hi.implicit_step()[0] == 0
    return d_lo, d_hi, g_lo, g_hi


def test_noalloc_matches_velocity_error_on_two_calls(env):
    torch, jfnk = env
    # first call: Taylor-Green 32^3 against 64^3; second, smaller: KH 16^2 against 32^2
    for name, n, r, axis in (("tg", 32, 2, 0), ("kh", 16, 2, 1)):
        print("case", name, n, r, axis, flush=True)
        d_lo, d_hi, g_lo, g_hi = _pair(jfnk, name, n, r)
        s_lo, s_hi = g_lo.get_state(), g_hi.get_state()
        dev_lo, dev_hi = torch.from_numpy(s_lo).cuda(), torch.from_numpy(s_hi).cuda()
        ref = g_lo.velocity_error(dev_hi, r, axis)
        got = g_lo.velocity_error_noalloc(dev_hi, r, axis)
        got_given = g_lo.velocity_error_noalloc(dev_hi, r, axis, u_low=dev_lo)
        orc = dg.velocity_error(s_lo, d_lo, s_hi, d_hi, axis)
        print(name, ref, got, got_given, orc, flush=True)
        assert ref > 0.0
        assert got == ref and got_given == ref
        assert got == pytest.approx(orc, rel=1e-12)
        g_lo.close()
        g_hi.close()


def test_noalloc_refuses_a_grid_beyond_its_scratch(env):
    torch, jfnk = env
    # 2048 x 2048 cells: 32 x 512 = 16384 blocks of partial sums, one more
    # than the 256 KiB scratch holds
    desc, opts, u = make_config("kh", n=2048, gmres_restart=2)
    g = jfnk.Problem(desc, opts, u)
    hi = torch.zeros(u.size, dtype=torch.float64, device="cuda")
    with pytest.raises(jfnk.JfnkError) as e:
        g.velocity_error_noalloc(hi, 1, 0)
    assert e.value.code == -4
    g.close()
