"""GPU (MI355X) tests of the continuous-batching request loop (jfnk_server_*).

Each request in a mix must give the same result as the same request run
alone through jfnk_create_problem / jfnk_implicit_step: the server issues
the same kernels with the same launch shapes and takes the same host
decisions, so the final states are compared bit for bit and the iteration
counts exactly.
"""
import time

import numpy as np
import pytest

from workloads import PREC_MIXED, make_config

pytestmark = pytest.mark.gpu

MIX = [  # (problem, n, steps, overrides)
    ("rt", None, 6, {}),
    ("kh", 64, 4, {"prec": PREC_MIXED}),
    ("tg", 16, 3, {}),
    ("rad", 32, 4, {}),
    ("kh", 32, 3, {}),
    ("tg", 32, 2, {"prec": PREC_MIXED}),
    ("rt", 16, 5, {"prec": PREC_MIXED}),
    ("kh", 128, 2, {}),
]


@pytest.fixture(scope="module")
def lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_10053_amd import jfnk
    jfnk.load()
    return jfnk


def _alone(jfnk, desc, opts, u, steps):
    p = jfnk.Problem(desc, opts, u)
    its = [0, 0]
    for _ in range(steps):
        rc, st = p.implicit_step()
        assert rc == 0
        its[0] += st["newton_its"]
        its[1] += st["gmres_its"]
    out = p.get_state()
    p.close()
    return out, its


def test_mix_matches_requests_run_alone(lib):
    jfnk = lib
    cases = [make_config(name, n=n, **over) + (steps,) for name, n, steps, over in MIX]
    sizes = [jfnk.footprint_bytes(d, o) for d, o, _, _ in cases]
    # room for about two of the largest at once: later requests queue
    srv = jfnk.Server(int(2.2 * max(sizes)), 3)
    ids = [srv.submit(d, o, u, k) for d, o, u, k in cases]
    results = [srv.wait(i) for i in ids]
    srv.close()
    for (d, o, u, k), (ug, st, ms), case in zip(cases, results, MIX):
        print("case", case, "status", st["status"], "steps", st["steps_done"], flush=True)
        assert st["status"] == 0 and st["steps_done"] == k and len(ms) == k
        ua, its = _alone(jfnk, d, o, u, k)
        assert (st["newton_its"], st["gmres_its"]) == tuple(its)
        assert np.array_equal(ug, ua), case
    # the requests overlapped in time, and the later ones waited for memory
    spans = sorted((r[1]["t_admit_ms"], r[1]["t_done_ms"]) for r in results)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert max(r[1]["t_admit_ms"] - r[1]["t_submit_ms"] for r in results) > 0


def test_requests_arriving_while_others_run_are_admitted(lib):
    jfnk = lib
    d1, o1, u1 = make_config("kh", n=128)
    d2, o2, u2 = make_config("rt")
    srv = jfnk.Server(4 * jfnk.footprint_bytes(d1, o1), 2)
    a = srv.submit(d1, o1, u1, 6)
    t0 = time.time()
    while srv.poll(a) == 0 and time.time() - t0 < 30:
        time.sleep(0.001)
    assert srv.poll(a) in (1, 2)
    b = srv.submit(d2, o2, u2, 4)
    ub, sb, _ = srv.wait(b)
    ua, sa, _ = srv.wait(a)
    srv.close()
    assert sa["status"] == 0 and sb["status"] == 0
    assert sb["t_submit_ms"] >= sa["t_admit_ms"]
    assert np.array_equal(ub, _alone(jfnk, d2, o2, u2, 4)[0])
    assert np.array_equal(ua, _alone(jfnk, d1, o1, u1, 6)[0])


def test_failed_request_does_not_disturb_the_others(lib):
    jfnk = lib
    dg, og, ug = make_config("kh", n=32)
    db, ob, ub = make_config("kh", n=32, newton_max=1, max_halvings=0)
    srv = jfnk.Server(8 * jfnk.footprint_bytes(dg, og), 2)
    ib = srv.submit(db, ob, ub, 3)
    ig = srv.submit(dg, og, ug, 3)
    rb = srv.wait(ib)
    rg = srv.wait(ig)
    srv.close()
    assert rb[1]["status"] == 1 and rb[1]["steps_done"] == 0
    assert np.array_equal(rb[0], ub)  # state restored to u^n
    assert rg[1]["status"] == 0 and np.array_equal(rg[0], _alone(jfnk, dg, og, ug, 3)[0])


def test_request_larger_than_the_arena_is_refused(lib):
    jfnk = lib
    d, o, u = make_config("kh", n=64)
    srv = jfnk.Server(jfnk.footprint_bytes(d, o) // 2, 1)
    with pytest.raises(jfnk.JfnkError):
        srv.submit(d, o, u, 1)
    srv.close()
