"""The -fopenmp build of the oracle (used only to time it on all host cores)
gives bit for bit the results of the serial build: its parallel loops write
each cell's outputs from inputs they do not write, and every reduction stays
serial."""
import os

import numpy as np
import pytest

# a few threads that sleep between parallel loops: the suite may run beside
# other test workers on the same cores (read when the threaded build loads)
os.environ.setdefault("OMP_NUM_THREADS", "3")
os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")

from oracle import Oracle
from workloads import PCS_ADI, make_config


@pytest.mark.parametrize("name,n,steps,over", [("tg", 16, 2, {}), ("rt", 16, 2, {}), ("rad", 16, 2, {}),
                                                ("srad", 16, 1, {}), ("kh", 32, 1, {"pc_solver": PCS_ADI}),
                                                ("kh", 32, 1, {"energy_form": 1})])
def test_threaded_oracle_is_bitwise_serial(name, n, steps, over):
    desc, opts, u = make_config(name, n=n, **over)
    a, b = Oracle(desc, opts, u), Oracle(desc, opts, u, threaded=True)
    for _ in range(steps):
        ra, sa = a.implicit_step()
        rb, sb = b.implicit_step()
        assert ra == rb == 0
        assert (sa["newton_its"], sa["gmres_its"], sa["dt"]) == (sb["newton_its"], sb["gmres_its"], sb["dt"])
    assert np.array_equal(a.get_state(), b.get_state())
    v = np.random.default_rng(1).uniform(-1, 1, u.size) * (u != 0)
    assert np.array_equal(a.rhs(u), b.rhs(u))
    dt = a.time_step(u)["dt"]
    b.time_step(u)
    assert np.array_equal(a.precond(u, dt, v), b.precond(u, dt, v))
