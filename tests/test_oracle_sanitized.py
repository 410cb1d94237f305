"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The checker itself must not read or write out of bounds or rely on undefined
arithmetic: a copy of `oracle/` is built with both sanitizers into a
temporary directory and driven, in a child process with the sanitizer
runtime preloaded, through implicit steps of every set-up (both energy
forms, the spherical shell, step halving, the time-step controller, passive
scalars with renormalisation) and through its component entry points.  Any
sanitizer report ends the child with a non-zero status.  Skipped where gcc
has no sanitizer runtime.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import sys
sys.path.insert(0, sys.argv[1])
sys.path.insert(1, sys.argv[2])
import numpy as np
import oracle
assert oracle.__file__.startswith(sys.argv[1]), oracle.__file__
from oracle import Oracle
from workloads import make_config
for name, n, over in (("rt", 16, {}), ("kh", 16, {}), ("tg", 8, {}), ("rad", 16, {}), ("srad", 8, {}),
                      ("rt", 16, dict(energy_form=1)), ("kh", 16, dict(newton_max=4, max_halvings=6)),
                      ("kh", 16, dict(dt_grow=1.5, newton_target=3, max_halvings=4)),
                      ("kh", 16, dict(gmres_forcing=1))):
    d, o, u = make_config(name, n=n, **over)
    orc = Oracle(d, o, u)
    for _ in range(2):
        rc, st = orc.implicit_step()
        assert rc == 0, (name, over, st)
d, o, u = make_config("rt", n=16)
orc = Oracle(d, o, u)
N = d["n"][0] * d["n"][1]
s = np.stack([np.linspace(0.0, 1.0, N), 1.0 - np.linspace(0.0, 1.0, N)])
orc.set_scalars(s.ravel(), 2, renormalize=True)
assert orc.implicit_step()[0] == 0
d, o, u = make_config("tg", n=8)
orc = Oracle(d, o, u)
dt = orc.time_step(u)["dt"]
v = np.random.default_rng(1).standard_normal(u.shape)
b = orc.cn_old(u, dt)
assert np.isfinite(orc.precond(u, dt, v)).all()
assert np.isfinite(orc.jv_eps(u, b, dt, v, 1e-8)).all()
assert np.isfinite(orc.residual(u, b, dt)).all()
print("sanitized oracle ok")
'''


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime")
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    src = os.path.join(ROOT, "oracle")
    for f in os.listdir(src):
        if f.endswith(".py") or f.endswith(".c"):
            shutil.copy2(os.path.join(src, f), pkg / f)
    lib = str(pkg / "liboracle.so")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-o", lib, str(pkg / "jfnk_oracle.c"), "-lm"]
    if subprocess.run(cmd, capture_output=True).returncode != 0:
        pytest.skip("sanitizer build not supported")
    shutil.copy2(lib, pkg / "liboracle_omp.so")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", SCRIPT, str(tmp_path), ROOT], env=env, capture_output=True,
                         text=True, timeout=900)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "sanitized oracle ok" in out.stdout
