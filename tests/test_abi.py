"""The C-ABI library builds, loads and exports every declared entry point
(no GPU needed: nothing here launches a kernel)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "jfnk.h")).read()
    return sorted(set(re.findall(r"\b(jfnk_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    from paper_1610_10053_amd import jfnk
    assert sorted(jfnk.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_1610_10053_amd import jfnk
    if not os.path.exists(jfnk.LIB_PATH):
        pytest.skip("libjfnk.so not built")
    lib = jfnk.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header_sizes(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct."""
    import ctypes as C
    import subprocess
    from paper_1610_10053_amd import jfnk
    pairs = [("jfnk_problem_desc", jfnk.ProblemDesc), ("jfnk_solver_opts", jfnk.SolverOpts),
             ("jfnk_step_stats", jfnk.StepStats), ("jfnk_request_stats", jfnk.RequestStats),
             ("jfnk_diagnostics", jfnk.Diagnostics)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "jfnk.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in pairs:
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)


def test_default_opts_and_footprint_are_host_only():
    from paper_1610_10053_amd import jfnk
    from workloads import make_config
    if not os.path.exists(jfnk.LIB_PATH):
        pytest.skip("libjfnk.so not built")
    o = jfnk.default_opts()
    assert o.newton_rtol == 1e-8 and o.gmres_restart == 30 and o.mg_nu1 == 2
    desc, opts, u = make_config("tg")
    b = jfnk.footprint_bytes(desc, opts)
    # 128^3 FP64: 31 basis vectors and 30 preconditioned ones of 84 MB dominate
    assert 61 * 83886080 < b < 8.0e9
    opts["prec"] = jfnk.MIXED
    assert jfnk.footprint_bytes(desc, opts) < b


def test_invalid_arguments_are_rejected_on_host():
    from paper_1610_10053_amd import jfnk
    from workloads import make_config
    if not os.path.exists(jfnk.LIB_PATH):
        pytest.skip("libjfnk.so not built")
    desc, opts, u = make_config("kh", n=16)
    bad = dict(desc, n=[15, 16, 1])
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.footprint_bytes(bad, opts)
    assert e.value.code == -1 and "even" in str(e.value)
    with pytest.raises(jfnk.JfnkError):
        jfnk.footprint_bytes(desc, dict(opts, gmres_restart=0))
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.footprint_bytes(desc, dict(opts, newton_target=-1))
    assert e.value.code == -1
    # the mixed form takes the line solves too
    assert jfnk.footprint_bytes(desc, dict(opts, prec=jfnk.MIXED, pc_solver=jfnk.PCS_ADI)) > 0


def test_server_arguments_are_rejected_on_host():
    from paper_1610_10053_amd import jfnk
    if not os.path.exists(jfnk.LIB_PATH):
        pytest.skip("libjfnk.so not built")
    for hbm, act in ((0, 2), (1 << 20, 0), (1 << 20, 65)):
        with pytest.raises(jfnk.JfnkError) as e:
            jfnk.Server(hbm, act)
        assert e.value.code == -1


def test_geometry_energy_and_light_options_are_checked_on_host():
    """spherical grids need 2D, walls on both axes, 0 < r, 0 < theta < pi,
    radial gravity and the multigrid preconditioner; unknown enum values and
    negative light-level sizes are bad arguments"""
    from paper_1610_10053_amd import jfnk
    from workloads import make_config
    if not os.path.exists(jfnk.LIB_PATH):
        pytest.skip("libjfnk.so not built")
    desc, opts, u = make_config("srad", n=8)
    assert jfnk.footprint_bytes(desc, opts) > 0
    cases = [(dict(desc, bc=[1, 0, 0]), opts, -4), (dict(desc, lo=[0.0, 0.5, 0.0]), opts, -1),
             (dict(desc, hi=[2.0, 3.2, 1.0]), opts, -1), (dict(desc, g=[-1.0, 0.5, 0.0]), opts, -4),
             (desc, dict(opts, pc_solver=jfnk.PCS_ADI), -4), (dict(desc, geometry=2), opts, -1),
             (dict(desc, energy_form=2), opts, -1), (desc, dict(opts, mg_light_cells=-1), -1)]
    d3, o3, _ = make_config("tg", n=8)
    cases.append((dict(d3, geometry=1), o3, -4))
    for d, o, code in cases:
        with pytest.raises(jfnk.JfnkError) as e:
            jfnk.footprint_bytes(d, o)
        assert e.value.code == code, (d, e.value)


def test_grid_beyond_32_bit_indexing_is_refused_before_any_allocation():
    """the size check precedes every device call, so it runs on the host"""
    import ctypes as C
    import numpy as np
    from paper_1610_10053_amd import jfnk
    from workloads import make_config
    if not os.path.exists(jfnk.LIB_PATH):
        pytest.skip("libjfnk.so not built")
    lib = jfnk.load()
    desc, opts, u = make_config("tg", n=8)
    big = dict(desc, n=[1024, 1024, 1024])
    one = np.zeros(1)
    h = C.c_void_p()
    rc = lib.jfnk_create_problem(C.byref(jfnk.make_desc(big)), C.byref(jfnk.make_opts(opts)),
                                 one.ctypes.data, 0, None, C.byref(h))
    assert rc == -4 and not h.value
