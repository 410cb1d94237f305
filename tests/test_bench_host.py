"""bench.py's host logic (no GPU needed): the one-GPU contract and the
counter-summary lookup that feeds roofline.traffic."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_bench(*args, env=None):
    e = dict(os.environ)
    if env:
        e.update(env)
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          cwd=ROOT, env=e, timeout=600)


def test_more_than_one_gpu_is_refused_with_a_message():
    for args, env in ((("--gpus", "2"), None), ((), {"WORLD_SIZE": "2"})):
        r = _run_bench(*args, env=env)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_traffic_lookup_follows_the_kernel_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.kernel_sources_sha()
    good = tmp_path / "good.md"
    good.write_text("summary\n```\nsources_sha256=%s\n"
                    "traffic class=mg_smooth kernel=k_gs<double, 3> bytes_per_launch=18388349\n"
                    "traffic class=residual_out kernel=k_out<3> bytes_per_launch=602964762\n```\n" % sha)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.measured_traffic("mg_smooth") == 18388349.0
    assert bench.measured_traffic("residual_out") == 602964762.0
    assert bench.measured_traffic("pc_back") is None
    stale = tmp_path / "stale.md"
    stale.write_text(good.read_text().replace(sha, "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic("mg_smooth") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("mg_smooth") is None


def test_committed_counter_summary_is_well_formed():
    """the committed summary carries a sources line and one traffic line per
    class, each with a positive byte count"""
    sys.path.insert(0, ROOT)
    import bench
    text = open(bench.TRAFFIC_FILE).read()
    lines = [ln for ln in text.splitlines() if ln.startswith(("sources_sha256=", "traffic class="))]
    assert lines[0].startswith("sources_sha256=") and len(lines[0].split("=", 1)[1]) == 64
    classes = [dict(t.split("=", 1) for t in ln.split()[1:] if "=" in t) for ln in lines[1:]]
    assert {"mg_smooth", "residual_out", "residual_mflux", "residual_prim", "residual_flux"} <= {c["class"] for c in classes}
    assert all(float(c["bytes_per_launch"]) > 0 for c in classes)


def test_whole_step_byte_model_reproduces_the_planning_figures():
    """The whole-step algorithmic byte model gives the planning figures of
    the Taylor-Green 128^3 byte budget: 3 Newton x 10 GMRES iterations,
    36.6 KB per cell-step in FP64 and 26.1 KB with an FP32 basis; and the
    round-1 measured counts (11.1 Newton, 31.45 GMRES) 27.7 KB."""
    sys.path.insert(0, ROOT)
    import bench
    assert abs(bench.model_bytes_per_cell(3, 30, 3, 1.0) - 36600.0) < 1e-9
    assert abs(bench.model_bytes_per_cell(3, 30, 3, 0.5) - 26100.0) < 1e-9
    assert abs(bench.model_bytes_per_cell(11.1, 31.45, 3, 1.0) - 27.7e3) < 50.0
    assert bench.model_bytes_per_cell(0, 0, 3, 1.0) == 120.0
