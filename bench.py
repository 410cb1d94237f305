"""Benchmark: implicit cell-steps per second of the Crank-Nicolson JFNK step
on the 3D Taylor-Green vortex at 128^3 (CFL_hydro 20, Newton rtol 1e-8,
GMRES(30), multigrid physics-based preconditioner), on one MI355X.

A step is one full implicit time step (time-step selection, Crank-Nicolson
old-time term, Newton iterations with preconditioned GMRES).  The state is
resident in HBM before the timed region.  Three forms are timed: plain FP64,
the mixed form (FP32 preconditioner and Krylov basis, FP64 residual,
Jacobian-free differences and orthogonalisation), and FP64 with the
internal-energy variable of eq. (2) as written.  A serving mix of
independent simulations through the continuous-batching request loop is
measured beside it (throughput and p50/p99 step latency).  Prints one JSON
line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "implicit cell-steps/s at Newton rtol 1e-8 (3D TG 128^3) + % HBM peak; p50/p99"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# timed-region kernel timing: windows of 4 consecutive launches carry events,
# a window opening at a launch with probability 1/251 (a fixed pseudo-random
# sequence, so the windows do not alias with the solver's periodic launch
# pattern), the dominant class counted after a window's first launch.  An
# evented launch costs about 5 us more than a plain one, so the windows are
# kept sparse: about 60 evented launches per step (< 1 % of the step time)
SAMPLE_PERIOD, SAMPLE_BURST = 251, 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(jfnk, torch, desc, opts, u0, steps, warmup, prof=True):
    dev = torch.from_numpy(u0).cuda()
    names = jfnk.profile_class_names()
    # warm-up: a separate instance takes the first `warmup` steps with every
    # kernel class timed (per-class table and the dominant class), then is
    # discarded
    table = {}
    if warmup > 0:
        wp = jfnk.Problem(desc, opts, dev)
        wp.profile_enable(names if prof else [])
        wp.profile_sample(1)
        for _ in range(warmup):
            rc, st = wp.implicit_step()
            if rc != 0:
                raise RuntimeError("warm-up step failed: %s" % st)
        table = wp.profile_read()
        wp.close()
    timed = {k: v for k, v in table.items() if v[2] > 0}
    dominant = max(timed, key=lambda k: timed[k][0]) if timed else "mg_smooth"
    # timed run: steps 1..K from t = 0 on a fresh instance; events on the
    # dispatches of sampled launch windows, the dominant class counted
    prob = jfnk.Problem(desc, opts, dev)
    prob.profile_enable([dominant] if prof else [])
    prob.profile_sample(SAMPLE_PERIOD, SAMPLE_BURST)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    stats = []
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        rc, st = prob.implicit_step()
        ev[k][1].record()
        if rc != 0:
            raise RuntimeError("timed step %d failed: %s" % (k, st))
        stats.append(st)
        log("  step %d dt %.4f newton %d gmres %d %.1f ms" % (k, st["dt"], st["newton_its"], st["gmres_its"],
                                                              st["wall_ms"]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom = prob.profile_read().get(dominant, (0.0, 0, 0.0))
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    state = prob.get_state()
    prob.close()
    return dict(wall=t1 - t0, step_ms=step_ms, stats=stats, table=table, dominant=dominant, dom=dom,
                state=state)


def serving_mix(nreq, steps_lo, steps_hi, seed):
    """Requests of the serving workload: problem uniform over rt/kh/tg/rad,
    2D size N uniform over 32, 48, 64, 96, 128, 192, 256, 384, 512 (rt N x 2N,
    kh N x N, rad N x 4N; sizes of the form 2^j or 3 * 2^j coarsen to a few
    cells per axis), 3D size uniform over 32/64/96/128, steps uniform over
    [steps_lo, steps_hi], precision FP64 or mixed with equal probability."""
    from workloads import PREC_FP64, PREC_MIXED
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nreq):
        name = ["rt", "kh", "tg", "rad"][rng.integers(4)]
        n = int(rng.choice([32, 64, 96, 128] if name == "tg" else [32, 48, 64, 96, 128, 192, 256, 384, 512]))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        prec = PREC_MIXED if rng.integers(2) else PREC_FP64
        out.append((name, n, steps, prec))
    return out


def run_serving(jfnk, mix, hbm_bytes, active, rate, seed):
    """Submit the mix at Poisson arrivals of the given rate (requests/s;
    0 = all at once) and wait for every request."""
    from workloads import make_config
    reqs = []
    for name, n, steps, prec in mix:
        d, o, u = make_config(name, n=n, prec=prec)
        reqs.append((d, o, u, steps))
    kinds = [m[0] for m in mix]
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1.0 / rate, len(reqs)) if rate > 0 else np.zeros(len(reqs))
    srv = jfnk.Server(hbm_bytes, active)
    t0 = time.perf_counter()
    t_next = t0
    ids = []
    for (d, o, u, k), gap in zip(reqs, gaps):
        t_next += gap
        delay = t_next - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(d, o, u, k))
    res = [srv.wait(i) for i in ids]
    wall = time.perf_counter() - t0
    srv.close()
    step_ms = np.concatenate([r[2] for r in res])
    cell_steps = sum(r[1]["cells"] * r[1]["steps_done"] for r in res)
    lat = np.array([r[1]["t_done_ms"] - r[1]["t_submit_ms"] for r in res])
    queue = np.array([r[1]["t_admit_ms"] - r[1]["t_submit_ms"] for r in res])
    by_kind = {}
    for kind, r in zip(kinds, res):
        b = by_kind.setdefault(kind, dict(requests=0, steps=0, cell_steps=0.0, step_ms=0.0, gmres=0))
        b["requests"] += 1
        b["steps"] += r[1]["steps_done"]
        b["cell_steps"] += r[1]["cells"] * r[1]["steps_done"]
        b["step_ms"] += float(np.sum(r[2]))
        b["gmres"] += r[1]["gmres_its"]
    for b in by_kind.values():
        b["mean_step_ms"] = b.pop("step_ms") / max(b["steps"], 1)
        b["gmres_per_step"] = b.pop("gmres") / max(b["steps"], 1)
    return dict(requests=len(res), failed=sum(1 for r in res if r[1]["status"] != 0), wall_s=wall,
                by_problem=by_kind,
                cell_steps_per_s=cell_steps / wall, requests_per_s=len(res) / wall,
                step_p50_ms=float(np.percentile(step_ms, 50)), step_p99_ms=float(np.percentile(step_ms, 99)),
                request_p50_ms=float(np.percentile(lat, 50)), request_p99_ms=float(np.percentile(lat, 99)),
                queue_p50_ms=float(np.percentile(queue, 50)), queue_p99_ms=float(np.percentile(queue, 99)),
                steps=int(sum(r[1]["steps_done"] for r in res)))


def serving(jfnk, args):
    lo, hi = (int(x) for x in args.serve_steps.split(","))
    mix = serving_mix(args.serve_requests, lo, hi, args.serve_seed)
    hbm = int(args.serve_hbm_gb * (1 << 30))
    log("serving: %d requests, saturated pass" % len(mix))
    sat = run_serving(jfnk, mix, hbm, args.serve_active, 0.0, args.serve_seed)
    out = {"workload": "serving mix: %d requests (rt/kh/tg/rad, 2D 32..512, 3D 32..128 cubed, %d..%d steps, "
                       "FP64 or mixed), seed %d" % (len(mix), lo, hi, args.serve_seed),
           "max_active": args.serve_active, "arena_gb": args.serve_hbm_gb, "saturated": sat}
    if args.serve_poisson:
        rate = 0.8 * sat["requests_per_s"]
        log("serving: Poisson arrivals at %.2f requests/s" % rate)
        poi = run_serving(jfnk, mix, hbm, args.serve_active, rate, args.serve_seed)
        poi["arrival_rate_per_s"] = rate
        out["poisson_0.8x"] = poi
    return out


def model_bytes_per_cell(newton, gmres, ndim, basis_bytes_ratio):
    """Algorithmic HBM bytes per cell of one implicit step with the given
    Newton and GMRES iteration counts (the step's method minimum, each vector
    read or written once): with S_v the bytes of one FP64 state vector per
    cell and S_b the basis bytes per cell (S_v, or S_v/2 for an FP32 basis),
    3 S_v for the time step and the Crank-Nicolson old-time term; per Newton
    iteration 3 S_v for F, k S_b + 6 S_v for the update (k = GMRES
    iterations per Newton iteration); per GMRES iteration 12 S_v (preconditioner
    about 4, Jacobian-free product 5, new basis vector 3) plus 3 j S_b for the
    fused CGS2 passes against the j vectors already in the basis."""
    sv = 8.0 * (2 + ndim)
    sb = sv * basis_bytes_ratio
    if newton <= 0:
        return 3.0 * sv
    k = gmres / newton
    return (3.0 * sv + newton * (3.0 * sv + k * sb + 6.0 * sv) + gmres * 12.0 * sv
            + newton * 1.5 * k * (k + 1.0) * sb)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tg128_fp64_hbm_traffic.md")


def kernel_sources_sha():
    """sha256 over the HIP kernel sources (csrc/*.hip, *.hpp, sorted by name)"""
    import glob
    import hashlib
    d = os.path.join(ROOT, "paper_1610_10053_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(d, "*.hip")) + glob.glob(os.path.join(d, "*.hpp"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(cls):
    """HBM bytes per launch of a kernel class from the committed counter
    summary, or None when it is absent or was taken on other kernel sources"""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    sha = None
    per = {}
    for line in text.splitlines():
        if line.startswith("sources_sha256="):
            sha = line.split("=", 1)[1].strip()
        elif line.startswith("traffic class="):
            kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
            per[kv.get("class")] = float(kv["bytes_per_launch"])
    if sha != kernel_sources_sha():
        return None
    return per.get(cls)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, steps, threaded):
    """The oracle (plain C, FP64) on the host: TG n^3, the benchmark's set-up,
    `steps` implicit steps from t = 0 on one core (the serial build), or
    with threaded=True its -fopenmp build on all the host threads OpenMP
    starts (same results bit for bit: parallel cell loops, serial
    reductions)."""
    import oracle
    from oracle import Oracle
    from workloads import make_config
    desc, opts, u0 = make_config("tg", n=n)
    orc = Oracle(desc, opts, u0, threaded=threaded)
    its = []
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, st = orc.implicit_step()
        if rc != 0:
            raise RuntimeError("oracle step failed")
        its.append((st["newton_its"], st["gmres_its"]))
    t = time.perf_counter() - t0
    cells = n ** 3
    nthr = oracle.threads(threaded)
    return dict(value=cells * steps / t, unit="cell-steps/s", cores=nthr, kind="oracle",
                sample="Taylor-Green %d^3 (the benchmark's set-up: CFL 20, Newton rtol 1e-8, GMRES(30), multigrid "
                       "preconditioner), %d implicit step(s) from t=0 (Newton/GMRES iterations %s), %s, %.1f s"
                       % (n, steps, its, "%d threads (-fopenmp build)" % nthr if threaded else "one core", t),
                nproc=os.cpu_count(), cpu_model=_cpu_model())


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--forms", default="fp64,mixed,internal",
                    help="fp64, mixed (FP32 preconditioner and basis), internal (FP64, energy variable rho e)")
    ap.add_argument("--cpu-n", type=int, default=128, help="grid of the one-core oracle leg")
    ap.add_argument("--cpu-steps", type=int, default=1, help="implicit steps of the one-core oracle leg")
    ap.add_argument("--cpu-n-all", type=int, default=128, help="grid of the all-cores oracle leg")
    ap.add_argument("--cpu-steps-all", type=int, default=3, help="implicit steps of the all-cores oracle leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-prof", action="store_true", help="no HIP-event timing (for external profilers)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-geometries", action="store_true",
                    help="skip the radiative layer in Cartesian and spherical geometry")
    ap.add_argument("--geo-steps", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-steps", default="20,200", help="lo,hi implicit steps per request")
    ap.add_argument("--serve-poisson", action="store_true",
                    help="also run the mix with Poisson arrivals at 0.8x the saturated request rate")
    # as many workers as the process's hardware queues (GPU_MAX_HW_QUEUES, 4 by
    # default): more concurrent requests only lengthen each step
    ap.add_argument("--serve-active", type=int, default=4)
    ap.add_argument("--serve-hbm-gb", type=float, default=64.0)
    ap.add_argument("--serve-seed", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the implicit step of one grid runs on one device, and several "
              "GPUs would need a domain-decomposed path, which is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1610_10053_amd import jfnk
    from workloads import make_config, ENERGY_INTERNAL, PREC_FP64, PREC_MIXED

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    jfnk.load()
    desc, opts, u0 = make_config("tg", n=args.n)
    cells = desc["n"][0] * desc["n"][1] * desc["n"][2]
    forms = [f for f in args.forms.split(",") if f]
    res = {}
    for f in forms:
        log("form", f)
        if f == "internal":
            d_i, o_i, u_i = make_config("tg", n=args.n, energy_form=ENERGY_INTERNAL)
            res[f] = run_form(jfnk, torch, d_i, o_i, u_i, args.steps, args.warmup, prof=not args.no_prof)
            continue
        o = dict(opts, prec=PREC_MIXED if f == "mixed" else PREC_FP64)
        res[f] = run_form(jfnk, torch, desc, o, u0, args.steps, args.warmup, prof=not args.no_prof)

    def summary(r, basis_ratio=1.0):
        ms = r["step_ms"]
        st = r["stats"]
        value = cells * len(ms) / r["wall"]
        model = sum(model_bytes_per_cell(s["newton_its"], s["gmres_its"], desc["ndim"], basis_ratio) for s in st)
        whole_gbs = model * cells / r["wall"] / 1e9
        ms_d, cnt, by = r["dom"]
        achieved = (by / (ms_d * 1e-3)) / 1e9 if ms_d > 0 else None
        kern = {}
        for k, (t, c, b) in sorted(r["table"].items(), key=lambda kv: -kv[1][0]):
            gbs = b / (t * 1e-3) / 1e9 if b > 0 and t > 0 else None
            kern[k] = dict(ms=round(t, 3), launches=c, avg_us=round(1e3 * t / c, 2),
                           gbs=round(gbs, 1) if gbs else None,
                           frac=round(gbs / PEAK_HBM_GBS, 3) if gbs else None)
        return dict(value=value, ms_per_step=1e3 * r["wall"] / len(ms), p50_ms=float(np.percentile(ms, 50)),
                    p99_ms=float(np.percentile(ms, 99)), first_step_ms=float(ms[0]),
                    newton_its_per_step=float(np.mean([s["newton_its"] for s in st])),
                    gmres_its_per_step=float(np.mean([s["gmres_its"] for s in st])),
                    dominant=r["dominant"], dominant_gbs=achieved,
                    dominant_avg_us=1e3 * ms_d / cnt if cnt else None, kernels=kern,
                    max_rel_res=float(max(s["rel_res"] for s in st)),
                    newton_exit_counts={"residual": sum(1 for s in st if s["newton_exit"] == 0),
                                        "density_correction": sum(1 for s in st if s["newton_exit"] == 1)},
                    whole_step={"model_bytes_per_cell_step": model / len(st), "achieved": whole_gbs,
                                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": whole_gbs / PEAK_HBM_GBS})

    main_form = forms[0]
    s0 = summary(res[main_form], 0.5 if main_form == "mixed" else 1.0)
    out = {
        "metric": METRIC, "value": s0["value"], "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": s0["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if main_form == "fp64" else "f64+f32", "data": "synthetic",
        "config": {"workload": "taylor_green_%d^3" % args.n, "cells": cells, "grid": desc["n"],
                   "cfl_hydro": opts["cfl_hydro"], "newton_rtol": opts["newton_rtol"],
                   "gmres_restart": opts["gmres_restart"], "preconditioner": "acoustic, %d multigrid V(2,2) cycle(s)" % opts["mg_cycles"],
                   "first_newton_iterate": ("u^n, or its extrapolation in time from the last two accepted states "
                                            "when that has the smaller residual; stopping test relative to F(u^n)"
                                            if opts.get("newton_extrapolate") else "u^n"),
                   "form": main_form, "timed_steps": "steps 1..%d of the run from t=0 (warm-up on a "
                   "separate instance)" % args.steps},
        "p50_ms": s0["p50_ms"], "p99_ms": s0["p99_ms"], "first_step_ms": s0["first_step_ms"],
        "newton_its_per_step": s0["newton_its_per_step"], "gmres_its_per_step": s0["gmres_its_per_step"],
        "max_rel_res": s0["max_rel_res"], "newton_exit_counts": s0["newton_exit_counts"],
        "roofline": {"bound": "hbm", "kernel": s0["dominant"], "achieved": s0["dominant_gbs"],
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": (s0["dominant_gbs"] / PEAK_HBM_GBS) if s0["dominant_gbs"] else None,
                     "avg_launch_us": s0["dominant_avg_us"], "traffic": measured_traffic(s0["dominant"]),
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                     "whole_step": s0["whole_step"]},
        "kernels": s0["kernels"],
    }
    for f in forms[1:]:
        sf = summary(res[f], 0.5 if f == "mixed" else 1.0)
        a, b = res[f]["state"], res[main_form]["state"]
        if f == "internal" or main_form == "internal":
            # the energy fields hold different variables: compare rho and m
            N = cells
            a = np.concatenate([a[:N], a[2 * N:]])
            b = np.concatenate([b[:N], b[2 * N:]])
            sf["rho_m_rel_l2_vs_%s" % main_form] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        else:
            sf["state_rel_l2_vs_%s" % main_form] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        sf.pop("kernels")
        sf["speedup_vs_%s" % main_form] = sf["value"] / s0["value"]
        out.setdefault("forms", {})[f] = sf
    if not args.no_geometries:
        # the radiative layer (conduction block in the preconditioner) as a
        # Cartesian box and as a spherical shell segment of the same cell count
        geo = {}
        for name in ("rad", "srad"):
            log("geometry", name)
            d_g, o_g, u_g = make_config(name)
            r = run_form(jfnk, torch, d_g, o_g, u_g, args.geo_steps, 1, prof=False)
            nc = d_g["n"][0] * d_g["n"][1] * d_g["n"][2]
            geo[name] = dict(grid=d_g["n"][:2], geometry="spherical (r, theta)" if name == "srad" else "cartesian",
                             steps=args.geo_steps, ms_per_step=1e3 * r["wall"] / args.geo_steps,
                             value=nc * args.geo_steps / r["wall"], unit="cell-steps/s",
                             newton_its_per_step=float(np.mean([st["newton_its"] for st in r["stats"]])),
                             gmres_its_per_step=float(np.mean([st["gmres_its"] for st in r["stats"]])))
        out["radiative_layer"] = geo
    if not args.no_serve:
        out["serving"] = serving(jfnk, args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one core)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.cpu_steps, threaded=False)
        log("cpu baseline (oracle, all cores)")
        out["cpu_baseline_all_cores"] = cpu_baseline(args.cpu_n_all, args.cpu_steps_all, threaded=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
