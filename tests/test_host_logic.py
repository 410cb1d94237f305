"""Host logic of the serving runtime, built with g++ and run on the CPU: the
first-fit range allocator over the device arena (against a brute-force model
of the free ranges) and the admission choice with its starvation bound.  The
driver is built with AddressSanitizer and UndefinedBehaviorSanitizer where
the compiler provides them, so that an out-of-range access or undefined
arithmetic in the allocator fails the run."""
import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1610_10053_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("adm") / "admission_driver")
    base = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-I", CSRC,
            os.path.join(HERE, "cpp", "admission_driver.cpp"), "-o", exe]
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
    if subprocess.run(base + san, capture_output=True).returncode != 0:
        subprocess.run(base, check=True)  # no sanitizer runtime: a plain build
    return exe


def run(exe, cmds):
    out = subprocess.run([exe], input="\n".join(cmds) + "\n", capture_output=True, text=True, check=True)
    return out.stdout.split("\n")[:len(cmds)]


def model_free(size, used):
    """free ranges (start, length) of [0, size) minus the used intervals"""
    free, pos = [], 0
    for o, b in sorted(used):
        if o > pos:
            free.append((pos, o - pos))
        pos = o + b
    if pos < size:
        free.append((pos, size - pos))
    return free


def test_first_fit_and_coalescing_against_a_model(driver):
    rng = random.Random(7)
    size = 1000
    for trial in range(20):
        used = []
        cmds, expect = ["init %d" % size], ["ok"]
        # build the sequence against the model, then check the driver replays it
        for step in range(60):
            if used and rng.random() < 0.4:
                o, b = used.pop(rng.randrange(len(used)))
                cmds.append("release %d %d" % (o, b))
                expect.append("ok")
            else:
                b = rng.randint(1, 200)
                fit = [f for f in model_free(size, used) if f[1] >= b]
                cmds.append("alloc %d" % b)
                if fit:
                    used.append((fit[0][0], b))
                    expect.append(str(fit[0][0]))
                else:
                    expect.append("-1")
            free = model_free(size, used)
            cmds.append("free")
            expect.append("%d %d" % (sum(f[1] for f in free), len(free)))
        assert run(driver, cmds) == expect, trial


def test_oldest_fitting_request_is_admitted(driver):
    # arena 100: a 70 and a 50 cannot both fit; the 20 behind the 50 passes it
    out = run(driver, ["init 100", "pick 100 70 50 20"])
    assert out[1].split() == ["0", "2"]


def test_a_request_passed_over_often_enough_blocks_later_arrivals(driver):
    # arena 100 with 60 taken: a 50 waits; with max_skips = 2 two requests of
    # 10 may pass it, the third may not
    out = run(driver, ["init 100", "alloc 60", "pick 2 50 10 10 10 10"])
    assert out[2].split() == ["1", "2"]
    out = run(driver, ["init 100", "alloc 60", "pick 100 50 10 10 10 10"])
    assert out[2].split() == ["1", "2", "3", "4"]


def test_exhausted_arena_admits_nothing(driver):
    out = run(driver, ["init 100", "alloc 100", "pick 1 1", "free"])
    assert out[1] == "0" and out[2] == "-" and out[3] == "0 0"
