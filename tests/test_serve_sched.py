"""The serving scheduler's state machine on the CPU: tests/serve_sim.cpp
drives paper_1401_6749_amd/csrc/serve_sched.h (the same header the serving
engine runs) with a simulated device on a virtual clock -- random Poisson
arrivals over four lattice sizes, workspace budgets from 1x to 4x the largest
request, 1 to 16 slots, overloads, and injected failures of batch creation,
chunk launches and completions, request set-up and finalization -- and stops
at the first state with no progress and no pending event."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_sim.cpp")
CSRC = os.path.join(ROOT, "paper_1401_6749_amd", "csrc")
INC = os.path.join(ROOT, "include")


def _build(tmp_path, csrc=CSRC, name="serve_sim", extra=()):
    exe = str(tmp_path / name)
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", *extra, "-I", csrc, "-I", INC, SRC, "-o", exe, "-lpthread"],
                   check=True, capture_output=True, text=True)
    return exe


@pytest.mark.parametrize("seed", [1, 7, 12])
def test_scheduler_never_stalls(tmp_path, seed):
    """40 random scenarios per seed, half of them with failures: every
    request finishes exactly once (results intact unless a failure was
    injected on its path), FIFO admission, the arena within its size and
    empty at the end, no batch destroyed while it holds work, and never a
    state without progress while requests are outstanding.  Built with the
    address and undefined-behaviour sanitizers (host code only)."""
    exe = _build(tmp_path, extra=("-fsanitize=address,undefined", "-fno-omit-frame-pointer"))
    r = subprocess.run([exe, str(seed), "40"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.count("seed ") == 40
    assert "failures on" in r.stdout and "failures off" in r.stdout


def test_harness_detects_a_stuck_scheduler(tmp_path):
    """The harness is sensitive: a scheduler that never releases idle batches
    (planted in a copy of the header) leaves the queue head waiting for memory
    that nothing will free, and the harness reports that state."""
    broken = tmp_path / "csrc"
    broken.mkdir()
    for f in ("serve_sched.h", "tm_arena.h", "tm_jobs.h", "tm_types.h"):
        txt = open(os.path.join(CSRC, f)).read()
        if f == "serve_sched.h":
            good = "        for (BatchRec *br : idle) drop_batch(br);\n        return !idle.empty();"
            assert good in txt
            txt = txt.replace(good, "        (void)idle;\n        return false;")
        (broken / f).write_text(txt)
    exe = _build(tmp_path, csrc=str(broken), name="serve_sim_broken")
    r = subprocess.run([exe, "1", "40"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 1
    assert "stuck" in r.stderr and "queue head" in r.stderr
