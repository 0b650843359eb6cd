"""Host-thread model of the two GPU solve schedules, under ThreadSanitizer.

tests/schedule_model.cpp replays the persistent schedule's protocol (queues,
epoch flags, done / p2c / rrd / crd counters, the ready3 shortcut, the
forwarding of band tiles that the next round reads) and the three-launch
schedule's lookahead (two streams, two events, per-parity operand panels,
the direct-copy fix-up list), one host thread per workgroup, on small
tiles, with random delays.  Clean runs must be race-free under TSan and
match the sequential blocked solve; each planted protocol mistake must be
caught (a TSan report or a wrong result).  The dependency structure follows
the paper's intra-round concurrency (Section 3.2, Opt-9) and the inter-round
overlap it names as future work (Section 5).  No GPU is involved.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "schedule_model.cpp")
ENV = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")

SHAPES = [  # n, T (tile edge = block), grid (workgroups), seed
    (4, 4, 2, 5),      # one round
    (7, 3, 3, 4),      # three rounds, ragged
    (13, 3, 2, 2),     # fewer workgroups than a round's items
    (22, 3, 9, 1),
    (40, 4, 16, 3),    # ten rounds
    (31, 5, 40, 6),    # more workgroups than items per round
]


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("model") / "schedule_model")
    subprocess.check_call(["g++", "-O1", "-g", "-fsanitize=thread", "-std=c++17", "-pthread", SRC, "-o", exe])
    return exe


def run(exe, sched, shape, reps, mutation=None, timeout=120):
    n, T, grid, seed = shape
    cmd = [exe, sched, str(n), str(T), str(grid), str(seed), str(reps)] + ([mutation] if mutation else [])
    return subprocess.run(cmd, env=ENV, capture_output=True, text=True, timeout=timeout)


@pytest.mark.parametrize("sched", ["persistent", "three", "three-general"])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{s[0]}T{s[1]}g{s[2]}" for s in SHAPES])
def test_schedule_is_race_free(model, sched, shape):
    r = run(model, sched, shape, reps=3)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert r.stdout.startswith("ok ")


MUTATIONS = [("persistent", m) for m in ("no-war", "no-done", "ready3-any", "keep-ready3", "no-diag")] + \
            [("three", m) for m in ("no-evb", "no-eva", "one-parity")]


@pytest.mark.parametrize("sched,mutation", MUTATIONS, ids=[f"{s}-{m}" for s, m in MUTATIONS])
def test_planted_protocol_mistake_is_caught(model, sched, mutation):
    caught = []
    for shape in [(22, 3, 9, 1), (40, 4, 16, 3)]:
        r = run(model, sched, shape, reps=3, mutation=mutation)
        caught.append(r.returncode != 0)
    assert any(caught), f"mutation {mutation!r} of the {sched} schedule was not detected"
