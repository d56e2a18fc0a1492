"""CPU tests of the serving loop's admission policy (sched_policy.hpp, the
host logic behind tsylv_submit), compiled with g++ from the library's own
header and driven with simulated queues: FIFO with head-of-line blocking,
rejection of requests that can never fit, batches of the batched method
formed from the consecutive compatible requests at the head, sized to the
arena and capped, and no admission without a free slot.  The admission
loop applies the policy until it waits, so the last test replays that loop
over a simulated arena."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_09233_amd", "csrc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = tmp_path_factory.mktemp("sp") / "sched_policy_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "sched_policy_check.cpp"),
                    "-o", str(out)], check=True)
    return str(out)


def decide(exe, scenarios):
    lines = []
    for slots, largest, cap, maxb, reqs in scenarios:
        lines.append("%d %d %d %d %d %s" % (slots, largest, cap, maxb, len(reqs), " ".join(reqs)))
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       check=True)
    return [tuple(l.split()) for l in r.stdout.strip().splitlines()]


def test_single_requests_fifo_and_head_of_line(exe):
    out = decide(exe, [
        (8, 120, 1000, 512, ["S100", "S50"]),   # head fits
        (8, 20, 1000, 512, ["S50", "S10"]),     # head waits; S10 behind it is not admitted
        (8, 1000, 1000, 512, ["S1000"]),        # exactly the free block
        (8, 500, 1000, 512, ["S2000", "S10"]),  # can never fit: rejected
        (0, 1000, 1000, 512, ["S10"]),          # no free slot
        (8, 1000, 1000, 512, []),               # empty queue
    ])
    assert out == [("single", "1"), ("wait", "0"), ("single", "1"), ("reject", "1"),
                   ("wait", "0"), ("wait", "0")]


def test_batches_from_the_head(exe):
    out = decide(exe, [
        (8, 1000, 1000, 512, ["B1:10", "B1:10", "B2:10", "B1:10"]),  # options class ends it
        (8, 1000, 1000, 512, ["B1:10", "S5", "B1:10"]),              # a single request ends it
        (8, 350, 1000, 512, ["B1:100", "B1:100", "B1:100", "B1:100"]),  # largest prefix that fits
        (8, 50, 1000, 512, ["B1:100", "B1:100"]),                    # even one waits
        (8, 50, 100, 512, ["B1:100", "B1:1"]),                       # one never fits: rejected
        (8, 10 ** 9, 10 ** 9, 512, ["B1:1"] * 600),                  # capped
        (0, 1000, 1000, 512, ["B1:10"]),                             # no free slot
        (8, 1000, 1000, 512, ["S10", "B1:10"]),                      # single at the head
    ])
    assert out == [("batch", "2"), ("batch", "1"), ("batch", "3"), ("wait", "0"),
                   ("reject", "1"), ("batch", "512"), ("wait", "0"), ("single", "1")]


def test_admission_loop_over_a_simulated_arena(exe):
    """Replays the scheduler's loop: apply decisions until 'wait', taking
    the admitted bytes from a single free block and a slot each time."""
    queue = ["S400", "B1:100", "B1:100", "B1:100", "S300", "S50"]
    free, cap, slots = 1000, 1000, 3
    admitted = []
    while True:
        kind, cnt = decide(exe, [(slots, free, cap, 512, queue)])[0]
        cnt = int(cnt)
        if kind == "wait":
            break
        taken, queue = queue[:cnt], queue[cnt:]
        if kind == "reject":
            admitted.append(("reject", taken))
            continue
        need = sum(int(t.split(":")[-1].lstrip("S")) for t in taken) + (16 if kind == "batch" else 0)
        free -= need
        slots -= 1
        admitted.append((kind, taken))
    assert admitted == [("single", ["S400"]), ("batch", ["B1:100", "B1:100", "B1:100"])]
    assert queue == ["S300", "S50"] and free == 1000 - 400 - 316  # S300 waits for memory
