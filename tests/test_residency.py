"""Host test of the admission rule that keeps channel pumps co-resident
(paper_2509_01425_amd/csrc/residency.h), compiled with g++ into a driver:
a pump launched while others run on other streams follows every one that
drives one of its rings, and the oldest others until everything that can be
in flight together fits the device at once."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("residency") / "residency_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2509_01425_amd", "csrc"),
                    os.path.join(ROOT, "tests", "residency_driver.cpp"), "-o", exe], check=True)

    def run(cases):
        text = ""
        for cap, nw, live in cases:
            text += f"{cap} {nw} {len(live)}\n"
            for w, d, s, c in live:
                text += f"{w} {int(d)} {int(s)} {int(c)}\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
        res = []
        for line in out.stdout.splitlines():
            v = [int(x) for x in line.split()]
            assert v[0] == len(v) - 1
            res.append(v[1:])
        return res
    return run


def test_fixed_cases(driver):
    cases = [
        (100, 40, []),                                              # nothing in flight
        (100, 40, [(30, 0, 0, 0), (30, 0, 0, 0)]),                  # 100 fits exactly
        (100, 40, [(30, 0, 0, 0), (31, 0, 0, 0)]),                  # oldest waited
        (100, 40, [(30, 0, 0, 0), (31, 0, 0, 0), (50, 0, 0, 0)]),   # two oldest
        (100, 40, [(90, 1, 0, 0), (60, 0, 0, 0)]),                  # done ones don't count
        (100, 40, [(90, 0, 1, 0), (60, 0, 0, 0)]),                  # same stream: ends first
        (100, 10, [(5, 0, 0, 0), (5, 0, 0, 1)]),                    # shared ring: always waited
        (100, 100, [(1, 0, 0, 0), (1, 0, 1, 0)]),                   # the whole device
    ]
    assert driver(cases) == [[], [], [0], [0, 1], [], [], [1], [0]]


def test_random_cases_keep_the_invariant(driver):
    g = np.random.default_rng(7)
    cases = []
    for _ in range(2000):
        cap = int(g.integers(1, 200))
        nw = int(g.integers(1, cap + 1))
        live = [(int(g.integers(1, cap + 1)), g.random() < 0.2, g.random() < 0.2,
                 g.random() < 0.1) for _ in range(int(g.integers(0, 8)))]
        cases.append((cap, nw, live))
    for (cap, nw, live), waits in zip(cases, driver(cases)):
        assert waits == sorted(set(waits))
        for i in waits:
            w, d, s, c = live[i]
            assert not d and not s  # never a finished or same-stream launch
        left = [i for i, (w, d, s, c) in enumerate(live) if not d and not s and i not in waits]
        # everything left in flight beside the new launch fits, and shares no ring
        assert sum(live[i][0] for i in left) + nw <= cap
        assert not any(live[i][3] for i in left)
        # capacity waits are the oldest: no skipped older launch could have stayed
        cap_waits = [i for i in waits if not live[i][3]]
        if cap_waits:
            last = cap_waits[-1]
            assert all(i in waits for i in range(last)
                       if not live[i][1] and not live[i][2])
