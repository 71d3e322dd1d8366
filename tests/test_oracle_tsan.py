"""The oracle under ThreadSanitizer (CPU only): many threads, each with its
own context over shared host buffers, as the benchmark's all-core CPU
baseline runs it (tests/oracle_tsan_driver.c).  No race may be reported; a
race planted in the driver (two threads copying into one range) must be."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tsan") / "oracle_tsan")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fsanitize=thread", "-pthread",
           "-fno-tree-loop-distribute-patterns", "-I", os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "oracle", "hicr_oracle.c"), os.path.join(HERE, "oracle_tsan_driver.c"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"no ThreadSanitizer build here: {r.stderr[-300:]}")
    return exe


def _run(exe, *args):
    env = dict(os.environ, TSAN_OPTIONS="exitcode=66 halt_on_error=0")
    return subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=300)


def test_threads_with_their_own_contexts_do_not_race(driver):
    r = _run(driver)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-2000:]
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    assert "all checks passed" in r.stdout


def test_a_planted_race_is_reported(driver):
    r = _run(driver, "overlap")
    assert "WARNING: ThreadSanitizer: data race" in r.stderr
    assert r.returncode == 66
