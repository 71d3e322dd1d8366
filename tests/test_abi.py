"""The C ABI: the built library loads and exports every function the public
headers declare; host-side argument checks that need no GPU."""
import ctypes
import os
import re

from paper_2509_01425_amd import hicr as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hicr_\w+)\s*\(", text, re.M))
    return names


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert {"hicr_memcpy_batch", "hicr_fence", "hicr_slot_register"} <= names
    lib = ctypes.CDLL(H.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    # the binding covers the same names
    assert names == set(H.exported_symbols())


def test_sched_classes_and_strerror():
    seen = set()
    for c in range(H.NUM_CLASSES):
        rc, s = H.hicr_sched_class(c)
        assert rc == H.OK
        seen.add((s.chunk_bytes, s.wgs_per_desc, s.unroll))
    assert seen == {(c, w, u) for c in (4096, 65536, 1 << 20) for w in (1, 4) for u in (2, 4)}
    assert H.hicr_sched_class(12)[0] == H.EINVAL
    for code in range(-10, 1):
        assert H.hicr_strerror(code) != "unknown error"


def test_ctx_create_rejects_bad_device():
    rc, ctx = H.hicr_ctx_create(10_000, 0)
    assert rc == H.EINVAL and ctx is None


def test_features_match_oracle():
    """The host-side batch feature equals the oracle's definition."""
    import numpy as np
    from oracle import mlp
    from workloads import memcpy as wm
    for b in range(20):
        d, _ = wm.family(b)
        rc, f = H.hicr_sched_features(d)
        assert rc == H.OK
        assert np.allclose(f, mlp.features(d["size"]), rtol=1e-6, atol=1e-6)
    rc, f = H.hicr_sched_features(np.zeros(0, dtype=H.DESC_DTYPE))
    assert rc == H.OK and not f.any()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
