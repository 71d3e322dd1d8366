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


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and every field offset of the header's structs, as the C
    compiler lays them out, equal the ctypes binding's (and the numpy
    descriptor dtype's)."""
    import subprocess
    structs = {"hicr_sched": H.hicr_sched, "hicr_channel_cfg": H.hicr_channel_cfg,
               "hicr_stream": H.hicr_stream, "hicr_pump_io": H.hicr_pump_io,
               "hicr_request": H.hicr_request, "hicr_serve_cfg": H.hicr_serve_cfg,
               "hicr_serve_stats": H.hicr_serve_stats, "hicr_dobj_handle": H.hicr_dobj_handle,
               "hicr_dev_ring": H.hicr_dev_ring}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hicr.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} sizeof %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            if f == "pad":
                continue
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append('printf("hicr_desc sizeof %zu\\n", sizeof(hicr_desc));')
    for f in H.DESC_DTYPE.names:
        lines.append(f'printf("hicr_desc {f} %zu\\n", offsetof(hicr_desc, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        name, field, v = ln.split()
        got[(name, field)] = int(v)
    for name, cls in structs.items():
        assert got[(name, "sizeof")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            if f != "pad":
                assert got[(name, f)] == getattr(cls, f).offset, (name, f)
    assert got[("hicr_desc", "sizeof")] == H.DESC_DTYPE.itemsize
    for f in H.DESC_DTYPE.names:
        assert got[("hicr_desc", f)] == H.DESC_DTYPE.fields[f][1], f
