"""Device-side input generation (fill) and the plain reference copy.

Loads ``workloads/libwlfill.so`` (built by ``workloads.device.build``).  This
is input plumbing for tests and benchmarks; it holds none of the data path.
"""
import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "fill.hip")
LIB = os.path.join(HERE, "libwlfill.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
           "-shared", "-Wall", "-Werror", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} missing; run workloads.device.build()")
        L = ctypes.CDLL(LIB)
        L.wl_fill.restype = ctypes.c_int
        L.wl_fill.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                              ctypes.c_void_p]
        L.wl_ref_copy.restype = ctypes.c_int
        L.wl_ref_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                  ctypes.c_uint32, ctypes.c_void_p]
        L.wl_ref_rows.restype = ctypes.c_int
        L.wl_ref_rows.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        L.wl_ref_stream.restype = ctypes.c_int
        L.wl_ref_stream.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                    ctypes.c_void_p]
        _lib = L
    return _lib


def fill(dev_ptr: int, n_bytes: int, seed: int, first_index: int = 0, stream: int = 0) -> None:
    rc = lib().wl_fill(dev_ptr, n_bytes, seed, first_index, stream or None)
    if rc != 0:
        raise RuntimeError(f"wl_fill failed ({rc})")


def ref_copy(dst: int, src: int, n_bytes: int, blocks: int = 4096, stream: int = 0) -> None:
    rc = lib().wl_ref_copy(dst, src, n_bytes, blocks, stream or None)
    if rc != 0:
        raise RuntimeError(f"wl_ref_copy failed ({rc})")


def ref_rows(dst_rows: int, src_rows: int, n_rows: int, row_bytes: int, blocks: int,
             stream: int = 0) -> None:
    """Plain copy of n_rows rows of row_bytes (a multiple of 16, at most 8 KiB)
    between the device addresses held in the device arrays dst_rows and
    src_rows (measurement only)."""
    rc = lib().wl_ref_rows(dst_rows, src_rows, n_rows, row_bytes // 16, blocks, stream or None)
    if rc != 0 or row_bytes % 16:
        raise RuntimeError(f"wl_ref_rows failed ({rc})")


REF_COPY, REF_READ, REF_WRITE, REF_MEMCPY = 0, 1, 2, 3


def ref_stream(kind: int, dst: int, src: int, n_bytes: int, blocks: int = 1024, sink: int = 0,
               stream: int = 0) -> None:
    """Reference HBM streams (measurement only): copy, read, write, or the
    runtime's device-to-device memcpy of n_bytes (a multiple of 64 KiB)."""
    rc = lib().wl_ref_stream(kind, dst or None, src or None, n_bytes, blocks, sink or None,
                             stream or None)
    if rc != 0:
        raise RuntimeError(f"wl_ref_stream failed ({rc})")


if __name__ == "__main__":
    print(build(verbose=True))
