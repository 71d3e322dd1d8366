"""Halo exchange of a 3-D Jacobi grid as a batch of memcpy requests.

The paper's Jacobi test case splits a cubic grid over instances and, every
iteration, copies each subdomain's boundary planes into its neighbours'
ghost layers.  Here the subdomains share one GPU: Py x Pz subdomains of N^3
interior cells (8-byte elements) with a one-cell ghost layer, (N+2)^3 cells
each, stored x-fastest and back to back in one pool.  The grid is split
along y and z only, so every face is N contiguous x-rows of N elements:

  ghost plane y = N+1 of subdomain (j, k)  <-  interior plane y = 1 of (j+1, k)
  ghost plane y = 0   of (j, k)            <-  interior plane y = N of (j-1, k)
  ghost plane z = N+1 of (j, k)            <-  interior plane z = 1 of (j, k+1)
  ghost plane z = 0   of (j, k)            <-  interior plane z = N of (j, k-1)

one request per row (x = 1..N), non-periodic.  Ghost cells are never a
source and interior cells never a destination, so a batch is hazard-free.
Only the request layout lives here; no stencil arithmetic.
"""
import numpy as np

from .memcpy import DESC_DTYPE


def sub_bytes(N: int, elem: int = 8) -> int:
    return (N + 2) ** 3 * elem


def cell(N: int, x, y, z, elem: int = 8):
    """Byte offset of cell (x, y, z) inside one subdomain."""
    return ((np.asarray(z, np.int64) * (N + 2) + y) * (N + 2) + x) * elem


def exchange(N: int, Py: int, Pz: int, elem: int = 8) -> np.ndarray:
    """Requests of one halo exchange; slot s = j + Py * k is subdomain (j, k),
    offsets are relative to the subdomain's first cell."""
    rows = np.arange(1, N + 1, dtype=np.int64)
    out = []

    def face(dst, src, dst_plane, src_plane, axis):
        d = np.zeros(N, dtype=DESC_DTYPE)
        d["dst_slot"], d["src_slot"] = dst, src
        if axis == "y":   # rows indexed by z
            d["dst_off"] = cell(N, 1, dst_plane, rows, elem)
            d["src_off"] = cell(N, 1, src_plane, rows, elem)
        else:             # rows indexed by y
            d["dst_off"] = cell(N, 1, rows, dst_plane, elem)
            d["src_off"] = cell(N, 1, rows, src_plane, elem)
        d["size"] = N * elem
        out.append(d)

    for k in range(Pz):
        for j in range(Py):
            s = j + Py * k
            if j + 1 < Py:
                face(s, s + 1, N + 1, 1, "y")
            if j > 0:
                face(s, s - 1, 0, N, "y")
            if k + 1 < Pz:
                face(s, s + Py, N + 1, 1, "z")
            if k > 0:
                face(s, s - Py, 0, N, "z")
    if not out:
        return np.zeros(0, dtype=DESC_DTYPE)
    return np.concatenate(out)


def n_faces(Py: int, Pz: int) -> int:
    return 2 * ((Py - 1) * Pz + Py * (Pz - 1))
