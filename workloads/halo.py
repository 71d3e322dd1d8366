"""Halo exchange of the paper's Jacobi test case as a batch of memcpy requests.

The test case splits a 704^3 grid of 8-byte cells, held in one allocation,
into lx x ly x lz local subgrids (1 x 2 x 22 in its best run) and, every
iteration, copies each subgrid's boundary planes into its neighbours' ghost
layers.  Here every subgrid has its own block of memory -- interior
nx x ny x nz cells plus a ghost layer h cells deep on every side, stored
x-fastest -- and the blocks lie back to back in one pool.  With the grid not
split along x (lx = 1), every face is a set of contiguous x-rows of nx cells:

  ghost planes y = ny+h .. ny+2h-1 of (j, k)  <-  planes y = h .. 2h-1 of (j+1, k)
  ghost planes y = 0 .. h-1          of (j, k)  <-  planes y = ny .. ny+h-1 of (j-1, k)
  ghost planes z = nz+h .. nz+2h-1 of (j, k)  <-  planes z = h .. 2h-1 of (j, k+1)
  ghost planes z = 0 .. h-1          of (j, k)  <-  planes z = nz .. nz+h-1 of (j, k-1)

one request per row, non-periodic.  Ghost cells are never a source and
interior cells never a destination, so a batch is hazard-free.  Only the
request layout lives here; no stencil arithmetic.
"""
import numpy as np

from .memcpy import DESC_DTYPE


def dims(N: int, Py: int, Pz: int):
    """Interior cells (nx, ny, nz) of one subgrid of an N^3 grid split 1 x Py x Pz."""
    assert N % Py == 0 and N % Pz == 0
    return N, N // Py, N // Pz


def sub_bytes(N: int, Py: int, Pz: int, h: int = 1, elem: int = 8) -> int:
    nx, ny, nz = dims(N, Py, Pz)
    return (nx + 2 * h) * (ny + 2 * h) * (nz + 2 * h) * elem


def cell(N: int, Py: int, Pz: int, h: int, x, y, z, elem: int = 8):
    """Byte offset of cell (x, y, z) (ghost layer included) inside one subgrid."""
    nx, ny, nz = dims(N, Py, Pz)
    return ((np.asarray(z, np.int64) * (ny + 2 * h) + y) * (nx + 2 * h) + x) * elem


def exchange(N: int, Py: int, Pz: int, h: int = 1, elem: int = 8) -> np.ndarray:
    """Requests of one halo exchange; slot s = j + Py * k is subgrid (j, k),
    offsets are relative to the subgrid's first byte."""
    nx, ny, nz = dims(N, Py, Pz)
    ys = np.arange(h, ny + h, dtype=np.int64)
    zs = np.arange(h, nz + h, dtype=np.int64)
    out = []

    def face(dst, src, dst_plane0, src_plane0, axis):
        for t in range(h):
            rows = zs if axis == "y" else ys
            d = np.zeros(len(rows), dtype=DESC_DTYPE)
            d["dst_slot"], d["src_slot"] = dst, src
            if axis == "y":   # plane y = const, rows indexed by z
                d["dst_off"] = cell(N, Py, Pz, h, h, dst_plane0 + t, rows, elem)
                d["src_off"] = cell(N, Py, Pz, h, h, src_plane0 + t, rows, elem)
            else:             # plane z = const, rows indexed by y
                d["dst_off"] = cell(N, Py, Pz, h, h, rows, dst_plane0 + t, elem)
                d["src_off"] = cell(N, Py, Pz, h, h, rows, src_plane0 + t, elem)
            d["size"] = nx * elem
            out.append(d)

    for k in range(Pz):
        for j in range(Py):
            s = j + Py * k
            if j + 1 < Py:
                face(s, s + 1, ny + h, h, "y")
            if j > 0:
                face(s, s - 1, 0, ny, "y")
            if k + 1 < Pz:
                face(s, s + Py, nz + h, h, "z")
            if k > 0:
                face(s, s - Py, 0, nz, "z")
    if not out:
        return np.zeros(0, dtype=DESC_DTYPE)
    return np.concatenate(out)


def n_requests(N: int, Py: int, Pz: int, h: int = 1) -> int:
    nx, ny, nz = dims(N, Py, Pz)
    return h * (2 * (Py - 1) * Pz * nz + 2 * Py * (Pz - 1) * ny)
