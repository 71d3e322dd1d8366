"""Seeded request traces for the serving loop.

Poisson arrivals (exponential gaps of mean 1/rate); each request is a memcpy
batch or a channel burst with probability 1/2.

* memcpy batch: n uniform in [8, 512] requests, sizes log-uniform in
  [64 B, 16 MiB], sources at uniform offsets of a shared source pool,
  destinations laid out back to back inside the request's own block with
  0..63-byte gaps (so they are unaligned and disjoint).
* channel burst: m uniform in [1, 256] messages, sizes log-uniform in
  [16 B, 256 KiB], sources at uniform offsets of the source pool, channel
  uniform over the server's channels; the output block holds the messages
  back to back.
"""
from dataclasses import dataclass

import numpy as np

from .memcpy import DESC_DTYPE, KiB, MiB, log_uniform, rng

REQ_DTYPE = np.dtype([("kind", "<u4"), ("channel", "<u4"), ("first", "<u8"), ("count", "<u8"),
                      ("hbm_bytes", "<u8"), ("arrival_ns", "<u8")], align=True)
assert REQ_DTYPE.itemsize == 40


@dataclass
class Trace:
    reqs: np.ndarray      # REQ_DTYPE
    descs: np.ndarray     # DESC_DTYPE (dst_off relative to the request block)
    msg_src_off: np.ndarray
    msg_size: np.ndarray

    def algorithmic_bytes(self) -> int:
        """Read + write bytes: 2 per copied byte; 4 per message byte plus the
        8-byte entry written and read per message."""
        tot = 2 * int(self.descs["size"].sum())
        tot += 4 * int(self.msg_size.sum()) + 16 * len(self.msg_size)
        return tot


def trace(duration_s=60.0, rate=2000.0, src_bytes=16 << 30, n_channels=1024, batch=0,
          copy_n=(8, 512), copy_size=(64, 16 * MiB), burst_m=(1, 256), burst_size=(16, 256 * KiB),
          n_max=None) -> Trace:
    g = rng(4, batch)
    n_est = int(duration_s * rate * 1.2) + 16
    gaps = g.exponential(1.0 / rate, size=n_est)
    t = np.cumsum(gaps)
    N = int(np.searchsorted(t, duration_s))
    if n_max is not None:
        N = min(N, n_max)
    t = t[:N]
    kinds = (g.random(N) >= 0.5).astype(np.uint32)  # 0 copy, 1 burst
    reqs = np.zeros(N, dtype=REQ_DTYPE)
    reqs["arrival_ns"] = np.round(t * 1e9).astype(np.uint64)
    reqs["kind"] = kinds
    descs, moff, msz = [], [], []
    nd = nm = 0
    for i in range(N):
        if kinds[i] == 0:
            n = int(g.integers(copy_n[0], copy_n[1] + 1))
            sz = log_uniform(g, copy_size[0], copy_size[1], n)
            so = np.floor(g.random(n) * (src_bytes - sz.astype(np.float64) + 1)).astype(np.uint64)
            gap = g.integers(0, 64, size=n).astype(np.uint64)
            ends = np.cumsum(gap + sz)
            do = ends - sz
            d = np.zeros(n, dtype=DESC_DTYPE)
            d["dst_off"], d["src_off"], d["size"] = do, so, sz
            descs.append(d)
            reqs[i]["first"], reqs[i]["count"] = nd, n
            reqs[i]["hbm_bytes"] = int(ends[-1])
            nd += n
        else:
            m = int(g.integers(burst_m[0], burst_m[1] + 1))
            sz = log_uniform(g, burst_size[0], burst_size[1], m)
            so = np.floor(g.random(m) * (src_bytes - sz.astype(np.float64) + 1)).astype(np.uint64)
            moff.append(so)
            msz.append(sz)
            reqs[i]["first"], reqs[i]["count"] = nm, m
            reqs[i]["channel"] = int(g.integers(0, n_channels))
            reqs[i]["hbm_bytes"] = int(sz.sum())
            nm += m
    cat = lambda xs, dt: np.concatenate(xs) if xs else np.zeros(0, dtype=dt)  # noqa: E731
    return Trace(reqs, cat(descs, DESC_DTYPE), cat(moff, np.uint64), cat(msz, np.uint64))
