"""Seeded channel workloads.

* ``tiny_schedule``: the tiny fixed-size SPSC channel (16 tokens of 256 B)
  carrying 1,000 tokens: a seeded sequence of push and pop attempts
  (p = 1/2 each; a push offers 1..4 tokens, a pop takes 1..4), generated
  until every token has been offered and consumed.  The attempts that find
  the ring full or empty are part of the sequence.
* ``plan``: many producer streams feeding variable-size channels.  The
  measured configuration is 1,024 SPSC channels plus 64 MPSC channels with 8
  producers each (1,536 streams), 1e6 messages in total (651 per stream, one
  more for the first 64 streams), sizes log-uniform in [16 B, 256 KiB].
  Every stream reads its messages from its own 2 MiB source slot, message j
  at a uniform offset.  Rings hold 1 MiB of payload and 64 size entries.
"""
from dataclasses import dataclass

import numpy as np

from .memcpy import KiB, MiB, log_uniform, rng


def tiny_schedule(n_attempts: int = 8000, batch: int = 0, max_k: int = 4):
    """A seeded list of ("push", k) / ("pop", k) attempts, p = 1/2 each, k
    uniform in [1, max_k].  A driver walks it until all tokens are through
    (offering at most the tokens that remain) and keeps popping after it."""
    g = rng(10, batch)
    kinds = g.random(n_attempts) < 0.5
    ks = g.integers(1, max_k + 1, size=n_attempts)
    return [("push" if kd else "pop", int(k)) for kd, k in zip(kinds, ks)]


@dataclass
class Plan:
    n_spsc: int
    n_mpsc: int
    K: int
    P: int                   # payload bytes per ring
    E: int                   # size entries per ring
    src_bytes: int           # source slot bytes per stream
    stream_channel: np.ndarray   # [S] channel index
    stream_producer: np.ndarray  # [S] producer index within the channel
    msg_begin: np.ndarray        # [S+1] first message of each stream
    msg_size: np.ndarray         # [M] bytes
    msg_src_off: np.ndarray      # [M] offset in the stream's source slot

    @property
    def n_streams(self):
        return len(self.stream_channel)

    @property
    def n_channels(self):
        return self.n_spsc + self.n_mpsc

    @property
    def n_msgs(self):
        return int(self.msg_begin[-1])

    def stream_bytes(self):
        return np.add.reduceat(self.msg_size, self.msg_begin[:-1]) if self.n_msgs else \
            np.zeros(self.n_streams, dtype=np.uint64)


def plan(n_spsc=1024, n_mpsc=64, K=8, total_msgs=1_000_000, lo=16, hi=256 * KiB,
         P=1 * MiB, E=64, src_bytes=2 * MiB, batch: int = 0) -> Plan:
    g = rng(2, batch)
    S = n_spsc + n_mpsc * K
    ch = np.concatenate([np.arange(n_spsc), n_spsc + np.repeat(np.arange(n_mpsc), K)])
    pr = np.concatenate([np.zeros(n_spsc, dtype=np.int64), np.tile(np.arange(K), n_mpsc)])
    per = np.full(S, total_msgs // S, dtype=np.int64)
    per[: total_msgs - int(per.sum())] += 1
    begin = np.concatenate([[0], np.cumsum(per)]).astype(np.int64)
    M = int(begin[-1])
    sizes = log_uniform(g, lo, hi, M)
    offs = np.floor(g.random(M) * (src_bytes - sizes.astype(np.float64) + 1)).astype(np.uint64)
    return Plan(n_spsc, n_mpsc, K, P, E, src_bytes, ch.astype(np.uint32), pr.astype(np.uint32),
                begin, sizes.astype(np.uint64), offs)
