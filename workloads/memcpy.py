"""Seeded memcpy workloads: slot layouts and request (descriptor) lists.

Every generator takes its randomness from ``rng(cfg, batch)``, a numpy
``Generator`` seeded with ``SeedSequence([0x48694352, cfg, batch])``.

Workloads (sizes follow the configurations the path is measured on):

* ``tiny``: 64 slots, sizes uniform in [1 KiB, 64 KiB], packed back to back
  in one byte pool (so slot bases are unaligned); 256 requests with random
  source/destination slots, unaligned offsets and sizes uniform in
  [1, 8 KiB].  Destinations are pairwise disjoint and disjoint from every
  source (no write/write or read/write conflict in the epoch).  Placement is
  an exact free-gap sampler; a request that fits nowhere has its size redrawn
  (up to 64 times from [1, 8 KiB], then from [1, largest free gap]).
* ``batched``: 8,192 slots over one pool of 64 GiB + 64 MiB.  Slot k is the
  window [k * 8 MiB, k * 8 MiB + 72 MiB), so windows overlap and any range of
  at most 64 MiB lies inside the window of the stride it starts in.  4,096
  requests, sizes log-uniform in [256 B, 64 MiB], no alignment.  The 4,096
  destination and 4,096 source ranges are laid out in a random order with
  random gaps, so all of them are pairwise disjoint.  (A 16 GiB pool cannot
  hold the ~22 GB of disjoint destinations such a batch draws; the pool is
  enlarged and the request law kept.)
* ``family``: the schedule-training distribution -- per batch a family
  (tiny-like uniform sizes or batched-like log-uniform sizes, p = 1/2), a
  request count log-uniform in [8, 4096] and a log-uniform sub-range of the
  family's size range, laid out like ``batched``.
"""
import numpy as np

# One request, in the argument order of memcpy(dst, dstOff, src, srcOff, size):
# the 32-byte record both the oracle and the GPU library accept.
DESC_DTYPE = np.dtype(
    [("dst_slot", "<u4"), ("src_slot", "<u4"), ("dst_off", "<u8"),
     ("src_off", "<u8"), ("size", "<u8")], align=True)

SEED_TAG = 0x48694352

KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30

# batched layout
B_SLOTS = 8192
B_STRIDE = 8 * MiB
B_WINDOW = 72 * MiB
B_POOL = (B_SLOTS - 1) * B_STRIDE + B_WINDOW  # 64 GiB + 64 MiB


def rng(cfg: int, batch: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_TAG, cfg, batch]))


def log_uniform(g: np.random.Generator, a: int, b: int, n: int) -> np.ndarray:
    """Integers in [a, b] whose logarithm is uniform: floor(exp(U(ln a, ln(b+1))))."""
    u = g.uniform(np.log(a), np.log(b + 1), size=n)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), a, b).astype(np.uint64)


# ------------------------------------------------------------------ tiny

def tiny_slots(g: np.random.Generator, n_slots: int = 64):
    sizes = g.integers(1 * KiB, 64 * KiB + 1, size=n_slots).astype(np.uint64)
    bases = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.uint64)
    return bases, sizes


def _free_starts(forbidden, lo, hi, s):
    """Feasible starts x in [lo, hi - s] with [x, x+s) avoiding every
    interval in ``forbidden`` (a sorted list of disjoint (a, b))."""
    out = []
    cur = lo
    for a, b in forbidden:
        if b <= lo or a >= hi:
            continue
        if a - cur >= s:
            out.append((cur, a - s))
        cur = max(cur, b)
    if hi - cur >= s:
        out.append((cur, hi - s))
    return out


def _merge(intervals):
    iv = sorted((a, b) for a, b in intervals if b > a)
    out = []
    for a, b in iv:
        if out and a <= out[-1][1]:
            out[-1] = (out[-1][0], max(out[-1][1], b))
        else:
            out.append((a, b))
    return out


def _pick_start(g, bases, sizes, forbidden, s):
    """Uniform over all feasible (slot, offset) pairs; None if there is none."""
    cands = []
    total = 0
    for k in range(len(bases)):
        lo, hi = int(bases[k]), int(bases[k] + sizes[k])
        for x0, x1 in _free_starts(forbidden, lo, hi, s):
            cnt = x1 - x0 + 1
            cands.append((k, x0, cnt))
            total += cnt
    if total == 0:
        return None
    r = int(g.integers(0, total))
    for k, x0, cnt in cands:
        if r < cnt:
            return k, x0 + r - int(bases[k])
        r -= cnt
    raise AssertionError


def _largest_gap(bases, sizes, forbidden):
    best = 0
    for k in range(len(bases)):
        lo, hi = int(bases[k]), int(bases[k] + sizes[k])
        cur = lo
        for a, b in forbidden:
            if b <= lo or a >= hi:
                continue
            best = max(best, a - cur)
            cur = max(cur, b)
        best = max(best, hi - cur)
    return best


def tiny_ops(g: np.random.Generator, bases, sizes, n_ops: int = 256, max_size: int = 8 * KiB):
    """Returns (descs, redraws)."""
    descs = np.zeros(n_ops, dtype=DESC_DTYPE)
    writes, reads = [], []
    redraws = 0
    for i in range(n_ops):
        s = int(g.integers(1, max_size + 1))
        tries = 0
        while True:
            # destination avoids every earlier destination and source
            forb_w = _merge(writes + reads)
            dst = _pick_start(g, bases, sizes, forb_w, s)
            src = None
            if dst is not None:
                dabs = int(bases[dst[0]]) + dst[1]
                forb_r = _merge(writes + [(dabs, dabs + s)])
                src = _pick_start(g, bases, sizes, forb_r, s)
            if dst is not None and src is not None:
                break
            redraws += 1
            tries += 1
            if tries < 64:
                s = int(g.integers(1, max_size + 1))
            else:
                big = min(_largest_gap(bases, sizes, forb_w), max_size)
                s = int(g.integers(1, max(big, 1) + 1))
        descs[i] = (dst[0], src[0], dst[1], src[1], s)
        dabs = int(bases[dst[0]]) + dst[1]
        sabs = int(bases[src[0]]) + src[1]
        writes.append((dabs, dabs + s))
        reads.append((sabs, sabs + s))
    return descs, redraws


def tiny(batch: int = 0):
    """The tiny workload: (slot bases, slot sizes, pool bytes, descs, redraws)."""
    g = rng(0, batch)
    bases, sizes = tiny_slots(g)
    descs, redraws = tiny_ops(g, bases, sizes)
    pool = int(bases[-1] + sizes[-1])
    return bases, sizes, pool, descs, redraws


# --------------------------------------------------------------- batched

def batched_slots():
    bases = (np.arange(B_SLOTS, dtype=np.uint64) * np.uint64(B_STRIDE))
    sizes = np.full(B_SLOTS, B_WINDOW, dtype=np.uint64)
    return bases, sizes


def layout_disjoint(g: np.random.Generator, sizes: np.ndarray, pool: int = B_POOL):
    """Place n destination and n source ranges of the given sizes in a random
    order with random gaps inside [0, pool); returns absolute starts
    (dst_abs, src_abs)."""
    n = len(sizes)
    both = np.concatenate([sizes, sizes]).astype(np.int64)
    free = pool - int(both.sum())
    if free < 0:
        raise ValueError("ranges do not fit the pool")
    order = g.permutation(2 * n)
    cuts = np.sort(g.integers(0, free + 1, size=2 * n))
    gaps = np.diff(np.concatenate([[0], cuts]))  # gap before each placed range
    placed = both[order]
    starts_in_order = np.cumsum(gaps) + np.concatenate([[0], np.cumsum(placed)[:-1]])
    starts = np.empty(2 * n, dtype=np.int64)
    starts[order] = starts_in_order
    return starts[:n].astype(np.uint64), starts[n:].astype(np.uint64)


def to_slot(abs_start: np.ndarray):
    """Slot whose window holds a range starting at abs_start (len <= 64 MiB)."""
    k = np.minimum(abs_start // np.uint64(B_STRIDE), np.uint64(B_SLOTS - 1))
    return k.astype(np.uint32), (abs_start - k * np.uint64(B_STRIDE)).astype(np.uint64)


def make_descs(g, sizes: np.ndarray):
    dabs, sabs = layout_disjoint(g, sizes)
    dk, doff = to_slot(dabs)
    sk, soff = to_slot(sabs)
    d = np.zeros(len(sizes), dtype=DESC_DTYPE)
    d["dst_slot"], d["dst_off"] = dk, doff
    d["src_slot"], d["src_off"] = sk, soff
    d["size"] = sizes
    return d


def batched(batch: int = 0, n: int = 4096, lo: int = 256, hi: int = 64 * MiB):
    g = rng(1, batch)
    sizes = log_uniform(g, lo, hi, n)
    return make_descs(g, sizes)


def family(batch: int, cfg_tag: int = 3):
    """One batch of the schedule-training distribution; returns (descs, family)."""
    g = rng(cfg_tag, batch)
    fam = int(g.integers(0, 2))
    if fam == 0:
        a, b = 1, 8 * KiB
    else:
        a, b = 256, 64 * MiB
    n = int(log_uniform(g, 8, 4096, 1)[0])
    lo, hi = sorted(int(x) for x in log_uniform(g, a, b, 2))
    if fam == 0:
        sizes = g.integers(lo, hi + 1, size=n).astype(np.uint64)
    else:
        sizes = log_uniform(g, lo, hi, n)
    while 2 * int(sizes.sum()) > 0.9 * B_POOL:
        sizes = sizes[: len(sizes) // 2]
    return make_descs(g, sizes), fam
