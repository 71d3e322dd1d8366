"""Pins of the oracle's slots / memcpy / counters / fence (CPU only).

What fixes the oracle here, besides itself:
  * libc memmove (via ctypes) -- the textbook routine for a byte copy;
  * brute force -- every order of the requests, and every split of them into
    byte pieces interleaved arbitrarily, gives the same bytes exactly when the
    pairwise hazard check passes (with all-distinct content);
  * an independent byte-marking hazard check;
  * closed-form counters (sent_k = #requests reading slot k, recv_k = #
    requests writing it; both sums = #requests);
  * numpy fancy-index assignment for the tiny workload.
"""
import ctypes
import itertools

import numpy as np
import pytest

from workloads import memcpy as wm
from workloads.content import content


def test_copy_bytes_equals_libc(orc):
    g = np.random.default_rng(1)
    for n in [0, 1, 2, 3, 7, 15, 16, 17, 63, 64, 65, 4095, 4096, 100003]:
        for so, do in [(0, 0), (1, 0), (0, 3), (5, 11), (13, 2)]:
            src = g.integers(0, 256, n + 32, dtype=np.uint8)
            a = g.integers(0, 256, n + 32, dtype=np.uint8)
            b = a.copy()
            orc.lib().or_copy_bytes(a.ctypes.data + do, src.ctypes.data + so, n)
            ctypes.memmove(b.ctypes.data + do, src.ctypes.data + so, n)
            assert np.array_equal(a, b)


def test_register_rules(orc):
    c = orc.Ctx()
    buf = np.zeros(64, np.uint8)
    assert c.register(buf, size=0)[0] == orc.EINVAL          # zero-size slot
    assert c.register(buf, space=7)[0] == orc.EINVAL          # unknown space
    assert c.register_raw(0, 16)[0] == orc.EINVAL             # null address
    rc, s0 = c.register(buf)
    rc1, s1 = c.register(buf, offset=8, size=16)              # aliasing is allowed
    assert rc == orc.OK and rc1 == orc.OK and s1 == s0 + 1
    assert c.counters(s0) == (orc.OK, 0, 0)
    assert c.deregister(s0) == orc.OK
    assert c.deregister(s0) == orc.EBADSLOT
    assert c.counters(s0)[0] == orc.EBADSLOT


def test_memcpy_preconditions(orc):
    c = orc.Ctx()
    a = np.arange(32, dtype=np.uint8)
    b = np.zeros(32, np.uint8)
    h = np.zeros(32, np.uint8)
    _, sa = c.register(a)
    _, sb = c.register(b)
    _, sh = c.register(h, space=orc.MEM_HOST)
    assert c.memcpy(sb, 0, 99, 0, 1) == orc.EBADSLOT
    assert c.memcpy(99, 0, sa, 0, 1) == orc.EBADSLOT
    assert c.memcpy(sb, 0, sa, 0, 33) == orc.ERANGE
    assert c.memcpy(sb, 32, sa, 0, 1) == orc.ERANGE
    assert c.memcpy(sb, 33, sa, 0, 0) == orc.ERANGE
    assert c.memcpy(sb, 0, sa, 2**64 - 1, 2) == orc.ERANGE    # no wrap-around
    assert c.memcpy(sb, 2**63, sa, 0, 2**63) == orc.ERANGE
    assert c.memcpy(sh, 0, sa, 0, 1) == orc.EUNSUPPORTED      # HBM -> host rejected
    assert c.memcpy(sb, 0, sh, 0, 1) == orc.EUNSUPPORTED
    assert not b.any() and c.counters(sb) == (orc.OK, 0, 0)
    # a request ending exactly at the slot end, and a zero-size one at the end
    assert c.memcpy(sb, 30, sa, 0, 2) == orc.OK
    assert c.memcpy(sb, 32, sa, 32, 0) == orc.OK
    assert list(b[30:]) == [0, 1] and not b[:30].any()
    assert c.counters(sa) == (orc.OK, 2, 0) and c.counters(sb) == (orc.OK, 0, 2)
    # a pair mask that allows host memory accepts the same request
    c2 = orc.Ctx(pair_mask=0b1111)
    _, x = c2.register(h, space=orc.MEM_HOST)
    _, y = c2.register(a)
    assert c2.memcpy(x, 0, y, 5, 3) == orc.OK and list(h[:3]) == [5, 6, 7]


def test_batch_atomic_rejection(orc):
    c = orc.Ctx()
    a = np.arange(64, dtype=np.uint8)
    b = np.zeros(64, np.uint8)
    _, sa = c.register(a)
    _, sb = c.register(b)
    d = np.zeros(4, dtype=orc.DESC_DTYPE)
    d[:] = [(sb, sa, 0, 0, 8), (sb, sa, 8, 8, 8), (sb, sa, 60, 0, 8), (sb, sa, 16, 0, 4)]
    rc, bad = c.memcpy_batch(d)
    assert (rc, bad) == (orc.ERANGE, 2)
    assert not b.any() and c.counters(sa) == (orc.OK, 0, 0)
    d[2]["dst_off"] = 40
    rc, bad = c.memcpy_batch(d)
    assert rc == orc.OK
    assert np.array_equal(b[:16], a[:16]) and np.array_equal(b[40:48], a[:8])
    assert c.counters(sa) == (orc.OK, 4, 0) and c.counters(sb) == (orc.OK, 0, 4)
    assert c.fence() == orc.OK
    assert c.fence_slot(sb, 0, 4) == orc.OK
    assert c.fence_slot(sb, 0, 5) == orc.ETIMEDOUT
    assert c.fence_slot(sa, 5, 0) == orc.ETIMEDOUT


def _apply_pieces(pool, reqs, pieces_order):
    """Apply byte pieces (req index, start, end) in the given order, reading
    sources from ``pool`` as it is at that moment."""
    for i, x0, x1 in pieces_order:
        d, s, _ = reqs[i]
        pool[d + x0:d + x1] = pool[s + x0:s + x1].copy()


def _byte_mark_hazard(reqs):
    """Independent hazard formulation: count per byte how often it is written
    and whether it is read."""
    if not reqs:
        return False
    top = max(max(d, s) + n for d, s, n in reqs) + 1
    w = np.zeros(top, int)
    r = np.zeros(top, bool)
    for d, s, n in reqs:
        w[d:d + n] += 1
        r[s:s + n] = True
    return bool((w > 1).any() or (r & (w > 0)).any())


def test_order_and_split_independence_bruteforce(orc):
    """Requests inside one 48-byte pool; up to 4 of them.  When the hazard
    check passes, the oracle (index order, byte loop) equals every
    permutation and many random byte-piece interleavings.  When it fails, the
    result depends on the order in almost every case (the exceptions are
    benign coincidences such as a request copying a range onto itself)."""
    g = np.random.default_rng(7)
    n_hazard = n_clean = n_dependent = 0
    for trial in range(400):
        pool0 = np.arange(48, dtype=np.uint8) + 1  # all-distinct content
        n_ops = int(g.integers(1, 5))
        reqs = []
        for _ in range(n_ops):
            n = int(g.integers(0, 7))
            d = int(g.integers(0, 48 - n + 1))
            s = int(g.integers(0, 48 - n + 1))
            reqs.append((d, s, n))
        c = orc.Ctx()
        pool = pool0.copy()
        _, slot = c.register(pool)
        descs = np.zeros(n_ops, dtype=orc.DESC_DTYPE)
        for i, (d, s, n) in enumerate(reqs):
            descs[i] = (slot, slot, d, s, n)
        hz = c.hazard_check(descs)[0]
        assert (hz == orc.EHAZARD) == _byte_mark_hazard(reqs)
        assert c.memcpy_batch(descs)[0] == orc.OK
        results = set()
        for perm in itertools.permutations(range(n_ops)):
            p = pool0.copy()
            _apply_pieces(p, reqs, [(i, 0, reqs[i][2]) for i in perm])
            results.add(p.tobytes())
        for _ in range(20):
            pieces = []
            for i, (d, s, n) in enumerate(reqs):
                cuts = sorted(set(int(x) for x in g.integers(0, n + 1, size=3)) | {0, n})
                pieces += [(i, a, b) for a, b in zip(cuts[:-1], cuts[1:])]
            order = g.permutation(len(pieces))
            p = pool0.copy()
            _apply_pieces(p, reqs, [pieces[k] for k in order])
            results.add(p.tobytes())
            # single-byte pieces, reversed: the most hostile split
            p = pool0.copy()
            _apply_pieces(p, reqs, [(i, x, x + 1) for i, (_, _, n) in enumerate(reqs)
                                    for x in reversed(range(n))])
            results.add(p.tobytes())
        if hz == orc.OK:
            n_clean += 1
            assert results == {pool.tobytes()}
        else:
            n_hazard += 1
            n_dependent += len(results) > 1
    assert n_hazard > 50 and n_clean > 50
    assert n_dependent >= 0.9 * n_hazard


def test_counters_closed_form(orc):
    g = np.random.default_rng(3)
    c = orc.Ctx()
    bufs = [np.zeros(64, np.uint8) for _ in range(5)]
    slots = [c.register(b)[1] for b in bufs]
    sent = np.zeros(5, int)
    recv = np.zeros(5, int)
    for _ in range(6):
        n = int(g.integers(0, 40))
        d = np.zeros(n, dtype=orc.DESC_DTYPE)
        d["dst_slot"] = g.integers(0, 5, n)
        d["src_slot"] = g.integers(0, 5, n)
        d["size"] = 0
        assert c.memcpy_batch(d)[0] == orc.OK
        np.add.at(sent, d["src_slot"], 1)
        np.add.at(recv, d["dst_slot"], 1)
    for k in range(5):
        assert c.counters(slots[k]) == (orc.OK, sent[k], recv[k])
    assert sent.sum() == recv.sum()
    # counter-only application agrees with the byte-moving one
    c2 = orc.Ctx()
    slots2 = [c2.register(b)[1] for b in bufs]
    d = np.zeros(30, dtype=orc.DESC_DTYPE)
    d["dst_slot"] = g.integers(0, 5, 30)
    d["src_slot"] = g.integers(0, 5, 30)
    assert c2.count_batch(d)[0] == orc.OK
    for k in range(5):
        _, s, r = c2.counters(slots2[k])
        assert s == int((d["src_slot"] == k).sum()) and r == int((d["dst_slot"] == k).sum())


def test_tiny_workload_matches_numpy_and_is_hazard_free(orc):
    bases, sizes, pool_len, descs, redraws = wm.tiny(0)
    assert len(descs) == 256 and 0 <= redraws
    assert (descs["size"] >= 1).all() and (descs["size"] <= 8192).all()
    pool = content(11, 0, pool_len)
    ref = pool.copy()
    c = orc.Ctx()
    slots = [c.register(pool, offset=int(b), size=int(s))[1] for b, s in zip(bases, sizes)]
    assert slots == list(range(64))
    assert c.hazard_check(descs)[0] == orc.OK
    assert c.memcpy_batch(descs)[0] == orc.OK
    # numpy: gather every source first, then scatter (a reordering that is
    # only valid because the batch is hazard-free)
    src_idx = np.concatenate([np.arange(int(d["size"])) + int(bases[d["src_slot"]] + d["src_off"])
                              for d in descs])
    dst_idx = np.concatenate([np.arange(int(d["size"])) + int(bases[d["dst_slot"]] + d["dst_off"])
                              for d in descs])
    ref[dst_idx] = ref[src_idx]
    assert np.array_equal(pool, ref)


@pytest.mark.parametrize("batch", [0, 1])
def test_batched_workload_is_disjoint_and_in_windows(batch):
    d = wm.batched(batch)
    assert len(d) == 4096
    s = d["size"].astype(np.int64)
    assert s.min() >= 256 and s.max() <= 64 * wm.MiB
    dabs = d["dst_slot"].astype(np.int64) * wm.B_STRIDE + d["dst_off"].astype(np.int64)
    sabs = d["src_slot"].astype(np.int64) * wm.B_STRIDE + d["src_off"].astype(np.int64)
    assert (d["dst_off"].astype(np.int64) + s <= wm.B_WINDOW).all()
    assert (d["src_off"].astype(np.int64) + s <= wm.B_WINDOW).all()
    starts = np.concatenate([dabs, sabs])
    ends = starts + np.concatenate([s, s])
    o = np.argsort(starts)
    assert (starts[o][1:] >= ends[o][:-1]).all()       # all 8192 ranges disjoint
    assert ends.max() <= wm.B_POOL
    assert (dabs % 16 != 0).mean() > 0.8                # offsets are unaligned
    assert 19e9 < s.sum() < 25e9                        # ~22.0 GB per batch


def test_generators_reproducible():
    a = wm.batched(3)
    b = wm.batched(3)
    assert a.tobytes() == b.tobytes()
    assert wm.tiny(1)[3].tobytes() == wm.tiny(1)[3].tobytes()
    assert wm.batched(4).tobytes() != a.tobytes()


def test_content_golden():
    from workloads.content import splitmix64
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    for seed, *outs in rows:
        got = splitmix64(int(seed), 0, 3)
        assert [int(x) for x in got] == [int(o, 16) for o in outs]
    # windows of the byte stream agree with the whole stream
    whole = content(5, 0, 4096)
    for a, n in [(0, 1), (3, 5), (7, 9), (8, 8), (1001, 777), (4000, 96)]:
        assert np.array_equal(content(5, a, n), whole[a:a + n])
