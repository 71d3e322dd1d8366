"""Step-level model of the channel ring protocol, with an exhaustive explorer.

TEST INFRASTRUCTURE ONLY.  The Channels frontend (paper Sec. 4.3) moves
messages through a circular buffer at the consumer: the producer writes a
message where the buffer has room, then makes it visible; the consumer reads
it, then tells the producer its room is free.  This module breaks that into
the individual memory steps a real producer and consumer perform and explores
every interleaving of them under sequential consistency, so that the
properties below are checked for all schedules, not just one:

  * the consumer never reads a byte that is not (yet) the message it expects;
  * the producer never overwrites a byte that the consumer has not read;
  * capacity: published bytes and entries never exceed the ring;
  * FIFO per producer, every message delivered exactly once;
  * no deadlock: while work remains some step is enabled.

Producer steps per message: take the lock (locking MPSC only), read the
consumer's counters and wait for room, write the payload one byte at a time,
write the size entry, publish the message counter, release the lock.
Consumer steps: read the message counter, read the size entry, read the
payload one byte at a time, publish the byte counter, publish the entry
counter.  On the GPU "publish" is a release store and "read counter" an
acquire load at device scope, which gives the same orders as this model.

``Variant`` switches let tests plant a mistake (publishing before writing,
releasing before reading, an off-by-one room check) and confirm that the
explorer catches it.
"""
from dataclasses import dataclass


@dataclass(frozen=True)
class Variant:
    publish_before_payload: bool = False   # producer bug
    free_before_read: bool = False         # consumer bug
    room_off_by_one: bool = False          # producer accepts one byte too many
    no_lock: bool = False                  # locking MPSC without the lock


class Violation(Exception):
    pass


def explore(P, E, msgs, locking=False, variant=Variant(), max_states=2_000_000):
    """Explore all interleavings.

    P: payload bytes; E: size entries; msgs: list over producers of lists of
    message sizes.  With one producer this is an SPSC ring; with several and
    ``locking`` it is the shared ring of a locking MPSC channel; with several
    and not ``locking`` every producer gets its own ring (non-locking MPSC).
    Returns the number of distinct states visited; raises Violation.
    """
    K = len(msgs)
    rings = 1 if (locking or K == 1) else K
    total = sum(len(m) for m in msgs)

    # shared state per ring: payload cells, size entries (size, producer, idx),
    # published counters tm (entries produced), hm/hb (consumed)
    # tb (bytes produced) is producer-private for SPSC rings and shared under
    # the lock for the locking ring.
    def ring_of(p):
        return 0 if rings == 1 else p

    init_rings = tuple(
        (tuple([None] * P), tuple([None] * E), 0, 0, 0, 0)  # cells, ents, tm, tb, hm, hb
        for _ in range(rings))
    # producer local: (msg index, phase, byte j, snapshot tm, tb, hm, hb)
    init_prod = tuple((0, "idle", 0, 0, 0) for _ in range(K))
    # consumer local: (phase, ring, size, byte j, producer, msg idx)
    init_cons = ("poll", 0, 0, 0, -1, -1)
    delivered = tuple(0 for _ in range(K))  # per-producer next expected msg
    lock = -1
    read_set = frozenset()  # markers (p, m, j) that the consumer has read
    start = (init_rings, init_prod, init_cons, delivered, lock, read_set, 0)

    seen = set()
    stack = [start]
    while stack:
        st = stack.pop()
        if st in seen:
            continue
        seen.add(st)
        if len(seen) > max_states:
            raise RuntimeError("state space too large")
        succ = list(_successors(st, P, E, msgs, K, rings, ring_of, locking, variant))
        rings_s, prods, cons, delv, lk, rset, npop = st
        done = npop == total and all(pr[0] == len(msgs[p]) for p, pr in enumerate(prods))
        if not succ and not done:
            raise Violation(f"deadlock in state {st}")
        for ring in rings_s:
            cells, ents, tm, tb, hm, hb = ring
            if tm - hm > E or tm - hm < 0:
                raise Violation("entry capacity exceeded")
            if tb - hb > P:
                raise Violation("byte capacity exceeded")
        stack.extend(succ)
    return len(seen)


def _set(t, i, v):
    lst = list(t)
    lst[i] = v
    return tuple(lst)


def _successors(st, P, E, msgs, K, rings, ring_of, locking, variant):
    rings_s, prods, cons, delv, lk, rset, npop = st
    # ---------------- producers
    for p in range(K):
        mi, phase, j, tb_loc, tm_loc = prods[p]
        if mi == len(msgs[p]):
            continue
        s = msgs[p][mi]
        r = ring_of(p)
        cells, ents, tm, tb, hm, hb = rings_s[r]
        shared = locking and K > 1
        if phase == "idle":
            if shared and not variant.no_lock:
                if lk != -1:
                    continue  # waiting for the lock
                yield (rings_s, _set(prods, p, (mi, "room", 0, 0, 0)), cons, delv, p, rset, npop)
            else:
                yield (rings_s, _set(prods, p, (mi, "room", 0, tb_loc, tm_loc)), cons, delv, lk,
                       rset, npop)
        elif phase == "room":
            # read consumer counters; with a shared ring also the producer side
            cur_tb = tb if shared else tb_loc
            cur_tm = tm if shared else tm_loc
            room = P - (cur_tb - hb)
            fits = (s <= room + 1) if variant.room_off_by_one else (s <= room)
            if cur_tm - hm < E and fits:
                nxt = "publish_early" if variant.publish_before_payload else "write"
                yield (rings_s, _set(prods, p, (mi, nxt, 0, cur_tb, cur_tm)), cons, delv, lk,
                       rset, npop)
            # else: spin (no state change) -> not a successor
        elif phase == "publish_early":
            ring = (cells, _set(ents, tm_loc % E, (s, p, mi)), tm, tb, hm, hb)
            ring = (ring[0], ring[1], tm_loc + 1, tb_loc + s, hm, hb)
            yield (_set(rings_s, r, ring), _set(prods, p, (mi, "write_late", 0, tb_loc, tm_loc)),
                   cons, delv, lk, rset, npop)
        elif phase in ("write", "write_late"):
            if j < s:
                pos = (tb_loc + j) % P
                old = cells[pos]
                if old is not None and old not in rset:
                    raise Violation(f"producer {p} overwrote unread byte {old}")
                ring = (_set(cells, pos, (p, mi, j)), ents, tm, tb, hm, hb)
                yield (_set(rings_s, r, ring), _set(prods, p, (mi, phase, j + 1, tb_loc, tm_loc)),
                       cons, delv, lk, rset, npop)
            elif phase == "write_late":
                yield (rings_s, _set(prods, p, (mi, "unlock", 0, tb_loc + s, tm_loc + 1)), cons,
                       delv, lk, rset, npop)
            else:
                yield (rings_s, _set(prods, p, (mi, "size", 0, tb_loc, tm_loc)), cons, delv, lk,
                       rset, npop)
        elif phase == "size":
            ring = (cells, _set(ents, tm_loc % E, (s, p, mi)), tm, tb, hm, hb)
            yield (_set(rings_s, r, ring), _set(prods, p, (mi, "publish", 0, tb_loc, tm_loc)),
                   cons, delv, lk, rset, npop)
        elif phase == "publish":
            ring = (cells, ents, tm_loc + 1, tb_loc + s, hm, hb)
            yield (_set(rings_s, r, ring), _set(prods, p, (mi, "unlock", 0, tb_loc + s, tm_loc + 1)),
                   cons, delv, lk, rset, npop)
        elif phase == "unlock":
            nlk = -1 if (shared and not variant.no_lock) else lk
            yield (rings_s, _set(prods, p, (mi + 1, "idle", 0, tb_loc, tm_loc)), cons, delv, nlk,
                   rset, npop)
    # ---------------- consumer
    cph, cr, cs, cj, cp, cm = cons
    if cph == "poll":
        for r in range(rings):
            cells, ents, tm, tb, hm, hb = rings_s[r]
            if tm > hm:  # acquire-read of the published entry counter
                yield (rings_s, prods, ("size", r, 0, 0, -1, -1), delv, lk, rset, npop)
    elif cph == "size":
        cells, ents, tm, tb, hm, hb = rings_s[cr]
        ent = ents[hm % E]
        if ent is None:
            raise Violation("consumer read an unwritten size entry")
        s, p, m = ent
        if m != delv[p]:
            raise Violation(f"FIFO broken: producer {p} message {m}, expected {delv[p]}")
        nxt = "free_early" if variant.free_before_read else "read"
        yield (rings_s, prods, (nxt, cr, s, 0, p, m), delv, lk, rset, npop)
    elif cph == "free_early":
        cells, ents, tm, tb, hm, hb = rings_s[cr]
        ring = (cells, ents, tm, tb, hm + 1, hb + cs)
        yield (_set(rings_s, cr, ring), prods, ("read_late", cr, cs, 0, cp, cm), delv, lk, rset,
               npop)
    elif cph in ("read", "read_late"):
        cells, ents, tm, tb, hm, hb = rings_s[cr]
        if cj < cs:
            base = hb if cph == "read" else hb - cs
            pos = (base + cj) % P
            if cells[pos] != (cp, cm, cj):
                raise Violation(f"consumer read {cells[pos]} expecting {(cp, cm, cj)}")
            yield (rings_s, prods, (cph, cr, cs, cj + 1, cp, cm), delv, lk,
                   rset | {(cp, cm, cj)}, npop)
        elif cph == "read_late":
            yield (rings_s, prods, ("poll", 0, 0, 0, -1, -1), _set(delv, cp, cm + 1), lk, rset,
                   npop + 1)
        else:
            yield (rings_s, prods, ("pub_hb", cr, cs, 0, cp, cm), delv, lk, rset, npop)
    elif cph == "pub_hb":
        cells, ents, tm, tb, hm, hb = rings_s[cr]
        ring = (cells, ents, tm, tb, hm, hb + cs)
        yield (_set(rings_s, cr, ring), prods, ("pub_hm", cr, cs, 0, cp, cm), delv, lk, rset, npop)
    elif cph == "pub_hm":
        cells, ents, tm, tb, hm, hb = rings_s[cr]
        ring = (cells, ents, tm, tb, hm + 1, hb)
        yield (_set(rings_s, cr, ring), prods, ("poll", 0, 0, 0, -1, -1), _set(delv, cp, cm + 1),
               lk, rset, npop + 1)
