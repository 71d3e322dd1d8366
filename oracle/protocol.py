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

With ``reserve=True`` the locking MPSC ring holds its lock only while it
checks room and reserves the next entry and byte range (shared reservation
counters rm/rb); each producer then writes its payload outside the lock and
publishes when the published counter reaches its reserved entry, i.e. in
lock order.

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
    unordered_publish: bool = False        # reservation mode without the turn wait


class Violation(Exception):
    pass


def explore(P, E, msgs, locking=False, variant=Variant(), max_states=2_000_000,
            reserve=False):
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
        # cells, ents, tm, tb, hm, hb, rm, rb (rm/rb: reservations, reserve mode)
        (tuple([None] * P), tuple([None] * E), 0, 0, 0, 0, 0, 0)
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
        succ = list(_successors(st, P, E, msgs, K, rings, ring_of, locking, variant, reserve))
        rings_s, prods, cons, delv, lk, rset, npop = st
        done = npop == total and all(pr[0] == len(msgs[p]) for p, pr in enumerate(prods))
        if not succ and not done:
            raise Violation(f"deadlock in state {st}")
        for ring in rings_s:
            cells, ents, tm, tb, hm, hb = ring[:6]
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


def _ring_set(ring, **kw):
    names = ("cells", "ents", "tm", "tb", "hm", "hb", "rm", "rb")
    lst = list(ring)
    for k, v in kw.items():
        lst[names.index(k)] = v
    return tuple(lst)


def _successors(st, P, E, msgs, K, rings, ring_of, locking, variant, reserve=False):
    rings_s, prods, cons, delv, lk, rset, npop = st
    shared = locking and K > 1
    use_lock = shared and not variant.no_lock
    # ---------------- producers
    for p in range(K):
        mi, phase, j, tb_loc, tm_loc = prods[p]
        if mi == len(msgs[p]):
            continue
        s = msgs[p][mi]
        r = ring_of(p)
        ring = rings_s[r]
        cells, ents, tm, tb, hm, hb, rm, rb = ring

        def go(new_phase, nj=0, ntb=tb_loc, ntm=tm_loc, nmi=mi, new_ring=None, new_lk=lk):
            rs = rings_s if new_ring is None else _set(rings_s, r, new_ring)
            return (rs, _set(prods, p, (nmi, new_phase, nj, ntb, ntm)), cons, delv, new_lk, rset,
                    npop)

        if phase == "idle":
            if use_lock:
                if lk != -1:
                    continue  # waiting for the lock
                yield go("room", new_lk=p)
            else:
                yield go("room")
        elif phase == "room":
            # read the consumer's counters; a shared ring also reads the
            # producer-side counters (reservations in reserve mode)
            if shared:
                cur_tm, cur_tb = (rm, rb) if reserve else (tm, tb)
            else:
                cur_tm, cur_tb = tm_loc, tb_loc
            room = P - (cur_tb - hb)
            fits = (s <= room + 1) if variant.room_off_by_one else (s <= room)
            if cur_tm - hm < E and fits:
                if shared and reserve:
                    yield go("reserve", ntb=cur_tb, ntm=cur_tm)
                else:
                    nxt = "publish_early" if variant.publish_before_payload else "write"
                    yield go(nxt, ntb=cur_tb, ntm=cur_tm)
            # else: spin (no state change) -> not a successor
        elif phase == "reserve":
            nr = _ring_set(ring, rm=tm_loc + 1, rb=tb_loc + s)
            yield go("write", new_ring=nr, new_lk=-1 if use_lock else lk)
        elif phase == "publish_early":
            nr = _ring_set(ring, ents=_set(ents, tm_loc % E, (s, p, mi)), tm=tm_loc + 1,
                           tb=tb_loc + s)
            yield go("write_late", new_ring=nr)
        elif phase in ("write", "write_late"):
            if j < s:
                pos = (tb_loc + j) % P
                old = cells[pos]
                if old is not None and old not in rset:
                    raise Violation(f"producer {p} overwrote unread byte {old}")
                nr = _ring_set(ring, cells=_set(cells, pos, (p, mi, j)))
                yield go(phase, nj=j + 1, new_ring=nr)
            elif phase == "write_late":
                yield go("unlock", ntb=tb_loc + s, ntm=tm_loc + 1)
            else:
                yield go("size")
        elif phase == "size":
            nr = _ring_set(ring, ents=_set(ents, tm_loc % E, (s, p, mi)))
            nxt = "turn" if (shared and reserve) else "publish"
            yield go(nxt, new_ring=nr)
        elif phase == "turn":
            # publish in reservation order: wait for the predecessors
            if variant.unordered_publish or tm == tm_loc:
                yield go("publish")
        elif phase == "publish":
            if shared and reserve:
                nr = _ring_set(ring, tm=max(tm, tm_loc + 1), tb=max(tb, tb_loc + s))
            else:
                nr = _ring_set(ring, tm=tm_loc + 1, tb=tb_loc + s)
            yield go("unlock", ntb=tb_loc + s, ntm=tm_loc + 1, new_ring=nr)
        elif phase == "unlock":
            release = use_lock and not reserve
            yield go("idle", nmi=mi + 1, new_lk=-1 if release else lk)
    # ---------------- consumer
    cph, cr, cs, cj, cp, cm = cons

    def cgo(new_cons, new_ring=None, ndelv=delv, nrset=rset, nnpop=npop):
        rs = rings_s if new_ring is None else _set(rings_s, cr, new_ring)
        return (rs, prods, new_cons, ndelv, lk, nrset, nnpop)

    if cph == "poll":
        for r in range(rings):
            tm, hm = rings_s[r][2], rings_s[r][4]
            if tm > hm:  # acquire-read of the published entry counter
                yield (rings_s, prods, ("size", r, 0, 0, -1, -1), delv, lk, rset, npop)
        return
    ring = rings_s[cr]
    cells, ents, tm, tb, hm, hb, rm, rb = ring
    if cph == "size":
        ent = ents[hm % E]
        if ent is None:
            raise Violation("consumer read an unwritten size entry")
        s, p, m = ent
        if m != delv[p]:
            raise Violation(f"FIFO broken: producer {p} message {m}, expected {delv[p]}")
        nxt = "free_early" if variant.free_before_read else "read"
        yield cgo((nxt, cr, s, 0, p, m))
    elif cph == "free_early":
        yield cgo(("read_late", cr, cs, 0, cp, cm), _ring_set(ring, hm=hm + 1, hb=hb + cs))
    elif cph in ("read", "read_late"):
        if cj < cs:
            base = hb if cph == "read" else hb - cs
            pos = (base + cj) % P
            if cells[pos] != (cp, cm, cj):
                raise Violation(f"consumer read {cells[pos]} expecting {(cp, cm, cj)}")
            yield cgo((cph, cr, cs, cj + 1, cp, cm), nrset=rset | {(cp, cm, cj)})
        elif cph == "read_late":
            yield cgo(("poll", 0, 0, 0, -1, -1), ndelv=_set(delv, cp, cm + 1), nnpop=npop + 1)
        else:
            yield cgo(("pub_hb", cr, cs, 0, cp, cm))
    elif cph == "pub_hb":
        yield cgo(("pub_hm", cr, cs, 0, cp, cm), _ring_set(ring, hb=hb + cs))
    elif cph == "pub_hm":
        yield cgo(("poll", 0, 0, 0, -1, -1), _ring_set(ring, hm=hm + 1),
                  ndelv=_set(delv, cp, cm + 1), nnpop=npop + 1)
