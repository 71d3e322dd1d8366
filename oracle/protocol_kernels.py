"""Step-level models of the ring protocols the device kernels run, with an
exhaustive interleaving explorer.

TEST INFRASTRUCTURE ONLY.  ``protocol`` models one message per publication.
The channel pump and the ping-pong kernel go further (paper Sec. 4.3, the
Channels frontend; Sec. 5, Test Case 1); each refinement is modelled here
step by step and explored under sequential consistency (on the device
"publish" is a release store and "read counter" an acquire load at device
scope, which give the same orders):

* ``explore_batched`` -- one producer publishes up to B messages with one
  counter store, after taking every leading message that fits the room it
  saw; one consumer takes up to C published messages at once and releases
  their room with two stores (bytes, then entries).  With S > 1 a full
  sub-batch of B messages may wait for up to S - 1 more before one store
  publishes them all (whether it waits is left open: both choices are
  explored, so every rule the kernel may use to decide is covered), and a
  producer that finds no room for its next message publishes what it holds
  first (the consumer cannot free room for messages it has not seen).
* ``explore_team`` -- a locking MPSC ring (ticket lock held only to check
  room and reserve entries and bytes) drained by a team of consumers: a
  member claims the next round number, defines the round once the previous
  one is defined (it starts where that one ends and takes up to C published
  messages), reads every message's ring position from the record its
  producer wrote before publishing, and releases the ring room in round
  order.
* ``explore_batched_abort`` -- the same ring with an abort request that may
  arrive at any moment: an actor that is waiting may then exit, one with
  work in hand carries on to its next wait; no actor may be left waiting
  forever (the pump's waits all look at its abort word).
* ``explore_striped`` -- ping-pong between two groups of W members over two
  one-message rings whose counters count stripes: a message is visible when
  all W stripes have arrived (counter >= W (k + 1)), a ring is free when all
  W stripes of the previous message were read (counter >= W k).

Every model checks, in every reachable state: no read of a byte (or stripe)
that does not hold the expected message, no overwrite of a byte not yet read,
entry capacity, every message delivered exactly once and FIFO per producer,
and no deadlock while work remains.  ``Bug`` flags plant one mistake each so
tests can confirm the explorer catches it.
"""
from dataclasses import dataclass


class Violation(Exception):
    pass


@dataclass(frozen=True)
class Bug:
    publish_before_payload: bool = False   # batched producer publishes, then writes
    release_before_read: bool = False      # batched consumer releases, then reads
    batch_room_first_only: bool = False    # batched producer checks room for message 0 only
    record_after_publish: bool = False     # team: producer writes the record after publishing
    no_round_order: bool = False           # team: a member releases without waiting its turn
    start_from_released: bool = False      # team: a round starts at the released counter
    count_messages: bool = False           # striped: counters waited on per message, not stripe
    signal_before_copy: bool = False       # striped: a stripe counted before it is copied
    no_publish_when_blocked: bool = False  # batched, S > 1: blocked with unpublished messages
    abort_ignored_by_producer: bool = False  # abort: the producer's room wait never exits
    abort_ignored_by_consumer: bool = False  # abort: the consumer's message wait never exits


def _dfs(start, succ, done, max_states):
    seen = set()
    stack = [start]
    while stack:
        st = stack.pop()
        if st in seen:
            continue
        seen.add(st)
        if len(seen) > max_states:
            raise RuntimeError("state space too large")
        nxt = list(succ(st))
        if not nxt and not done(st):
            raise Violation(f"deadlock in state {st}")
        stack.extend(nxt)
    return len(seen)


def _set(t, i, v):
    lst = list(t)
    lst[i] = v
    return tuple(lst)


# ------------------------------------------------------------ batched ring

def explore_batched(P, E, sizes, B, C, bug=Bug(), max_states=3_000_000, S=1):
    """One producer stream of messages ``sizes`` through one ring of P bytes
    and E entries; producer sub-batches of at most B messages, up to S of
    them per publication; consumer batches of at most C.  Returns the number
    of states visited."""
    start, succ, done = _batched_model(P, E, sizes, B, C, bug, S)
    return _dfs(start, succ, done, max_states)


def explore_batched_abort(P, E, sizes, B, C, bug=Bug(), max_states=3_000_000, S=1):
    """``explore_batched`` with an abort request that may arrive in any state.
    Once it has arrived, an actor that has no move of its own -- a producer
    waiting for room, a consumer waiting for messages: the waits in which a
    kernel wave looks at its abort word -- may exit; an actor with work in
    hand goes on to its next wait or to its end.  Every reachable state
    keeps the safety checks of ``explore_batched``, and a state without
    moves must have every actor finished or exited (no wave left waiting
    forever).  Returns the number of states visited."""
    n = len(sizes)
    inner_start, inner_succ, inner_done = _batched_model(P, E, sizes, B, C, bug, S)

    def prod_done(st):
        return st[5][0] == n

    def cons_done(st):
        return st[8] == n

    def succ(xst):
        st, aborted, p_out, c_out = xst
        p_moves, c_moves = [], []
        for nx in inner_succ(st):
            (p_moves if nx[5] != st[5] else c_moves).append(nx)
        if not p_out:
            for nx in p_moves:
                yield (nx, aborted, p_out, c_out)
        if not c_out:
            for nx in c_moves:
                yield (nx, aborted, p_out, c_out)
        if not aborted:
            yield (st, True, p_out, c_out)
        else:
            if (not p_out and not p_moves and not prod_done(st)
                    and not bug.abort_ignored_by_producer):
                yield (st, aborted, True, c_out)
            if (not c_out and not c_moves and not cons_done(st)
                    and not bug.abort_ignored_by_consumer):
                yield (st, aborted, p_out, True)

    def done(xst):
        st, aborted, p_out, c_out = xst
        if inner_done(st):
            return True
        return aborted and (p_out or prod_done(st)) and (c_out or cons_done(st))

    return _dfs((inner_start, False, False, False), succ, done, max_states)


def _batched_model(P, E, sizes, B, C, bug, S):
    """Start state, successor function and end predicate of the batched
    single-producer ring (see ``explore_batched``)."""
    n = len(sizes)
    offs = [sum(sizes[:i]) for i in range(n)]  # stream byte offset of message i

    # shared: cells (P markers), ents (E), tm (published), hm, hb (released)
    # producer: (m, phase, j, my_tm, my_tb, hm_seen, cur msg, cur byte, pend)
    #   (my_tm, my_tb count the messages copied, published or not; pend is
    #   the number of full sub-batches copied and not yet published)
    # consumer: (phase, hm_loc, hb_loc, k, cur msg, cur byte)
    # rset: frozenset of markers read
    start = (tuple([None] * P), tuple([None] * E), 0, 0, 0,
             (0, "rd_hm", 0, 0, 0, 0, 0, 0, 0), ("poll", 0, 0, 0, 0, 0), frozenset(), 0)

    def succ(st):
        cells, ents, tm, hm, hb, pr, co, rset, ndone = st
        m, ph, j, my_tm, my_tb, hm_seen, cm, cb, pend = pr

        def P_(**kw):
            v = dict(m=m, ph=ph, j=j, my_tm=my_tm, my_tb=my_tb, hm_seen=hm_seen, cm=cm, cb=cb,
                     pend=pend)
            v.update(kw)
            return (v["m"], v["ph"], v["j"], v["my_tm"], v["my_tb"], v["hm_seen"], v["cm"],
                    v["cb"], v["pend"])

        # ---- producer
        if m < n:
            if ph == "rd_hm":
                yield (cells, ents, tm, hm, hb, P_(ph="rd_hb", hm_seen=hm), co, rset, ndone)
            elif ph == "rd_hb":
                # leading messages that fit the room seen (hm read first, hb now)
                take, run = 0, 0
                for i in range(min(B, n - m)):
                    run += sizes[m + i]
                    fits_e = my_tm + i + 1 - hm_seen <= E
                    fits_b = my_tb + run - hb <= P
                    if i > 0 and bug.batch_room_first_only:
                        fits_e = fits_b = True
                    if not (fits_e and fits_b):
                        break
                    take += 1
                if take:
                    nxt = "pub_early" if bug.publish_before_payload else "ents"
                    yield (cells, ents, tm, hm, hb, P_(ph=nxt, j=take), co, rset, ndone)
                elif pend and not bug.no_publish_when_blocked:
                    # no room: publish what is held, then look again
                    yield (cells, ents, my_tm, hm, hb, P_(ph="rd_hm", pend=0), co, rset, ndone)
                elif hm != hm_seen:
                    # the room seen was stale: look again
                    yield (cells, ents, tm, hm, hb, P_(ph="rd_hm"), co, rset, ndone)
            elif ph in ("ents", "pub_early"):
                ne = ents
                for i in range(j):
                    ne = _set(ne, (my_tm + i) % E, (sizes[m + i], m + i))
                if ph == "pub_early":
                    yield (cells, ne, my_tm + j, hm, hb, P_(ph="pay_late", cm=0, cb=0), co, rset,
                           ndone)
                else:
                    yield (cells, ne, tm, hm, hb, P_(ph="pay", cm=0, cb=0), co, rset, ndone)
            elif ph in ("pay", "pay_late"):
                while cm < j and cb == sizes[m + cm]:
                    cm, cb = cm + 1, 0
                if cm < j:
                    pos = (my_tb + offs[m + cm] - offs[m] + cb) % P
                    old = cells[pos]
                    if old is not None and old not in rset:
                        raise Violation(f"producer overwrote unread byte {old}")
                    nc = _set(cells, pos, (m + cm, cb))
                    yield (nc, ents, tm, hm, hb, P_(cm=cm, cb=cb + 1), co, rset, ndone)
                else:
                    nb = my_tb + offs[m + j - 1] + sizes[m + j - 1] - offs[m]
                    if ph == "pay" and j == B and pend + 1 < S and m + j < n:
                        # a full sub-batch, more to come: it may be held for the next one
                        yield (cells, ents, tm, hm, hb,
                               P_(m=m + j, ph="rd_hm", my_tm=my_tm + j, my_tb=nb, pend=pend + 1),
                               co, rset, ndone)
                    if ph == "pay":
                        yield (cells, ents, my_tm + j, hm, hb,
                               P_(m=m + j, ph="rd_hm", my_tm=my_tm + j, my_tb=nb, pend=0), co,
                               rset, ndone)
                    else:
                        yield (cells, ents, tm, hm, hb,
                               P_(m=m + j, ph="rd_hm", my_tm=my_tm + j, my_tb=nb), co, rset, ndone)
        # ---- consumer
        cph, hm_loc, hb_loc, k, qm, qb = co
        if cph == "poll":
            if tm > hm_loc:
                k2 = min(C, tm - hm_loc)
                yield (cells, ents, tm, hm, hb, pr, ("ents", hm_loc, hb_loc, k2, 0, 0), rset,
                       ndone)
        elif cph == "ents":
            for i in range(k):
                e = ents[(hm_loc + i) % E]
                if e is None or e[1] != hm_loc + i:
                    raise Violation(f"consumer read entry {e} for message {hm_loc + i}")
            nxt = "rel_hb_early" if bug.release_before_read else "pay"
            yield (cells, ents, tm, hm, hb, pr, (nxt, hm_loc, hb_loc, k, 0, 0), rset, ndone)
        elif cph in ("pay", "pay_late"):
            while qm < k and qb == sizes[hm_loc + qm]:
                qm, qb = qm + 1, 0
            if qm < k:
                mi = hm_loc + qm
                pos = (hb_loc + offs[mi] - offs[hm_loc] + qb) % P
                if cells[pos] != (mi, qb):
                    raise Violation(f"consumer read {cells[pos]} expecting {(mi, qb)}")
                yield (cells, ents, tm, hm, hb, pr, (cph, hm_loc, hb_loc, k, qm, qb + 1),
                       rset | {(mi, qb)}, ndone)
            elif cph == "pay":
                yield (cells, ents, tm, hm, hb, pr, ("rel_hb", hm_loc, hb_loc, k, 0, 0), rset,
                       ndone)
            else:
                nb = hb_loc + offs[hm_loc + k - 1] + sizes[hm_loc + k - 1] - offs[hm_loc]
                yield (cells, ents, tm, hm, hb, pr, ("poll", hm_loc + k, nb, 0, 0, 0), rset,
                       ndone + k)
        elif cph in ("rel_hb", "rel_hb_early"):
            nb = hb_loc + offs[hm_loc + k - 1] + sizes[hm_loc + k - 1] - offs[hm_loc]
            nxt = "rel_hm" if cph == "rel_hb" else "rel_hm_early"
            yield (cells, ents, tm, hm, nb, pr, (nxt, hm_loc, hb_loc, k, 0, 0), rset, ndone)
        elif cph == "rel_hm":
            nb = hb_loc + offs[hm_loc + k - 1] + sizes[hm_loc + k - 1] - offs[hm_loc]
            yield (cells, ents, tm, hm_loc + k, hb, pr, ("poll", hm_loc + k, nb, 0, 0, 0), rset,
                   ndone + k)
        elif cph == "rel_hm_early":
            yield (cells, ents, tm, hm_loc + k, hb, pr, ("pay_late", hm_loc, hb_loc, k, 0, 0),
                   rset, ndone)

    def done(st):
        return st[8] == n and st[5][0] == n

    def checked_succ(st):
        cells, ents, tm, hm, hb, pr, co, rset, ndone = st
        if tm - hm > E or tm < hm:
            raise Violation("entry capacity exceeded")
        return succ(st)

    return start, checked_succ, done


# ------------------------------------------------- locking ring, team drain

def explore_team(P, E, msgs, T, C, bug=Bug(), max_states=3_000_000):
    """A locking MPSC ring of P bytes and E entries fed by len(msgs)
    producers (msgs[p]: message sizes) and drained by a team of T members
    with rounds of at most C messages.  Returns the number of states."""
    K = len(msgs)
    total = sum(len(x) for x in msgs)
    max_rounds = total + T + 1

    # shared: cells, ents, recs (per sequence: (pos, p, mi)), tm, rm, rb,
    #         ticket, serving, hm, hb, claim, rounds (end + 1, 0 undefined)
    # producer p: (mi, phase, my_ticket, my_rm, my_rb, byte)
    # member t: (phase, k, start, end, cur idx, cur byte, bend)
    # consumed: tuple of consume counts per sequence number; rset: read markers
    sh0 = (tuple([None] * P), tuple([None] * E), tuple([None] * total), 0, 0, 0, 0, 0, 0, 0, 0,
           tuple([0] * max_rounds))
    pr0 = tuple((0, "ticket", 0, 0, 0, 0) for _ in range(K))
    me0 = tuple(("claim", 0, 0, 0, 0, 0, 0) for _ in range(T))
    start = (sh0, pr0, me0, tuple([0] * total), frozenset())

    def succ(st):
        sh, prs, mes, consumed, rset = st
        cells, ents, recs, tm, rm, rb, ticket, serving, hm, hb, claim, rounds = sh

        def SH(**kw):
            names = ("cells", "ents", "recs", "tm", "rm", "rb", "ticket", "serving", "hm", "hb",
                     "claim", "rounds")
            v = list(sh)
            for a, b in kw.items():
                v[names.index(a)] = b
            return tuple(v)

        # ---- producers
        for p in range(K):
            mi, ph, tk, my_rm, my_rb, jb = prs[p]
            if mi == len(msgs[p]):
                continue
            s = msgs[p][mi]

            def PR(**kw):
                v = dict(mi=mi, ph=ph, tk=tk, my_rm=my_rm, my_rb=my_rb, jb=jb)
                v.update(kw)
                return _set(prs, p, (v["mi"], v["ph"], v["tk"], v["my_rm"], v["my_rb"], v["jb"]))

            if ph == "ticket":
                yield (SH(ticket=ticket + 1), PR(ph="turn_lock", tk=ticket), mes, consumed, rset)
            elif ph == "turn_lock":
                if serving == tk:
                    yield (sh, PR(ph="room"), mes, consumed, rset)
            elif ph == "room":
                if rm - hm < E and rb + s - hb <= P:
                    yield (SH(rm=rm + 1, rb=rb + s, serving=serving + 1),
                           PR(ph="ent", my_rm=rm, my_rb=rb), mes, consumed, rset)
            elif ph == "ent":
                ne = _set(ents, my_rm % E, (s, p, mi))
                nxt = "pay" if bug.record_after_publish else "rec"
                yield (SH(ents=ne), PR(ph=nxt, jb=0), mes, consumed, rset)
            elif ph == "rec" or ph == "rec_late":
                nr = _set(recs, my_rm, (my_rb, p, mi))
                if ph == "rec":
                    yield (SH(recs=nr), PR(ph="pay", jb=0), mes, consumed, rset)
                else:
                    yield (SH(recs=nr), PR(mi=mi + 1, ph="ticket"), mes, consumed, rset)
            elif ph == "pay":
                if jb < s:
                    pos = (my_rb + jb) % P
                    old = cells[pos]
                    if old is not None and old not in rset:
                        raise Violation(f"producer {p} overwrote unread byte {old}")
                    yield (SH(cells=_set(cells, pos, (p, mi, jb))), PR(jb=jb + 1), mes, consumed,
                           rset)
                else:
                    yield (sh, PR(ph="turn_pub"), mes, consumed, rset)
            elif ph == "turn_pub":
                if tm == my_rm:  # publish in reservation order
                    nxt = "rec_late" if bug.record_after_publish else "ticket"
                    nmi = mi if bug.record_after_publish else mi + 1
                    yield (SH(tm=my_rm + 1), PR(mi=nmi, ph=nxt), mes, consumed, rset)
        # ---- team members
        for t in range(T):
            ph, k, rs, re, ci, cb, bend = mes[t]

            def ME(**kw):
                v = dict(ph=ph, k=k, rs=rs, re=re, ci=ci, cb=cb, bend=bend)
                v.update(kw)
                return _set(mes, t, (v["ph"], v["k"], v["rs"], v["re"], v["ci"], v["cb"],
                                     v["bend"]))

            if ph == "claim":
                if claim < max_rounds:
                    yield (SH(claim=claim + 1), prs, ME(ph="start", k=claim), consumed, rset)
            elif ph == "start":
                if bug.start_from_released:
                    yield (sh, prs, ME(ph="define", rs=hm), consumed, rset)
                elif k == 0:
                    yield (sh, prs, ME(ph="define", rs=0), consumed, rset)
                elif rounds[k - 1]:
                    yield (sh, prs, ME(ph="define", rs=rounds[k - 1] - 1), consumed, rset)
            elif ph == "define":
                if rs >= total:
                    # nothing left: the round is defined empty and the member stops
                    yield (SH(rounds=_set(rounds, k, rs + 1)), prs, ME(ph="exit"), consumed, rset)
                elif tm > rs:
                    e = min(rs + C, tm, total)
                    yield (SH(rounds=_set(rounds, k, e + 1)), prs, ME(ph="read", re=e, ci=rs, cb=0),
                           consumed, rset)
            elif ph == "read":
                if ci < re:
                    ent = ents[ci % E]
                    rec = recs[ci]
                    if ent is None or rec is None:
                        raise Violation(f"member {t} read an unwritten entry or record of {ci}")
                    sz, p, mi = ent
                    pos, rp, rmi = rec
                    if (rp, rmi) != (p, mi):
                        raise Violation(f"record {rec} does not match entry {ent}")
                    if cb < sz:
                        at = (pos + cb) % P
                        if cells[at] != (p, mi, cb):
                            raise Violation(f"member {t} read {cells[at]} expecting {(p, mi, cb)}")
                        yield (sh, prs, ME(cb=cb + 1), consumed, rset | {(p, mi, cb)})
                    else:
                        if consumed[ci]:
                            raise Violation(f"message {ci} consumed twice")
                        yield (sh, prs, ME(ci=ci + 1, cb=0, bend=pos + sz), _set(consumed, ci, 1),
                               rset)
                else:
                    yield (sh, prs, ME(ph="turn_rel"), consumed, rset)
            elif ph == "turn_rel":
                if bug.no_round_order or hm == rs:
                    yield (sh, prs, ME(ph="rel_hb"), consumed, rset)
            elif ph == "rel_hb":
                nb = bend if re > rs else hb
                yield (SH(hb=max(hb, nb) if bug.no_round_order else nb), prs, ME(ph="rel_hm"),
                       consumed, rset)
            elif ph == "rel_hm":
                yield (SH(hm=max(hm, re) if bug.no_round_order else re), prs, ME(ph="claim"),
                       consumed, rset)

    def done(st):
        sh, prs, mes, consumed, rset = st
        return all(consumed) and all(p[0] == len(msgs[i]) for i, p in enumerate(prs)) and \
            all(m[0] == "exit" for m in mes)

    def checked_succ(st):
        sh = st[0]
        tm, hm = sh[3], sh[8]
        if tm - hm > E or tm < hm:
            raise Violation("entry capacity exceeded")
        if any(c > 1 for c in st[3]):
            raise Violation("a message was consumed twice")
        return succ(st)

    return _dfs(start, checked_succ, done, max_states)


# --------------------------------------------------- striped ping-pong

def explore_striped(W, reps, bug=Bug(), max_states=3_000_000):
    """Ping-pong over two one-message rings A and B between a pinger and a
    ponger group of W members each; member i owns stripe i.  Counters:
    A arrived, A freed, B arrived, B freed, each raised by one per stripe.
    Returns the number of states."""
    need = (lambda k: k) if bug.count_messages else (lambda k: W * k)

    # shared: ringA, ringB, buf (markers per stripe), ctr (4), read sets
    # member: (k, step)
    start = (tuple([None] * W), tuple([None] * W), tuple([None] * W), (0, 0, 0, 0),
             tuple((0, 0) for _ in range(W)), tuple((0, 0) for _ in range(W)),
             frozenset(), frozenset())

    def succ(st):
        A, Bq, buf, ctr, pi, po, readA, readB = st
        for i in range(W):
            k, s = pi[i]
            if k == reps:
                continue
            npi = lambda ns, nk=k: _set(pi, i, (nk, ns))
            if s == 0:          # wait until A is free of message k - 1
                if ctr[1] >= need(k):
                    yield (A, Bq, buf, ctr, npi(1), po, readA, readB)
            elif s == 1:        # copy stripe i of message k into A (or count first)
                if bug.signal_before_copy:
                    yield (A, Bq, buf, _set(ctr, 0, ctr[0] + 1), npi(11), po, readA, readB)
                else:
                    old = A[i]
                    if old is not None and old not in readA:
                        raise Violation(f"pinger {i} overwrote unread stripe {old} of A")
                    yield (_set(A, i, (k, i)), Bq, buf, ctr, npi(2), po, readA, readB)
            elif s == 11:       # (bug) copy after counting
                old = A[i]
                if old is not None and old not in readA:
                    raise Violation(f"pinger {i} overwrote unread stripe {old} of A")
                yield (_set(A, i, (k, i)), Bq, buf, ctr, npi(3), po, readA, readB)
            elif s == 2:        # A: stripe arrived
                yield (A, Bq, buf, _set(ctr, 0, ctr[0] + 1), npi(3), po, readA, readB)
            elif s == 3:        # wait for the echo
                if ctr[2] >= need(k + 1):
                    yield (A, Bq, buf, ctr, npi(4), po, readA, readB)
            elif s == 4:        # read stripe i of the echo
                if Bq[i] != (k, i):
                    raise Violation(f"pinger {i} read {Bq[i]} of B expecting {(k, i)}")
                yield (A, Bq, buf, ctr, npi(5), po, readA, readB | {(k, i)})
            elif s == 5:        # B: stripe freed
                yield (A, Bq, buf, _set(ctr, 3, ctr[3] + 1), _set(pi, i, (k + 1, 0)), po, readA,
                       readB)
        for i in range(W):
            k, s = po[i]
            if k == reps:
                continue
            npo = lambda ns, nk=k: _set(po, i, (nk, ns))
            if s == 0:          # wait for message k in A
                if ctr[0] >= need(k + 1):
                    yield (A, Bq, buf, ctr, pi, npo(1), readA, readB)
            elif s == 1:        # take stripe i of A into the buffer
                if A[i] != (k, i):
                    raise Violation(f"ponger {i} read {A[i]} of A expecting {(k, i)}")
                yield (A, Bq, _set(buf, i, A[i]), ctr, pi, npo(2), readA | {(k, i)}, readB)
            elif s == 2:        # A: stripe freed
                yield (A, Bq, buf, _set(ctr, 1, ctr[1] + 1), pi, npo(3), readA, readB)
            elif s == 3:        # wait until B is free of message k - 1
                if ctr[3] >= need(k):
                    yield (A, Bq, buf, ctr, pi, npo(4), readA, readB)
            elif s == 4:        # copy the buffer's stripe into B
                old = Bq[i]
                if old is not None and old not in readB:
                    raise Violation(f"ponger {i} overwrote unread stripe {old} of B")
                yield (A, _set(Bq, i, buf[i]), buf, ctr, pi, npo(5), readA, readB)
            elif s == 5:        # B: stripe arrived
                yield (A, Bq, buf, _set(ctr, 2, ctr[2] + 1), pi, _set(po, i, (k + 1, 0)), readA,
                       readB)

    def done(st):
        return all(k == reps for k, _ in st[4]) and all(k == reps for k, _ in st[5])

    return _dfs(start, succ, done, max_states)
