"""Exhaustive interleaving checks of the protocols the device kernels run
(oracle/protocol_kernels.py; CPU only): batched publication and
consumption, the team drain of a locking ring, and ping-pong's striped
counters.  Each accepted configuration is explored completely; each planted
mistake must be caught."""
import pytest

from oracle import protocol_kernels as pk

BATCHED = [
    (4, 4, [2, 1, 3, 2], 2, 1),
    (4, 3, [2, 1, 3, 2, 1], 2, 2),
    (5, 4, [1, 2, 3, 1, 2], 3, 2),
    (4, 4, [1, 3, 1, 2, 1], 2, 1),
    (6, 3, [2, 3, 1, 4, 2], 2, 2),
    (3, 3, [3, 0, 2, 1], 3, 1),       # a zero-byte message, a message as large as the ring
]


@pytest.mark.parametrize("cfg", BATCHED)
def test_batched_ring_accepts(cfg):
    assert pk.explore_batched(*cfg) > 0


@pytest.mark.parametrize("bug", ["publish_before_payload", "release_before_read",
                                 "batch_room_first_only"])
@pytest.mark.parametrize("cfg", BATCHED[:5])
def test_batched_ring_catches(cfg, bug):
    with pytest.raises(pk.Violation):
        pk.explore_batched(*cfg, pk.Bug(**{bug: True}))


# abort: every wave that waits looks at the pump's abort word, so once a
# request has arrived no actor of a ring (Sec. 4.3) is left waiting; the
# BATCHED rings, and two with deferred publication
ABORT = [cfg + (1,) for cfg in BATCHED] + [(4, 4, [2, 2, 1, 1], 2, 1, 2), (3, 2, [1, 1, 1, 1], 2, 2, 3)]


@pytest.mark.parametrize("cfg", ABORT)
def test_abort_leaves_no_actor_waiting(cfg):
    P, E, sizes, B, C, S = cfg
    plain = pk.explore_batched(P, E, sizes, B, C, S=S)
    # the abort adds states (a request in any state, exits from waits)
    assert pk.explore_batched_abort(P, E, sizes, B, C, S=S) > plain


@pytest.mark.parametrize("bug", ["abort_ignored_by_producer", "abort_ignored_by_consumer"])
@pytest.mark.parametrize("cfg", ABORT)
def test_abort_catches_a_wait_that_ignores_it(cfg, bug):
    P, E, sizes, B, C, S = cfg
    with pytest.raises(pk.Violation, match="deadlock"):
        pk.explore_batched_abort(P, E, sizes, B, C, pk.Bug(**{bug: True}), S=S)
    # the same bug changes nothing without an abort
    assert pk.explore_batched(P, E, sizes, B, C, pk.Bug(**{bug: True}), S=S) > 0


# deferred publication: (P, E, sizes, B, C, S) -- sub-batches of B messages,
# up to S per publication
DEFERRED = [
    (4, 4, [1, 1, 1, 1, 2], 2, 1, 2),
    (4, 6, [1, 1, 1, 1, 1, 1], 2, 2, 3),
    (5, 4, [1, 2, 1, 1, 2], 2, 1, 2),
    (3, 4, [1, 1, 1, 1], 1, 2, 3),
    (2, 4, [1, 1, 1], 2, 1, 2),          # a full sub-batch fills the ring's bytes
    (4, 4, [2, 2, 1, 1], 2, 1, 2),       # ... with messages of two bytes
    (3, 2, [1, 1, 1, 1], 2, 2, 3),       # ... fills the ring's entries
]


@pytest.mark.parametrize("cfg", DEFERRED)
def test_deferred_publication_accepts(cfg):
    P, E, sizes, B, C, S = cfg
    assert pk.explore_batched(P, E, sizes, B, C, S=S) > 0


@pytest.mark.parametrize("cfg", DEFERRED[4:])
def test_deferred_publication_catches_a_blocked_producer_that_holds_messages(cfg):
    # these configurations reach a state where a full sub-batch is held and
    # the next message does not fit
    P, E, sizes, B, C, S = cfg
    with pytest.raises(pk.Violation, match="deadlock"):
        pk.explore_batched(P, E, sizes, B, C, pk.Bug(no_publish_when_blocked=True), S=S)


@pytest.mark.parametrize("bug", ["publish_before_payload", "release_before_read",
                                 "batch_room_first_only"])
@pytest.mark.parametrize("cfg", [(6, 4, [1, 1, 3, 2, 1, 2], 2, 1, 2),
                                 (5, 6, [1, 1, 2, 2, 1, 1], 2, 1, 3)])
def test_deferred_publication_catches(cfg, bug):
    P, E, sizes, B, C, S = cfg
    # the configuration reaches held sub-batches (its state space differs
    # from the one of immediate publication)
    assert pk.explore_batched(P, E, sizes, B, C, S=S) != pk.explore_batched(P, E, sizes, B, C)
    with pytest.raises(pk.Violation):
        pk.explore_batched(P, E, sizes, B, C, pk.Bug(**{bug: True}), S=S)


TEAM = [
    (4, 2, [[1, 2], [2, 1]], 2, 2),
    (3, 3, [[1, 1], [2, 1]], 2, 1),
    (5, 3, [[2, 0], [1, 3]], 2, 2),    # a zero-byte message
    (3, 2, [[1], [1], [2]], 2, 2),     # three producers
]


@pytest.mark.parametrize("cfg", TEAM)
def test_team_drain_accepts(cfg):
    assert pk.explore_team(*cfg) > 1000


@pytest.mark.parametrize("bug", ["record_after_publish", "no_round_order",
                                 "start_from_released"])
@pytest.mark.parametrize("cfg", TEAM)
def test_team_drain_catches(cfg, bug):
    with pytest.raises(pk.Violation):
        pk.explore_team(*cfg, pk.Bug(**{bug: True}))


@pytest.mark.parametrize("W,reps", [(2, 2), (3, 2), (2, 3), (4, 1)])
def test_striped_pingpong_accepts(W, reps):
    assert pk.explore_striped(W, reps) > 0


@pytest.mark.parametrize("bug", ["count_messages", "signal_before_copy"])
@pytest.mark.parametrize("W,reps", [(2, 2), (3, 2), (4, 1)])
def test_striped_pingpong_catches(W, reps, bug):
    with pytest.raises(pk.Violation):
        pk.explore_striped(W, reps, pk.Bug(**{bug: True}))
