"""Host-side model of the queued loop's round protocol (the step kernel's state
machine in gr_kernels.hip).  Each phase of a round reads and clears rotating
counters: the per-round queue counters (3 slots), the candidate-list counters
(3 rows) and the small-round expanded-vertex counters (3 rows).  The model
replays random schedules of normal rounds, small rounds and overflow fallbacks
and checks that every counter a phase adds into was cleared since its last use
and that every read sees the round it expects -- and that dropping one of the
clears the kernel does is detected."""
import random


def replay(seed, rounds=60, clear_slot_in_small=True):
    rnd = random.Random(seed)
    slot = {0: ("w", 0), 1: ("z",), 2: ("z",)}  # queue counters: slot r % 3 holds round r's totals
    cc = {0: ("z",), 1: ("z",), 2: ("z",)}     # candidate counters: row (r + 1) % 3 gets round r's appends
    act = {0: ("z",), 1: ("z",), 2: ("z",)}    # expanded-vertex counters of small round r: row r % 3
    r, phase, forced_small = 0, "advance", False
    for _ in range(400):
        if r >= rounds:
            return
        if phase == "advance":
            assert slot[r % 3] == ("w", r), "advance reads round %d's totals" % r
            cc[(r + 2) % 3] = ("z",)
            assert cc[(r + 1) % 3] == ("z",), "push appends into a cleared row"
            cc[(r + 1) % 3] = ("a", r)
            phase = "filter"
        elif phase == "filter":
            assert slot[(r + 1) % 3] == ("z",), "filter adds into a cleared slot"
            slot[(r + 1) % 3] = ("w", r + 1)
            slot[(r + 2) % 3] = ("z",)
            assert cc[(r + 1) % 3] == ("a", r)
            if rnd.random() < 0.6:  # the list did not overflow: next round is small
                act[(r + 1) % 3] = ("z",)
                r, phase, forced_small = r + 1, "after-small", True
            else:
                r, phase = r + 1, "advance"
        else:  # after-small: the candidates of round r - 1 decide round r
            assert cc[r % 3] == ("a", r - 1), "round %d reads round %d's candidates" % (r, r - 1)
            overflow = rnd.random() < 0.3 and not forced_small  # the filter checked the same counters
            forced_small = False
            if not overflow:  # small round r
                act[(r + 1) % 3] = ("z",)
                cc[(r + 2) % 3] = ("z",)
                if clear_slot_in_small:
                    slot[(r + 2) % 3] = ("z",)
                assert cc[(r + 1) % 3] == ("z",), "small round appends into a cleared row"
                assert act[r % 3] == ("z",), "small round counts into a cleared row"
                cc[(r + 1) % 3] = ("a", r)
                act[r % 3] = ("a", r)
                r += 1
            else:  # round r - 1's filter, then a normal round r
                assert slot[r % 3] == ("z",), "fallback filter adds into a cleared slot"
                slot[r % 3] = ("w", r)
                slot[(r + 1) % 3] = ("z",)
                phase = "advance"


def test_protocol_invariants_hold():
    for seed in range(1500):
        replay(seed)


def test_model_detects_a_missing_clear():
    caught = 0
    for seed in range(200):
        try:
            replay(seed, clear_slot_in_small=False)
        except AssertionError:
            caught += 1
    assert caught > 0
