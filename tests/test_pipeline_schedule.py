"""Host logic of pipeline.run_in_flight (no GPU): slots whose detections
end in a scripted order stand in for streams.  Every batch is started and
finished exactly once, on the slot that started it, finished only after its
detection has ended, the slot refilled at once; a slot whose detection is
held back holds back no other slot; results come back in batch order."""

import pytest

from paper_2101_05012_amd import pipeline


class FakeEvent:
    def __init__(self, clock, at):
        self.clock, self.at = clock, at

    def query(self):
        return self.clock[0] >= self.at


def run(n_slots, n_batches, durations):
    """durations[b]: polls until batch b's detection ends once started"""
    clock = [0]
    bufs = [{} for _ in range(n_slots)]
    log = []
    slot_of = {}

    def start_fn(i, b):
        assert b not in slot_of
        slot_of[b] = i
        bufs[i]["detected"] = FakeEvent(clock, clock[0] + durations[b])
        log.append(("start", i, b, clock[0]))

    def finish_fn(i, b):
        assert slot_of[b] == i
        assert bufs[i]["detected"].query()
        log.append(("finish", i, b, clock[0]))
        return ("result", b)

    real_ready = pipeline.ready

    def ticking_ready(bf):
        clock[0] += 1
        return real_ready(bf)

    pipeline.ready = ticking_ready
    try:
        out = pipeline.run_in_flight(n_slots, n_batches, start_fn, finish_fn, bufs, poll_s=0.0)
    finally:
        pipeline.ready = real_ready
    return out, log, slot_of


@pytest.mark.parametrize("n_slots,n_batches", [(1, 1), (1, 5), (4, 3), (4, 4), (4, 17), (16, 64)])
def test_every_batch_once_in_order(n_slots, n_batches):
    durations = [(7 * b) % 13 + 1 for b in range(n_batches)]
    out, log, slot_of = run(n_slots, n_batches, durations)
    assert out == [("result", b) for b in range(n_batches)]
    starts = [e for e in log if e[0] == "start"]
    finishes = [e for e in log if e[0] == "finish"]
    assert sorted(e[2] for e in starts) == list(range(n_batches))
    assert sorted(e[2] for e in finishes) == list(range(n_batches))
    # batches start in order, and a slot starts its next batch right after
    # finishing one (nothing else logged in between)
    assert [e[2] for e in starts] == list(range(n_batches))
    for k, e in enumerate(log):
        if e[0] == "finish" and any(s[2] > e[2] and s[1] == e[1] for s in starts):
            nxt = log[k + 1]
            assert nxt[0] == "start" and nxt[1] == e[1], (e, nxt)
    assert len(set(slot_of.values())) == min(n_slots, n_batches)


def test_held_slot_holds_back_no_other():
    # slot 0's first batch takes very long; the other three slots keep
    # cycling through every later batch meanwhile
    n_slots, n_batches = 4, 12
    durations = [1000] + [3] * (n_batches - 1)
    out, log, slot_of = run(n_slots, n_batches, durations)
    assert out == [("result", b) for b in range(n_batches)]
    fin = {e[2]: e[3] for e in log if e[0] == "finish"}
    assert all(fin[b] < fin[0] for b in range(1, n_batches))
    assert all(slot_of[b] != 0 for b in range(1, n_batches))
