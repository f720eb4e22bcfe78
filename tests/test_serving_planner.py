"""Host logic of the serving loop: batch formation, admission by footprint, factor cache."""

from types import SimpleNamespace as NS

from paper_2501_06748_amd.serving import BatchPlanner


def _req(rid, key, steps=100, n_rec=4):
    return NS(rid=rid, model=NS(key=key), n_steps=steps, n_rec=n_rec)


def _fp(factor=100, run=10):
    return lambda key, shots, steps: (factor, run * shots)


def test_batches_group_same_model_and_steps_in_arrival_order():
    p = BatchPlanner(10_000, _fp(), max_shots=3)
    for i, (k, st) in enumerate([("a", 100), ("b", 100), ("a", 100), ("a", 200), ("a", 100), ("a", 100)]):
        p.add(_req(i, k, st))
    b, ev = p.next_batch()
    assert [r.rid for r in b.requests] == [0, 2, 4] and not ev        # capped at 3 shots
    b2, _ = p.next_batch()
    assert [r.rid for r in b2.requests] == [1]                       # model "a" busy: "b" goes next
    b3, _ = p.next_batch()
    assert b3 is None                                                # the rest is for the busy model
    p.finish(b)
    b4, _ = p.next_batch()
    assert [r.rid for r in b4.requests] == [3]                       # oldest first: the 200-step shot
    p.finish(b4)
    b5, _ = p.next_batch()
    assert [r.rid for r in b5.requests] == [5]


def test_admission_waits_for_memory_and_runs_alone_above_budget():
    p = BatchPlanner(250, _fp(factor=100, run=60))
    p.add(_req(0, "a"))
    p.add(_req(1, "b"))
    b0, _ = p.next_batch()
    assert b0 is not None and p.used == 160
    b1, _ = p.next_batch()
    assert b1 is None                                                # 160 + 160 > 250: wait
    p.finish(b0)                                                     # a's factors stay cached (100)
    b1, ev = p.next_batch()
    assert b1 is not None and [r.rid for r in b1.requests] == [1]
    assert len(ev) == 1 and p.used == 160                            # idle "a" evicted to make room
    p.finish(b1)
    q = BatchPlanner(50, _fp(factor=100, run=60))
    q.add(_req(7, "z"))
    bz, _ = q.next_batch()
    assert bz is not None                                            # alone it runs above the budget


def test_cache_reuse_and_no_cache_mode():
    p = BatchPlanner(10_000, _fp(factor=100, run=10))
    p.add(_req(0, "a"))
    b, _ = p.next_batch()
    assert b.factor_bytes == 100
    p.cache["a"].value = object()                                    # factors built by the worker
    assert p.finish(b) is None and p.used == 100                     # kept resident
    p.add(_req(1, "a"))
    b, _ = p.next_batch()
    assert b.factor_bytes == 0 and p.used == 110                     # reused, not re-added
    p.finish(b)
    q = BatchPlanner(10_000, _fp(factor=100, run=10), batching=False, cache=False)
    q.add(_req(0, "a"))
    q.add(_req(1, "a"))
    b, _ = q.next_batch()
    assert len(b.requests) == 1
    ent = q.finish(b)
    assert ent is not None and q.used == 0 and "a" not in q.cache
