"""Host logic of the serving loop: batch packing and HBM-budget admission."""
from collections import deque

import pytest

from paper_2310_20285_amd.serving import HBMBudget, Ticket, admit_fits, plan_batch


def _pred(rid, rows):
    return Ticket(rid, "predict", 0.0, rows)


def _fit(rid, nbytes):
    t = Ticket(rid, "fit", 0.0, 100)
    t.bytes = nbytes
    return t


def test_plan_batch_packs_in_arrival_order_and_splits_large_queries():
    q = deque([_pred(0, 3), _pred(1, 5), _pred(2, 10), _pred(3, 1)])
    b1 = plan_batch(q, 12)
    assert [(t.rid, a, k) for t, a, k in b1] == [(0, 0, 3), (1, 0, 5), (2, 0, 4)]
    assert [t.rid for t in q] == [2, 3] and q[0].served_rows == 4
    b2 = plan_batch(q, 12)
    assert [(t.rid, a, k) for t, a, k in b2] == [(2, 4, 6), (3, 0, 1)]
    assert not q


def test_plan_batch_rows_cover_every_query_exactly_once():
    sizes = [1, 4096, 7, 300, 8191, 2, 8192, 5000]
    q = deque(_pred(i, n) for i, n in enumerate(sizes))
    seen = {i: [] for i in range(len(sizes))}
    while q:
        batch = plan_batch(q, 8192)
        assert 0 < sum(k for _, _, k in batch) <= 8192
        for t, a, k in batch:
            seen[t.rid].append((a, k))
    for i, n in enumerate(sizes):
        pos = 0
        for a, k in seen[i]:
            assert a == pos and k > 0
            pos += k
        assert pos == n


def test_budget_reserve_release():
    b = HBMBudget(100)
    assert b.try_reserve(60) and not b.try_reserve(50) and b.try_reserve(40)
    assert b.free == 0
    b.release(60)
    assert b.free == 60
    with pytest.raises(RuntimeError):
        b.release(1000)


def test_admission_refuses_oversized_and_keeps_arrival_order():
    b = HBMBudget(100)
    q = deque([_fit(0, 40), _fit(1, 150), _fit(2, 50), _fit(3, 20)])
    start, refused = admit_fits(q, b, capacity=100, free_workers=4)
    assert [t.rid for t in start] == [0, 2] and [t.rid for t in refused] == [1]
    # fit 3 needs 20 bytes and 10 are left: it waits
    assert [t.rid for t in q] == [3] and b.used == 90
    start, refused = admit_fits(q, b, capacity=100, free_workers=4)
    assert not start and not refused
    b.release(40)
    start, _ = admit_fits(q, b, capacity=100, free_workers=4)
    assert [t.rid for t in start] == [3] and b.used == 70


def test_admission_respects_worker_count_and_head_of_line():
    b = HBMBudget(1000)
    q = deque([_fit(0, 10), _fit(1, 10), _fit(2, 10)])
    start, _ = admit_fits(q, b, capacity=1000, free_workers=2)
    assert [t.rid for t in start] == [0, 1] and len(q) == 1
    b2 = HBMBudget(100)
    q2 = deque([_fit(0, 90), _fit(1, 80), _fit(2, 5)])
    start, _ = admit_fits(q2, b2, capacity=100, free_workers=4)
    # the head waits for budget and blocks the small fit behind it
    assert [t.rid for t in start] == [0] and [t.rid for t in q2] == [1, 2]
