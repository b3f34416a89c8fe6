"""The request loop's scheduling on the host (fake server: no device, zero
results): FIFO admission, memory admission against the budget, slots,
batching of same-matrix requests into one launch group, queue limits and
ticket semantics."""
import time

import numpy as np
import pytest

import paper_2405_03456_amd as hm
from paper_2405_03456_amd import _lib


def block_bytes(n, cols):
    return 2 * ((n * cols * 8 + 255) // 256 * 256)


def test_fake_server_completes_everything_in_fifo_groups():
    S = hm.Server(mem_budget=1 << 24, max_slots=8, max_queue=100, max_cols=64, fake=True, fake_us=2000)
    a, b = S.register_shape(1000), S.register_shape(3000)
    tickets = []
    for i in range(20):
        t, Y = S.submit(a if i % 2 else b, np.ones((1000 if i % 2 else 3000, 1 + i % 5)))
        tickets.append((t, Y))
    stats = [S.wait(t) for t, _ in tickets]
    for (t, Y), st in zip(tickets, stats):
        assert np.all(Y == 0.0)
        assert st["latency_ms"] >= st["queue_ms"] >= 0.0 and st["run_ms"] > 0.0
        assert 1 <= st["group_requests"] <= 8
    # FIFO per matrix: a matrix's requests run in groups of non-decreasing id
    # (a later request of an idle matrix may join a group formed while an
    # earlier request of a busy matrix still waits)
    for parity in (0, 1):
        gid = [st["group_id"] for i, st in enumerate(stats) if i % 2 == parity]
        assert gid == sorted(gid)
    # requests for the same matrix share a block: its columns are summed
    assert max(st["group_cols"] for st in stats) > 5
    s = S.stats()
    assert s["submitted"] == s["completed"] == 20
    assert s["peak_inflight"] <= 8 and s["max_group_requests"] <= 8
    S.close()


def test_memory_admission_respects_the_budget():
    n = 4096
    budget = 3 * block_bytes(n, 4)          # at most three 4-column blocks at once
    S = hm.Server(mem_budget=budget, max_slots=64, max_queue=100, max_cols=4, fake=True, fake_us=3000)
    ids = [S.register_shape(n) for _ in range(6)]
    ts = [S.submit(ids[i % 6], np.ones((n, 4)))[0] for i in range(18)]
    for t in ts:
        S.wait(t)
    s = S.stats()
    assert s["peak_arena_bytes"] <= budget
    assert s["completed"] == 18 and s["groups"] >= 6
    with pytest.raises(hm.HMError) as ex:   # wider than max_cols: its workspace was never sized for it
        S.submit(ids[0], np.ones((n, 5)))
    assert ex.value.status == _lib.HM_EINVAL
    S.close()
    # a request within max_cols that could never fit the budget
    S = hm.Server(mem_budget=block_bytes(n, 4), max_slots=4, max_queue=10, max_cols=16, fake=True, fake_us=10)
    m = S.register_shape(n)
    with pytest.raises(hm.HMError) as ex:
        S.submit(m, np.ones((n, 13)))
    assert ex.value.status == _lib.HM_ENOMEM
    S.close()


def test_queue_limit_and_ticket_errors():
    S = hm.Server(mem_budget=1 << 20, max_slots=1, max_queue=3, max_cols=8, fake=True, fake_us=200000)
    m = S.register_shape(100)
    first = S.submit(m, np.ones(100))[0]
    time.sleep(0.05)                         # the first request is now running
    ts = [S.submit(m, np.ones(100))[0] for _ in range(3)]
    with pytest.raises(hm.HMError) as ex:
        S.submit(m, np.ones(100))
    assert ex.value.status == _lib.HM_EBUSY
    assert S.poll(ts[0]) is None             # still queued behind the running one
    for t in [first] + ts:
        S.wait(t)
    with pytest.raises(hm.HMError):          # released after done
        S.poll(first)
    with pytest.raises(hm.HMError):          # unknown matrix
        S.submit(99, np.ones(100))
    S.close()


def test_bad_options_and_register_rules():
    with pytest.raises(hm.HMError):
        hm.Server(mem_budget=0, fake=True)
    with pytest.raises(hm.HMError):
        hm.Server(max_slots=0, fake=True)
    S = hm.Server(fake=True)
    with pytest.raises(hm.HMError):
        S.register_shape(0)
    S.close()


def test_destroy_drains_pending_requests():
    S = hm.Server(mem_budget=1 << 22, max_slots=2, max_queue=50, max_cols=8, fake=True, fake_us=1000)
    m = S.register_shape(500)
    pend = [S.submit(m, np.ones((500, 2))) for _ in range(10)]
    S.close()                                # waits for all ten
    for _, Y in pend:
        assert np.all(Y == 0.0)
