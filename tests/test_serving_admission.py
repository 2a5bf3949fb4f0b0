"""Host logic of the serving loop's admission (no device needed): requests
wait while their staging does not fit in free memory, except that an idle
server admits one, so the loop always makes progress."""
import collections
import time

import numpy as np

from paper_2407_19562_amd import inputs, serving


def _server(free, m=1 << 20):
    srv = serving.Server.__new__(serving.Server)   # no graphs, no device
    srv.reserve = 1 << 20
    srv._free_bytes = lambda: free
    srv.inserted = [0]
    srv.slack = [serving.spare_slots(m)]
    srv.growth = [serving.growth_bytes(m)]
    return srv


def _requests(k):
    e = np.zeros(3, np.int32)
    b = inputs.Batch(e, e, e, e)
    return collections.deque(serving.Request(0, b, 0.0) for _ in range(k))


def test_admits_what_fits():
    srv = _server(free=1 << 30)
    rep, pending, queues = serving.Report(), _requests(3), [collections.deque()]
    srv._admit(rep, pending, queues, time.perf_counter(), open_loop=False)
    assert len(queues[0]) == 3 and not pending and rep.admission_waits == 0


def test_waits_when_memory_is_short_unless_idle():
    srv = _server(free=0)
    rep, pending, queues = serving.Report(), _requests(3), [collections.deque()]
    srv._admit(rep, pending, queues, time.perf_counter(), open_loop=False)
    assert len(queues[0]) == 0 and len(pending) == 3 and rep.admission_waits == 1
    srv._admit(rep, pending, queues, time.perf_counter(), open_loop=False, idle=True)
    assert len(queues[0]) == 1 and len(pending) == 2


def test_open_loop_respects_arrival_times():
    srv = _server(free=1 << 30)
    e = np.zeros(1, np.int32)
    b = inputs.Batch(e, e, e, e)
    pending = collections.deque([serving.Request(0, b, 0.0), serving.Request(0, b, 1e6)])
    rep, queues = serving.Report(), [collections.deque()]
    srv._admit(rep, pending, queues, time.perf_counter(), open_loop=True)
    assert len(queues[0]) == 1 and len(pending) == 1


def test_growth_counts_when_insertions_overflow_the_slack():
    # a graph of 4096 edges has 1024 spare slots: the batch of 1000
    # insertions fits, the next one would overflow and needs the growth
    # bytes too
    m = 4096
    e = np.zeros(1000, np.int32)
    big = inputs.Batch(np.zeros(0, np.int32), np.zeros(0, np.int32), e, e)
    staging = 48 * 1000
    free = (1 << 20) + 2 * staging + serving.growth_bytes(m) // 2
    srv = _server(free=free, m=m)
    pending = collections.deque([serving.Request(0, big, 0.0), serving.Request(0, big, 0.0)])
    rep, queues = serving.Report(), [collections.deque()]
    srv._admit(rep, pending, queues, time.perf_counter(), open_loop=False)
    assert len(queues[0]) == 1 and len(pending) == 1 and rep.admission_waits == 1
    assert srv.inserted[0] == 1000
    # with room for the growth it is admitted, and the slack doubles
    srv._free_bytes = lambda: (1 << 20) + staging + serving.growth_bytes(m)
    srv._admit(rep, pending, queues, time.perf_counter(), open_loop=False)
    assert len(queues[0]) == 2 and not pending
    assert srv.slack[0] == 2 * serving.spare_slots(m) and srv.inserted[0] == 1000
