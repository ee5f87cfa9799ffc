"""The serving scheduler on the CPU: an oracle-backed executor and a fake clock
(tests/fake_executor.py) check admission by memory budget, continuous batching
of BFS queries into shared sessions, sharing of whole-graph jobs, cancellation
and the latency report; every answer is compared with the oracle."""
import numpy as np
import pytest

import graphgen as gg
import oracle as orc
from fake_executor import FakeClock, FakeExecutor
from paper_2201_08560_amd.serve import Query, Server

GRAPHS = [gg.rmat(9, 8, seed=3), gg.path(40), gg.er_gnm(300, 900, seed=4), gg.star(50)]


def expected(q):
    g = GRAPHS[q.graph]
    return {"bfs": lambda: orc.bfs(g, q.source), "sssp": lambda: orc.sssp_unit(g, q.source),
            "cc": lambda: orc.cc(g), "tc": lambda: orc.tc(g)}[q.kind]()


def check(q):
    assert q.status == "done", (q.qid, q.status)
    exp = expected(q)
    if q.kind == "tc":
        assert int(q.result) == exp
    else:
        assert np.array_equal(np.asarray(q.result, dtype=np.uint32), exp), (q.qid, q.kind)


def stream(n, seed, kinds=("bfs", "bfs", "sssp", "cc", "tc"), rate=50.0):
    r = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(n):
        t += r.exponential(1.0 / rate)
        g = int(r.integers(len(GRAPHS)))
        out.append(Query(i, kinds[int(r.integers(len(kinds)))], g, int(r.integers(GRAPHS[g].n)), t))
    return out


def run(queries, budget=1 << 30, clock=None, **kw):
    clock = clock or FakeClock()
    ex = FakeExecutor(GRAPHS, **kw)
    srv = Server(ex, budget, clock=clock)
    srv.run(queries, sleep=clock.sleep, max_ticks=100000)
    return srv, ex


def test_every_query_answered_like_the_oracle():
    srv, ex = run(stream(200, 1))
    assert len(srv.done) == 200 and srv.in_use == 0
    for q in srv.done:
        check(q)
    st = srv.stats()
    assert st["done"] == 200 and st["p99_ms"] >= st["p50_ms"] >= 0
    assert ex.opened == ex.closed


def test_bfs_queries_join_a_running_session():
    """Queries that arrive while a session runs join its next step instead of
    waiting for it to finish (continuous batching)."""
    clock = FakeClock()
    ex = FakeExecutor(GRAPHS)
    srv = Server(ex, 1 << 30, clock=clock)
    a = Query(0, "bfs", 1, 0, 0.0)       # path graph: 40 levels
    srv.submit(a)
    for _ in range(5):
        srv.tick()
    b = Query(1, "bfs", 1, 39, 0.0)
    srv.submit(b)
    srv.tick()
    assert ex.opened == 1 and b.joined_step == 5 and a.status == "running"
    while not srv.idle:
        srv.tick()
    check(a), check(b)
    assert ex.opened == 1
    assert max(ex.sessions[0].steps_with) == 2


def test_more_than_64_queries_reuse_slots():
    qs = [Query(i, "bfs", 2, i % GRAPHS[2].n, 0.0) for i in range(150)]
    srv, ex = run(qs)
    for q in srv.done:
        check(q)
    assert ex.opened == 1 and max(ex.sessions[0].steps_with) == 64


def test_budget_rejects_what_can_never_fit_and_delays_the_rest():
    n2, n3 = GRAPHS[2].n, GRAPHS[3].n
    # room for graph 2's session and two results, not for graph 3's session beside it
    budget = 280 * n2 + 1024 + 2 * 4 * n2 + 64
    assert 280 * n2 + 1024 + 280 * n3 + 1024 + 4 * (n2 + n3) > budget
    a, b, c = Query(0, "bfs", 2, 0, 0.0), Query(1, "bfs", 3, 0, 0.0), Query(2, "bfs", 2, 5, 0.0)
    srv, ex = run([a, b, c], budget=budget, clock=FakeClock(tick=1e-3))
    for q in (a, b, c):
        check(q)
    assert srv.peak_in_use <= budget and srv.in_use == 0
    assert b.admitted >= a.finished and c.admitted < a.finished  # c joined a's session; b waited
    assert b.waited_for_memory and not a.waited_for_memory and not c.waited_for_memory
    assert srv.stats()["waited_for_memory"] == 1
    # graph 0's session (512 vertices) is larger than the whole budget: rejected
    srv2 = Server(FakeExecutor(GRAPHS), 1000, clock=FakeClock())
    q = Query(9, "bfs", 0, 0, 0.0)
    srv2.submit(q)
    assert q.status == "rejected" and srv2.queue == []


def test_waiting_query_admitted_when_memory_frees():
    n = GRAPHS[2].n
    budget = 280 * n + 1024 + 4 * n  # one session, one result
    clock = FakeClock(tick=1e-3)
    ex = FakeExecutor(GRAPHS)
    srv = Server(ex, budget, clock=clock)
    a, b = Query(0, "bfs", 2, 0, 0.0), Query(1, "bfs", 2, 1, 0.0)
    srv.submit(a), srv.submit(b)
    srv.tick()
    assert a.status == "running" and b.status == "queued"
    while not srv.idle:
        srv.tick()
    check(a), check(b)
    assert b.admitted >= a.finished


def test_whole_graph_jobs_are_shared_and_cached():
    qs = [Query(i, "cc", 2, 0, 0.0) for i in range(5)] + [Query(5, "tc", 0, 0, 0.0), Query(6, "tc", 0, 0, 1.0)]
    srv, ex = run(qs, job_ticks=4)
    for q in srv.done:
        check(q)
    assert sorted(k for k, _, _ in ex.jobs_run) == ["cc", "tc"]


def test_cancel_queued_and_running():
    clock = FakeClock()
    ex = FakeExecutor(GRAPHS, job_ticks=50)
    srv = Server(ex, 1 << 30, clock=clock)
    a, b, c = Query(0, "bfs", 1, 0, 0.0), Query(1, "sssp", 2, 3, 0.0), Query(2, "bfs", 1, 7, 0.0)
    for q in (a, b, c):
        srv.submit(q)
    srv.tick()
    srv.cancel(a)   # running in a session
    srv.cancel(b)   # running as a job
    while not srv.idle:
        srv.tick()
    assert a.status == b.status == "cancelled"
    check(c)
    assert srv.in_use == 0 and ex.opened == ex.closed


def test_results_same_alone_and_in_the_mix():
    qs = stream(120, 7)
    srv, _ = run([Query(q.qid, q.kind, q.graph, q.source, q.arrival) for q in qs])
    mixed = {q.qid: q.result for q in srv.done}
    for q in qs[:40]:
        alone, _ = run([Query(q.qid, q.kind, q.graph, q.source, 0.0)])
        a = alone.done[0].result
        if q.kind == "tc":
            assert int(a) == int(mixed[q.qid])
        else:
            assert np.array_equal(np.asarray(a), np.asarray(mixed[q.qid]))


def test_bad_queries():
    srv = Server(FakeExecutor(GRAPHS), 1 << 30, clock=FakeClock())
    with pytest.raises(ValueError):
        srv.submit(Query(0, "diameter", 0))
    with pytest.raises(ValueError):
        srv.submit(Query(1, "bfs", 0, GRAPHS[0].n))


def test_admission_scan_stops_after_scan_limit_waiting_queries():
    """A round stops looking after scan_limit queries that cannot start; the
    rest keep their order and start in later rounds, every answer unchanged."""
    n = GRAPHS[2].n
    budget = 280 * n + 1024 + 4 * n  # one session of graph 2 and one result
    clock = FakeClock(tick=1e-3)
    srv = Server(FakeExecutor(GRAPHS), budget, clock=clock, scan_limit=2)
    qs = [Query(i, "bfs", 2, i, 0.0) for i in range(4)] + [Query(4, "cc", 1, 0, 0.0)]
    for q in qs:
        srv.submit(q)
    srv.tick()
    # q0 runs; q1 and q2 cannot start (no memory for a second result) and end the
    # scan, so q3 and the CC query are not looked at in this round
    assert qs[0].status == "running"
    assert [q.qid for q in srv.queue] == [1, 2, 3, 4]
    while not srv.idle:
        srv.tick()
    for q in qs:
        check(q)
    assert srv.peak_in_use <= budget and srv.in_use == 0
