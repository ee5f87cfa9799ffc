"""Serving on the GPU: continuous BFS sessions through the C ABI, and the
scheduler with the device executor.  Every answer equals the oracle's, and
each query's result is the same alone and in a mixed stream where queries join
running sessions and whole-graph jobs overlap them on other streams."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as orc

pytestmark = pytest.mark.gpu
b2 = pytest.importorskip("paper_2201_08560_amd")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2201_08560_amd.serve import GpuExecutor, Query, Server  # noqa: E402

GRAPHS = [gg.rmat(12, 16, seed=5), gg.path(300), gg.er_gnm(2049, 6000, seed=7), gg.king_grid(30, 41),
          gg.rmat(10, 8, seed=6), gg.disjoint_union(gg.complete(20), gg.path(1), gg.cycle(37))]
TILES = [32, 8, 16, 4, 8, 32]


@pytest.fixture(scope="module")
def pool():
    # TC operands of two graphs are left to the executor to build on first use
    return [(b2.B2SR.from_graph(g, t), None if i in (1, 4) else b2.B2SR.from_graph(g, GpuExecutor.tc_tile(t), lower=True))
            for i, (g, t) in enumerate(zip(GRAPHS, TILES))]


def expected(q):
    g = GRAPHS[q.graph]
    return {"bfs": lambda: orc.bfs(g, q.source), "sssp": lambda: orc.sssp_unit(g, q.source),
            "cc": lambda: orc.cc(g), "tc": lambda: orc.tc(g)}[q.kind]()


def host(q):
    if q.kind == "tc":
        return int(b2.as_u64(q.result)[0])
    return b2.as_u32(q.result)


def test_session_slots_join_between_levels(pool):
    """Slots join at different steps and leave when done; each one's levels
    equal a plain BFS from its source."""
    A = pool[1][0]   # a path: long BFS
    g = GRAPHS[1]
    s = b2.BfsSession(A)
    try:
        starts = {0: 0, 5: 299, 63: 150}
        s.join(0, starts[0])
        steps, done, joined = 0, {}, {0}
        while len(done) < 3:
            if steps == 3:
                s.join(5, starts[5]), joined.add(5)
            if steps == 10:
                s.join(63, starts[63]), joined.add(63)
            s.step()
            steps += 1
            alive = s.alive()
            for slot in list(joined):
                if not (alive >> slot) & 1:
                    print(f"slot {slot} done at step {steps}", flush=True)
                    done[slot] = b2.as_u32(s.extract(slot))
                    joined.discard(slot)
        for slot, src in starts.items():
            assert np.array_equal(done[slot], orc.bfs(g, src)), slot
        st, busy = s.info()
        assert st == steps and busy == 0
        # a freed slot is reused by a new query on the same session
        s.join(0, 10)
        while (s.step() or True) and (s.alive() & 1):
            pass
        assert np.array_equal(b2.as_u32(s.extract(0)), orc.bfs(g, 10))
    finally:
        s.close()


def test_session_64_sources_and_cancel(pool):
    A, g = pool[0][0], GRAPHS[0]
    srcs = gg.sample_sources(g, 64, seed=3)
    s = b2.BfsSession(A)
    try:
        for k, v in enumerate(srcs):
            s.join(k, int(v))
        s.step()
        s.alive()
        s.cancel(7)                       # leaves mid-flight; its bits are cleared on the next join
        live = set(range(64)) - {7}
        out = {}
        while live:
            s.step()
            a = s.alive()
            for k in list(live):
                if not (a >> k) & 1:
                    out[k] = b2.as_u32(s.extract(k))
                    live.discard(k)
        for k in out:
            assert np.array_equal(out[k], orc.bfs(g, int(srcs[k]))), k
        s.join(7, int(srcs[0]))          # the cancelled slot starts over cleanly
        while (s.step() or True) and (s.alive() >> 7) & 1:
            pass
        assert np.array_equal(b2.as_u32(s.extract(7)), orc.bfs(g, int(srcs[0])))
    finally:
        s.close()


def stream(n, seed, rate):
    r = np.random.default_rng(seed)
    t, out = 0.0, []
    kinds = ("bfs", "bfs", "bfs", "sssp", "cc", "tc")
    for i in range(n):
        t += r.exponential(1.0 / rate)
        gi = int(r.integers(len(GRAPHS)))
        out.append(Query(i, kinds[int(r.integers(len(kinds)))], gi, int(r.integers(GRAPHS[gi].n)), t))
    return out


def test_server_mixed_stream_matches_oracle_and_alone(pool):
    ex = GpuExecutor(pool, GRAPHS, streams=3, workers=2)
    try:
        qs = stream(150, 11, rate=2000.0)
        budget = sum(ex.session_bytes(i) for i in range(len(GRAPHS))) // 2  # admission is exercised
        srv = Server(ex, budget)
        srv.run([Query(q.qid, q.kind, q.graph, q.source, q.arrival) for q in qs])
        torch.cuda.synchronize()
        assert all(q.status == "done" for q in srv.done), [q.status for q in srv.done if q.status != "done"]
        mixed = {q.qid: q for q in srv.done}
        for q in qs:
            got = host(mixed[q.qid])
            exp = expected(q)
            if q.kind == "tc":
                assert got == exp, q
            else:
                assert np.array_equal(got, exp), (q.qid, q.kind, q.graph)
        st = srv.stats()
        print(st, flush=True)
        assert st["peak_bytes_in_use"] <= budget and srv.in_use == 0
        # alone: each query through an empty server gives the same result
        for q in qs[:30]:
            solo = Server(ex, budget, cache=False)
            solo.run([Query(q.qid, q.kind, q.graph, q.source, 0.0)])
            torch.cuda.synchronize()
            a = host(solo.done[0])
            m = host(mixed[q.qid])
            assert (a == m) if q.kind == "tc" else np.array_equal(a, m), (q.qid, q.kind)
    finally:
        ex.shutdown()
