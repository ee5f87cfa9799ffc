"""Batched multi-graph 64-source BFS on the GPU: every mode (per-level launches,
one persistent cooperative kernel, a replayed hipGraph plan) against the oracle's
per-source BFS and against per-graph launches, alone and in the mix."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as orc

pytestmark = pytest.mark.gpu
b2 = pytest.importorskip("paper_2201_08560_amd")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2201_08560_amd.batch import GraphBatch  # noqa: E402
from paper_2201_08560_amd import autotune  # noqa: E402


def make_graphs():
    gs = [gg.chung_lu(int(n), k, 2.1, seed=1000 + i)
          for i, (n, k) in enumerate([(1024, 4), (3000, 12), (5000, 30), (1100, 8), (20000, 6), (1500, 20)])]
    gs += [gg.er_gnm(2049, 6000, seed=7), gg.path(700), gg.king_grid(33, 40), gg.star(900),
           gg.disjoint_union(gg.complete(20), gg.path(50)), gg.mycielski(9)]
    return gs


GRAPHS = make_graphs()
TILES = [(4, 8, 16, 32, 64)[i % 5] for i in range(len(GRAPHS))]


def sources_for(g, k, seed):
    cand = np.flatnonzero(g.degrees() > 0)
    r = gg.rng(seed)
    return r.choice(cand, size=min(k, cand.size), replace=False).astype(np.uint32)


@pytest.fixture(scope="module")
def batch():
    B = GraphBatch(GRAPHS, TILES)
    B.set_sources([sources_for(g, 64 if i % 3 else 37, i) for i, g in enumerate(GRAPHS)])
    return B


def check_all(B, levels):
    for i, g in enumerate(GRAPHS):
        print(f"graph {i} {g.name} T={TILES[i]}", flush=True)
        ref = orc.bfs_multi(g, B.sources[i])
        assert np.array_equal(B.levels_of_host(levels, i), ref), g.name
    # padding vertices between graphs are never reached
    lv = b2.as_u32(levels)
    for i, g in enumerate(GRAPHS):
        pad = lv[int(B.offsets[i]) + g.n:int(B.offsets[i + 1])]
        assert np.all(pad == b2.UNREACHED)


def test_batch_levels_mode(batch):
    lv, it = batch.run(b2.BATCH_LEVELS)
    assert it >= 2
    check_all(batch, lv)


def test_batch_persistent_mode(batch):
    lv, it = batch.run(b2.BATCH_PERSISTENT)
    lv2, it2 = batch.run(b2.BATCH_LEVELS)
    assert it == it2
    assert torch.equal(lv, lv2)
    check_all(batch, lv)


@pytest.mark.parametrize("mode", ["levels", "persistent"])
def test_batch_graph_plan_replays(batch, mode):
    """The hipGraph plan replayed three times, with eager work and a change of
    sources between replays; every replay matches the eager result.  The path
    graph needs hundreds of levels, so the per-level plan replays its
    continuation graph many times."""
    eager, eager_it = batch.run(b2.BATCH_LEVELS)
    eager = eager.clone()
    plan = batch.plan(b2.BATCH_LEVELS if mode == "levels" else b2.BATCH_PERSISTENT)
    try:
        for rep in range(3):
            it = plan.launch(want_iters=(rep == 1))
            torch.cuda.synchronize()
            assert torch.equal(plan.out, eager), rep
            if rep == 1:
                assert it == eager_it
            junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work between replays
            torch.cuda.synchronize()
            del junk
        old = [s.copy() for s in batch.sources]
        batch.set_sources([sources_for(g, 64 if i % 3 else 37, 100 + i) for i, g in enumerate(GRAPHS)])
        it = plan.launch(want_iters=True)
        assert it >= 2
        check_all(batch, plan.out)
        batch.set_sources(old)
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(plan.out, eager)
        # enqueue only, then read the status once
        plan.launch(check=False)
        assert plan.status() == eager_it
        assert torch.equal(plan.out, eager)
    finally:
        plan.close()


def _flags_word(n):
    """Index (in 32-bit words) of the batch workspace's flag words: after the
    F, V, Y frontier arrays and the active bit vector, each 256-byte aligned."""
    off = 0
    for nbytes in (n * 8, n * 8, n * 8, (n + 31) // 32 * 4):
        off = (off + 255) & ~255
        off += nbytes
    return ((off + 255) & ~255) // 4


def test_persistent_plan_reports_a_timed_out_barrier(batch):
    """The time-out flag set from the host (as a barrier wait that ran out would
    set it) makes a persistent replay stop at its first barrier; an enqueue-only
    launch returns at once, the status read reports the time-out and clears the
    flag, and the next replay is whole again."""
    eager, _ = batch.run(b2.BATCH_LEVELS)
    plan = batch.plan(b2.BATCH_PERSISTENT)
    try:
        plan.launch()
        assert torch.equal(plan.out, eager)
        plan.ws.view(torch.int32)[_flags_word(batch.n) + 5] = 1
        plan.launch(check=False)
        with pytest.raises(b2.B2SRError):
            plan.status()
        plan.launch()
        assert torch.equal(plan.out, eager)
    finally:
        plan.close()


def test_batch_equals_per_graph_launches(batch):
    """Each graph's result is the same alone (its own B2SR, b2sr_msbfs) and in the mix."""
    mixed, _ = batch.run(b2.BATCH_PERSISTENT)
    for i, g in enumerate(GRAPHS):
        A = b2.B2SR.from_graph(g, TILES[i])
        alone, _ = b2.b2sr_msbfs(A, batch.sources[i])
        assert torch.equal(alone, batch.levels_of(mixed, i)), g.name


def test_autotune_exact_counts_match_oracle():
    for g in GRAPHS[:4]:
        T, rep = autotune.choose_tile(g)
        assert T in autotune.TILES
        for k in autotune.TILES:
            assert rep["ntiles"][k] == orc.b2sr_count_tiles(g, k)


def test_batch_tile_is_the_least_summed_cost():
    """One width for a batch: the argmin over T of the per-graph modelled costs
    summed (each graph's cost table from choose_tile), ties to the smaller T."""
    graphs = [gg.rmat(10, 8, seed=3), gg.king_grid(40, 50), gg.complete(40), gg.er_gnm(3000, 9000, seed=5)]
    total = {T: 0.0 for T in autotune.TILES}
    for g in graphs:
        cost = autotune.choose_tile(g, nsample=128)[1]["cost"]
        for T in total:
            total[T] += cost[T]
    T, rep = autotune.choose_batch_tile(graphs)
    assert rep["cost"] == pytest.approx(total)
    assert T == min(total, key=lambda k: (total[k], k))


def test_persistent_phase_timestamps(batch):
    """The timed persistent launch gives the same levels, and its per-level
    phase times are non-negative and add up within the run."""
    ref, it = batch.run(b2.BATCH_PERSISTENT)
    lv, it2, ph = b2.b2sr_msbfs_batch_timed(batch.n, batch.groups, batch.seed_vertex, batch.seed_bit)
    assert it2 == it and torch.equal(lv, ref)
    check_all(batch, lv)
    assert set(ph) == {"product", "product_median_block", "barrier1_wait", "update", "barrier2_wait"}
    for k, v in ph.items():
        assert v.shape == (min(it, 64),) and np.all(v >= 0), k
    assert np.all(ph["product_median_block"] <= ph["product"] + 1e-6)
