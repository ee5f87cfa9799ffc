"""The measured autotuner and the work split it sets: every split gives the
same products (bit, count and min results bit-exact; float sums within the
oracle's tolerance), and tune() returns the argmin of the times it records."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as orc
from helpers import EPS32, TILES, pack_bits, unpack_bits

pytestmark = pytest.mark.gpu
b2 = pytest.importorskip("paper_2201_08560_amd")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2201_08560_amd import autotune  # noqa: E402

GRAPHS = [gg.rmat(13, 16, seed=13), gg.star(20000), gg.er_gnm(4099, 12000, seed=2)]


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_products_under_every_split(gi, T):
    g = GRAPHS[gi]
    r = gg.rng(40 + gi)
    x = r.random(g.n) < 0.3
    xf = r.random(g.n).astype(np.float32)
    xu = np.where(r.random(g.n) < 0.5, r.integers(0, 50, g.n), 0xFFFFFFFF).astype(np.uint32)
    mask = r.random(g.n) < 0.2
    want_or = orc.spmv_or(g, x, mask, True)
    want_cnt = orc.spmv_count(g, x)
    want_plus = orc.spmv_plus(g, xf.astype(np.float64))
    bound = (g.degrees() + 2) * EPS32 * want_plus + 1e-30
    xb = torch.from_numpy(pack_bits(x).view(np.int32)).cuda()
    mb = torch.from_numpy(pack_bits(mask).view(np.int32)).cuda()
    xft = torch.from_numpy(xf).cuda()
    xut = torch.from_numpy(xu.view(np.int32)).cuda()
    A0 = b2.B2SR.from_graph(g, T)
    ref_min = b2.as_u32(b2.spmv_bin_full(A0, b2.MIN_PLUS_U32, xut, self_loop=True, alpha=1.0))
    for k in (1, 3, 64):
        print(f"split {g.name} T={T} chunk_blocks={k}", flush=True)
        A = A0.with_split(k)
        assert np.array_equal(unpack_bits(b2.as_u32(b2.spmv_bin_bin(A, xb, mb, complement=True)), g.n), want_or)
        assert np.array_equal(b2.as_u32(b2.spmv_bin_bin(A, xb, count=True)), want_cnt)
        y = b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, xft).cpu().numpy()
        assert np.all(np.abs(y - want_plus) <= bound)
        assert np.array_equal(b2.as_u32(b2.spmv_bin_full(A, b2.MIN_PLUS_U32, xut, self_loop=True, alpha=1.0)), ref_min)


def test_tune_returns_the_measured_argmin():
    g = gg.rmat(13, 16, seed=13)
    T, k, rep = autotune.tune(g, reps=3)
    times = rep["times_ms"]
    assert set(times) == {f"T{t}/k{s}" for t in rep["candidates"] for s in rep["splits"]}
    assert set(rep["candidates"]) <= set(autotune.TILES)
    best = min(times, key=lambda key: times[key])
    assert times[f"T{T}/k{k}"] == times[best]
    assert rep["choice"] == {"tile": T, "chunk_blocks": k}
    # the chosen matrix computes the same product as the default split
    A = b2.B2SR.from_graph(g, T)
    ones = torch.full(((g.n + 31) // 32,), -1, dtype=torch.int32, device="cuda")
    assert torch.equal(b2.spmv_bin_bin(A.with_split(k), ones), b2.spmv_bin_bin(A, ones))
