"""spmv_bin_full_noalloc (the variant for callers that cannot allocate: its
workspace is the library's per-device scratch array) against spmv_bin_full on
the same inputs: two calls in a row, the second on a smaller matrix, for the
plus-times product (the kind that uses the workspace) with and without column
scaling, and the other semirings, which pass straight through."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as orc
from helpers import EPS32, pack_bits

pytestmark = pytest.mark.gpu
b2 = pytest.importorskip("paper_2201_08560_amd")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def _inputs(g, seed):
    r = gg.rng(seed)
    x = torch.from_numpy(r.random(g.n).astype(np.float32)).cuda()
    s = torch.from_numpy((1.0 / np.maximum(g.degrees(), 1)).astype(np.float32)).cuda()
    mask = torch.from_numpy(pack_bits(r.random(g.n) < 0.3).view(np.int32)).cuda()
    return x, s, mask


@pytest.mark.parametrize("T", (8, 32, 64))
def test_noalloc_equals_workspace_call_twice(T):
    for g, seed in ((gg.rmat(15, 16, seed=15), 1), (gg.er_gnm(2049, 6000, seed=7), 2)):  # the second smaller
        print(f"noalloc {g.name} T={T}", flush=True)
        A = b2.B2SR.from_graph(g, T)
        x, s, mask = _inputs(g, seed)
        for kw in ({}, {"col_scale": s}, {"col_scale": s, "mask": mask, "complement": True, "alpha": 0.85,
                                          "beta": 0.15 / g.n}):
            ref = b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, x, **kw)
            out = torch.full_like(ref, float("nan"))
            b2.spmv_bin_full_noalloc(A, b2.PLUS_TIMES_F32, x, out=out, **kw)
            assert torch.equal(out, ref), kw  # the same kernels in the same order: identical sums
        # the product itself against the oracle (tolerance of an f32 sum of non-negative terms)
        y = b2.spmv_bin_full_noalloc(A, b2.PLUS_TIMES_F32, x).cpu().numpy()
        want = orc.spmv_plus(g, x.cpu().numpy().astype(np.float64))
        assert np.all(np.abs(y - want) <= (g.degrees() + 2) * EPS32 * want + 1e-30)
        # the other semirings need no workspace and pass through
        xd = torch.from_numpy(np.where(gg.rng(seed + 9).random(g.n) < 0.5, 3.0, np.inf).astype(np.float32)).cuda()
        assert torch.equal(b2.spmv_bin_full_noalloc(A, b2.MIN_PLUS_F32, xd, self_loop=True, alpha=1.0),
                           b2.spmv_bin_full(A, b2.MIN_PLUS_F32, xd, self_loop=True, alpha=1.0))
        xu = torch.from_numpy(gg.rng(seed + 5).integers(0, 2**63, g.n, dtype=np.int64)).cuda()
        assert torch.equal(b2.spmv_bin_full_noalloc(A, b2.OR_U64, xu), b2.spmv_bin_full(A, b2.OR_U64, xu))


def test_noalloc_through_the_c_abi():
    """A direct ctypes call, status codes included: too large a workspace is
    refused with B2SR_ENOSPC before anything is launched."""
    g = gg.rmat(12, 8, seed=3)
    A = b2.B2SR.from_graph(g, 16)
    x, s, _ = _inputs(g, 4)
    ref = b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, x, col_scale=s)
    out = torch.empty_like(ref)
    L = b2.lib()
    rc = L.spmv_bin_full_noalloc(A.view, b2.PLUS_TIMES_F32, b2._ptr(x), b2._ptr(s), None, None, 0, 1.0, 0.0,
                                 b2._ptr(out), b2._stream())
    assert rc == 0 and torch.equal(out, ref)
    big = b2.b2sr_matrix(1 << 26, 64, 1 << 31, 0, 0x1000, 0x1000, 0x1000)  # partials of 4 GiB
    assert L.spmv_bin_full_noalloc(ctypes.byref(big), b2.PLUS_TIMES_F32, ctypes.c_void_p(0x1000), None, None, None,
                                   0, 1.0, 0.0, ctypes.c_void_p(0x2000), None) == -3
