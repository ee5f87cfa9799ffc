"""C-ABI checks that need no GPU: the library loads, exports every function
include/b2sr.h declares, and rejects bad arguments on the host before any
launch."""
import ctypes
import os
import subprocess

import pytest

import paper_2201_08560_amd as b2

L = b2.lib()
FAKE = 0x1000  # never dereferenced: every call below fails host validation first


def mat(n=64, tile=8, ntiles=4, rp=FAKE, ci=FAKE, bits=FAKE, chunk_blocks=0):
    return b2.b2sr_matrix(n, tile, ntiles, chunk_blocks, rp, ci, bits)


def test_every_declared_function_is_exported():
    names = b2.header_functions()
    assert {"b2sr_from_csr", "spmv_bin_bin", "spmv_bin_full", "spgemm_masked"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", b2.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {line.split()[-1] for line in out.stdout.splitlines() if " T " in line}
    missing = [f for f in names if f not in exported]
    assert not missing, missing
    for f in names:
        assert hasattr(L, f)


def test_strerror_and_version():
    assert b2.b2sr_strerror(0) == "success"
    assert "invalid" in b2.b2sr_strerror(-1)
    assert "workspace" in b2.b2sr_strerror(-3)
    assert b2.b2sr_strerror(-99) == "unknown status"
    assert L.b2sr_version() >= 100


def test_matrix_validation():
    S = None
    x = ctypes.c_void_p(FAKE)
    assert L.spmv_bin_bin(None, x, None, 0, x, S) == -1
    for bad in (mat(tile=6), mat(tile=128), mat(chunk_blocks=65), mat(rp=0), mat(ci=0), mat(bits=0),
                mat(tile=32, bits=FAKE + 4), mat(tile=64, bits=FAKE + 8), mat(ntiles=10**6, n=64, tile=32)):
        assert L.spmv_bin_bin(ctypes.byref(bad), x, None, 0, x, S) == -1
    assert L.spmv_bin_bin(ctypes.byref(mat(n=0xFFFFFFF0)), x, None, 0, x, S) == -2


def test_spmv_argument_errors():
    A = ctypes.byref(mat())
    x = ctypes.c_void_p(FAKE)
    y = ctypes.c_void_p(FAKE + 4096)
    assert L.spmv_bin_bin(A, None, None, 0, y, None) == -1                 # x NULL
    assert L.spmv_bin_bin(A, x, None, 0, None, None) == -1                 # y NULL
    assert L.spmv_bin_bin(A, x, None, 0x100, y, None) == -1                # unknown flag
    assert L.spmv_bin_full(A, 1, ctypes.c_void_p(FAKE + 4), None, None, None, 0, 1.0, 0.0, y, None, 0, None) == -1  # x misaligned
    assert L.spmv_bin_bin(A, x, None, 0, x, None) == -1                    # y aliases x
    assert L.spmv_bin_full(A, 9, x, None, None, None, 0, 1.0, 0.0, y, None, 0, None) == -5   # unknown semiring
    assert L.spmv_bin_full(A, 1, x, None, None, None, b2.SELF, 1.0, 0.0, y, None, 0, None) == -1  # SELF on plus
    assert L.spmv_bin_full(A, 3, x, None, None, None, 0, 1.5, 0.0, y, None, 0, None) == -1   # non-integral u32 weight
    assert L.spmv_bin_full(A, 3, x, ctypes.c_void_p(FAKE), None, None, 0, 1.0, 0.0, y, None, 0, None) == -1  # scale on min
    need = L.spmv_bin_full_workspace_bytes(A, 1)
    assert need > 0
    assert L.spmv_bin_full(A, 1, x, None, None, None, 0, 1.0, 0.0, y, None, 0, None) == -3   # no workspace
    base = need - 4 * 64                     # without col_scale the scaled copy of x is not needed
    assert base > 0
    assert L.spmv_bin_full(A, 1, x, None, None, None, 0, 1.0, 0.0, y, x, base - 1, None) == -3
    s = ctypes.c_void_p(FAKE + 8192)
    assert L.spmv_bin_full(A, 1, x, s, None, None, 0, 1.0, 0.0, y, x, need - 1, None) == -3
    assert L.spmv_bin_full(A, 1, x, s, None, None, 0, 1.0, 0.0, y, ctypes.c_void_p(FAKE + 8), need, None) == -1  # ws misaligned
    assert L.spmv_bin_full_workspace_bytes(A, 2) == 0
    assert L.spmv_bin_full(A, 2, x, None, y, None, 0, 1.0, 0.0, y, None, 0, None) == -1   # x_active aliases y


def test_spgemm_and_build_argument_errors():
    A = ctypes.byref(mat())
    B16 = ctypes.byref(mat(tile=16))
    Bn = ctypes.byref(mat(n=65))
    s = ctypes.c_void_p(FAKE)
    assert L.spgemm_masked(A, B16, None, 0, s, None, 0, None) == -1     # tile mismatch
    assert L.spgemm_masked(A, Bn, None, 0, s, None, 0, None) == -1      # n mismatch
    assert L.spgemm_masked(A, A, A, 0, None, None, 0, None) == -1       # no output
    assert L.spgemm_masked(A, A, A, 0x8, s, None, 0, None) == -1        # unknown flag
    assert L.spgemm_masked_workspace_bytes(A, A) >= 4 * 8 * 8       # orientation lists (optional)
    assert L.spgemm_masked_workspace_bytes(A, None) == 2 * 8 * 8 * 4
    assert L.spgemm_masked(A, A, None, 0, s, None, 0, None) == -3       # unmasked needs workspace
    assert L.spgemm_masked_rows(A, A, None, 0, 8, 0, s, None) == -1      # mask required
    assert L.spgemm_masked_rows(A, A, A, 3, 2, 0, s, None) == -1         # begin > end
    assert L.spgemm_masked_rows(A, A, A, 0, 9, 0, s, None) == -1         # end past the 8 tile-rows
    assert L.spgemm_masked_rows(A, B16, A, 0, 8, 0, s, None) == -1       # tile mismatch
    assert L.spgemm_masked_rows(A, A, A, 0, 8, 0, None, None) == -1      # no output
    nt = ctypes.c_uint64(0)
    p = ctypes.c_void_p(FAKE)
    assert L.b2sr_count_tiles(10, 5, p, p, 5, 0, p, ctypes.byref(nt), None) == -1       # tile 5
    assert L.b2sr_count_tiles(10, 5, p, p, 8, 2, p, ctypes.byref(nt), None) == -1       # unknown flag
    assert L.b2sr_count_tiles(10, 1 << 32, p, p, 8, 0, p, ctypes.byref(nt), None) == -2  # nnz too large
    assert L.b2sr_count_tiles(10, 5, None, p, 8, 0, p, ctypes.byref(nt), None) == -1
    assert L.b2sr_from_csr(10, 5, p, p, 8, 0, p, 1 << 32, p, p, None) == -2
    assert L.b2sr_from_csr(10, 5, p, p, 8, 0, p, 3, p, ctypes.c_void_p(FAKE + 2), None) == -1
    assert L.b2sr_pack_bits(10, None, p, None) == -1


def test_algorithm_argument_errors():
    A = ctypes.byref(mat())
    need = L.b2sr_algo_workspace_bytes(A, b2.ALGO_BFS)
    assert need > 0
    for algo in (b2.ALGO_BFS, b2.ALGO_SSSP, b2.ALGO_CC, b2.ALGO_PAGERANK, b2.ALGO_MSBFS, b2.ALGO_MIS, b2.ALGO_COLOR):
        assert L.b2sr_algo_workspace_bytes(A, algo) > 0
    assert L.b2sr_algo_workspace_bytes(A, 99) == 0
    p = ctypes.c_void_p(FAKE)
    it = ctypes.c_uint32(0)
    assert L.b2sr_bfs(A, 0, p, None, 0, ctypes.byref(it), None) == -3             # no workspace
    assert L.b2sr_bfs(A, 0, p, p, need - 1, ctypes.byref(it), None) == -3
    assert L.b2sr_bfs(A, 64, p, p, need, ctypes.byref(it), None) == -1            # src >= n
    wsm = L.b2sr_algo_workspace_bytes(A, b2.ALGO_MSBFS)
    srcs = (ctypes.c_uint32 * 3)(1, 2, 1)
    assert L.b2sr_msbfs(A, srcs, 3, p, p, wsm, ctypes.byref(it), None) == -1      # repeated source
    srcs65 = (ctypes.c_uint32 * 65)(*range(65))
    assert L.b2sr_msbfs(A, srcs65, 65, p, p, wsm, ctypes.byref(it), None) == -1   # > 64 sources
    wpr = L.b2sr_algo_workspace_bytes(A, b2.ALGO_PAGERANK)
    assert L.b2sr_pagerank(A, ctypes.c_float(1.5), 3, p, p, wpr, None) == -1      # damping > 1


def test_library_has_no_cpu_fallback_symbols():
    """The product library links the HIP runtime and nothing from the oracle."""
    out = subprocess.run(["nm", "-D", b2.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "orc_" not in out
    ldd = subprocess.run(["ldd", b2.LIB_PATH], capture_output=True, text=True).stdout
    assert "amdhip64" in ldd and "oracle" not in ldd


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(b2, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b2, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        b2.lib()


def test_batch_argument_errors():
    A = mat()
    groups = (b2.b2sr_matrix * 2)(A, A)
    p = ctypes.c_void_p(FAKE)
    it = ctypes.c_uint32(0)
    need = L.b2sr_msbfs_batch_workspace_bytes(64)
    assert need >= 3 * 64 * 8
    assert L.b2sr_msbfs_batch(64, 0, groups, 1, p, p, p, 0, p, need, ctypes.byref(it), None) == -1   # no groups
    assert L.b2sr_msbfs_batch(64, 9, groups, 1, p, p, p, 0, p, need, ctypes.byref(it), None) == -1   # > 8 groups
    assert L.b2sr_msbfs_batch(64, 2, groups, 1, p, p, p, 7, p, need, ctypes.byref(it), None) == -1   # bad mode
    assert L.b2sr_msbfs_batch(64, 2, groups, 1, p, p, p, 0, p, need - 1, ctypes.byref(it), None) == -3
    assert L.b2sr_msbfs_batch(65, 2, groups, 1, p, p, p, 0, p, 1 << 20, ctypes.byref(it), None) == -1  # n mismatch
    assert L.b2sr_msbfs_batch(64, 2, groups, 1, None, p, p, 0, p, need, ctypes.byref(it), None) == -1  # no seeds
    bad = (b2.b2sr_matrix * 1)(mat(tile=5))
    assert L.b2sr_msbfs_batch(64, 1, bad, 1, p, p, p, 0, p, need, ctypes.byref(it), None) == -1
    h = ctypes.c_void_p(0)
    assert L.b2sr_msbfs_batch_plan_create(64, 2, groups, 1, p, p, p, 0, p, need, None) == -1
    assert L.b2sr_msbfs_batch_plan_create(64, 0, groups, 1, p, p, p, 0, p, need, ctypes.byref(h)) == -1
    assert L.b2sr_msbfs_batch_plan_create(64, 2, groups, 1, p, p, p, 7, p, need, ctypes.byref(h)) == -1  # bad mode
    assert h.value is None
    assert L.b2sr_msbfs_batch_plan_launch(None, None, None) == -1
    assert L.b2sr_msbfs_batch_plan_destroy(None) == 0


def test_sampling_profile_closed_form():
    """One nonzero per row: every sampled row touches one chunk, so the estimate is
    (w + (4 + (k-1) w) / k) / 8 for each tile width k (the reading of Algorithm 1)."""
    import graphgen as gg
    from paper_2201_08560_amd import autotune
    g = gg.path(2)  # rows {1}, {0}
    est = autotune.sampling_profile(g.rowptr, g.colind, g.n, nsample=2)
    for k, w in ((4, 1), (8, 1), (16, 2), (32, 4)):
        assert est[k] == pytest.approx((w + (4 + (k - 1) * w) / k) / 8.0)
    m = gg.cycle(1000)
    est = autotune.sampling_profile(m.rowptr, m.colind, m.n, nsample=500, seed=3)
    assert est[32] < est[4] * 8  # monotone sanity: wider tiles share chunks between neighbours


def test_session_argument_errors():
    """Serving sessions reject bad handles and sizes on the host."""
    n = 1000
    need = L.b2sr_bfs_session_bytes(n)
    assert need >= n * (3 * 8 + 64 * 4)
    assert L.b2sr_bfs_session_bytes(2 * n) > need
    A = mat(n=n, tile=8)
    h = ctypes.c_void_p(0)
    assert L.b2sr_bfs_session_create(ctypes.byref(A), None, need, None, None) == -1       # no handle out
    assert L.b2sr_bfs_session_create(ctypes.byref(A), None, need, None, ctypes.byref(h)) == -3   # no workspace
    assert L.b2sr_bfs_session_create(ctypes.byref(A), FAKE, need - 1, None, ctypes.byref(h)) == -3
    bad = mat(n=n, tile=5)
    assert L.b2sr_bfs_session_create(ctypes.byref(bad), FAKE, need, None, ctypes.byref(h)) == -1
    assert h.value is None
    assert L.b2sr_bfs_session_join(None, 0, 0, None) == -1
    assert L.b2sr_bfs_session_step(None, None, None) == -1
    assert L.b2sr_bfs_session_extract(None, 0, None, None) == -1
    assert L.b2sr_bfs_session_info(None, None, None) == -1
    assert L.b2sr_bfs_session_destroy(None) == 0


def test_transpose_argument_errors():
    need = L.b2sr_csr_transpose_workspace_bytes(100)
    assert need >= 400
    p = FAKE
    assert L.b2sr_csr_transpose(100, 10, None, p, p, p, p, need, None) == -1
    assert L.b2sr_csr_transpose(100, 10, p, None, p, p, p, need, None) == -1
    assert L.b2sr_csr_transpose(100, 10, p, p, p, None, p, need, None) == -1
    assert L.b2sr_csr_transpose(100, 10, p, p, p, p, None, need, None) == -3
    assert L.b2sr_csr_transpose(100, 10, p, p, p, p, p, need - 1, None) == -3
    assert L.b2sr_csr_transpose(100, 1 << 32, p, p, p, p, p, need, None) == -2
    A = mat(n=64, tile=5)
    assert L.b2sr_pagerank_directed(ctypes.byref(A), 0.85, 1, p, p, 1 << 20, None) == -1


def test_mis_color_argument_errors():
    A = mat(n=64, tile=8)
    need = L.b2sr_algo_workspace_bytes(ctypes.byref(A), 6)
    assert need >= 64 * 16 and L.b2sr_algo_workspace_bytes(ctypes.byref(A), 7) == need
    p = FAKE
    assert L.b2sr_mis(ctypes.byref(A), None, p, p, need, None, None) == -1
    assert L.b2sr_mis(ctypes.byref(A), p, None, p, need, None, None) == -1
    assert L.b2sr_mis(ctypes.byref(A), p, p, None, need, None, None) == -3
    assert L.b2sr_color(ctypes.byref(A), p, None, p, need, None, None) == -1
    assert L.b2sr_color(ctypes.byref(A), p, p, p, need - 1, None, None) == -3


def test_stream_read_argument_errors():
    assert L.b2sr_stream_read(None, 64, FAKE, None) == -1
    assert L.b2sr_stream_read(FAKE, 64, None, None) == -1
    assert L.b2sr_stream_read(FAKE + 4, 64, FAKE, None) == -1   # not 16-byte aligned
    assert L.b2sr_stream_read(FAKE, 8, FAKE, None) == 0         # under one vector: nothing to read


def test_eccentricity_argument_errors():
    A = mat(n=64, tile=8)
    need = L.b2sr_algo_workspace_bytes(ctypes.byref(A), 8)
    assert need >= 3 * 64 * 8
    srcs = (ctypes.c_uint32 * 2)(0, 64)   # 64 is out of range
    ecc = (ctypes.c_uint32 * 2)()
    assert L.b2sr_eccentricity(ctypes.byref(A), srcs, 2, ecc, FAKE, need, None) == -1
    assert L.b2sr_eccentricity(ctypes.byref(A), None, 2, ecc, FAKE, need, None) == -1
    assert L.b2sr_eccentricity(ctypes.byref(A), srcs, 1, ecc, None, need, None) == -3
    assert L.b2sr_diameter(ctypes.byref(A), None, FAKE, need, None) == -1


def test_lgc_argument_errors():
    A = mat(n=64, tile=8)
    need = L.b2sr_algo_workspace_bytes(ctypes.byref(A), b2.ALGO_LGC)
    assert need >= 64 * (6 * 4 + 2 * 8)          # keys, ids (twice), rank, degrees; volumes and cuts
    p = FAKE
    f = ctypes.c_float
    assert L.b2sr_lgc(ctypes.byref(A), 64, f(0.85), 5, p, p, p, p, need, None) == -1     # seed >= n
    assert L.b2sr_lgc(ctypes.byref(A), 0, f(1.5), 5, p, p, p, p, need, None) == -1       # alpha > 1
    assert L.b2sr_lgc(ctypes.byref(A), 0, f(0.85), 5, None, p, p, p, need, None) == -1   # no ppr output
    assert L.b2sr_lgc(ctypes.byref(A), 0, f(0.85), 5, p, p, None, p, need, None) == -1   # no stats
    assert L.b2sr_lgc(ctypes.byref(A), 0, f(0.85), 5, p, p, p, p, need - 1, None) == -3
    assert L.b2sr_sweep_cut(ctypes.byref(A), None, p, p, p, p, need, None) == -1         # no score
    assert L.b2sr_sweep_cut(ctypes.byref(A), p, p, p, None, p, need, None) == -1         # no stats
    assert L.b2sr_sweep_cut(ctypes.byref(A), p, p, p, p, None, need, None) == -3
