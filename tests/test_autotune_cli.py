"""The Algorithm 1 sampling profile from the command line (no GPU needed)."""
import json

import numpy as np

import graphgen as gg
from paper_2201_08560_amd import autotune


def test_cli_sampling_profile(capsys, tmp_path):
    assert autotune.main(["er:2000:8000:3", "--no-exact", "--sample", "256"]) == 0
    out = json.loads(capsys.readouterr().out)
    assert out["n"] == 2000 and out["nnz"] == 16000
    est = out["sampling_estimate_b2sr_over_csr"]
    assert set(est) == {"4", "8", "16", "32", "64"} and all(v > 0 for v in est.values())
    g = gg.king_grid(20, 30)
    f = tmp_path / "king.npz"
    np.savez(f, n=g.n, rowptr=g.rowptr, colind=g.colind)
    assert autotune.main([str(f), "--no-exact"]) == 0
    assert json.loads(capsys.readouterr().out)["nnz"] == g.nnz


def test_cli_rejects_unknown_spec():
    import pytest
    with pytest.raises(ValueError):
        autotune.main(["torus:3", "--no-exact"])


def test_prune_keeps_the_widths_near_the_best_estimate():
    from paper_2201_08560_amd import autotune
    est = {4: 0.50, 8: 0.30, 16: 0.31, 32: 0.40, 64: 0.70}
    assert autotune.prune(est) == [8, 16, 32]                 # within 1.5x of 0.30
    assert autotune.prune(est, slack=1.1) == [8, 16]
    assert autotune.prune(est, keep=1) == [8]
    assert autotune.prune({k: 0.0 for k in autotune.TILES}) == list(autotune.TILES)  # nothing sampled
