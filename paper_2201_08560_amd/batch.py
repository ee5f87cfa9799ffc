"""Batched multi-source BFS over many graphs: host-side layout only.

Graphs are placed one after another in a shared vertex space, each starting at
a multiple of 64 so no 64-bit frontier word or 32-bit bit-vector word spans two
graphs.  Graphs that use the same tile width form one group: a block-diagonal
B2SR matrix over the whole space, built on the device by b2sr_from_csr.  The
BFS itself runs in libb2sr.so (b2sr_msbfs_batch or a MsbfsPlan).
"""
from __future__ import annotations

import numpy as np
import torch

from . import B2SR, BATCH_LEVELS, MsbfsPlan, as_u32, b2sr_msbfs_batch

ALIGN = 64


class GraphBatch:
    def __init__(self, graphs, tiles):
        if len(graphs) != len(tiles):
            raise ValueError("one tile width per graph")
        self.graphs = list(graphs)
        self.tiles = [int(t) for t in tiles]
        sizes = np.array([(g.n + ALIGN - 1) // ALIGN * ALIGN for g in self.graphs], dtype=np.int64)
        self.offsets = np.zeros(len(graphs) + 1, dtype=np.int64)
        np.cumsum(sizes, out=self.offsets[1:])
        self.n = int(self.offsets[-1])
        if self.n >= 2**32 - 256:
            raise ValueError("vertex space exceeds 32 bits")
        self.groups = []
        self.group_tiles = sorted(set(self.tiles))
        for T in self.group_tiles:
            members = [i for i, t in enumerate(self.tiles) if t == T]
            counts = np.zeros(self.n, dtype=np.int64)
            cols = []
            for i in members:
                g, off = self.graphs[i], int(self.offsets[i])
                counts[off:off + g.n] = g.degrees()
                cols.append(g.colind.astype(np.int64) + off)
            rowptr = np.zeros(self.n + 1, dtype=np.int64)
            np.cumsum(counts, out=rowptr[1:])
            colind = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64)
            self.groups.append(B2SR.from_csr(rowptr.astype(np.uint32), colind.astype(np.uint32), self.n, T))
        self.sources = None
        self.seed_vertex = self.seed_bit = None

    def set_sources(self, sources):
        """sources[i]: up to 64 distinct vertex ids of graph i (bit s = position s)."""
        sv, sb = [], []
        for i, src in enumerate(sources):
            src = np.asarray(src, dtype=np.int64)
            if src.size > 64:
                raise ValueError("at most 64 sources per graph")
            sv.append(src + int(self.offsets[i]))
            sb.append(np.arange(src.size, dtype=np.int64))
        self.sources = [np.asarray(s, dtype=np.uint32) for s in sources]
        vert = np.concatenate(sv).astype(np.uint32)
        bit = np.concatenate(sb).astype(np.uint32)
        if self.seed_vertex is not None and self.seed_vertex.numel() == vert.size:
            # rewrite in place so existing plans see the new sources
            self.seed_vertex.copy_(torch.from_numpy(vert.view(np.int32)))
            self.seed_bit.copy_(torch.from_numpy(bit.view(np.int32)))
        else:
            self.seed_vertex = torch.from_numpy(vert.view(np.int32)).cuda()
            self.seed_bit = torch.from_numpy(bit.view(np.int32)).cuda()

    def run(self, mode=BATCH_LEVELS, out=None, ws=None):
        return b2sr_msbfs_batch(self.n, self.groups, self.seed_vertex, self.seed_bit, mode, out, ws)

    def plan(self, mode=BATCH_LEVELS, out=None, ws=None) -> MsbfsPlan:
        return MsbfsPlan(self.n, self.groups, self.seed_vertex, self.seed_bit, mode, out, ws)

    def levels_of(self, levels: torch.Tensor, i: int) -> torch.Tensor:
        """Levels of graph i as a (nsrc, n_i) device tensor, the layout of b2sr_msbfs."""
        off, n = int(self.offsets[i]), self.graphs[i].n
        k = self.sources[i].size
        return levels[off:off + n, :k].t()

    def levels_of_host(self, levels: torch.Tensor, i: int) -> np.ndarray:
        return as_u32(self.levels_of(levels, i).contiguous())
