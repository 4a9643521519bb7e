"""Batched evaluation of queries whose frozen layers have different widths and depths.

Every query is one ciphertext of the same CKKS context. Layer l of a query with widths
(w_0..w_d) uses the dense layer (l, w_l, w_{l+1}) whose diagonal plaintext bank is shared by all
queries with that shape: all queries use one slot layout (a fixed block stride) and layer l always
runs at the same level, so a bank per (position, w_in, w_out) serves every query. The batch is
evaluated position by position: the ciphertexts at a position are grouped by bank and each group
is one batched dense call; the x^2 of every continuing query is one batched call; replicate is
grouped by the next layer's padded width. With graphs=True each group's dense launch sequence is
captured once into a HIP graph (on static buffers, after the workspace has reached its size and
been frozen) and replayed.

Orchestration only: every arithmetic step runs in the library's kernels.
"""
from __future__ import annotations

import collections
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import CTL_ACT_NONE, Context, Keys, Model


class MixEngine:
    def __init__(self, ctx: Context, keys: Keys, bank: Callable[[int, int, int, int], np.ndarray],
                 t1_of: Dict[int, int], block: int, raw: bool = False, lazy: bool = True,
                 graphs: bool = False, qp: bool = True):
        """bank(pos, w_in, w_out, t) gives the layer's float64 weights [w_out][w_in] (raw=False) or
        its int64 [t][N] encoded diagonal plaintexts (raw=True). lazy / qp: the dense-layer variant
        (single-ModDown giant steps; baby steps over Q*P as well)."""
        self.c, self.keys, self.bank, self.t1_of = ctx, keys, bank, t1_of
        self.block, self.raw, self.lazy, self.graphs, self.qp = block, raw, lazy, graphs, qp
        self.models: Dict[Tuple[int, int, int], Model] = {}
        self._graphs: Dict[Tuple, Tuple] = {}
        self._frozen = False
        import torch
        self.torch = torch

    def level(self, pos: int) -> int:
        return self.c.nq - 2 * pos

    def model(self, pos: int, w_in: int, w_out: int) -> Model:
        key = (pos, w_in, w_out)
        if key not in self.models:
            t = max(w_in, w_out)
            layer = [(w_in, w_out, self.t1_of[t], CTL_ACT_NONE)]
            src = self.bank(pos, w_in, w_out, t)
            kw = dict(lazy=self.lazy, qp=self.qp, block=self.block, k_in=self.level(pos))
            self.models[key] = (self.c.load_model_ex(layer, pts=[src], **kw) if self.raw
                                else self.c.load_model_ex(layer, weights=[src], **kw))
        return self.models[key]

    @staticmethod
    def rotations(queries, t1_of) -> List[int]:
        rots = set()
        for q in queries:
            for l in range(q.depth):
                t = max(q.widths[l], q.widths[l + 1])
                t1 = t1_of[t]
                rots.update(range(1, t1))
                rots.update(k2 * t1 for k2 in range(1, t // t1))
                if l + 1 < q.depth:
                    rots.add(-max(q.widths[l + 1], q.widths[l + 2]))
        return sorted(rots)

    # ------------------------------------------------------------------ graphs
    def freeze(self):
        """Stop workspace growth (call after one eager run of the largest batch)."""
        self.c.workspace_freeze(True)
        self._frozen = True

    def _dense(self, model: Model, x):
        if not self.graphs or not self._frozen:
            return self.c.dense(model, 0, self.keys, x)
        torch = self.torch
        key = (id(model), x.shape[0])
        if key not in self._graphs:
            sin = torch.empty_like(x)
            sout = self.c.empty_ct(x.shape[0], x.shape[2] - 1)
            sin.copy_(x)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self.c.dense(model, 0, self.keys, sin, out=sout)
            self._graphs[key] = (g, sin, sout)
        g, sin, sout = self._graphs[key]
        sin.copy_(x)
        g.replay()
        return sout.clone()

    # ------------------------------------------------------------------ evaluation
    def run(self, cts, queries: Sequence) -> List:
        """cts: [Q][2][n_q][N] top-level ciphertexts (query i in row i). Returns one [2][k][N]
        tensor per query (k = n_q - 2 depth + 1)."""
        torch = self.torch
        Q = len(queries)
        out: List[Optional[object]] = [None] * Q
        cur = {i: None for i in range(Q)}
        rows = cts
        idx_of = {i: i for i in range(Q)}       # row of query i in `rows`
        active = list(range(Q))
        for pos in range(max(q.depth for q in queries)):
            act = [i for i in active if queries[i].depth > pos]
            if not act:
                break
            k = self.level(pos)
            dense_out = {}
            groups = collections.defaultdict(list)
            for i in act:
                groups[(queries[i].widths[pos], queries[i].widths[pos + 1])].append(i)
            for (w_in, w_out), members in sorted(groups.items()):
                sel = torch.tensor([idx_of[i] for i in members], device=rows.device)
                x = rows.index_select(0, sel)[:, :, :k].contiguous()
                y = self._dense(self.model(pos, w_in, w_out), x)
                for r, i in enumerate(members):
                    dense_out[i] = y[r]
            cont = [i for i in act if queries[i].depth > pos + 1]
            for i in act:
                if queries[i].depth == pos + 1:
                    out[i] = dense_out[i]
            if not cont:
                break
            sq_in = torch.stack([dense_out[i] for i in cont])
            sq = self.c.square(self.keys, sq_in)
            sq_row = {i: r for r, i in enumerate(cont)}
            rgroups = collections.defaultdict(list)
            for i in cont:
                rgroups[max(queries[i].widths[pos + 1], queries[i].widths[pos + 2])].append(i)
            nxt = self.c.empty_ct(len(cont), k - 2)
            new_idx = {}
            r0 = 0
            for width, members in sorted(rgroups.items()):
                sel = torch.tensor([sq_row[i] for i in members], device=sq.device)
                rep = self.c.replicate(self.keys, sq.index_select(0, sel).contiguous(), width)
                nxt[r0:r0 + len(members)] = rep
                for r, i in enumerate(members):
                    new_idx[i] = r0 + r
                r0 += len(members)
            rows, idx_of, active = nxt, new_idx, cont
        return out
