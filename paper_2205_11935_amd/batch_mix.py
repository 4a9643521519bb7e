"""Batched evaluation of queries whose frozen layers have different widths and depths.

Every query is one ciphertext of the same CKKS context. Layer l of a query with widths
(w_0..w_d) uses the dense layer (l, w_l, w_{l+1}) whose diagonal plaintext bank is shared by all
queries with that shape: all queries use one slot layout (a fixed block stride) and layer l always
runs at the same level, so a bank per (position, w_in, w_out) serves every query. The batch is
evaluated position by position: the ciphertexts at a position are ordered by bank and every bank's
dense layer runs in one ctl_dense_groups call (one ModUp of every ciphertext, the giant steps'
ModUp, ModDown and rescale shared by all widths; key products and plaintext products per bank);
the x^2 of every continuing query is one batched call; replicate is grouped by the next layer's
padded width. With graphs=True the whole chain of a position (dense groups, x^2, replicates) is
captured once per shape signature into a HIP graph (on static buffers, after the workspace has
reached its size and been frozen) and replayed.

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

    def _chain(self, pos: int, models, counts, sq_rows, rep_widths):
        """The work of one position on its input x ([n][2][k][N], rows in group order): every
        group's dense layer in one ctl_dense_groups call, then x^2 of the rows that continue (in
        the order of their next layer's width) and one replicate per width. Returns a function
        x -> (dense output [n][2][k-1][N], next input [m][2][k-2][N] or None)."""
        torch = self.torch
        k = self.level(pos)
        sel = torch.tensor(sq_rows, dtype=torch.int64, device="cuda:%d" % self.c.device) if sq_rows else None

        def dense(x):
            if self.qp:
                return self.c.dense_groups(models, counts, self.keys, x)
            y = self.c.empty_ct(x.shape[0], k - 1)          # other variants: one call per bank
            r0 = 0
            for m, cnt in zip(models, counts):
                self.c.dense(m, 0, self.keys, x[r0:r0 + cnt], out=y[r0:r0 + cnt])
                r0 += cnt
            return y

        def chain(x):
            y = dense(x)
            if sel is None:
                return y, None
            sq = self.c.square(self.keys, y.index_select(0, sel))
            nxt = self.c.empty_ct(len(sq_rows), k - 2)
            r0 = 0
            for width, cnt in rep_widths:
                self.c.replicate(self.keys, sq[r0:r0 + cnt], width, out=nxt[r0:r0 + cnt])
                r0 += cnt
            return y, nxt
        # a captured graph's index_select reads `sel` at every replay: whoever keeps the graph must
        # keep this tensor alive with it
        chain.index = sel
        return chain

    def _run_position(self, pos: int, models, counts, sq_rows, rep_widths, x):
        if not self.graphs or not self._frozen:
            return self._chain(pos, models, counts, sq_rows, rep_widths)(x)
        torch = self.torch
        key = (pos, tuple(id(m) for m in models), tuple(counts), tuple(sq_rows), tuple(rep_widths))
        if key not in self._graphs:
            chain = self._chain(pos, models, counts, sq_rows, rep_widths)
            sin = torch.empty_like(x)
            sin.copy_(x)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                y, nxt = chain(sin)
            # the chain (and its index tensor, read by the graph's gather at every replay) lives
            # as long as the graph
            self._graphs[key] = (g, sin, y, nxt, chain)
        g, sin, y, nxt, _ = self._graphs[key]
        sin.copy_(x)
        g.replay()
        return y.clone(), (nxt.clone() if nxt is not None else None)

    # ------------------------------------------------------------------ evaluation
    def run(self, cts, queries: Sequence, done_events: Optional[List] = None) -> List:
        """cts: [Q][2][n_q][N] top-level ciphertexts (query i in row i). Returns one [2][k][N]
        tensor per query (k = n_q - 2 depth + 1). With done_events (a list of Q entries), entry i
        receives a CUDA event recorded on the current stream once query i's last layer is done."""
        torch = self.torch
        Q = len(queries)
        out: List[Optional[object]] = [None] * Q
        rows = cts
        idx_of = {i: i for i in range(Q)}       # row of query i in `rows`
        active = list(range(Q))
        for pos in range(max(q.depth for q in queries)):
            act = [i for i in active if queries[i].depth > pos]
            if not act:
                break
            k = self.level(pos)
            groups = collections.defaultdict(list)
            for i in act:
                groups[(queries[i].widths[pos], queries[i].widths[pos + 1])].append(i)
            shapes = sorted(groups)
            order = [i for sh in shapes for i in groups[sh]]                  # rows in group order
            models = [self.model(pos, w_in, w_out) for (w_in, w_out) in shapes]
            counts = [len(groups[sh]) for sh in shapes]
            rgroups = collections.defaultdict(list)
            for i in order:
                if queries[i].depth > pos + 1:
                    rgroups[max(queries[i].widths[pos + 1], queries[i].widths[pos + 2])].append(i)
            widths = sorted(rgroups)
            rorder = [i for wd in widths for i in rgroups[wd]]               # continuing, by next width
            at = {i: r for r, i in enumerate(order)}
            sel = torch.tensor([idx_of[i] for i in order], device=rows.device)
            x = rows.index_select(0, sel)[:, :, :k].contiguous()
            y, nxt = self._run_position(pos, models, counts, [at[i] for i in rorder],
                                        [(wd, len(rgroups[wd])) for wd in widths], x)
            finished = [i for i in order if queries[i].depth == pos + 1]
            if done_events is not None and finished:
                ev = torch.cuda.Event(enable_timing=True)
                ev.record()
                for i in finished:
                    done_events[i] = ev
            for i in finished:
                out[i] = y[at[i]]
            if not rorder:
                break
            rows, idx_of, active = nxt, {i: r for r, i in enumerate(rorder)}, rorder
        return out
