"""Serving loop for encrypted queries: continuous batching over several CKKS parameter sets on one GPU.

The setting is the paper's MLaaS one (Section 1 and the Classify protocol of Section 3): clients
upload CKKS ciphertexts, the server evaluates its frozen layers (ClassifyHE) and returns encrypted
results. Each client's evaluation keys and every admitted ciphertext stay resident in HBM.

* Admission by memory. Each parameter set owns a pool of ciphertext slots (input and output
  residues of one query) sized from a byte budget; a query is admitted when a slot is free and its
  client's evaluation keys are resident or can be made resident inside the key budget. Keys are
  kept in LRU order and only clients with no admitted or running query can be evicted. Queries
  that cannot be admitted wait in arrival order; beyond `max_pending` waiting queries a new one is
  rejected.
* Continuous batching. A parameter set has one or more lanes, each a library context with its own
  stream and workspace (keys and plaintext banks are shared between the lanes). Whenever a lane
  is idle it takes the oldest admitted queries of its parameter set (up to `max_batch`), whatever
  their clients, groups them by client and launches one batched forward pass
  (ctl_forward_multi: key products per client run, everything else over the whole batch). With
  `mix_clients=False` a batch holds one client's queries only (the client whose oldest admitted
  query arrived first). Queries that arrive while other batches run are admitted into free slots
  at once and join the next batch; the lanes of both parameter sets run concurrently on their own
  streams, so their work overlaps on the device.
* Every arithmetic step runs in the library; this module only schedules, copies ciphertexts
  between slots and batch buffers, and records times.

`KeyCache` and `Scheduler` are host logic with no device dependency; `GpuServer` runs them on the
GPU through the library.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import math
import time
from typing import Callable, Deque, Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    client: int
    pset: str
    ct: object = None                 # the uploaded ciphertext [2][k_in][N] (device tensor)
    t_arrive: float = math.nan
    t_admit: float = math.nan
    t_launch: float = math.nan
    t_done: float = math.nan
    status: str = "new"               # new | pending | admitted | running | done | rejected
    slot: int = -1
    batch: int = -1
    out: object = None                # result [2][k_out][N], filled when `keep_outputs` is set

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


# ----------------------------------------------------------------------------------------- keys
class KeyCache:
    """LRU residency of per-client evaluation keys under a device byte budget.

    load(client) -> (handle, nbytes) makes a client's keys resident; unload(handle) frees them.
    acquire(client) pins the client's keys (one pin per admitted query) and returns False when they
    cannot be made resident without evicting a pinned client."""

    def __init__(self, budget: int, size_of: Callable[[int], int], load: Callable[[int], Tuple[object, int]],
                 unload: Callable[[object], None]):
        self.budget, self.size_of, self._load, self._unload = budget, size_of, load, unload
        self._res: "collections.OrderedDict[int, Tuple[object, int]]" = collections.OrderedDict()
        self._pins: Dict[int, int] = collections.Counter()
        self.loads = self.evictions = 0

    @property
    def used(self) -> int:
        return sum(b for _, b in self._res.values())

    def resident(self) -> List[int]:
        return list(self._res)

    def handle(self, client: int):
        return self._res[client][0]

    def acquire(self, client: int) -> bool:
        if client in self._res:
            self._res.move_to_end(client)
            self._pins[client] += 1
            return True
        need = self.size_of(client)
        if need > self.budget:
            raise ValueError("client %d needs %d key bytes, more than the whole budget %d" % (client, need, self.budget))
        free = self.budget - self.used
        victims = []
        for c, (_, b) in self._res.items():          # least recently used first
            if free >= need:
                break
            if self._pins[c] == 0:
                victims.append(c)
                free += b
        if free < need:
            return False
        for c in victims:
            h, _ = self._res.pop(c)
            self._unload(h)
            self.evictions += 1
        h, nbytes = self._load(client)
        self._res[client] = (h, nbytes)
        self._pins[client] += 1
        self.loads += 1
        return True

    def release(self, client: int):
        if self._pins[client] <= 0:
            raise RuntimeError("release of client %d without a pin" % client)
        self._pins[client] -= 1

    def clear(self):
        for h, _ in self._res.values():
            self._unload(h)
        self._res.clear()


# ------------------------------------------------------------------------------------ scheduling
@dataclasses.dataclass
class PsetConfig:
    name: str
    slots: int          # ciphertext slots (admitted + running queries) of this parameter set
    max_batch: int
    lanes: int = 2


class Scheduler:
    """Admission, batch formation and completion bookkeeping (no device work)."""

    def __init__(self, configs: Sequence[PsetConfig], keys: KeyCache, max_pending: int = 1 << 20,
                 mix_clients: bool = True):
        self.cfg = {c.name: c for c in configs}
        self.keys = keys
        self.max_pending = max_pending
        self.mix_clients = mix_clients
        self.pending: Dict[str, Deque[Request]] = {c.name: collections.deque() for c in configs}
        self.admitted: Dict[str, "collections.OrderedDict[int, Deque[Request]]"] = {
            c.name: collections.OrderedDict() for c in configs}
        self.free_slots: Dict[str, List[int]] = {c.name: list(range(c.slots - 1, -1, -1)) for c in configs}
        self.rejected = 0
        self._batch_id = 0

    def arrive(self, r: Request, now: float) -> bool:
        if r.pset not in self.cfg:
            raise ValueError("unknown parameter set %r" % r.pset)
        r.t_arrive = now if math.isnan(r.t_arrive) else r.t_arrive
        if sum(len(q) for q in self.pending.values()) >= self.max_pending:
            r.status = "rejected"
            self.rejected += 1
            return False
        r.status = "pending"
        self.pending[r.pset].append(r)
        return True

    def admit(self, now: float) -> List[Request]:
        """Admit waiting queries in arrival order while slots are free; a query whose client's keys
        cannot be made resident now stays waiting and later queries of other clients may pass it."""
        out = []
        for name, q in self.pending.items():
            kept: Deque[Request] = collections.deque()
            while q:
                if not self.free_slots[name]:
                    break
                r = q.popleft()
                if not self.keys.acquire(r.client):
                    kept.append(r)
                    continue
                r.slot = self.free_slots[name].pop()
                r.status, r.t_admit = "admitted", now
                self.admitted[name].setdefault(r.client, collections.deque()).append(r)
                out.append(r)
            kept.extend(q)
            self.pending[name] = kept
        return out

    def next_batch(self, pset: str, now: float) -> List[Request]:
        """mix_clients: the oldest admitted queries (at most max_batch), grouped by client in order
        of each client's oldest one, arrival order within a client. Otherwise the admitted queries
        of the client whose oldest admitted query arrived first (at most max_batch)."""
        adm = self.admitted[pset]
        if not adm:
            return []
        cap = self.cfg[pset].max_batch
        if self.mix_clients:
            heap = [(q[0].t_arrive, i, c) for i, (c, q) in enumerate(adm.items())]
            heapq.heapify(heap)
            runs: Dict[int, List[Request]] = {}          # insertion order = order of first pick
            n = 0
            while heap and n < cap:
                _, i, c = heapq.heappop(heap)
                q = adm[c]
                runs.setdefault(c, []).append(q.popleft())
                n += 1
                if q:
                    heapq.heappush(heap, (q[0].t_arrive, i, c))
            for c in runs:
                if not adm[c]:
                    del adm[c]
            batch = [r for rs in runs.values() for r in rs]
        else:
            client = min(adm, key=lambda c: adm[c][0].t_arrive)
            q = adm[client]
            batch = [q.popleft() for _ in range(min(len(q), cap))]
            if not q:
                del adm[client]
        self._batch_id += 1
        for r in batch:
            r.status, r.t_launch, r.batch = "running", now, self._batch_id
        return batch

    def finish(self, batch: Iterable[Request], now: float):
        for r in batch:
            r.status, r.t_done = "done", now
            self.free_slots[r.pset].append(r.slot)
            self.keys.release(r.client)

    def idle(self) -> bool:
        return not any(self.pending.values()) and not any(self.admitted.values())


def latency_stats(reqs: Sequence[Request]) -> Dict[str, float]:
    done = [r for r in reqs if r.status == "done"]
    if not done:
        return {"completed": 0}
    lat = np.array([r.latency for r in done]) * 1e3
    t0 = min(r.t_arrive for r in done)
    t1 = max(r.t_done for r in done)
    return {"completed": len(done), "rejected": sum(r.status == "rejected" for r in reqs),
            "throughput_qps": len(done) / max(t1 - t0, 1e-9),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "mean_batch": len(done) / max(len({(r.pset, r.batch) for r in done}), 1)}


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64([seed, 77]))
    return np.cumsum(g.exponential(1.0 / rate, size=count))


# --------------------------------------------------------------------------------------- device
@dataclasses.dataclass
class PsetSpec:
    """One parameter set served by the GPU: its context parameters, model and pool sizes."""
    name: str
    workload: object                    # a workloads.Workload (parameters and layer shapes)
    weights: List[np.ndarray]
    slot_bytes_budget: int              # device bytes for the ciphertext slots
    max_batch: int = 64
    lanes: int = 2
    lazy: bool = True
    qp: bool = True              # baby steps over Q*P (dense-layer variant)
    raw_banks: Optional[List[np.ndarray]] = None    # already-encoded int64 [t][N] plaintexts per layer
                                                    # (used instead of `weights` when given)


class _Lane:
    def __init__(self, ctx, stream, max_batch, k_in, k_out, torch):
        self.ctx, self.stream = ctx, stream
        self.inp = ctx.empty_ct(max_batch, k_in)
        self.out = ctx.empty_ct(max_batch, k_out)
        self.idx_host = torch.empty(max_batch, dtype=torch.int64, pin_memory=True)
        self.idx = torch.empty(max_batch, dtype=torch.int64, device=self.inp.device)
        self.batch: List[Request] = []
        self.event = None


class GpuServer:
    """Runs the scheduler on the GPU. Clients register the evaluation keys they would upload; the
    server holds them on the host and loads them into HBM on demand (KeyCache)."""

    def __init__(self, specs: Sequence[PsetSpec], key_budget: int, max_pending: int = 1 << 20,
                 keep_outputs: bool = False, device: int = 0, mix_clients: bool = True):
        import torch
        from . import Context
        self.torch = torch
        self.keep_outputs = keep_outputs
        self.specs = {s.name: s for s in specs}
        self.lanes: Dict[str, List[_Lane]] = {}
        self.models = {}
        self.pool_in, self.pool_out = {}, {}
        self.client_pset: Dict[int, str] = {}
        self.client_keys: Dict[int, Dict[int, np.ndarray]] = {}
        cfgs = []
        for s in specs:
            w = s.workload
            ctxs = [Context.for_workload(w, device=device) for _ in range(s.lanes)]
            layers = [(l.n_in, l.n_out, l.t1) for l in w.layers]
            m = (ctxs[0].load_model_raw(layers, s.raw_banks, lazy=s.lazy, qp=s.qp) if s.raw_banks is not None
                 else ctxs[0].load_model(layers, s.weights, lazy=s.lazy, qp=s.qp))
            self.models[s.name] = m
            k_in, k_out = m.info.k_in, m.info.k_out
            per_slot = 2 * (k_in + k_out) * ctxs[0].n * 8
            slots = max(1, s.slot_bytes_budget // per_slot)
            self.pool_in[s.name] = ctxs[0].empty_ct(slots, k_in)
            self.pool_out[s.name] = ctxs[0].empty_ct(slots, k_out)
            self.lanes[s.name] = [_Lane(c, torch.cuda.Stream(device=device), s.max_batch, k_in, k_out, torch)
                                  for c in ctxs]
            cfgs.append(PsetConfig(s.name, slots, s.max_batch, s.lanes))
        self.keys = KeyCache(key_budget, self._key_size, self._load_keys, self._unload_keys)
        self.sched = Scheduler(cfgs, self.keys, max_pending, mix_clients)

    # ------------------------------------------------------------------ clients and keys
    def register_client(self, client: int, pset: str, evaluation_keys: Dict[int, np.ndarray]):
        self.client_pset[client] = pset
        self.client_keys[client] = evaluation_keys

    def _key_size(self, client: int) -> int:
        return sum(a.nbytes for a in self.client_keys[client].values())

    def _load_keys(self, client: int):
        ctx = self.lanes[self.client_pset[client]][0].ctx
        k = ctx.import_keys(self.client_keys[client])
        return k, k.nbytes()

    def _unload_keys(self, keys):
        # only clients without admitted or running queries are evicted, so no queued work reads
        # these keys; the synchronization keeps that true even for work enqueued by other callers
        self.torch.cuda.synchronize()
        del keys

    def warmup(self):
        """Grow every lane's workspace to its largest batch, then freeze it: from here on a forward
        pass never allocates."""
        torch = self.torch
        for name, lanes in self.lanes.items():
            client = next(c for c, p in self.client_pset.items() if p == name)
            assert self.keys.acquire(client)
            keys = self.keys.handle(client)
            for ln in lanes:
                ln.inp.zero_()
                with torch.cuda.stream(ln.stream):
                    # the largest batch, and one query (small batches split their transforms
                    # through a buffer of their own)
                    ln.ctx.forward(self.models[name], keys, ln.inp, out=ln.out, stream=ln.stream)
                    ln.ctx.forward(self.models[name], keys, ln.inp[:1], out=ln.out[:1], stream=ln.stream)
                ln.stream.synchronize()
                ln.ctx.workspace_freeze(True)
            self.keys.release(client)
        torch.cuda.synchronize()

    # ------------------------------------------------------------------ loop
    def submit(self, r: Request, now: float) -> bool:
        return self.sched.arrive(r, now)

    def step(self, now: float, clock: Optional[Callable[[], float]] = None) -> int:
        """One pass of the loop: admit, launch on idle lanes, retire finished batches (stamped with
        clock(), default `now`). Returns the number of queries retired."""
        torch = self.torch
        for r in self.sched.admit(now):
            self.pool_in[r.pset][r.slot].copy_(r.ct)
            r.ct = None                          # the upload buffer is no longer needed
        cur = torch.cuda.current_stream()
        for name, lanes in self.lanes.items():
            for ln in lanes:
                if ln.batch:
                    continue
                batch = self.sched.next_batch(name, now)
                if not batch:
                    break
                n = len(batch)
                ln.idx_host.numpy()[:n] = [r.slot for r in batch]
                keys = [self.keys.handle(r.client) for r in batch]
                with torch.cuda.stream(ln.stream):
                    ln.stream.wait_stream(cur)       # the slot copies above
                    ln.idx[:n].copy_(ln.idx_host[:n], non_blocking=True)
                    torch.index_select(self.pool_in[name], 0, ln.idx[:n], out=ln.inp[:n])
                    ln.ctx.forward_multi(self.models[name], keys, ln.inp[:n], out=ln.out[:n], stream=ln.stream)
                    self.pool_out[name].index_copy_(0, ln.idx[:n], ln.out[:n])
                    ln.event = torch.cuda.Event()
                    ln.event.record(ln.stream)
                ln.batch = batch
        retired = 0
        for name, lanes in self.lanes.items():
            for ln in lanes:
                if ln.batch and ln.event.query():
                    t = clock() if clock is not None else now
                    if self.keep_outputs:
                        for r in ln.batch:
                            r.out = self.pool_out[name][r.slot].clone()
                    self.sched.finish(ln.batch, t)
                    retired += len(ln.batch)
                    ln.batch = []
        return retired

    def run_trace(self, reqs: Sequence[Request], offsets: Sequence[float], timeout: float = 600.0) -> float:
        """Submit reqs[i] at offsets[i] seconds after the start (busy loop, wall clock) and run
        until every query is done or rejected. Returns the elapsed seconds."""
        order = np.argsort(np.asarray(offsets), kind="stable")
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0       # noqa: E731
        nxt = 0
        left = len(reqs)
        while left:
            now = time.perf_counter() - t0
            while nxt < len(order) and offsets[order[nxt]] <= now:
                r = reqs[order[nxt]]
                r.t_arrive = offsets[order[nxt]]
                if not self.submit(r, now):
                    left -= 1
                nxt += 1
            left -= self.step(clock(), clock)
            if now > timeout:
                raise TimeoutError("serving trace did not drain in %.0f s" % timeout)
        self.torch.cuda.synchronize()
        return time.perf_counter() - t0

    def close(self):
        self.torch.cuda.synchronize()
        for lanes in self.lanes.values():
            for ln in lanes:
                ln.ctx.workspace_freeze(False)
        self.keys.clear()
