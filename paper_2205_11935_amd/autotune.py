"""Autotuner for the library's launch knobs (ctl_knob_set), keyed by GPU architecture, ring degree
and prime chain.

The knobs choose how work is divided among kernels (the MAC's giant-step chunk and ciphertexts per
workgroup, the key product's workgroup numbering, when transforms split or loop); every choice
computes the same residues. The
tuner times the caller's own workload — typically one batched forward pass — for each candidate
value, one knob at a time starting from the current settings (coordinate descent), keeps the
fastest, and checks that every candidate's output equals the first one bit for bit. Results can be
cached in a JSON file so that later contexts with the same key start tuned.

Orchestration only: the timed work runs in the library's kernels.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Callable, Dict, List, Optional, Sequence

CANDIDATES: Dict[str, List[int]] = {
    "mac_chunk": [16, 12, 8, 6, 4],
    "mac_cts": [8, 16, 4, 2],
    "keyip_xcd": [1, 0],
    "ntt_xcd": [1, 0],
    "mac_limb": [1, 0],
    "keyip_rr": [8, 6, 4, 2, 1],
    "ntt_split": [128, 64, 256, 0],
    "ntt_loop": [8, 4, 16, 0],
    "fuse_rescale": [1, 0],
}


def cache_key(arch: str, log2n: int, primes: Sequence[int]) -> str:
    h = hashlib.sha1(",".join(str(int(p)) for p in primes).encode()).hexdigest()[:12]
    return "%s/N=2^%d/%s" % (arch, log2n, h)


def context_key(ctx) -> str:
    import torch
    arch = torch.cuda.get_device_properties(ctx.device).gcnArchName.split(":")[0]
    return cache_key(arch, ctx.log2n, ctx.primes)


def load(path: str, key: str) -> Optional[Dict[str, int]]:
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    entry = data.get(key)
    return dict(entry["knobs"]) if entry else None


def save(path: str, key: str, result: Dict) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key] = result
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(ctx, knobs: Dict[str, int]) -> None:
    for name, value in knobs.items():
        ctx.knob(name, value)


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def pick(times: Dict[int, float], entry: int, margin: float) -> int:
    """The fastest value of `times` ({value: ms}), unless it is within `margin` of `entry`'s."""
    fastest = min(times, key=times.get)
    if entry in times and times[fastest] >= (1.0 - margin) * times[entry]:
        return entry
    return fastest


def tune(ctx, run: Callable[[], object], reps: int = 3,
         candidates: Optional[Dict[str, List[int]]] = None, margin: float = 0.01) -> Dict:
    """run() enqueues the workload on the current stream and returns its output tensor. Returns
    {"knobs": best settings (applied to ctx), "baseline_ms": time with the settings on entry,
    "best_ms": time with the best ones, "trials": {knob: {value: ms}}}. A knob leaves the value it
    had on entry only for one that is faster by more than `margin` (a fraction): differences
    within run-to-run noise, e.g. of a knob the workload does not exercise, change nothing."""
    import torch
    candidates = candidates or CANDIDATES
    stream = torch.cuda.current_stream()

    def timed() -> float:
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            run()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return _median(ms)

    ref = run().clone()
    torch.cuda.synchronize()
    best = {name: ctx.knob(name) for name in candidates}
    baseline = timed()
    trials: Dict[str, Dict[int, float]] = {}
    for name, values in candidates.items():
        trials[name] = {}
        entry = ctx.knob(name)
        for v in values:
            ctx.knob(name, v)
            out = run()
            torch.cuda.synchronize()
            if not torch.equal(out, ref):
                ctx.knob(name, best[name])
                raise RuntimeError("knob %s=%d changed the result" % (name, v))
            trials[name][v] = timed()
        best[name] = pick(trials[name], entry, margin)
        ctx.knob(name, best[name])
    return {"knobs": best, "baseline_ms": baseline, "best_ms": timed(),
            "trials": {k: {str(v): round(t, 3) for v, t in d.items()} for k, d in trials.items()}}
