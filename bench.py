#!/usr/bin/env python3
"""Benchmark of the encrypted frozen-layer forward pass (CryptoTL's ClassifyHE) on one MI355X.

One step = one ClassifyHE pass over a batch of ciphertexts of the large workload: N = 2^14,
ciphertext primes {60,40,40,40,40,60} bits plus a 60-bit special prime, scale 2^40, frozen layers
768 -> 256 -> 64 with x^2 between, weights N(0, 0.05^2), inputs N(0,1) clipped to [-3,3], 5 items
per ciphertext, 64 ciphertexts per launch sequence. Inputs are encrypted and resident in HBM
before the timed region starts; keys and the plaintext bank are resident too.

Prints one JSON line: batched encrypted forward passes/s (value), the one-ciphertext-per-sequence
("plain") rate, p50/p99 latencies, NTT GB/s, per-kernel times measured with HIP events on the
launch stream, the roofline of the dominant kernel, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

# MI355X figures used for the roofline: HBM3E 8 TB/s (published). The integer work runs on the
# vector ALU: 256 CUs at 2.4 GHz, each issuing one 64-lane VALU instruction per clock at full rate.
HBM_PEAK_GBS = 8000.0
CUS, CLOCK_HZ, LANES_PER_CU_CLK = 256, 2.4e9, 64
VALU_PEAK = CUS * CLOCK_HZ * LANES_PER_CU_CLK          # 39.3e12 lane-instructions / s
# VALU lane-instructions per unit of algorithmic work. Residues modulo primes below 2^41 are
# processed in exact FP64 arithmetic (full rate on gfx950), the others as 64-bit integers on the
# 32-bit integer VALU (64-bit add/sub/compare = 2 instructions):
#   NTT butterfly, FP64: product y w (mul, fma for the exact low part, mul by 1/q, rint, fma) 5
#     + x + t + x - t 2 ... + 1 for the sum of the product's two parts                  = 8
#   NTT butterfly, integer (Harvey, Shoup product by the twiddle): Shoup product 16 (high half
#     of x w': 1 mul_hi + 3 mad_u64_u32 + 1 add; low halves of x w and h q: 2 x (1 mad + 2 mul_lo
#     + 1 add); subtract 2) + lazy correction 5 + add 2 + subtract with offset 4              = 27
#   multiply-accumulate, FP64: exact product 6 + accumulate 1                              = 7
#   multiply-accumulate, integer, into a 128-bit sum: 64x64->128 product 7 + 128-bit add 4 = 11
SLOTS_BFLY = {"fp": 8, "int": 27}
SLOTS_MAC = {"fp": 7, "int": 11}
NTT_FAMILIES = ("k_ntt_fwd", "k_ntt_inv", "k_modup", "k_drop", "k_int_ntt")


def _percentile(xs, p):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), p)) if xs else None


def _src_digest():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "ctl_internal.h"):
        with open(os.path.join(ROOT, "paper_2205_11935_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, digest: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if taken on this source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != digest:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("bytes_per_launch")


_ORACLE_WORKLOAD = None
_ORACLE_VARIANT = "qp"


def _oracle_job(i: int):
    """One ciphertext of the large workload through the C oracle's forward pass, in a pool worker:
    set-up (keys, banks, encryption) untimed, then the forward pass timed on the host clock."""
    from oracle import CKKSOracle
    w = _ORACLE_WORKLOAD
    o = CKKSOracle.for_workload(w)
    v = _variant_flags(_ORACLE_VARIANT)
    plan = o.plan([(l.n_in, l.n_out, l.t1) for l in w.layers], **v)
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    keys = o.keygen_rotations(w.seed_keys, s, plan.rotations)
    rlk = o.keygen_relin(w.seed_keys, s)
    ws = W.weights(w)
    banks = [o.bank_ntt(o.layer_bank(plan, li, ws[li]), plan.layers[li].k, ext=v["qp"]) for li in range(len(ws))]
    x = W.inputs(w, i + 1, plan.items, stream=7)[i]
    ct = o.encrypt(pk, o.encode(o.input_slots(plan, x), o.scale), w.seed_encrypt + i)
    t0 = time.time()
    o.forward(plan, ct, banks, keys, rlk)
    return t0, time.time()


def cpu_pool(workers: int, variant: str):
    """Fork the oracle workers now, before this process touches the GPU; they stay idle until
    cpu_baseline hands them work."""
    import multiprocessing as mp
    global _ORACLE_WORKLOAD, _ORACLE_VARIANT
    _ORACLE_WORKLOAD = W.LARGE
    _ORACLE_VARIANT = variant
    return mp.get_context("fork").Pool(workers)


def cpu_baseline(pool, workers: int):
    """The CPU oracle as it stands: one ciphertext of the large workload per worker process, all
    at once, the same dense-layer variant as the GPU headline. Throughput = ciphertexts / (last
    end - first start) of the forward passes; set-up is excluded."""
    spans = pool.map(_oracle_job, range(workers), chunksize=1)
    pool.close()
    pool.join()
    t0, t1 = min(a for a, _ in spans), max(b for _, b in spans)
    per = [b - a for a, b in spans]
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": workers / (t1 - t0), "unit": "encrypted forward passes/s", "cores": workers,
            "kind": "oracle", "single_ct_s": round(sorted(per)[len(per) // 2], 3),
            "host": {"cpu": cpu, "nproc": os.cpu_count()},
            "sample": "%d ciphertexts of the large workload, one per worker process, through the C "
                      "oracle's forward pass (%s variant) run together (%.1f s wall; key generation, "
                      "bank encoding and encryption excluded)" % (workers, _ORACLE_VARIANT, t1 - t0)}


VARIANTS = ("qp", "lazy", "per-step")


def _variant_flags(v: str):
    return {"lazy": v != "per-step", "qp": v == "qp"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=W.LARGE.batch)
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=16,
                    help="oracle worker processes for the CPU leg, one ciphertext each, capped at the host's "
                         "cores (0: skip)")
    ap.add_argument("--no-profile", action="store_true", help="do not bracket launches with events")
    ap.add_argument("--variant", choices=VARIANTS, default="qp",
                    help="dense-layer variant: baby steps kept over Q*P with one ModDown per giant step "
                         "(qp), single-ModDown giant steps (lazy) or one ModDown per rotation (per-step); "
                         "the other two are timed too, without profiling")
    ap.add_argument("--other-steps", type=int, default=3, help="timed steps of each other variant")
    ap.add_argument("--workload", choices=("large", "mix", "serve", "cnn"), default="large",
                    help="large: the 768->256->64 stack, batch 64 (the headline); mix: 512 queries of "
                         "1-3 layers with widths from {128,256,512,768}; serve: the serving loop alone; "
                         "cnn: the paper's frozen CNN stack at its two parameter sets")
    ap.add_argument("--autotune", type=int, default=1,
                    help="tune the launch knobs on the timed workload before timing it (0: library defaults)")
    ap.add_argument("--paper-stack", type=int, default=1,
                    help="also time the paper's frozen CNN stack (Conv1D, Dense+ReLU approx., AvgPool, "
                         "Dense) at CryptoTL_p1 and _p2 and report it beside the headline (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="serving sweep: seconds of Poisson arrivals per rate (0: skip the sweep)")
    ap.add_argument("--serve-rates", default="10,100,500,1000,2000", help="serving sweep: arrival rates, q/s")
    ap.add_argument("--mix-queries", type=int, default=512)
    ap.add_argument("--graphs", action="store_true", help="mix: replay captured HIP graphs of the dense calls")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the timed region, copy a buffer of this many MiB once (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU (the encrypted forward pass would shard by ciphertext with "
              "no exchange between GPUs, and no multi-GPU run is made); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    pool, workers = None, 0
    if args.cpu_sample > 0 and args.workload == "large":
        workers = max(1, min(args.cpu_sample, os.cpu_count() or 1, 16))
        pool = cpu_pool(workers, args.variant)

    import torch
    import paper_2205_11935_amd as ctl

    if args.workload == "mix":
        return bench_mix(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "cnn":
        return bench_cnn(args)

    w = W.LARGE
    B = args.batch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    c = ctl.Context.for_workload(w)
    layers = [(l.n_in, l.n_out, l.t1) for l in w.layers]
    t_setup = time.perf_counter()
    model = c.load_model(layers, W.weights(w), **_variant_flags(args.variant))
    others = {v: c.load_model(layers, W.weights(w), **_variant_flags(v))
              for v in VARIANTS if v != args.variant} if args.other_steps > 0 else {}
    keys = c.keygen(w.seed_keys, model.info.rotations, relin=True)
    x = W.inputs(w, B, model.info.items)
    ct = c.empty_ct(B, c.nq)
    for i in range(B):
        c.encrypt(keys, c.encode_items(model, x[i]), w.seed_encrypt + i, out=ct[i])
    out = c.empty_ct(B, model.info.k_out)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        c.forward(model, keys, ct, out=out)
    torch.cuda.synchronize()
    tuning = None
    if args.autotune:
        from paper_2205_11935_amd import autotune
        tuning = autotune.tune(c, lambda: c.forward(model, keys, ct, out=out), reps=2)
        tuning = {"knobs": tuning["knobs"], "default_ms": round(tuning["baseline_ms"], 3),
                  "tuned_ms": round(tuning["best_ms"], 3), "trials": tuning["trials"]}

    # ---------------------------------------------------------------- timed region (batched)
    if not args.no_profile:
        c.profile_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for s in range(args.steps):
        c.forward(model, keys, ct, out=out)
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = [ev[s].elapsed_time(ev[s + 1]) for s in range(args.steps)]
    prof = c.profile_read() if not args.no_profile else {}
    prof_bytes = c.profile_bytes() if not args.no_profile else {}
    c.profile_enable(False)
    value = B * args.steps / elapsed

    if args.copy_calibration_mib > 0:
        words = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(words, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---------------------------------------------------------------- the other dense-layer variants
    other_lines = []
    for v, other in others.items():
        c.forward(other, keys, ct, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.other_steps):
            c.forward(other, keys, ct, out=out)
        torch.cuda.synchronize()
        other_elapsed = time.perf_counter() - t0
        other_lines.append({"variant": v, "steps": args.other_steps,
                            "value": round(B * args.other_steps / other_elapsed, 3),
                            "ms_per_step": round(other_elapsed / args.other_steps * 1e3, 3)})
    if others:
        c.forward(model, keys, ct, out=out)     # leave the headline variant's output in `out`

    # decrypted spot check of the last step (ciphertext 0) against the FP64 forward pass
    res = c.decrypt(keys, out[0], model.info.k_out)
    y = c.decode_items(model, res)
    ref = x[0]
    for li, wm in enumerate(W.weights(w)):
        ref = ref @ wm.T
        if li + 1 < len(w.layers):
            ref = ref * ref
    rel_err = float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))

    # ---------------------------------------------------------------- plain: one ciphertext per sequence
    plain = None
    one = one_out = None
    if args.plain_steps > 0:
        one, one_out = ct[:1].contiguous(), c.empty_ct(1, model.info.k_out)
        for _ in range(2):
            c.forward(model, keys, one, out=one_out)
        torch.cuda.synchronize()
        pev = [torch.cuda.Event(enable_timing=True) for _ in range(args.plain_steps + 1)]
        t0 = time.perf_counter()
        pev[0].record(stream)
        for s in range(args.plain_steps):
            c.forward(model, keys, one, out=one_out)
            pev[s + 1].record(stream)
        torch.cuda.synchronize()
        plain_elapsed = time.perf_counter() - t0
        plain_ms = [pev[s].elapsed_time(pev[s + 1]) for s in range(args.plain_steps)]
        plain = {"value": round(args.plain_steps / plain_elapsed, 3), "unit": "encrypted forward passes/s",
                 "p50_ms": _percentile(plain_ms, 50), "p99_ms": _percentile(plain_ms, 99)}
        # the same single-ciphertext pass replayed from a captured graph (the library's launch
        # sequence with the host's per-launch work removed); the workspace is frozen meanwhile so
        # that nothing is allocated under capture, and every replay must equal the eager result
        want = one_out.clone()
        c.workspace_freeze(True)
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                c.forward(model, keys, one, out=one_out)
            gev = [torch.cuda.Event(enable_timing=True) for _ in range(args.plain_steps + 1)]
            same = True
            for s in range(args.plain_steps):
                one_out.zero_()
                gev[s].record(stream)
                g.replay()
                gev[s + 1].record(stream)
                torch.cuda.synchronize()
                same = same and bool(torch.equal(one_out, want))
            gms = [gev[s].elapsed_time(gev[s + 1]) for s in range(args.plain_steps)]
            plain["graph"] = {"p50_ms": _percentile(gms, 50), "p99_ms": _percentile(gms, 99),
                              "replays_equal_eager": same}
            del g
        except RuntimeError as e:          # capture refused: report it, keep the eager figures
            plain["graph"] = {"error": str(e)[:200]}
        finally:
            c.workspace_freeze(False)
        torch.cuda.synchronize()

    # ---------------------------------------------------------------- standalone batched NTT
    n = c.n
    res_cnt = 64 * (c.nq + 1)
    buf = torch.randint(0, 1 << 40, (res_cnt, n), dtype=torch.int64, device=dev)
    pidx = [r % (c.nq + 1) for r in range(res_cnt)]
    c.ntt(buf, pidx)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record(stream)
    for _ in range(reps):
        c.ntt(buf, pidx)
    e1.record(stream)
    torch.cuda.synchronize()
    ntt_ms = e0.elapsed_time(e1) / reps
    ntt_gbs = 16.0 * n * res_cnt / (ntt_ms * 1e-3) / 1e9

    # ---------------------------------------------------------------- kernels and roofline
    kernels = {}
    total_ms = sum(v[1] for v in prof.values()) or 1.0
    for name, (cnt, ms, work, fpw) in prof.items():
        if cnt:
            kernels[name] = {"launches": cnt, "ms": round(ms, 3), "share": round(ms / total_ms, 4),
                             "avg_ms": round(ms / cnt, 4), "work": work, "fp64_share": round(fpw / work, 3)}
    logn = int(math.log2(n))
    butterflies_per_ntt = (n // 2) * logn
    ntt_res = sum(prof[f][2] for f in NTT_FAMILIES if f in prof)
    ntt_time = sum(prof[f][1] for f in NTT_FAMILIES if f in prof)
    ntt_gbs_fwd = 16.0 * n * ntt_res / (ntt_time * 1e-3) / 1e9 if ntt_time else None
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms"])
        cnt, ms, work, fpw = prof[dom]
        avg_s = ms / cnt * 1e-3
        if dom in NTT_FAMILIES:
            slots = (fpw * SLOTS_BFLY["fp"] + (work - fpw) * SLOTS_BFLY["int"]) / cnt * butterflies_per_ntt
            alg_bytes = work / cnt * 16.0 * n
            ops = "NTT butterflies x (%d FP64 | %d integer) VALU lane-instructions" % (SLOTS_BFLY["fp"], SLOTS_BFLY["int"])
        elif dom in ("k_mac", "k_mac_fp", "k_mac_direct", "k_keyip", "k_tensor"):
            slots = (fpw * SLOTS_MAC["fp"] + (work - fpw) * SLOTS_MAC["int"]) / cnt
            # the library's per-launch model: digits, keys, outputs (key product); ciphertexts,
            # rotations, bank, outputs (MAC); see ctl_profile_read_bytes
            alg_bytes = prof_bytes.get(dom, 0.0) / cnt or None
            ops = "modular multiply-accumulates x (%d FP64 | %d integer) VALU lane-instructions" % (
                SLOTS_MAC["fp"], SLOTS_MAC["int"])
        else:
            slots, alg_bytes, ops = 0.0, work / cnt * 16.0, "residue words"
        digest = _src_digest()
        alu = slots / avg_s / 1e12
        alu_peak = VALU_PEAK / 1e12
        hbm = alg_bytes / avg_s / 1e9 if alg_bytes else 0.0
        # the binding roofline is the one the kernel is closer to: its time at that peak is the
        # larger of the two model times
        if hbm / HBM_PEAK_GBS > alu / alu_peak:
            bound, achieved, peak, unit = "hbm", hbm, HBM_PEAK_GBS, "GB/s"
        else:
            bound, achieved, peak, unit = "alu", alu, alu_peak, "T VALU-lane-instr/s"
        roofline = {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": round(peak, 2),
                    "unit": unit, "frac": round(achieved / peak, 4),
                    "traffic": _traffic(dom, digest), "avg_launch_ms": round(ms / cnt, 4),
                    "work_per_launch": work / cnt, "ops": ops, "source_digest": digest,
                    "alu_achieved": round(alu, 3), "alu_frac": round(alu / alu_peak, 4)}
        if alg_bytes:
            roofline["alg_bytes_per_launch"] = alg_bytes
            roofline["hbm_gbs"] = round(hbm, 1)
            roofline["hbm_frac"] = round(hbm / HBM_PEAK_GBS, 4)

    line = {
        "metric": "encrypted fwd passes/sec at N=2^14 (batched vs plain) + NTT GB/s; p50/p99",
        "value": round(value, 3),
        "unit": "encrypted forward passes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "large: N=2^14, q={60,40,40,40,40,60}+P60, scale 2^40, 768->256->64 x^2, "
                               "%d ciphertexts per launch sequence" % B,
                   "global_batch": B, "items_per_ct": model.info.items, "layers": "768->256->64",
                   "variant": args.variant, "t1": [l.t1 for l in w.layers], "parallelism": "single GPU"},
        "other_variants": other_lines,
        "autotune": tuning,
        "items_per_s": round(value * model.info.items, 2),
        "batched_step_ms": {"p50": _percentile(step_ms, 50), "p99": _percentile(step_ms, 99)},
        "plain": plain,
        "ntt_gbs": {"standalone": round(ntt_gbs, 1), "in_forward": round(ntt_gbs_fwd, 1) if ntt_gbs_fwd else None,
                    "bytes_per_ntt": 16 * n},
        "decrypt_check_rel_err": rel_err,
        "kernels": kernels,
        "roofline": roofline,
        "setup_s": round(setup_s, 2),
        "workspace_gib": round(c.workspace_bytes() / 2 ** 30, 2),
    }
    if args.serve_seconds > 0 or args.paper_stack:
        del c, model, others, keys, ct, out, one, one_out, buf
        import gc
        gc.collect()
        torch.cuda.empty_cache()
    if args.serve_seconds > 0:
        line["serving"] = serving_sweep(args)
    if args.paper_stack:
        line["paper_stack"] = {name: cnn_measure(name, args.batch, max(2, args.steps // 2), plain_steps=5)
                               for name in ("cnn_p1", "cnn_p2")}
    if pool is not None:
        try:
            line["cpu_baseline"] = cpu_baseline(pool, workers)
        except Exception as e:          # noqa: BLE001 -- the GPU line is still worth printing
            line["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)


def serving_sweep(args):
    """The serving loop under Poisson load: 80% of queries on the mid parameter set (N=2^13,
    512->128->128) and 20% on the large one (N=2^14, 768->256->64), four clients per set with
    their evaluation keys resident in HBM, continuous batching on two lanes per set."""
    import torch
    import paper_2205_11935_amd as ctl
    from paper_2205_11935_amd.serving import GpuServer, PsetSpec, Request, latency_stats, poisson_arrivals
    t0 = time.perf_counter()
    wl = {"mid": W.MID, "large": W.LARGE}
    specs = [PsetSpec("mid", W.MID, W.weights(W.MID), slot_bytes_budget=1 << 30, max_batch=64, lanes=2),
             PsetSpec("large", W.LARGE, W.weights(W.LARGE), slot_bytes_budget=2 << 30, max_batch=64, lanes=2)]
    clients = {c: ("mid" if c < 4 else "large") for c in range(8)}
    cctx = {p: ctl.Context.for_workload(wl[p]) for p in wl}
    cmodel = {p: cctx[p].load_model([(l.n_in, l.n_out, l.t1) for l in wl[p].layers], W.weights(wl[p]), lazy=True, qp=True)
              for p in wl}
    uploads, cts = {}, {}
    g = np.random.Generator(np.random.PCG64(W.MIX_SEED + 9))
    for c, p in clients.items():
        k = cctx[p].keygen(wl[p].seed_keys + 100 * c, cmodel[p].info.rotations, relin=True)
        uploads[c] = k.evaluation_keys()
        m = cmodel[p]
        cts[c] = []
        for j in range(4):
            x = g.uniform(-1.0, 1.0, size=(m.info.items, m.info.n_in))
            cts[c].append(cctx[p].encrypt(k, cctx[p].encode_items(m, x), seed=7000 + 10 * c + j))
        del k
    key_budget = sum(sum(a.nbytes for a in u.values()) for u in uploads.values()) + (64 << 20)
    srv = GpuServer(specs, key_budget=key_budget)
    for c, p in clients.items():
        srv.register_client(c, p, uploads[c])
    srv.warmup()
    for c in clients:                               # every client's keys resident before the load
        assert srv.keys.acquire(c)
        srv.keys.release(c)
    # one untimed pass of the loop itself (first calls of the gather/scatter paths on every lane)
    warm = [Request(-1 - i, c, p, ct=cts[c][0]) for i, (c, p) in enumerate(list(clients.items()) * 2)]
    srv.run_trace(warm, [0.0] * len(warm), timeout=120)
    setup_s = time.perf_counter() - t0
    sweep = []
    rid = 0
    for rate in [float(r) for r in args.serve_rates.split(",")]:
        n = int(min(max(rate * args.serve_seconds, 50), 4 * rate * args.serve_seconds))
        offs = poisson_arrivals(rate, n, seed=int(rate))
        reqs = []
        for i in range(n):
            p = "mid" if g.random() < 0.8 else "large"
            c = int(g.integers(0, 4)) + (0 if p == "mid" else 4)
            reqs.append(Request(rid, c, p, ct=cts[c][i % 4]))
            rid += 1
        wall = srv.run_trace(reqs, offs, timeout=300)
        st = latency_stats(reqs)
        per = {p: latency_stats([r for r in reqs if r.pset == p]) for p in wl}
        sweep.append({"rate_qps": rate, "queries": n, "wall_s": round(wall, 3),
                      "throughput_qps": round(st["throughput_qps"], 1),
                      "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                      "mean_batch": round(st["mean_batch"], 2), "rejected": st["rejected"],
                      "p99_ms_by_set": {p: round(per[p]["p99_ms"], 3) for p in per if per[p]["completed"]}})
        print("serving rate %.0f q/s: %s" % (rate, json.dumps(sweep[-1])), file=sys.stderr, flush=True)
    srv.close()
    return {"workload": "Poisson arrivals, 80% mid (N=2^13, 512->128->128) / 20% large (N=2^14, "
                        "768->256->64), 4 clients per set, keys resident, 2 lanes per set, batches of up to 64 "
                        "of the oldest queries across clients",
            "sweep": sweep, "key_bytes": key_budget, "setup_s": round(setup_s, 2)}


PAPER_KB = {"cnn_p1": [235.3, 82.4], "cnn_p2": [838.1, 262.3]}
PAPER_T_S = {"cnn_p1": {"avx512_s": 1.08, "portable_s": 2.72}, "cnn_p2": {"avx512_s": 2.56, "portable_s": 5.93}}


def cnn_measure(name: str, batch: int, steps: int, plain_steps: int = 5):
    """The paper's frozen layers (Conv1D f=9, Dense 768 + cubic ReLU approximation, AvgPool 3,
    Dense 766) at one of Table 2's parameter sets: batched throughput, one-ciphertext latency (the
    paper's t_S, single-threaded CPU there) and a decrypted check against FP64."""
    import torch
    import paper_2205_11935_amd as ctl
    w = W.CNN_WORKLOADS[name]
    t0 = time.perf_counter()
    c = ctl.Context(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    layers = [ctl.Layer.conv1d(w.width, w.f_conv),
              ctl.Layer.dense(w.width, w.width, w.t1, act=ctl.CTL_ACT_POLY3, coef=W.RELU3_COEF),
              ctl.Layer.avgpool(w.width, w.f_pool),
              ctl.Layer.dense(w.pooled, w.pooled, w.t1)]
    taps, w1, w2 = W.cnn_weights(w)
    m = c.load_model(layers, [taps, w1, None, w2], lazy=True, qp=True)
    keys = c.keygen(w.seed_keys, m.info.rotations, relin=True)
    x = W.cnn_inputs(w, batch, m.info.items)
    ct = c.empty_ct(batch, c.nq)
    for i in range(batch):
        c.encrypt(keys, c.encode_items(m, x[i]), 800 + i, out=ct[i])
    out = c.empty_ct(batch, m.info.k_out)
    setup_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    c.forward(m, keys, ct, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.forward(m, keys, ct, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    one, one_out = ct[:1].contiguous(), c.empty_ct(1, m.info.k_out)
    c.forward(m, keys, one, out=one_out)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(plain_steps + 1)]
    ev[0].record(stream)
    for i in range(plain_steps):
        c.forward(m, keys, one, out=one_out)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    lat = [ev[i].elapsed_time(ev[i + 1]) for i in range(plain_steps)]
    y = c.decode_items(m, c.decrypt(keys, out[0], m.info.k_out))
    ref = []
    for b in range(m.info.items):                     # FP64 forward pass of the same layers
        z = w1 @ np.convolve(x[0][b], taps[::-1], mode="same")
        a = np.polyval(np.array(W.RELU3_COEF)[::-1], z)
        ref.append(w2 @ np.convolve(a, np.ones(w.f_pool) / w.f_pool, mode="valid"))
    ref = np.stack(ref)
    err = float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))
    value = batch * steps / el
    t_s = _percentile(lat, 50) / 1e3
    up = ctl.ct_packed_bytes(w.log2n, w.q_bits, w.p_bits, len(w.q_bits), 1)      # seeded c0 + seed
    down = ctl.ct_packed_bytes(w.log2n, w.q_bits, w.p_bits, m.info.k_out, 2)
    return {"params": "N=2^%d, log2 q=%d, Delta=2^%d, p=%d" % (w.log2n, sum(x.bit_length() for x in c.primes),
                                                                 w.log2_scale, m.info.items),
            "batch": batch, "fwd_per_s": round(value, 2), "items_per_s": round(value * m.info.items, 1),
            "ms_per_batch": round(el / steps * 1e3, 2), "t_s_one_ct_ms": {"p50": _percentile(lat, 50),
                                                                           "p99": _percentile(lat, 99)},
            "paper_t_s": PAPER_T_S[name], "speedup_vs_paper_avx512_t_s": round(PAPER_T_S[name]["avx512_s"] / t_s, 1),
            "message_kB": {"client_to_server": round(up / 1000, 1), "server_to_client": round(down / 1000, 1),
                           "paper": PAPER_KB[name]},
            "decrypt_check_rel_err": err, "setup_s": round(setup_s, 2)}


def bench_cnn(args):
    res = {name: cnn_measure(name, args.batch, args.steps, plain_steps=10) for name in ("cnn_p1", "cnn_p2")}
    p2 = res["cnn_p2"]
    line = {"metric": "encrypted fwd passes/sec of the paper's frozen CNN layers (CryptoTL_p2, N=2^14)",
            "value": p2["fwd_per_s"], "unit": "encrypted forward passes/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": p2["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "Conv1D f=9 -> Dense 768 + ReLU approx. (degree 3) -> AvgPool 3 -> Dense 766, "
                                   "batch %d" % args.batch},
            "paper_stack": res}
    print(json.dumps(line), flush=True)


def bench_serve(args):
    if args.serve_rates == "10,100,500,1000,2000":       # the full sweep of the serving workload
        args.serve_rates = "10,20,50,100,200,500,1000,2000"
        args.serve_seconds = max(args.serve_seconds, 5.0)
    sv = serving_sweep(args)
    top = sv["sweep"][-1]
    line = {"metric": "p50/p99 latency and throughput of the serving loop under Poisson load",
            "value": top["throughput_qps"], "unit": "queries/s", "n_gpus": 1, "steps": len(sv["sweep"]),
            "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u64", "data": "synthetic", "config": {"workload": sv["workload"]},
            "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"], "serving": sv}
    print(json.dumps(line), flush=True)


def bench_mix(args):
    """Throughput of the batched mix: queries of 1-3 dense layers with widths drawn from
    {128,256,512,768}, evaluated position by position with banks shared per shape."""
    import torch
    import paper_2205_11935_amd as ctl
    from paper_2205_11935_amd.batch_mix import MixEngine
    w = W.LARGE
    c = ctl.Context.for_workload(w)
    queries = W.mix_queries(args.mix_queries)
    t0 = time.perf_counter()
    keys = c.keygen(w.seed_keys, MixEngine.rotations(queries, W.MIX_T1), relin=True)
    eng = MixEngine(c, keys, lambda p, a, b, t: W.mix_weights(p, a, b), W.MIX_T1, W.MIX_BLOCK, lazy=True,
                    graphs=args.graphs)
    items = (c.n // 2) // W.MIX_BLOCK
    xs = W.mix_inputs(queries, items)
    dev = c.empty_ct(len(queries), c.nq)
    for i, q in enumerate(queries):
        c.encrypt(keys, c.encode_items(eng.model(0, q.widths[0], q.widths[1]), xs[i]), 9000 + i, out=dev[i])
    for q in queries:                       # every bank the batch touches, before timing
        for l in range(q.depth):
            eng.model(l, q.widths[l], q.widths[l + 1])
    setup_s = time.perf_counter() - t0
    eng.run(dev, queries)
    torch.cuda.synchronize()
    if args.graphs:
        eng.freeze()
        eng.run(dev, queries)               # capture
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        eng.run(dev, queries)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    depth_hist = {d: sum(1 for q in queries if q.depth == d) for d in (1, 2, 3)}
    line = {
        "metric": "encrypted fwd passes/sec at N=2^14, batched mix of layer widths and depths",
        "value": round(len(queries) * args.steps / dt, 3), "unit": "encrypted forward passes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "mix: %d queries, 1-3 dense layers, widths from {128,256,512,768}, N=2^14, "
                               "block 1536 (5 items per ciphertext)" % len(queries),
                   "depths": depth_hist, "banks": len(eng.models), "graphs": bool(args.graphs)},
        "setup_s": round(setup_s, 2),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
