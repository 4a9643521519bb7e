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
# vector ALU: 256 CUs at 2.4 GHz, each issuing one 64-lane VALU instruction per clock at full rate
# (the unit-count figure); the rates each instruction class really issues at are measured by the
# library's issue-rate probe (ctl_probe_valu) in every run and the ALU roof uses those.
HBM_PEAK_GBS = 8000.0
CUS, CLOCK_HZ, LANES_PER_CU_CLK = 256, 2.4e9, 64
VALU_PEAK = CUS * CLOCK_HZ * LANES_PER_CU_CLK          # 39.3e12 lane-instructions / s
# VALU lane-operations per unit of algorithmic work, by instruction class (add32: full-rate 32-bit
# integer and logic ops, mul32: v_mul_lo/hi_u32, mad64: v_mad_u64_u32, fma64: FP64 ops). Residues
# modulo primes below 2^41 are processed in exact FP64 arithmetic, the others as 64-bit integers on
# the 32-bit integer VALU (64-bit add/sub/compare = 2 instructions):
#   NTT butterfly, FP64: product y w (mul, fma for the exact low part, mul by 1/q, rint, fma) 5
#     + x + t, x - t 2 + 1 for the sum of the product's two parts                      = 8 fma64
#   NTT butterfly, integer (Harvey, Shoup product by the twiddle): high half of x w' 1 mul_hi
#     + 3 mad + 1 add; low halves of x w and h q 2 x (1 mad + 2 mul_lo + 1 add); subtract 2;
#     lazy correction 5, add 2, subtract with offset 4               = 5 mad64 + 5 mul32 + 17 add32
#   product in the FP64 MAC and key product: exact product 5 + accumulate 1, plus the final
#     conversion of each sum spread over its terms                                     = 7 fma64
#   product in the integer MAC (30-bit limbs): 4 v_mad_u64_u32 into column sums, + the operand
#     split and column normalization spread over the terms                    = 4 mad64 + 1 add32
#   product in the integer key product (30-bit limbs): 4 mad64, + the reduction of each sum
#     (carries, a Shoup product by 2^60 mod q, two conditional subtracts) spread over its K = 4..6
#     terms                                                                  = 4.7 mad64 + 3.5 add32
UNIT_OPS = {
    "bfly": {"fp": {"fma64": 8}, "int": {"mad64": 5, "mul32": 5, "add32": 17}},
    "mac": {"fp": {"fma64": 7}, "int": {"mad64": 4, "add32": 1}},
    "keyip": {"fp": {"fma64": 7}, "int": {"mad64": 4.7, "add32": 3.5}},
}
NTT_FAMILIES = ("k_ntt_fwd", "k_ntt_inv", "k_modup", "k_drop", "k_int_ntt",
                "k_ntt_fwd_fp", "k_ntt_inv_fp", "k_modup_fp", "k_drop_fp")
MAC_FAMILIES = ("k_mac", "k_mac_fp", "k_mac_direct", "k_tensor")


def _percentile(xs, p):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), p)) if xs else None


def _src_digest():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "ctl_internal.h"):
        with open(os.path.join(ROOT, "paper_2205_11935_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, site: str, digest: str):
    """HBM bytes per launch of a kernel instance from the committed rocprofv3 counter summary, if
    it was taken on this source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != digest:
        return None
    k = rec.get("instances", {}).get("%s @ %s" % (kernel, site))
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


def valu_rates(c):
    """Measured lane-operations per second of each instruction class (the library's probe)."""
    return {k: c.probe_valu(k) for k in ("add32", "mul32", "mad64", "fma64")}


def _alu_ops(family: str, work: float, fp_work: float, n: int):
    """Model lane-operations of a launch by instruction class ({class: ops})."""
    if family in NTT_FAMILIES:
        units, model = (n // 2) * int(math.log2(n)), UNIT_OPS["bfly"]
    elif family in MAC_FAMILIES:
        units, model = 1, UNIT_OPS["mac"]
    elif family in ("k_keyip", "k_keyip_fp"):
        units, model = 1, UNIT_OPS["keyip"]
    else:
        return {}
    ops = {}
    for part, w in (("fp", fp_work), ("int", work - fp_work)):
        for cls, per in model[part].items():
            ops[cls] = ops.get(cls, 0.0) + per * w * units
    return ops


def _alg_bytes(family: str, work: float, model_bytes: float, n: int) -> float:
    """Algorithmic HBM bytes of a launch: the library's model (key product, MAC), one read and one
    write of a residue per transform (NTT-bearing kernels), else 0 (not modelled)."""
    if model_bytes:
        return model_bytes
    if family in NTT_FAMILIES:
        return 16.0 * n * work
    return 0.0


def instances(launches, steps: int, n: int, rates):
    """Per kernel instance (family, layer, phase, work per launch) per step: time, algorithmic bytes,
    model ALU operations, and the HBM and ALU fractions of its roofs (ALU roof: every class at its
    measured rate)."""
    groups = {}
    for r in launches:
        key = (r["family"], r["layer"], r["phase"], r["work"])
        g = groups.setdefault(key, {"launches": 0, "ms": 0.0, "fp_work": 0.0, "bytes": 0.0})
        g["launches"] += 1
        g["ms"] += r["ms"]
        g["fp_work"] += r["fp_work"]
        g["bytes"] += r["bytes"]
    out = []
    for (fam, layer, phase, work), g in groups.items():
        cnt = g["launches"]
        avg_s = g["ms"] / cnt * 1e-3
        fpw = g["fp_work"] / cnt
        alg = _alg_bytes(fam, work, g["bytes"] / cnt, n)
        ops = _alu_ops(fam, work, fpw, n)
        alu_s = sum(v / rates[k] for k, v in ops.items()) if ops else 0.0
        tot_ops = sum(ops.values())
        site = ("layer %d " % layer if layer >= 0 else "") + (phase or "")
        out.append({"kernel": fam, "site": site.strip(), "launches_per_step": cnt / steps,
                    "ms_per_step": round(g["ms"] / steps, 4), "avg_launch_ms": round(g["ms"] / cnt, 4),
                    "work_per_launch": work, "fp64_share": round(fpw / work, 3) if work else 0.0,
                    "alg_bytes_per_launch": alg, "hbm_gbs": round(alg / avg_s / 1e9, 1) if avg_s else 0.0,
                    "hbm_frac": round(alg / avg_s / 1e9 / HBM_PEAK_GBS, 4) if avg_s else 0.0,
                    "alu_ops_per_launch": tot_ops, "alu_tops": round(tot_ops / avg_s / 1e12, 3) if avg_s else 0.0,
                    "alu_frac": round(alu_s / avg_s, 4) if avg_s else 0.0})
    out.sort(key=lambda x: -x["ms_per_step"])
    return out


def roofline_of(inst, traffic):
    """The roofline object of one kernel instance: the binding roof is the one whose model time is
    the larger (HBM at 8 TB/s on its algorithmic bytes; ALU at the measured class rates)."""
    if inst["hbm_frac"] >= inst["alu_frac"]:
        bound, achieved, peak, unit = "hbm", inst["hbm_gbs"], HBM_PEAK_GBS, "GB/s"
    else:
        # achieved model lane-ops per second against the rate they would run at on the measured
        # class peaks (peak = achieved / alu_frac)
        bound, achieved, unit = "alu", inst["alu_tops"], "T VALU lane-ops/s"
        peak = round(inst["alu_tops"] / inst["alu_frac"], 3) if inst["alu_frac"] else None
    return {"bound": bound, "kernel": inst["kernel"], "site": inst["site"], "achieved": achieved, "peak": peak,
            "unit": unit, "frac": round(max(inst["hbm_frac"], inst["alu_frac"]), 4), "traffic": traffic,
            "avg_launch_ms": inst["avg_launch_ms"], "alg_bytes_per_launch": inst["alg_bytes_per_launch"],
            "hbm_gbs": inst["hbm_gbs"], "hbm_frac": inst["hbm_frac"], "alu_tops": inst["alu_tops"],
            "alu_frac": inst["alu_frac"]}


VARIANTS = ("qp", "lazy", "per-step")


def _variant_flags(v: str):
    return {"lazy": v != "per-step", "qp": v == "qp"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=W.LARGE.batch)
    ap.add_argument("--plain-steps", type=int, default=50)
    ap.add_argument("--cpu-sample", type=int, default=16,
                    help="oracle worker processes for the CPU leg, one ciphertext each, capped at the host's "
                         "cores (0: skip)")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the instrumented pass (launches bracketed with events) after the timed region")
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
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="serving sweep: seconds of Poisson arrivals per rate, unless --serve-queries come "
                         "sooner (0: skip the sweep)")
    ap.add_argument("--serve-queries", type=int, default=5000,
                    help="serving sweep: queries per rate, unless --serve-seconds of arrivals come sooner")
    ap.add_argument("--serve-rates", default="10,20,50,100,200,500,1000,2000,5000,10000,20000",
                    help="serving sweep: arrival rates, q/s")
    ap.add_argument("--mix-queries", type=int, default=512,
                    help="batched mix: queries per pass (0: leave the mix out of the default line)")
    ap.add_argument("--mix-steps", type=int, default=3, help="batched mix: timed passes in the default line")
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
    # no instrumentation here: the kernel breakdown comes from a separate pass below
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
    value = B * args.steps / elapsed

    # ---------------------------------------------------------------- instrumented pass: per-launch events
    prof, prof_bytes, launches = {}, {}, []
    if not args.no_profile:
        c.profile_enable(True)
        for _ in range(args.steps):
            c.forward(model, keys, ct, out=out)
        torch.cuda.synchronize()
        prof, prof_bytes, launches = c.profile_read(), c.profile_bytes(), c.profile_launches()
        c.profile_enable(False)
    rates = valu_rates(c)

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
        for _ in range(20):                 # some 25 ms of single-ciphertext passes before timing
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
        if not args.no_profile:               # where one ciphertext's time goes (instrumented pass)
            c.profile_enable(True)
            for _ in range(3):
                c.forward(model, keys, one, out=one_out)
            torch.cuda.synchronize()
            pl = c.profile_launches()
            c.profile_enable(False)
            by_fam = {}
            for r in pl:
                f = by_fam.setdefault(r["family"], [0, 0.0])
                f[0] += 1
                f[1] += r["ms"]
            plain["kernels"] = {f: {"launches": v[0] / 3, "ms": round(v[1] / 3, 4)}
                                for f, v in sorted(by_fam.items(), key=lambda x: -x[1][1])}
            plain["launches"] = len(pl) / 3
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
            kernels[name] = {"launches": cnt, "ms_per_step": round(ms / args.steps, 3), "share": round(ms / total_ms, 4),
                             "avg_ms": round(ms / cnt, 4), "work": work, "fp64_share": round(fpw / work, 3)}
    ntt_res = sum(prof[f][2] for f in NTT_FAMILIES if f in prof)
    ntt_time = sum(prof[f][1] for f in NTT_FAMILIES if f in prof)
    ntt_gbs_fwd = 16.0 * n * ntt_res / (ntt_time * 1e-3) / 1e9 if ntt_time else None
    digest = _src_digest()
    inst = instances(launches, args.steps, n, rates) if launches else []
    roofline = None
    if inst:
        top = inst[0]
        roofline = roofline_of(top, _traffic(top["kernel"], top["site"], digest))
        roofline["source_digest"] = digest
        roofline["valu_rates_tops"] = {k: round(v / 1e12, 2) for k, v in rates.items()}
        roofline["valu_peak_unit_count_tops"] = round(VALU_PEAK / 1e12, 2)
        roofline["top_instances"] = [{k: i[k] for k in ("kernel", "site", "ms_per_step", "avg_launch_ms", "hbm_frac",
                                                        "alu_frac", "hbm_gbs", "alu_tops")} for i in inst[:4]]

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
        "instances": inst,
        "roofline": roofline,
        "setup_s": round(setup_s, 2),
        "workspace_gib": round(c.workspace_bytes() / 2 ** 30, 2),
    }
    if args.serve_seconds > 0 or args.paper_stack or args.mix_queries > 0:
        del c, model, others, keys, ct, out, one, one_out, buf
        import gc
        gc.collect()
        torch.cuda.empty_cache()
    if args.mix_queries > 0:
        line["mix"] = mix_measure(args.mix_steps, args.mix_queries)
        print("mix: %s" % json.dumps(line["mix"]), file=sys.stderr, flush=True)
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
        # at least serve_seconds of arrivals or serve_queries queries, whichever comes first
        n = max(1, int(min(args.serve_queries, round(rate * args.serve_seconds))))
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
        sweep.append({"rate_qps": rate, "queries": n, "arrival_span_s": round(float(offs[-1]), 2),
                      "wall_s": round(wall, 3), "throughput_qps": round(st["throughput_qps"], 1),
                      "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                      "p99_samples": st["completed"],
                      "mean_batch": round(st["mean_batch"], 2), "rejected": st["rejected"],
                      "by_set": {p: {"p50_ms": round(per[p]["p50_ms"], 3), "p99_ms": round(per[p]["p99_ms"], 3),
                                     "samples": per[p]["completed"]} for p in per if per[p]["completed"]}})
        print("serving rate %.0f q/s: %s" % (rate, json.dumps(sweep[-1])), file=sys.stderr, flush=True)
    srv.close()
    # the first offered rate the loop does not keep up with (throughput below 95% of it)
    knee = next((p["rate_qps"] for p in sweep if p["throughput_qps"] < 0.95 * p["rate_qps"]), None)
    return {"workload": "Poisson arrivals, 80% mid (N=2^13, 512->128->128) / 20% large (N=2^14, "
                        "768->256->64), 4 clients per set, keys resident, 2 lanes per set, batches of up to 64 "
                        "of the oldest queries across clients",
            "per_rate": "min(%d queries, %g s of arrivals)" % (args.serve_queries, args.serve_seconds),
            "sweep": sweep, "saturation_qps": knee if knee is not None else "above %g q/s (the highest rate swept)"
            % max(p["rate_qps"] for p in sweep),
            "key_bytes": key_budget, "setup_s": round(setup_s, 2)}


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
    sv = serving_sweep(args)
    top = sv["sweep"][-1]
    line = {"metric": "p50/p99 latency and throughput of the serving loop under Poisson load",
            "value": top["throughput_qps"], "unit": "queries/s", "n_gpus": 1, "steps": len(sv["sweep"]),
            "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u64", "data": "synthetic", "config": {"workload": sv["workload"]},
            "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"], "serving": sv}
    print(json.dumps(line), flush=True)


def mix_measure(steps: int, n_queries: int, graphs: bool = False):
    """The batched mix: queries of 1-3 dense layers with widths drawn from {128,256,512,768},
    evaluated position by position with banks shared per shape. Throughput over `steps` passes of
    the whole batch, and per-query latency within a pass (from the pass's start to the event
    recorded after the dense group that finishes the query)."""
    import torch
    import paper_2205_11935_amd as ctl
    from paper_2205_11935_amd.batch_mix import MixEngine
    w = W.LARGE
    c = ctl.Context.for_workload(w)
    queries = W.mix_queries(n_queries)
    t0 = time.perf_counter()
    keys = c.keygen(w.seed_keys, MixEngine.rotations(queries, W.MIX_T1), relin=True)
    eng = MixEngine(c, keys, lambda p, a, b, t: W.mix_weights(p, a, b), W.MIX_T1, W.MIX_BLOCK, lazy=True,
                    graphs=graphs)
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
    if graphs:
        eng.freeze()
        eng.run(dev, queries)               # capture
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        eng.run(dev, queries)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # one more pass with a completion event per query
    start, done = torch.cuda.Event(enable_timing=True), [None] * len(queries)
    start.record()
    eng.run(dev, queries, done_events=done)
    torch.cuda.synchronize()
    lat = [start.elapsed_time(e) for e in done]
    if graphs:
        c.workspace_freeze(False)
    depth_hist = {d: sum(1 for q in queries if q.depth == d) for d in (1, 2, 3)}
    return {"workload": "mix: %d queries, 1-3 dense layers, widths from {128,256,512,768}, N=2^14, "
                        "block 1536 (5 items per ciphertext)" % len(queries),
            "queries": len(queries), "steps": steps, "value": round(len(queries) * steps / dt, 3),
            "unit": "encrypted forward passes/s", "ms_per_pass": round(dt / steps * 1e3, 3),
            "query_latency_ms": {"p50": _percentile(lat, 50), "p99": _percentile(lat, 99), "max": max(lat)},
            "depths": depth_hist, "banks": len(eng.models), "graphs": bool(graphs), "setup_s": round(setup_s, 2)}


def bench_mix(args):
    mx = mix_measure(args.steps, args.mix_queries, graphs=args.graphs)
    line = {
        "metric": "encrypted fwd passes/sec at N=2^14, batched mix of layer widths and depths",
        "value": mx["value"], "unit": mx["unit"],
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": mx["ms_per_pass"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": mx["workload"], "depths": mx["depths"], "banks": mx["banks"], "graphs": mx["graphs"]},
        "mix": mx,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
