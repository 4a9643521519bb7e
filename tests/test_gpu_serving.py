"""GPU test of the serving loop: queries of two parameter sets (N=2^13 and N=2^14) from four
clients arrive as a Poisson stream and are served with continuous batching (batches mix clients,
each evaluated with its own keys), with a key budget
that holds only one N=2^14 client's keys at a time (so keys are evicted and uploaded again). Every
result must equal, bit for bit, the same query evaluated alone with the client's own keys, and the
decrypted results must match the FP64 forward pass. A second run serves a model of seeded integer
plaintexts and checks served results against the CPU oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import normwise_error

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_serving_results_equal_alone_and_in_the_mix():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_11935_amd as ctl
    from paper_2205_11935_amd.serving import GpuServer, PsetSpec, Request, latency_stats, poisson_arrivals

    specs = [PsetSpec("mid", W.MID, W.weights(W.MID), slot_bytes_budget=8 << 20, max_batch=4, lanes=2),
             PsetSpec("large", W.LARGE, W.weights(W.LARGE), slot_bytes_budget=16 << 20, max_batch=4, lanes=2)]
    clients = {0: "mid", 1: "mid", 2: "large", 3: "large"}
    # client side: own context, keys, encrypted inputs
    cctx = {"mid": ctl.Context.for_workload(W.MID), "large": ctl.Context.for_workload(W.LARGE)}
    wl = {"mid": W.MID, "large": W.LARGE}
    cmodel = {p: cctx[p].load_model([(l.n_in, l.n_out, l.t1) for l in wl[p].layers], W.weights(wl[p]), lazy=True, qp=True)
              for p in cctx}
    ckeys, uploads = {}, {}
    for c, p in clients.items():
        ckeys[c] = cctx[p].keygen(wl[p].seed_keys + 100 * c, cmodel[p].info.rotations, relin=True)
        uploads[c] = ckeys[c].evaluation_keys()
    key_bytes = {c: sum(a.nbytes for a in uploads[c].values()) for c in clients}
    budget = key_bytes[0] + key_bytes[1] + max(key_bytes[2], key_bytes[3]) + (1 << 20)
    srv = GpuServer(specs, key_budget=budget, keep_outputs=True)
    for c, p in clients.items():
        srv.register_client(c, p, uploads[c])
    srv.warmup()

    n_req = 40
    g = np.random.Generator(np.random.PCG64(11))
    reqs, xs = [], []
    for i in range(n_req):
        p = "mid" if g.random() < 0.8 else "large"
        c = int(g.choice([k for k, v in clients.items() if v == p]))
        if i < 2:
            c, p = 2 + i, "large"                 # both N=2^14 clients early: forces an eviction
        m = cmodel[p]
        x = np.clip(g.normal(0.0, 1.0, size=(m.info.items, m.info.n_in)), -3, 3) if p == "large" \
            else g.uniform(-1.0, 1.0, size=(m.info.items, m.info.n_in))
        ct = cctx[p].encrypt(ckeys[c], cctx[p].encode_items(m, x), seed=9100 + i)
        reqs.append(Request(i, c, p, ct=ct))
        xs.append(x)
    # a burst of 20 at once (batches of several queries are certain), then 20 more arriving as a
    # Poisson stream while those run
    offsets = np.concatenate([np.zeros(20), poisson_arrivals(300.0, n_req - 20, seed=12)])
    inputs = [r.ct.clone() for r in reqs]
    srv.run_trace(reqs, offsets, timeout=120)
    st = latency_stats(reqs)
    assert st["completed"] == n_req, st
    assert srv.keys.evictions >= 1 and srv.keys.loads >= 3
    assert st["mean_batch"] > 1.0, st
    by_batch = {}
    for r in reqs:
        by_batch.setdefault(r.batch, set()).add(r.client)
    assert any(len(cs) > 1 for cs in by_batch.values())      # batches mixing clients ran

    for r, x, ct in zip(reqs, xs, inputs):
        m = cmodel[r.pset]
        alone = cctx[r.pset].forward(m, ckeys[r.client], ct[None])[0]
        assert torch.equal(alone, r.out), (r.rid, r.client, r.pset)
    for r, x in list(zip(reqs, xs))[:6]:
        m = cmodel[r.pset]
        y = cctx[r.pset].decode_items(m, cctx[r.pset].decrypt(ckeys[r.client], r.out, m.info.k_out))
        ref = x
        ws = W.weights(wl[r.pset])
        for li, wmat in enumerate(ws):
            ref = ref @ wmat.T
            if li + 1 < len(ws):
                ref = ref * ref
        assert normwise_error(y, ref) < 2.0 ** -20, r.rid
    srv.close()


def test_served_results_match_oracle():
    """Both parameter sets served from integer plaintext banks (the bit-exact contract leaves FP64
    encoding out): a burst of 8 queries from one client per set, then 4 more arriving while those
    run; two served results per set equal the oracle's forward pass with that client's keys."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from concurrent.futures import ThreadPoolExecutor
    import paper_2205_11935_amd as ctl
    from oracle import CKKSOracle
    from paper_2205_11935_amd.serving import GpuServer, PsetSpec, Request, latency_stats, poisson_arrivals

    wl = {"mid": W.MID, "large": W.LARGE}
    orc = {p: CKKSOracle.for_workload(wl[p]) for p in wl}
    plans = {p: orc[p].plan([(l.n_in, l.n_out, l.t1) for l in wl[p].layers], lazy=True, qp=True) for p in wl}
    raw = {p: [W.raw_plaintexts(91 + li, L.t, orc[p].n, bound_bits=45, stream=li) for li, L in enumerate(plans[p].layers)]
           for p in wl}
    specs = [PsetSpec("mid", W.MID, None, slot_bytes_budget=8 << 20, max_batch=4, lanes=2, raw_banks=raw["mid"]),
             PsetSpec("large", W.LARGE, None, slot_bytes_budget=16 << 20, max_batch=4, lanes=2, raw_banks=raw["large"])]
    clients = {0: "mid", 1: "large"}
    cctx = {p: ctl.Context.for_workload(wl[p]) for p in wl}
    ckeys = {c: cctx[p].keygen(wl[p].seed_keys + 100 * c, plans[p].rotations, relin=True) for c, p in clients.items()}
    srv = GpuServer(specs, key_budget=1 << 34, keep_outputs=True)
    for c, p in clients.items():
        srv.register_client(c, p, ckeys[c].evaluation_keys())
    srv.warmup()
    reqs, msgs = [], []
    for i in range(12):
        c = i % 2
        p = clients[c]
        m = W.raw_plaintexts(95 + i, 1, orc[p].n, bound_bits=40)[0]
        reqs.append(Request(i, c, p, ct=cctx[p].encrypt(ckeys[c], m, seed=9500 + i)))
        msgs.append(m)
    offsets = np.concatenate([np.zeros(8), poisson_arrivals(200.0, 4, seed=13)])
    srv.run_trace(reqs, offsets, timeout=120)
    assert latency_stats(reqs)["completed"] == 12
    srv.close()

    picks = [0, 2, 1, 11]                                 # two of each parameter set
    oref = {}
    for c, p in clients.items():
        o, seed = orc[p], wl[p].seed_keys + 100 * c
        s = o.keygen_secret(seed)
        oref[c] = (o.keygen_public(seed, s), o.keygen_rotations(seed, s, plans[p].rotations), o.keygen_relin(seed, s),
                   [o.bank_ntt(raw[p][li], L.k, ext=True) for li, L in enumerate(plans[p].layers)])

    def oracle(i):
        r = reqs[i]
        o = orc[r.pset]
        pk, okeys, rlk, banks = oref[r.client]
        return o.forward(plans[r.pset], o.encrypt(pk, msgs[i], 9500 + i), banks, okeys, rlk)

    with ThreadPoolExecutor(max_workers=4) as ex:      # the C oracle releases the interpreter lock
        wants = list(ex.map(oracle, picks))
    for i, want in zip(picks, wants):
        assert np.array_equal(ctl.to_numpy_u64(reqs[i].out), want), (i, reqs[i].pset)
