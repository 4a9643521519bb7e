"""GPU tests of the batched mix of layer widths and depths (one context, one slot layout, banks
shared per (position, w_in, w_out)): bit-exact against the oracle query by query, HIP-graph replays
identical to eager runs, and decrypted outputs within 2^-20 of the FP64 forward pass."""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import CKKSOracle, normwise_error

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _raw_bank(n):
    def bank(pos, w_in, w_out, t):
        return W.raw_plaintexts(W.MIX_SEED + pos * 7919 + w_in * 31 + w_out, t, n, bound_bits=40)
    return bank


@functools.lru_cache(maxsize=None)
def _setup(widths, nq_queries):
    """A small mix (few widths so the raw banks stay small) with keys on both sides."""
    _need_gpu()
    import paper_2205_11935_amd as ctl
    from paper_2205_11935_amd.batch_mix import MixEngine
    w = W.LARGE
    c = ctl.Context.for_workload(w)
    o = CKKSOracle.for_workload(w)
    queries = W.mix_queries(nq_queries, widths=widths)
    rots = MixEngine.rotations(queries, W.MIX_T1)
    keys = c.keygen(w.seed_keys, rots, relin=True)
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    okeys = o.keygen_rotations(w.seed_keys, s, rots)
    rlk = o.keygen_relin(w.seed_keys, s)
    return c, o, queries, keys, (s, pk, okeys, rlk)


def _oracle_query(o, q, ct, bank, okeys, rlk, banks_ntt=None):
    for l in range(q.depth):
        w_in, w_out = q.widths[l], q.widths[l + 1]
        t = max(w_in, w_out)
        k = o.nq - 2 * l
        pts = (banks_ntt[(l, w_in, w_out)] if banks_ntt is not None
               else o.bank_ntt(bank(l, w_in, w_out, t), k, ext=True))
        ct = o.dense(ct, pts, W.MIX_T1[t], okeys, lazy=True, qp=True)
        if l + 1 < q.depth:
            ct = o.square(ct, rlk)
            ct = o.replicate(ct, max(q.widths[l + 1], q.widths[l + 2]), okeys)
    return ct


def test_mix_bit_exact_against_oracle():
    from paper_2205_11935_amd.batch_mix import MixEngine
    import paper_2205_11935_amd as ctl
    c, o, queries, keys, (s, pk, okeys, rlk) = _setup((128, 256), 12)
    bank = _raw_bank(o.n)
    eng = MixEngine(c, keys, bank, W.MIX_T1, W.MIX_BLOCK, raw=True, lazy=True)
    msgs = W.raw_plaintexts(77, len(queries), o.n, bound_bits=40)
    dev = c.empty_ct(len(queries), o.nq)
    for i in range(len(queries)):
        c.encrypt(keys, msgs[i], 500 + i, out=dev[i])
    outs = eng.run(dev, queries)
    assert sorted({q.depth for q in queries}) == [1, 2, 3]
    for i, q in enumerate(queries):
        want = _oracle_query(o, q, o.encrypt(pk, msgs[i], 500 + i), bank, okeys, rlk)
        got = ctl.to_numpy_u64(outs[i])
        assert got.shape == want.shape == (2, o.nq - 2 * q.depth + 1, o.n)
        assert np.array_equal(got, want), (i, q)


def test_mix_bit_exact_wide_layers():
    """Widths 512 and 768 only (t1 = 64, the largest banks), at every position: 10 queries of depth
    1-3 on the shared 1536-slot block, each against the oracle."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_2205_11935_amd.batch_mix import MixEngine
    import paper_2205_11935_amd as ctl
    c, o, queries, keys, (s, pk, okeys, rlk) = _setup((512, 768), 10)
    bank = _raw_bank(o.n)
    eng = MixEngine(c, keys, bank, W.MIX_T1, W.MIX_BLOCK, raw=True, lazy=True)
    msgs = W.raw_plaintexts(79, len(queries), o.n, bound_bits=40)
    dev = c.empty_ct(len(queries), o.nq)
    for i in range(len(queries)):
        c.encrypt(keys, msgs[i], 800 + i, out=dev[i])
    outs = [ctl.to_numpy_u64(x) for x in eng.run(dev, queries)]
    shapes = {(l, q.widths[l], q.widths[l + 1]) for q in queries for l in range(q.depth)}
    assert {sh[0] for sh in shapes} == {0, 1, 2} and {sh[1] for sh in shapes} == {512, 768}
    with ThreadPoolExecutor(max_workers=8) as ex:
        # the C oracle releases the interpreter lock and keeps no shared mutable state
        banks_ntt = dict(zip(sorted(shapes), ex.map(
            lambda sh: o.bank_ntt(bank(sh[0], sh[1], sh[2], max(sh[1], sh[2])), o.nq - 2 * sh[0], ext=True),
            sorted(shapes))))
        wants = list(ex.map(lambda i: _oracle_query(o, queries[i], o.encrypt(pk, msgs[i], 800 + i), bank, okeys,
                                                    rlk, banks_ntt), range(len(queries))))
    for i, q in enumerate(queries):
        assert outs[i].shape == wants[i].shape == (2, o.nq - 2 * q.depth + 1, o.n)
        assert np.array_equal(outs[i], wants[i]), (i, q)


def test_mix_graph_replays_match_eager():
    from paper_2205_11935_amd.batch_mix import MixEngine
    import paper_2205_11935_amd as ctl
    c, o, queries, keys, _ = _setup((128, 256), 12)
    eng = MixEngine(c, keys, _raw_bank(o.n), W.MIX_T1, W.MIX_BLOCK, raw=True, lazy=True, graphs=True)
    msgs = W.raw_plaintexts(78, len(queries), o.n, bound_bits=40)
    dev = c.empty_ct(len(queries), o.nq)
    for i in range(len(queries)):
        c.encrypt(keys, msgs[i], 600 + i, out=dev[i])
    eager = [ctl.to_numpy_u64(x) for x in eng.run(dev, queries)]
    eng.freeze()
    try:
        for rep in range(3):
            got = [ctl.to_numpy_u64(x) for x in eng.run(dev, queries)]
            for a, b in zip(got, eager):
                assert np.array_equal(a, b), rep
            # eager library work between replays must not disturb the captured graphs
            c.rescale(dev[:2].contiguous())
            torch.cuda.synchronize()
        assert eng._graphs, "no graph was captured"
    finally:
        c.workspace_freeze(False)


def test_mix_fp64_tolerance():
    """Real weights per (position, w_in, w_out) encoded by the library; every width and depth."""
    from paper_2205_11935_amd.batch_mix import MixEngine
    _need_gpu()
    import paper_2205_11935_amd as ctl
    w = W.LARGE
    c = ctl.Context.for_workload(w)
    queries = W.mix_queries(16)
    keys = c.keygen(w.seed_keys, MixEngine.rotations(queries, W.MIX_T1), relin=True)
    eng = MixEngine(c, keys, lambda p, a, b, t: W.mix_weights(p, a, b), W.MIX_T1, W.MIX_BLOCK, lazy=True)
    items = (c.n // 2) // W.MIX_BLOCK
    xs = W.mix_inputs(queries, items)
    dev = c.empty_ct(len(queries), c.nq)
    for i, q in enumerate(queries):
        m0 = eng.model(0, q.widths[0], q.widths[1])
        c.encrypt(keys, c.encode_items(m0, xs[i]), 700 + i, out=dev[i])
    outs = eng.run(dev, queries)
    q_primes = c.primes[: c.nq]
    for i, q in enumerate(queries):
        scale = c.scale
        for l in range(q.depth - 1):
            scale = scale * scale / q_primes[c.nq - 2 * l - 2]
        k_out = c.nq - 2 * q.depth + 1
        z = c.decode(c.decrypt(keys, outs[i], k_out), scale)
        y = np.stack([z[b * W.MIX_BLOCK: b * W.MIX_BLOCK + q.widths[-1]] for b in range(items)])
        ref = xs[i]
        for l in range(q.depth):
            ref = ref @ W.mix_weights(l, q.widths[l], q.widths[l + 1]).T
            if l + 1 < q.depth:
                ref = ref * ref
        assert normwise_error(y, ref) < 2.0 ** -20, (i, q)


def test_dense_groups_equals_dense_per_model():
    """ctl_dense_groups over banks of all four widths at positions 0 and 1 (groups of 3, 1, 2 and
    2 ciphertexts) equals ctl_dense of each model on its own ciphertexts, bit for bit; a model
    without baby steps over Q*P, or one at another level, is rejected before anything runs."""
    _need_gpu()
    import paper_2205_11935_amd as ctl
    from paper_2205_11935_amd.batch_mix import MixEngine
    c, o, queries, keys, _ = _setup((128, 256, 512, 768), 24)
    eng = MixEngine(c, keys, _raw_bank(o.n), W.MIX_T1, W.MIX_BLOCK, raw=True, lazy=True)
    for pos, shapes in ((0, [(128, 768), (768, 256), (512, 512), (256, 128)]),
                        (1, [(256, 512), (768, 768), (128, 128), (512, 256)])):
        models = [eng.model(pos, a, b) for a, b in shapes]
        counts = [3, 1, 2, 2]
        k = eng.level(pos)
        msgs = W.raw_plaintexts(80 + pos, sum(counts), o.n, bound_bits=40)
        top = c.empty_ct(sum(counts), o.nq)
        for i in range(sum(counts)):
            c.encrypt(keys, msgs[i], 900 + 10 * pos + i, out=top[i])
        x = top[:, :, :k].contiguous()
        got = ctl.to_numpy_u64(c.dense_groups(models, counts, keys, x))
        r0 = 0
        for m, cnt in zip(models, counts):
            want = ctl.to_numpy_u64(c.dense(m, 0, keys, x[r0:r0 + cnt].contiguous()))
            assert np.array_equal(got[r0:r0 + cnt], want), (pos, r0)
            r0 += cnt
    lazy_only = c.load_model_ex([(128, 128, 32, 0)], pts=[_raw_bank(o.n)(0, 128, 128, 128)], lazy=True,
                                block=W.MIX_BLOCK)
    out = c.empty_ct(2, o.nq - 1)
    out.fill_(3)
    x2 = top[:2].contiguous()
    with pytest.raises(ctl.CtlError) as ei:
        c.dense_groups([eng.model(0, 128, 128), lazy_only], [1, 1], keys, x2, out=out)
    assert ei.value.code == -1
    with pytest.raises(ctl.CtlError) as ei:
        c.dense_groups([eng.model(0, 128, 128), eng.model(1, 128, 128)], [1, 1], keys, x2, out=out)
    assert ei.value.code == -3
    torch.cuda.synchronize()
    assert torch.all(out == 3)
