"""GPU parity: every HIP path result against the CPU oracle on the same seeded inputs.

Integer results (NTT residues, keys, ciphertexts after every homomorphic operation) must be
bit-exact. Decrypted outputs must match the FP64 forward pass normwise within 2^-20 (2^-12 for the
small workload, whose 2^30 scale is noise-limited). Encoding (FP64 -> integer) must agree with the
oracle's to within one unit per coefficient.
"""
import functools
import os

import numpy as np
import pytest

import workloads as W
from oracle import CKKSOracle, normwise_error

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@functools.lru_cache(maxsize=None)
def _ctx(name):
    _need_gpu()
    import paper_2205_11935_amd as ctl
    return ctl.Context.for_workload(W.WORKLOADS[name])


@functools.lru_cache(maxsize=None)
def _orc(name):
    return CKKSOracle.for_workload(W.WORKLOADS[name])


def _u64(t):
    import paper_2205_11935_amd as ctl
    return ctl.to_numpy_u64(t)


def _dev(a):
    import paper_2205_11935_amd as ctl
    return ctl.from_numpy_u64(a)


def _plan(name, lazy=False):
    """lazy: False (one ModDown per giant step), True (single-ModDown giant steps) or "qp" (baby
    steps over Q*P as well)."""
    w = W.WORKLOADS[name]
    return _orc(name).plan([(l.n_in, l.n_out, l.t1) for l in w.layers], lazy=bool(lazy), qp=lazy == "qp")


@functools.lru_cache(maxsize=None)
def _keys(name):
    """Library keys and oracle keys from the same seed (the tests below check they agree)."""
    w = W.WORKLOADS[name]
    o, c = _orc(name), _ctx(name)
    plan = _plan(name)
    rots = plan.rotations + [3, -5]
    lk = c.keygen(w.seed_keys, rots, relin=True)
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    okeys = o.keygen_rotations(w.seed_keys, s, rots)
    rlk = o.keygen_relin(w.seed_keys, s)
    return lk, s, pk, okeys, rlk


def _fresh_ct(name, seed, count=1):
    """count encryptions of random integer messages, on both sides."""
    o, c = _orc(name), _ctx(name)
    lk, s, pk, _, _ = _keys(name)
    msgs = W.raw_plaintexts(seed, count, o.n, bound_bits=40)
    dev = c.empty_ct(count, o.nq)
    ref = []
    for i in range(count):
        c.encrypt(lk, msgs[i], seed * 1000 + i, out=dev[i])
        ref.append(o.encrypt(pk, msgs[i], seed * 1000 + i))
    torch.cuda.synchronize()
    return dev, np.stack(ref)


# ------------------------------------------------------------------ NTT
@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_ntt_forward_inverse_bit_exact(name):
    o, c = _orc(name), _ctx(name)
    rng = np.random.default_rng(1)
    # every prime, ragged residue counts, edge values
    idx = [i % o.np for i in range(2 * o.np + 3)]
    host = np.stack([rng.integers(0, o.primes[p], size=o.n, dtype=np.uint64) for p in idx])
    host[0, :4] = [0, 1, o.primes[idx[0]] - 1, 0]
    host[1, :] = o.primes[idx[1]] - 1
    dev = _dev(host)
    c.ntt(dev, idx, inverse=False)
    got = _u64(dev)
    want = np.stack([o.ntt(host[r], idx[r]) for r in range(len(idx))])
    assert np.array_equal(got, want)
    c.ntt(dev, idx, inverse=True)
    assert np.array_equal(_u64(dev), host)
    back = np.stack([o.ntt(host[r], idx[r], inverse=True) for r in range(len(idx))])
    dev2 = _dev(host)
    c.ntt(dev2, idx, inverse=True)
    assert np.array_equal(_u64(dev2), back)


@pytest.mark.parametrize("name", ["small", "large"])
def test_parity_hooks(name):
    """ctl_ct_export / ctl_ct_import in both forms and ctl_pt_import against the oracle's NTT of the
    same integers; an unreduced word is rejected with nothing written."""
    import paper_2205_11935_amd as ctl
    o, c = _orc(name), _ctx(name)
    rng = np.random.default_rng(5)
    k = o.nq
    coef = np.stack([np.stack([rng.integers(0, o.q[i], size=o.n, dtype=np.uint64) for i in range(k)])
                     for _ in range(2)])
    ntt = np.stack([np.stack([o.ntt(coef[p, i], i) for i in range(k)]) for p in range(2)])
    dev = c.ct_import(coef, coeff=True)
    assert np.array_equal(_u64(dev), ntt)
    assert np.array_equal(c.ct_export(dev), ntt)
    assert np.array_equal(c.ct_export(dev, coeff=True), coef)
    dev2 = c.ct_import(ntt)
    assert np.array_equal(_u64(dev2), ntt)
    bad = ntt.copy()
    bad[1, k - 1, 7] = o.q[k - 1]
    before = _u64(dev2).copy()
    with pytest.raises(ctl.CtlError) as ei:
        c.ct_import(bad, out=dev2)
    assert ei.value.code == -1
    assert np.array_equal(_u64(dev2), before)
    pts = W.raw_plaintexts(77, 3, o.n, bound_bits=45)
    for ext in (False, True):
        got = _u64(c.pt_import(pts, k - 1, ext=ext))
        assert np.array_equal(got, o.bank_ntt(pts, k - 1, ext=ext)), ext


# ------------------------------------------------------------------ keys and encryption
@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_keygen_bit_exact(name):
    o = _orc(name)
    lk, s, pk, okeys, rlk = _keys(name)
    assert np.array_equal(lk.secret(), s)
    assert np.array_equal(lk.public(), pk)
    gl = sorted(lk.galois_elements())
    assert gl == sorted(list(okeys) + [0])
    for g in sorted(okeys)[:3] + sorted(okeys)[-2:]:
        assert np.array_equal(lk.galois_key(g), okeys[g]), g
    assert np.array_equal(lk.galois_key(0), rlk)


@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_encrypt_decrypt_bit_exact(name):
    o, c = _orc(name), _ctx(name)
    lk, s, _, _, _ = _keys(name)
    dev, ref = _fresh_ct(name, 11, count=2)
    assert np.array_equal(_u64(dev), ref)
    for k in (o.nq, 1):
        got = c.decrypt(lk, dev[1, :, :k].contiguous(), k)
        assert np.array_equal(got, o.decrypt(s, np.ascontiguousarray(ref[1][:, :k])))


# ------------------------------------------------------------------ single operations
@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_rescale_bit_exact(name):
    o, c = _orc(name), _ctx(name)
    dev, ref = _fresh_ct(name, 12, count=3)
    for k in (o.nq, 2):
        got = _u64(c.rescale(dev[:, :, :k].contiguous()))
        for b in range(3):
            assert np.array_equal(got[b], o.rescale(np.ascontiguousarray(ref[b][:, :k])))


@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_rotate_bit_exact(name):
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, _ = _keys(name)
    dev, ref = _fresh_ct(name, 13, count=2)
    for r in (1, 3, -5):
        g = o.galois_elt(r)
        for k in (o.nq, 1):
            got = _u64(c.rotate(lk, dev[:, :, :k].contiguous(), r))
            for b in range(2):
                assert np.array_equal(got[b], o.rotate(np.ascontiguousarray(ref[b][:, :k]), okeys[g], g)), (r, k, b)


@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_square_bit_exact(name):
    o, c = _orc(name), _ctx(name)
    lk, _, _, _, rlk = _keys(name)
    dev, ref = _fresh_ct(name, 14, count=2)
    for k in (o.nq, 2):
        got = _u64(c.square(lk, dev[:, :, :k].contiguous()))
        for b in range(2):
            assert np.array_equal(got[b], o.square(np.ascontiguousarray(ref[b][:, :k]), rlk)), (k, b)


@pytest.mark.parametrize("name", ["mid", "large"])
def test_replicate_bit_exact(name):
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, _ = _keys(name)
    plan = _plan(name)
    w = plan.layers[0].next_t
    dev, ref = _fresh_ct(name, 15, count=2)
    k = o.nq - 2
    got = _u64(c.replicate(lk, dev[:, :, :k].contiguous(), w))
    for b in range(2):
        assert np.array_equal(got[b], o.replicate(np.ascontiguousarray(ref[b][:, :k]), w, okeys))


# ------------------------------------------------------------------ dense layer and forward pass
def _raw_model(name, seed=21, lazy=False):
    """The same random integer plaintext banks on both sides."""
    o, c = _orc(name), _ctx(name)
    w = W.WORKLOADS[name]
    plan = _plan(name)
    banks = [W.raw_plaintexts(seed + li, L.t, o.n, bound_bits=45, stream=li) for li, L in enumerate(plan.layers)]
    layers = [(l.n_in, l.n_out, l.t1) for l in w.layers]
    model = c.load_model_raw(layers, banks, lazy=bool(lazy), qp=lazy == "qp")
    banks_ntt = [o.bank_ntt(banks[li], L.k, ext=lazy == "qp") for li, L in enumerate(plan.layers)]
    return model, banks_ntt


@pytest.mark.parametrize("name,lazy", [("small", False), ("mid", False), ("large", False),
                                       ("mid", True), ("large", True),
                                       ("small", "qp"), ("mid", "qp"), ("large", "qp")])
def test_dense_bit_exact(name, lazy):
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, _ = _keys(name)
    plan = _plan(name, lazy)
    model, banks_ntt = _raw_model(name, lazy=lazy)
    assert model.info.items == plan.items and model.info.block == plan.block
    assert model.info.k_out == plan.k_out
    assert sorted(model.info.rotations) == sorted(plan.rotations)
    dev, ref = _fresh_ct(name, 16, count=2)
    for li, L in enumerate(plan.layers):
        x = dev[:, :, :L.k].contiguous()
        got = _u64(c.dense(model, li, lk, x))
        for b in range(2):
            want = o.dense(np.ascontiguousarray(ref[b][:, :L.k]), banks_ntt[li], L.t1, okeys, bool(lazy),
                           qp=lazy == "qp")
            assert np.array_equal(got[b], want), (li, b)


@pytest.mark.parametrize("name,lazy", [("small", False), ("mid", False), ("large", False), ("large", True),
                                       ("mid", "qp"), ("large", "qp")])
def test_forward_bit_exact(name, lazy):
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, rlk = _keys(name)
    plan = _plan(name, lazy)
    model, banks_ntt = _raw_model(name, seed=31, lazy=lazy)
    dev, ref = _fresh_ct(name, 17, count=2)
    got = _u64(c.forward(model, lk, dev))
    assert got.shape == (2, 2, plan.k_out, o.n)
    for b in range(2):
        assert np.array_equal(got[b], o.forward(plan, ref[b], banks_ntt, okeys, rlk)), b


def _oracle_many(fn, items):
    """fn over items on host threads (the C oracle releases the interpreter lock and keeps no
    shared mutable state)."""
    from concurrent.futures import ThreadPoolExecutor
    items = list(items)
    with ThreadPoolExecutor(max_workers=min(8, len(items))) as ex:
        return list(ex.map(fn, items))


# ciphertexts on both sides of the MAC workgroup boundaries: 8 ciphertexts per integer-prime
# (limb) MAC workgroup, 16 per FP64-prime MAC workgroup, and the last one of the batch
BOUNDARY_CTS = (0, 7, 8, 15, 16, 63)


@pytest.mark.parametrize("lazy", [False, True, "qp"])
def test_forward_full_batch(lazy):
    """The large workload's batch of 64 ciphertexts in one launch sequence, as the benchmark times
    it: ciphertexts 0, 7, 8, 15, 16 and 63 equal the oracle's forward pass, and every one of the
    64 equals its own evaluation alone (a batch of one takes the unstaged MAC and one-ciphertext
    key products, so this compares two kernel paths on every ciphertext). For the headline variant
    every value the autotuner may try for each launch knob gives the same batch bit for bit."""
    from paper_2205_11935_amd import autotune
    name = "large"
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, rlk = _keys(name)
    plan = _plan(name, lazy)
    model, banks_ntt = _raw_model(name, seed=41, lazy=lazy)
    B = W.LARGE.batch
    assert B == BOUNDARY_CTS[-1] + 1
    dev, ref = _fresh_ct(name, 18, count=B)
    got = _u64(c.forward(model, lk, dev))
    for b in range(B):
        one = _u64(c.forward(model, lk, dev[b:b + 1].contiguous()))
        assert np.array_equal(one[0], got[b]), b
    if lazy == "qp":
        defaults = {kn: c.knob(kn) for kn in autotune.CANDIDATES}
        try:
            for kn, values in autotune.CANDIDATES.items():
                for v in values:
                    c.knob(kn, v)
                    assert np.array_equal(_u64(c.forward(model, lk, dev)), got), (kn, v)
                c.knob(kn, defaults[kn])
        finally:
            autotune.apply(c, defaults)
    wants = _oracle_many(lambda b: o.forward(plan, ref[b], banks_ntt, okeys, rlk), BOUNDARY_CTS)
    for b, want in zip(BOUNDARY_CTS, wants):
        assert np.array_equal(got[b], want), b


@pytest.mark.parametrize("lazy", [True, "qp"])
def test_forward_ragged_batch(lazy):
    """13 ciphertexts of the mid workload: not a multiple of the MACs' ciphertexts per workgroup
    (8 by default; fewer than 16, the FP64 MAC's largest workgroup), and odd for the key
    product's pairs; ciphertexts 0, 7 and 12 against the oracle, every one against its own
    evaluation alone."""
    name = "mid"
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, rlk = _keys(name)
    plan = _plan(name, lazy)
    model, banks_ntt = _raw_model(name, seed=51, lazy=lazy)
    B = 13
    dev, ref = _fresh_ct(name, 19, count=B)
    got = _u64(c.forward(model, lk, dev))
    for b in (0, 7, 12):
        assert np.array_equal(got[b], o.forward(plan, ref[b], banks_ntt, okeys, rlk)), b
    for b in range(B):
        assert np.array_equal(_u64(c.forward(model, lk, dev[b:b + 1].contiguous()))[0], got[b]), b


@pytest.mark.parametrize("name", ["small", "large"])
def test_split_transforms_equal_one_workgroup_form(name):
    """Launches of few transforms split each one over N/1024 workgroups (the ntt_split knob): a
    forward pass of 1 and 3 ciphertexts and a batch of residue transforms give the same residues
    with splitting on (default) and off."""
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, rlk = _keys(name)
    model, _ = _raw_model(name, seed=31, lazy="qp")
    dev, _ = _fresh_ct(name, 25, count=3)
    rng = np.random.default_rng(9)
    idx = [i % o.np for i in range(2 * o.np + 1)]
    host = np.stack([rng.integers(0, o.primes[p], size=o.n, dtype=np.uint64) for p in idx])
    before = c.knob("ntt_split")
    try:
        outs = {}
        for split in (before, 0):
            c.knob("ntt_split", split)
            res = [_u64(c.forward(model, lk, dev[:1].contiguous())), _u64(c.forward(model, lk, dev))]
            buf = _dev(host)
            c.ntt(buf, idx)
            res.append(_u64(buf))
            c.ntt(buf, idx, inverse=True)
            res.append(_u64(buf))
            outs[split] = res
    finally:
        c.knob("ntt_split", before)
    assert before > 2 * o.np + 1
    for a, b in zip(outs[before], outs[0]):
        assert np.array_equal(a, b)
    assert np.array_equal(outs[0][3], host)


@pytest.mark.parametrize("name", ["small", "large"])
def test_looped_transforms_equal_one_workgroup_form(name):
    """Launches of many transforms run a grid of resident workgroups that loop over them (the
    ntt_loop knob): a forward pass of 16 ciphertexts and 2050 residue transforms (the prime pattern
    ends in a partial period) give the same residues looped (every launch with at least one
    transform per CU in each class) and in the one-workgroup-per-transform form."""
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, rlk = _keys(name)
    model, _ = _raw_model(name, seed=33, lazy="qp")
    dev, _ = _fresh_ct(name, 27, count=16)
    rng = np.random.default_rng(11)
    idx = [i % o.np for i in range(2050)]
    host = np.stack([rng.integers(0, o.primes[p], size=o.n, dtype=np.uint64) for p in idx])
    before = c.knob("ntt_loop")
    try:
        outs, recs = {}, {}
        for loop in (1, 0):
            c.knob("ntt_loop", loop)
            c.profile_enable(True)
            res = [_u64(c.forward(model, lk, dev))]
            recs[loop] = c.profile_read()                # synchronizes the recorded events
            c.profile_enable(False)
            buf = _dev(host)
            c.ntt(buf, idx)
            res.append(_u64(buf))
            c.ntt(buf, idx, inverse=True)
            res.append(_u64(buf))
            outs[loop] = res
    finally:
        c.profile_enable(False)
        c.knob("ntt_loop", before)
    for a, b in zip(outs[1], outs[0]):
        assert np.array_equal(a, b)
    assert np.array_equal(outs[1][2], host)
    # a looped launch is one kernel per prime class, each with a record of its own: the FP64-prime
    # kernels under the _fp families, none of them unlooped (the large chain has both classes, and
    # its 16-ciphertext ModUp has more than one transform per CU of each)
    assert recs[0]["k_modup_fp"][0] == 0 and recs[0]["k_modup"][0] > 0
    if name == "large":
        assert any(q < (1 << 41) for q in c.primes) and any(q >= (1 << 41) for q in c.primes)
        assert recs[1]["k_modup_fp"][0] > 0 and recs[1]["k_modup"][0] > 0


@pytest.mark.parametrize("count,loop", [(1, 0), (16, 0), (128, 1)])
def test_moddown_rescale_one_pass_equals_two(count, loop):
    """The ModDown by P that ends a key switch and the rescale after it, as one pass (the
    fuse_rescale knob) and as two: the same residues for squares of uniform residues at k = n_q and
    k = 2 (the relinearization adds d0, d1: the addend path) and for the forward pass (no addend),
    with the transforms split (1 ciphertext: the split chain, both coefficient rows' inverse top
    passes in the forward top pass's workgroups), one workgroup each (16) and looped (128
    ciphertexts, ntt_loop 1: at least one transform per CU in each class of every launch)."""
    name = "large"
    o, c = _orc(name), _ctx(name)
    lk = _keys(name)[0]
    rng = np.random.default_rng(1000 + count)
    host = np.stack([np.stack([np.stack([rng.integers(0, o.primes[i], size=o.n, dtype=np.uint64)
                                         for i in range(o.nq)]) for _ in range(2)]) for _ in range(count)])
    dev = _dev(host)
    model = None
    if count <= 16:
        model, _ = _raw_model(name, seed=35, lazy="qp")
    before = (c.knob("fuse_rescale"), c.knob("ntt_loop"))
    try:
        outs = {}
        c.knob("ntt_loop", 1 if loop else before[1])
        for fuse in (1, 0):
            c.knob("fuse_rescale", fuse)
            res = [_u64(c.square(lk, dev[:, :, :k].contiguous())) for k in (o.nq, 2)]
            if model is not None:
                res.append(_u64(c.forward(model, lk, dev)))
            outs[fuse] = res
    finally:
        c.knob("fuse_rescale", before[0])
        c.knob("ntt_loop", before[1])
    assert len(outs[1]) == len(outs[0])
    for a, b in zip(outs[1], outs[0]):
        assert a.shape == b.shape and np.array_equal(a, b)


def test_profile_bytes_model():
    """The algorithmic bytes the library records for a key product: one rotation of 3 ciphertexts
    reads 3 k(k+1) digit rows and one key set's 2 k(k+1) key rows and writes 3 2(k+1) rows, N
    words each; families that do not model bytes report 0."""
    name = "mid"
    c = _ctx(name)
    lk = _keys(name)[0]
    dev, _ = _fresh_ct(name, 23, count=3)
    k, n = dev.shape[2], c.n
    c.profile_enable(True)
    try:
        c.rotate(lk, dev, 3)
        torch.cuda.synchronize()
        launches = c.profile_read()
        pb = c.profile_bytes()
    finally:
        c.profile_enable(False)
    # one launch per arithmetic class present among the k + 1 rows (FP64 primes / integer primes),
    # each with the bytes of its own rows
    fams = [f for f in ("k_keyip_fp", "k_keyip") if launches.get(f, (0,))[0]]
    assert fams and all(launches[f][0] == 1 for f in fams) and launches["k_ntt_inv"][0] >= 1
    assert sum(pb[f] for f in fams) == 8.0 * n * (3 * k * (k + 1) + 2 * k * (k + 1) + 3 * 2 * (k + 1))
    assert pb["k_ntt_inv"] == 0.0


def test_forward_key_product_rotation_groups():
    """Hoisted rotations per key-product workgroup (the keyip_rr knob, 1..8; 6 and 8 reach the
    FP64 rows only, the limb rows stop at 4): every setting gives the same residues, the oracle's,
    on the large workload with a batch of 5 (odd for the key product's ciphertext pairs); 63 and 31
    baby rotations leave a short last group for every group size but 1."""
    name, lazy = "large", "qp"
    o, c = _orc(name), _ctx(name)
    lk, _, _, okeys, rlk = _keys(name)
    plan = _plan(name, lazy)
    model, banks_ntt = _raw_model(name, seed=61, lazy=lazy)
    dev, ref = _fresh_ct(name, 20, count=5)
    before = c.knob("keyip_rr")
    try:
        outs = {}
        for rr in (1, 2, 3, 4, 6, 8):
            c.knob("keyip_rr", rr)
            outs[rr] = _u64(c.forward(model, lk, dev))
    finally:
        c.knob("keyip_rr", before)
    for rr in (1, 2, 3, 6, 8):
        assert np.array_equal(outs[rr], outs[4]), rr
    for b in (0, 4):
        assert np.array_equal(outs[4][b], o.forward(plan, ref[b], banks_ntt, okeys, rlk)), b


# ------------------------------------------------------------------ encoding and end-to-end tolerance
@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_encode_matches_oracle(name):
    o, c = _orc(name), _ctx(name)
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, o.n // 2)
    a, b = c.encode(z, o.scale), o.encode(z, o.scale)
    d = np.abs(a - b)
    assert d.max() <= 1
    assert (d != 0).mean() < 1e-3
    dec = c.decode(np.stack([(a % q).astype(np.uint64) for q in o.q[:1]]), o.scale)
    assert np.max(np.abs(dec - z)) < 2.0 ** -20


@pytest.mark.parametrize("name,tol_log2,lazy", [("small", -12, False), ("mid", -20, False), ("large", -20, False),
                                                ("mid", -20, True), ("large", -20, True),
                                                ("mid", -20, "qp"), ("large", -20, "qp")])
def test_forward_fp64_tolerance(name, tol_log2, lazy):
    """Encode real inputs and weights with the library, run ClassifyHE on the GPU, decrypt and
    decode: the result matches the plain FP64 forward pass normwise."""
    w = W.WORKLOADS[name]
    o, c = _orc(name), _ctx(name)
    lk = _keys(name)[0]
    ws = W.weights(w)
    layers = [(l.n_in, l.n_out, l.t1) for l in w.layers]
    model = c.load_model(layers, ws, lazy=bool(lazy), qp=lazy == "qp")
    n_ct = 2
    x = W.inputs(w, n_ct, model.info.items)
    dev = c.empty_ct(n_ct, o.nq)
    for i in range(n_ct):
        c.encrypt(lk, c.encode_items(model, x[i]), w.seed_encrypt + i, out=dev[i])
    out = c.forward(model, lk, dev)
    for i in range(n_ct):
        res = c.decrypt(lk, out[i], model.info.k_out)
        y = c.decode_items(model, res)
        err = normwise_error(y, o.forward_fp64(ws, x[i]))
        assert err < 2.0 ** tol_log2, (i, err)
