"""GPU parity of the paper's frozen CNN layers (Section 3.1 algorithms, Section 4.1 network) at the
two parameter sets of Table 2: every residue bit-exact against the oracle for seeded raw plaintexts,
ciphertext products and the degree-3 activation op by op, and decrypted outputs of the library's
own encoding within the FP64 tolerance of each parameter set."""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import CKKSOracle, normwise_error
from oracle import cnn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _layers(ctl, w):
    return [ctl.Layer.conv1d(w.width, w.f_conv),
            ctl.Layer.dense(w.width, w.width, w.t1, act=ctl.CTL_ACT_POLY3, coef=W.RELU3_COEF),
            ctl.Layer.avgpool(w.width, w.f_pool),
            ctl.Layer.dense(w.pooled, w.pooled, w.t1)]


@functools.lru_cache(maxsize=None)
def _setup(name):
    _need_gpu()
    import paper_2205_11935_amd as ctl
    w = W.CNN_WORKLOADS[name]
    c = ctl.Context(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    o = CKKSOracle(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    p = cnn.plan(o, w.width, w.f_conv, w.f_pool, w.t1, W.RELU3_COEF)
    raw = {"conv": W.raw_plaintexts(w.seed_base + 11, w.f_conv, o.n, 40),
           "dense1": W.raw_plaintexts(w.seed_base + 12, w.width, o.n, 40),
           "pool": W.raw_plaintexts(w.seed_base + 13, 1, o.n, 40)[0],
           "dense2": W.raw_plaintexts(w.seed_base + 14, w.width, o.n, 40)}
    m = c.load_model_raw(_layers(ctl, w), [raw["conv"], raw["dense1"], raw["pool"][None], raw["dense2"]], lazy=True,
                         qp=True)
    keys = c.keygen(w.seed_keys, m.info.rotations, relin=True)
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    okeys = o.keygen_rotations(w.seed_keys, s, p.rotations)
    rlk = o.keygen_relin(w.seed_keys, s)
    return ctl, w, c, o, p, raw, m, keys, (s, pk, okeys, rlk)


@pytest.mark.parametrize("name", ["cnn_p1", "cnn_p2"])
def test_plan_matches_oracle(name):
    ctl, w, c, o, p, raw, m, keys, _ = _setup(name)
    assert c.primes == o.primes
    assert m.info.items == p.items and m.info.block == p.block
    assert m.info.layer_k == [p.k_conv, p.k_dense1, p.k_pool, p.k_dense2]
    assert m.info.k_out == p.k_out == 1
    assert set(m.info.rotations) == set(p.rotations)
    assert m.info.scale_out == p.scale_act_out


@pytest.mark.parametrize("name", ["cnn_p1", "cnn_p2"])
def test_mul_and_poly3_bit_exact(name):
    ctl, w, c, o, p, raw, m, keys, (s, pk, okeys, rlk) = _setup(name)
    k = p.k_act
    g = np.random.Generator(np.random.PCG64(21))
    cts = [o.encrypt(pk, g.integers(-2 ** 40, 2 ** 40, o.n), 300 + i)[:, :k].copy() for i in range(3)]
    dev = ctl.from_numpy_u64(np.stack(cts))
    got = ctl.to_numpy_u64(c.mul(keys, dev[:2].contiguous(), dev[1:].contiguous()))
    for i in range(2):
        assert np.array_equal(got[i], o.mul(cts[i], cts[i + 1], rlk)), i
    out, s3 = c.poly3(keys, dev, p.scale_in, W.RELU3_COEF)
    got = ctl.to_numpy_u64(out)
    for i in range(3):
        want, ws3 = o.poly3(cts[i], p.scale_in, W.RELU3_COEF, rlk)
        assert s3 == ws3
        assert np.array_equal(got[i], want), i


@pytest.mark.parametrize("name", ["cnn_p1", "cnn_p2"])
def test_each_layer_bit_exact(name):
    """Convolution and average pool alone (ctl_dense on their layer index, rotations over Q*P)
    against the oracle."""
    ctl, w, c, o, p, raw, m, keys, (s, pk, okeys, rlk) = _setup(name)
    g = np.random.Generator(np.random.PCG64(22))
    ct = o.encrypt(pk, g.integers(-2 ** 40, 2 ** 40, o.n), 400)
    got = ctl.to_numpy_u64(c.dense(m, 0, keys, ctl.from_numpy_u64(ct[None])))[0]
    conv = np.stack([o.plaintext(x, p.k_conv, ext=True) for x in raw["conv"]])
    assert np.array_equal(got, o.conv1d(ct, conv, okeys, qp=True))
    ct3 = ct[:, : p.k_pool].copy()
    got = ctl.to_numpy_u64(c.dense(m, 2, keys, ctl.from_numpy_u64(ct3[None])))[0]
    assert np.array_equal(got, o.avgpool(ct3, o.plaintext(raw["pool"], p.k_pool, ext=True), p.f_pool, okeys,
                                         qp=True))


@pytest.mark.parametrize("name", ["cnn_p1", "cnn_p2"])
def test_stack_bit_exact(name):
    ctl, w, c, o, p, raw, m, keys, (s, pk, okeys, rlk) = _setup(name)
    g = np.random.Generator(np.random.PCG64(23))
    msgs = [g.integers(-2 ** 40, 2 ** 40, o.n) for _ in range(3)]
    dev = c.empty_ct(3, o.nq)
    for i, mm in enumerate(msgs):
        c.encrypt(keys, mm, 500 + i, out=dev[i])
    got = ctl.to_numpy_u64(c.forward(m, keys, dev))
    assert got.shape == (3, 2, 1, o.n)
    for i in (0, 2):                                   # the oracle takes seconds per ciphertext
        want = cnn.forward(p, o, o.encrypt(pk, msgs[i], 500 + i), raw, okeys, rlk, W.RELU3_COEF, qp=True)
        assert np.array_equal(got[i], want), i


@pytest.mark.parametrize("name,tol", [("cnn_p1", 2.0 ** -8), ("cnn_p2", 2.0 ** -20)])
def test_stack_fp64_tolerance(name, tol):
    """Real weights encoded by the library; p1's Delta = 2^25 leaves about 2^-11 (fresh noise
    2^-10.6 of a unit slot), p2's Delta = 2^50 about 2^-35."""
    _need_gpu()
    import paper_2205_11935_amd as ctl
    w = W.CNN_WORKLOADS[name]
    c = ctl.Context(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    taps, w1, w2 = W.cnn_weights(w)
    m = c.load_model(_layers(ctl, w), [taps, w1, None, w2], lazy=True, qp=True)
    keys = c.keygen(w.seed_keys, m.info.rotations, relin=True)
    n_ct = 4
    x = W.cnn_inputs(w, n_ct, m.info.items)
    dev = c.empty_ct(n_ct, c.nq)
    for i in range(n_ct):
        c.encrypt(keys, c.encode_items(m, x[i]), 600 + i, out=dev[i])
    out = c.forward(m, keys, dev)
    for i in range(n_ct):
        y = c.decode_items(m, c.decrypt(keys, out[i], m.info.k_out))
        ref = np.stack([cnn.forward_fp64(x[i][b], taps, w1, w2, W.RELU3_COEF, w.f_pool) for b in range(m.info.items)])
        assert normwise_error(y, ref) < tol, i
