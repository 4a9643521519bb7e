"""GPU tests of the client side and the wire format: seeded symmetric encryption bit-exact against
the oracle, and the whole protocol of Section 3 through serialized messages at CryptoTL_p1 — the
client encrypts, sends c0 and the seed; the server expands, runs the frozen layers and sends the
result back; the client decrypts within the p1 tolerance."""
import numpy as np
import pytest

import workloads as W
from oracle import CKKSOracle, normwise_error
from oracle import cnn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("w", [W.LARGE, W.CNN_P1], ids=["large", "cnn_p1"])
def test_encrypt_sym_bit_exact(w):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_11935_amd as ctl
    c = ctl.Context(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    o = CKKSOracle(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    keys = c.keygen(w.seed_keys, [], relin=False)
    s = o.keygen_secret(w.seed_keys)
    m = W.raw_plaintexts(41, 1, o.n, 40)[0]
    got = ctl.to_numpy_u64(c.encrypt_sym(keys, m, 777))
    assert np.array_equal(got, o.encrypt_sym(s, m, 777))
    assert np.array_equal(ctl.to_numpy_u64(c.expand_seeded(got[0], 777)), got)


def test_protocol_through_the_wire_format_p1():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_11935_amd as ctl
    w = W.CNN_P1
    wire = (w.log2n, w.q_bits, w.p_bits)
    layers = [ctl.Layer.conv1d(w.width, w.f_conv),
              ctl.Layer.dense(w.width, w.width, w.t1, act=ctl.CTL_ACT_POLY3, coef=W.RELU3_COEF),
              ctl.Layer.avgpool(w.width, w.f_pool),
              ctl.Layer.dense(w.pooled, w.pooled, w.t1)]
    taps, w1, w2 = W.cnn_weights(w)
    # client and server hold separate contexts; only bytes pass between them (and the evaluation
    # keys, uploaded once per session)
    client = ctl.Context(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    server = ctl.Context(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    cm = client.load_model(layers, [taps, w1, None, w2], lazy=True, qp=True)
    sm = server.load_model(layers, [taps, w1, None, w2], lazy=True, qp=True)
    ck = client.keygen(w.seed_keys, cm.info.rotations, relin=True)
    sk = server.import_keys(ck.evaluation_keys())
    x = W.cnn_inputs(w, 1, cm.info.items)[0]
    full = client.encrypt_sym(ck, client.encode_items(cm, x), 4242)
    up = ctl.ct_pack(*wire, ctl.to_numpy_u64(full)[:1], seed=4242)
    assert len(up) == ctl.ct_packed_bytes(*wire, len(w.q_bits), 1)
    c0, seed = ctl.ct_unpack(*wire, up)
    ct = server.expand_seeded(c0[0], seed)
    assert torch.equal(ct, full)
    out = server.forward(sm, sk, ct[None])[0]
    down = ctl.ct_pack(*wire, ctl.to_numpy_u64(out))
    assert len(down) == ctl.ct_packed_bytes(*wire, 1, 2)
    res, _ = ctl.ct_unpack(*wire, down)
    y = client.decode_items(cm, client.decrypt(ck, ctl.from_numpy_u64(res), 1))
    ref = np.stack([cnn.forward_fp64(x[b], taps, w1, w2, W.RELU3_COEF, w.f_pool) for b in range(cm.info.items)])
    assert normwise_error(y, ref) < 2.0 ** -8
