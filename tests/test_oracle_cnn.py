"""Pins of the oracle's CNN layers (Section 3.1: 1D convolution, average pooling, the degree-3
ReLU approximation; Section 4.1: the frozen server stack) against independent definitions:
numpy's convolution routines, exact decryption linearity, closed-form special cases and
brute-force polynomial evaluation."""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import CKKSOracle, normwise_error
from oracle import cnn

LOGN, QB, PB, LS = 12, (40, 30, 30, 30, 30), 40, 30


@functools.lru_cache(maxsize=None)
def _small():
    o = CKKSOracle(LOGN, QB, PB, LS)
    s = o.keygen_secret(77)
    pk = o.keygen_public(77, s)
    rots = [r for r in range(-4, 5) if r != 0] + [-1, -2]
    keys = o.keygen_rotations(77, s, sorted(set(rots)))
    rlk = o.keygen_relin(77, s)
    return o, s, pk, keys, rlk


def _enc(o, pk, z, seed, scale=None):
    return o.encrypt(pk, o.encode(z, scale or o.scale), seed)


def _dec(o, s, ct, scale):
    return o.decrypt_decode(s, ct, scale).real


def test_mul_of_equal_operands_equals_square():
    o, s, pk, keys, rlk = _small()
    g = np.random.Generator(np.random.PCG64(1))
    ct = _enc(o, pk, g.uniform(-1, 1, o.n // 2), 3)
    assert np.array_equal(o.mul(ct, ct, rlk), o.square(ct, rlk))


def test_mul_decrypts_to_slot_product():
    o, s, pk, keys, rlk = _small()
    g = np.random.Generator(np.random.PCG64(2))
    a, b = g.uniform(-1, 1, o.n // 2), g.uniform(-1, 1, o.n // 2)
    out = o.mul(_enc(o, pk, a, 4), _enc(o, pk, b, 5), rlk)
    k = o.nq
    got = _dec(o, s, out, o.scale * o.scale / o.q[k - 1])
    assert np.max(np.abs(got - a * b)) < 2.0 ** -14


@pytest.mark.parametrize("mul,add,k_out", [(3, 0, 0), (-7, 12345, 0), (1, -99, 3), (-(2 ** 40) - 1, 2 ** 45, 2)])
def test_affine_is_exact_on_decryptions(mul, add, k_out):
    """Dec(ct * m + a) = m Dec(ct) + a X^0, residue by residue (decryption is linear)."""
    o, s, pk, keys, rlk = _small()
    g = np.random.Generator(np.random.PCG64(6))
    ct = _enc(o, pk, g.uniform(-1, 1, o.n // 2), 7)
    out = o.affine(ct, mul, add, k_out)
    kk = k_out or o.nq
    d_in, d_out = o.decrypt(s, ct), o.decrypt(s, out)
    for i in range(kk):
        q = o.q[i]
        want = [(mul * int(v)) % q for v in d_in[i]]
        want[0] = (want[0] + add) % q
        assert [int(v) for v in d_out[i]] == want


def _cnn_small_plan(width=64, f_conv=9, f_pool=3):
    o = _small()[0]
    block = 2 * width
    return cnn.CnnPlan(width, f_conv, f_pool, 8, block, (o.n // 2) // block, o.nq, 0, 0, 0, 0, 0, o.scale, 0.0, [])


def test_conv1d_matches_numpy_same_convolution():
    o, s, pk, keys, rlk = _small()
    p = _cnn_small_plan()
    g = np.random.Generator(np.random.PCG64(8))
    x = g.uniform(-1, 1, (p.items, p.width))
    taps = g.normal(0, 0.3, p.f_conv)
    ct = _enc(o, pk, cnn.input_slots(p, o, x), 9)
    k = o.nq
    pts = np.stack([o.plaintext(o.encode(cnn.conv_tap_slots(p, o, taps, i), float(o.q[k - 1])), k)
                    for i in range(p.f_conv)])
    z = _dec(o, s, o.conv1d(ct, pts, keys), o.scale)
    for b in range(p.items):
        ref = np.convolve(x[b], taps[::-1], mode="same")          # correlation, 'same' padding
        base = b * p.block
        assert np.max(np.abs(z[base: base + p.width] - ref)) < 2.0 ** -12
        assert np.max(np.abs(z[base + p.width: base + 2 * p.width] - ref)) < 2.0 ** -12


def test_conv1d_single_tap_is_one_plaintext_product():
    o, s, pk, keys, rlk = _small()
    g = np.random.Generator(np.random.PCG64(10))
    ct = _enc(o, pk, g.uniform(-1, 1, o.n // 2), 11)
    k = o.nq
    pt = o.plaintext(o.encode(g.uniform(-1, 1, o.n // 2), float(o.q[k - 1])), k)
    prod = np.zeros_like(ct)
    for p_ in range(2):
        for i in range(k):
            q = o.q[i]
            prod[p_, i] = np.array([(int(a) * int(b)) % q for a, b in zip(ct[p_, i], pt[i])], dtype=np.uint64)
    assert np.array_equal(o.conv1d(ct, pt[None], keys), o.rescale(prod))


def test_avgpool_matches_numpy_valid_mean():
    o, s, pk, keys, rlk = _small()
    p = _cnn_small_plan()
    g = np.random.Generator(np.random.PCG64(12))
    x = g.uniform(-1, 1, (p.items, p.width))
    ct = _enc(o, pk, cnn.input_slots(p, o, x), 13)
    k = o.nq
    pt = o.plaintext(o.encode(cnn.pool_slots(p, o), float(o.q[k - 1])), k)
    z = _dec(o, s, o.avgpool(ct, pt, p.f_pool, keys), o.scale)
    for b in range(p.items):
        base = b * p.block
        ref = np.convolve(x[b], np.ones(p.f_pool) / p.f_pool, mode="valid")
        assert np.max(np.abs(z[base + p.f_pool - 1: base + p.width] - ref)) < 2.0 ** -12
        assert np.max(np.abs(z[base: base + p.f_pool - 1])) < 2.0 ** -12       # cleared by the mask
        assert np.max(np.abs(z[base + p.width: base + p.block])) < 2.0 ** -12


# ------------------------------------------------------------------ rotations kept over Q*P
def _unit_pts(o, k, f, i, ext):
    raw = np.zeros((f, o.n), dtype=np.int64)
    raw[i, 0] = 1
    return np.stack([o.plaintext(m, k, ext) for m in raw])


@pytest.mark.parametrize("i", [0, 3, 4, 8])
def test_conv1d_qp_with_a_unit_tap_equals_plain_rotation(i):
    """One tap equal to 1, the others 0: the Q*P sum is ct~_{i-4}, whose ModDown is exactly
    rot_{i-4}(ct), so both variants give the same bits."""
    o, s, pk, keys, rlk = _small()
    g = np.random.Generator(np.random.PCG64(31))
    ct = _enc(o, pk, g.uniform(-1, 1, o.n // 2), 32)
    k = o.nq
    a = o.conv1d(ct, _unit_pts(o, k, 9, i, False), keys)
    b = o.conv1d(ct, _unit_pts(o, k, 9, i, True), keys, qp=True)
    assert np.array_equal(a, b)


def test_conv1d_and_pool_qp_single_term_equal_plain():
    """f = 1: the only term is P ct, which ModDown returns exactly, for any plaintext."""
    o, s, pk, keys, rlk = _small()
    g = np.random.Generator(np.random.PCG64(33))
    ct = _enc(o, pk, g.uniform(-1, 1, o.n // 2), 34)
    k = o.nq
    m = o.encode(g.uniform(-1, 1, o.n // 2), float(o.q[k - 1]))
    assert np.array_equal(o.conv1d(ct, o.plaintext(m, k)[None], keys),
                          o.conv1d(ct, o.plaintext(m, k, True)[None], keys, qp=True))
    assert np.array_equal(o.avgpool(ct, o.plaintext(m, k), 1, keys),
                          o.avgpool(ct, o.plaintext(m, k, True), 1, keys, qp=True))


def test_conv1d_and_pool_qp_match_numpy():
    o, s, pk, keys, rlk = _small()
    p = _cnn_small_plan()
    g = np.random.Generator(np.random.PCG64(35))
    x = g.uniform(-1, 1, (p.items, p.width))
    taps = g.normal(0, 0.3, p.f_conv)
    ct = _enc(o, pk, cnn.input_slots(p, o, x), 36)
    k = o.nq
    pts = np.stack([o.plaintext(o.encode(cnn.conv_tap_slots(p, o, taps, i), float(o.q[k - 1])), k, True)
                    for i in range(p.f_conv)])
    z = _dec(o, s, o.conv1d(ct, pts, keys, qp=True), o.scale)
    ptp = o.plaintext(o.encode(cnn.pool_slots(p, o), float(o.q[k - 1])), k, True)
    zp = _dec(o, s, o.avgpool(ct, ptp, p.f_pool, keys, qp=True), o.scale)
    for b in range(p.items):
        base = b * p.block
        ref = np.convolve(x[b], taps[::-1], mode="same")
        assert np.max(np.abs(z[base: base + p.width] - ref)) < 2.0 ** -12
        refp = np.convolve(x[b], np.ones(p.f_pool) / p.f_pool, mode="valid")
        assert np.max(np.abs(zp[base + p.f_pool - 1: base + p.width] - refp)) < 2.0 ** -12


@pytest.mark.parametrize("coef", [(0.75, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), W.RELU3_COEF,
                                  (-0.3, 0.2, -0.05, 0.01)])
def test_poly3_evaluates_the_polynomial(coef):
    """Each monomial alone (closed forms: constant, z, z^2, z^3), the printed ReLU approximation and
    a mixed cubic, against direct evaluation on the encrypted values."""
    o, s, pk, keys, rlk = _small()
    g = np.random.Generator(np.random.PCG64(14))
    z = g.uniform(-4, 5, o.n // 2)
    ct = _enc(o, pk, z, 15)
    out, s3 = o.poly3(ct, o.scale, coef, rlk)
    assert out.shape[1] == o.nq - 2
    got = _dec(o, s, out, s3)
    ref = coef[0] + coef[1] * z + coef[2] * z ** 2 + coef[3] * z ** 3
    # measured 2^-15.3 .. 2^-16.7 (fresh noise at 2^30); a scale off by q/Delta (about 2^-13.6 here) fails
    assert np.max(np.abs(got - ref)) < 2.0 ** -14 * max(1.0, np.max(np.abs(ref)))


def test_relu3_coefficients_are_the_cubic_through_relu_points():
    """The printed coefficients agree with -(z+1)(z+4)(z-20)/162, the cubic that meets ReLU at
    z = -4, -1, 2, 5, to the five digits printed."""
    c = np.array(W.RELU3_COEF)
    exact = np.array([40 / 81, 16 / 27, 5 / 54, -1 / 162])
    assert np.max(np.abs(c - exact) / np.abs(exact)) < 1e-4
    for zz in (-4.0, -1.0, 2.0, 5.0):
        assert abs(np.polyval(c[::-1], zz) - max(zz, 0.0)) < 1e-3


def test_fp64_stack_matches_numpy_routines():
    g = np.random.Generator(np.random.PCG64(16))
    n, f = 40, 9
    x, taps = g.normal(size=n), g.normal(size=f)
    w1, w2 = g.normal(size=(n, n)), g.normal(size=(n - 2, n - 2))
    y = w1 @ np.convolve(x, taps[::-1], mode="same")
    a = np.polyval(np.array(W.RELU3_COEF)[::-1], y)
    ref = w2 @ np.convolve(a, np.ones(3) / 3, mode="valid")
    got = cnn.forward_fp64(x, taps, w1, w2, W.RELU3_COEF, 3)
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("qp", [False, True])
def test_frozen_stack_p1_end_to_end(qp):
    """The whole frozen stack at CryptoTL_p1 (N = 2^13, Delta = 2^25, 2 items) against FP64, with
    every hoisted rotation lowered per rotation or kept over Q*P. Fresh encryption noise alone is
    about 2^-10.6 of a unit slot at this scale; measured 2^-11."""
    w = W.CNN_P1
    o = CKKSOracle(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)
    assert sum(x.bit_length() for x in o.primes) == 218            # Table 2's log2 q
    p = cnn.plan(o, w.width, w.f_conv, w.f_pool, w.t1, W.RELU3_COEF)
    assert p.items == 2                                             # Table 2's p
    taps, w1, w2 = W.cnn_weights(w)
    raw = cnn.banks(p, o, taps, w1, w2)
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    keys = o.keygen_rotations(w.seed_keys, s, p.rotations)
    rlk = o.keygen_relin(w.seed_keys, s)
    x = W.cnn_inputs(w, 1, p.items)[0]
    ct = o.encrypt(pk, o.encode(cnn.input_slots(p, o, x), o.scale), 11)
    out = cnn.forward(p, o, ct, raw, keys, rlk, W.RELU3_COEF, qp=qp)
    assert out.shape == (2, 1, o.n)
    y = cnn.output_values(p, o.decrypt_decode(s, out, p.scale_act_out), w.pooled)
    ref = np.stack([cnn.forward_fp64(x[b], taps, w1, w2, W.RELU3_COEF, w.f_pool) for b in range(p.items)])
    assert normwise_error(y, ref) < 2.0 ** -8
