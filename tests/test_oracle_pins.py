"""Pins of the CPU oracle against independent definitions (no GPU).

Each test checks the oracle against something other than itself: a textbook definition written
with Python integers (oracle/bigint.py), a published test vector, an algebraic law, a closed-form
noise bound, or the FP64 matrix product the paper's Eq. (1) must reproduce.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import CKKSOracle, bigint, chacha20_block, find_primes, min_psi, normwise_error

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def tiny():
    # N = 2^6 with one 30-bit, one 40-bit and one 60-bit ciphertext prime, special prime 61 bits
    return CKKSOracle(6, (30, 40, 60), 61, 20)


def _rand_res(rng, q, n):
    return rng.integers(0, q, size=n, dtype=np.uint64, endpoint=False)


# ------------------------------------------------------------------ primes and roots
@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_primes_definition(name):
    w = W.WORKLOADS[name]
    o = CKKSOracle.for_workload(w)
    bits = list(w.q_bits) + [w.p_bits]
    two_n = 2 * o.n
    assert len(set(o.primes)) == len(o.primes)
    for i, (q, b) in enumerate(zip(o.primes, bits)):
        assert bigint.is_prime(q)
        assert q % two_n == 1
        assert q.bit_length() == b
        # maximality: every larger candidate below 2^b is composite or taken earlier
        c = (1 << b) - two_n + 1
        while c > q:
            assert (not bigint.is_prime(c)) or c in o.primes[:i]
            c -= two_n


def test_primes_survey_values():
    # the large workload's chain begins and ends with these (found independently by hand)
    p = find_primes(14, [60, 40, 40, 40, 40, 60, 60])
    assert p[0] == 0xffffffffffe8001 and p[1] == 0xffffe80001 and p[6] == 0xffffffffffc0001


@pytest.mark.parametrize("logn", [4, 6, 12])
def test_psi_minimal_primitive(logn):
    n = 1 << logn
    for q in find_primes(logn, [30, 40, 60]):
        psi = min_psi(q, logn)
        assert pow(psi, n, q) == q - 1
        roots = [pow(psi, e, q) for e in range(1, 2 * n, 2)]   # all primitive 2N-th roots
        assert psi == min(roots)
        assert len(set(roots)) == n


# ------------------------------------------------------------------ NTT
@pytest.mark.parametrize("logn", [2, 3, 5, 8])
def test_ntt_matches_quadratic_definition(logn):
    o = CKKSOracle(logn, (30, 40, 60), 61, 20)
    rng = np.random.default_rng(logn)
    for pi, q in enumerate(o.primes):
        a = _rand_res(rng, q, o.n)
        a[0], a[-1] = q - 1, 0
        got = o.ntt(a, pi)
        assert [int(x) for x in got] == bigint.ntt_definition([int(x) for x in a], q, o.psis[pi])


@pytest.mark.parametrize("logn", [2, 4, 6])
def test_ntt_convolution_theorem(logn):
    o = CKKSOracle(logn, (30, 60), 61, 20)
    rng = np.random.default_rng(100 + logn)
    for pi, q in enumerate(o.primes):
        a, b = _rand_res(rng, q, o.n), _rand_res(rng, q, o.n)
        lhs = [(int(x) * int(y)) % q for x, y in zip(o.ntt(a, pi), o.ntt(b, pi))]
        prod = bigint.negacyclic_product([int(x) for x in a], [int(x) for x in b], q)
        assert lhs == [int(x) for x in o.ntt(np.array(prod, dtype=np.uint64), pi)]


@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_ntt_roundtrip(name):
    o = CKKSOracle.for_workload(W.WORKLOADS[name])
    rng = np.random.default_rng(7)
    for pi, q in enumerate(o.primes):
        a = _rand_res(rng, q, o.n)
        a[:3] = [0, 1, q - 1]
        assert np.array_equal(o.ntt(o.ntt(a, pi), pi, inverse=True), a)
        assert np.array_equal(o.ntt(o.ntt(a, pi, inverse=True), pi), a)


# ------------------------------------------------------------------ automorphisms
def test_automorphism_definition_and_laws(tiny):
    o = tiny
    rng = np.random.default_rng(3)
    two_n = 2 * o.n
    for pi, q in enumerate(o.primes):
        a = _rand_res(rng, q, o.n)
        for g in (3, 5, 25, two_n - 1, o.galois_elt(-3)):
            coef = o.automorph_coef(a, pi, g)
            assert [int(x) for x in coef] == bigint.automorph_definition([int(x) for x in a], g, q)
            # NTT-domain gather equals the NTT of the coefficient-domain automorphism
            assert np.array_equal(o.automorph_ntt(o.ntt(a, pi), g), o.ntt(coef, pi))
        # composition law sigma_g o sigma_h = sigma_{gh mod 2N}
        g, h = 5, 3 * 5 % two_n
        lhs = o.automorph_coef(o.automorph_coef(a, pi, h), pi, g)
        assert np.array_equal(lhs, o.automorph_coef(a, pi, g * h % two_n))


def test_galois_elements(tiny):
    o = tiny
    two_n, half = 2 * o.n, o.n // 2
    assert o.galois_elt(0) == 1 and o.galois_elt(1) == 5 and o.galois_elt(2) == 25
    for r in range(1, half):
        assert o.galois_elt(r) * o.galois_elt(-r) % two_n == 1
    assert o.galois_elt(half) == 1   # 5 has order N/2 modulo 2N


def test_rotation_direction_in_slots():
    # decode(sigma_{5^r}(encode z)) is z rotated LEFT by r (the paper's rot_j, Section 3.1)
    o = CKKSOracle(8, (40, 40), 60, 30)
    rng = np.random.default_rng(5)
    z = rng.uniform(-1, 1, o.n // 2)
    m = o.encode(z, 2.0 ** 30)
    for r in (1, 3, -2, 17):
        g = o.galois_elt(r)
        mg = [int(x) for x in bigint.automorph_definition([int(x) for x in m], g, 1 << 62)]
        mg = [x - (1 << 62) if x >= (1 << 61) else x for x in mg]
        zz = o.decode_coeffs(mg, 2.0 ** 30).real
        assert np.max(np.abs(zz - np.roll(z, -r))) < 1e-6


# ------------------------------------------------------------------ encoding
def test_encode_matches_direct_evaluation():
    o = CKKSOracle(5, (40,), 60, 30)
    rng = np.random.default_rng(11)
    z = rng.uniform(-1, 1, o.n // 2)
    m = o.encode_real(z)
    zeta = np.exp(1j * np.pi / o.n)
    for j, e in enumerate(o.slot_exponents()):
        val = sum(m[k] * zeta ** (int(e) * k) for k in range(o.n))
        assert abs(val - z[j]) < 1e-12


def test_encode_decode_roundtrip():
    o = CKKSOracle.for_workload(W.MID)
    rng = np.random.default_rng(12)
    z = rng.uniform(-1, 1, o.n // 2)
    dec = o.decode_coeffs(o.encode(z, o.scale), o.scale)
    assert np.max(np.abs(dec.real - z)) < 2.0 ** -30
    assert np.max(np.abs(dec.imag)) < 2.0 ** -30


# ------------------------------------------------------------------ randomness
def test_chacha20_rfc8439_vector():
    rec = {}
    for line in open(os.path.join(GOLDEN, "chacha20_block.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        rec[k] = v
    key = [int(x, 16) for x in rec["key"]]
    nonce = [int(x, 16) for x in rec["nonce"]]
    out = chacha20_block(key, int(rec["counter"][0]), nonce)
    assert out.hex() == rec["out"][0]


def test_gaussian_table_and_moments():
    o = CKKSOracle.for_workload(W.SMALL)
    cdt = [int(x) for x in o.cdt()]
    sigma = 3.2
    rho = [math.exp(-(e * e) / (2 * sigma * sigma)) for e in range(-19, 20)]
    tot = math.fsum(rho)
    for m in range(39):
        c = math.fsum(rho[: m + 1]) / tot
        assert abs(cdt[m] / 2.0 ** 53 - c) < 1e-14
    assert cdt == sorted(cdt) and cdt[-1] == 1 << 53
    e = o.sample(42, 3, 0, 1, 0, 200000)
    assert e.min() >= -19 and e.max() <= 19
    assert abs(e.mean()) < 0.05
    assert abs(e.var() / sigma ** 2 - 1) < 0.02


def test_ternary_and_uniform_samplers():
    o = CKKSOracle.for_workload(W.SMALL)
    s = o.sample(9, 1, 0, 0, 0, 300000)
    counts = np.array([(s == v).sum() for v in (-1, 0, 1)])
    assert set(np.unique(s)) <= {-1, 0, 1}
    assert np.all(np.abs(counts / len(s) - 1 / 3) < 0.005)
    q = o.q[1]
    u = o.sample(9, 2, 0, 2, q, 200000).astype(np.uint64)
    assert int(u.max()) < q
    hist = np.histogram(u.astype(np.float64) / q, bins=16, range=(0, 1))[0]
    assert np.all(np.abs(hist / len(u) - 1 / 16) < 0.004)
    # different purpose tags and indices give different streams
    assert not np.array_equal(o.sample(9, 1, 0, 0, 0, 64), o.sample(9, 1, 1, 0, 0, 64))


# ------------------------------------------------------------------ exact rounding steps
def test_moddown_is_rounded_division(tiny):
    o = tiny
    rng = np.random.default_rng(21)
    k = o.nq
    mods = o.q + [o.P]
    # a random pair over Q * P given by coefficient residues
    coef = np.stack([np.stack([_rand_res(rng, m, o.n) for m in mods]) for _ in range(2)])
    coef[0, :, 0] = 0
    u = np.stack([np.stack([o.ntt(coef[p, i], i if i < k else k) for i in range(k + 1)])
                  for p in range(2)])
    got = o.moddown(u)
    for p in range(2):
        res = np.stack([o.ntt(got[p, i], i, inverse=True) for i in range(k)])
        for x in range(o.n):
            X = bigint.crt([int(coef[p, i, x]) for i in range(k + 1)], mods)
            want = bigint.round_div(X, o.P)
            for i in range(k):
                assert int(res[i, x]) == want % o.q[i]


def test_rescale_is_rounded_division(tiny):
    o = tiny
    rng = np.random.default_rng(22)
    k = o.nq
    coef = np.stack([np.stack([_rand_res(rng, m, o.n) for m in o.q]) for _ in range(2)])
    ct = np.stack([np.stack([o.ntt(coef[p, i], i) for i in range(k)]) for p in range(2)])
    got = o.rescale(ct)
    for p in range(2):
        res = np.stack([o.ntt(got[p, i], i, inverse=True) for i in range(k - 1)])
        for x in range(o.n):
            X = bigint.crt([int(coef[p, i, x]) for i in range(k)], o.q)
            want = bigint.round_div(X, o.q[k - 1])
            for i in range(k - 1):
                assert int(res[i, x]) == want % o.q[i]


def test_modup_digits_are_centered_lifts(tiny):
    o = tiny
    rng = np.random.default_rng(23)
    k = o.nq
    coef = np.stack([_rand_res(rng, q, o.n) for q in o.q])
    d = np.stack([o.ntt(coef[i], i) for i in range(k)])
    dig = o.modup(d)
    mods = o.q + [o.P]
    for j in range(k):
        for t in range(k + 1):
            pi = t if t < k else k
            res = o.ntt(dig[j, t], pi, inverse=True)
            want = [bigint.centered(int(v), o.q[j]) % mods[t] for v in coef[j]]
            assert [int(v) for v in res] == want


# ------------------------------------------------------------------ encryption and key switching
@pytest.fixture(scope="module")
def mid_keys():
    w = W.MID
    o = CKKSOracle.for_workload(w)
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    return o, s, pk


def test_decrypt_encrypt_noise(mid_keys):
    o, s, pk = mid_keys
    rng = np.random.default_rng(31)
    m = rng.integers(-2 ** 40, 2 ** 40, size=o.n, dtype=np.int64)
    ct = o.encrypt(pk, m, 77)
    got = np.array(o.compose(o.decrypt(s, ct)), dtype=object)
    noise = np.array([int(a) - int(b) for a, b in zip(got, m)], dtype=np.float64)
    var = 3.2 ** 2 * (4 * o.n / 3 + 1)
    assert 0.85 < noise.var() / var < 1.15
    assert np.max(np.abs(noise)) < 8 * math.sqrt(var)


def test_keyswitch_of_zero_is_zero(mid_keys):
    o, s, pk = mid_keys
    key = o.keygen_galois(5, s, 5)
    for k in (1, 2, o.nq):
        out = o.keyswitch(np.zeros((k, o.n), dtype=np.uint64), key)
        assert not out.any()


def test_rotation_decrypts_to_rotated_slots(mid_keys):
    o, s, pk = mid_keys
    rng = np.random.default_rng(32)
    z = rng.uniform(-1, 1, o.n // 2)
    ct = o.encrypt(pk, o.encode(z, o.scale), 78)
    for r in (1, 7, -33):
        g = o.galois_elt(r)
        key = o.keygen_galois(5, s, g)
        for k in (o.nq, 2):
            dec = o.decrypt_decode(s, o.rotate(ct[:, :k], key, g), o.scale).real
            assert np.max(np.abs(dec - np.roll(z, -r))) < 2.0 ** -20


def test_hoisted_rotation_equals_unhoisted(mid_keys):
    o, s, pk = mid_keys
    rng = np.random.default_rng(33)
    m = rng.integers(-2 ** 40, 2 ** 40, size=o.n, dtype=np.int64)
    ct = o.encrypt(pk, m, 79)
    for k in (o.nq, 3):
        c = np.ascontiguousarray(ct[:, :k])
        dig = o.modup(np.ascontiguousarray(c[1]))
        for r in (1, 5, -128):
            g = o.galois_elt(r)
            key = o.keygen_galois(5, s, g)
            assert np.array_equal(o.rotate_hoisted(c, dig, key, g), o.rotate(c, key, g))


def test_square_relin_rescale(mid_keys):
    o, s, pk = mid_keys
    rng = np.random.default_rng(34)
    z = rng.uniform(-1, 1, o.n // 2)
    ct = o.encrypt(pk, o.encode(z, o.scale), 80)
    rlk = o.keygen_relin(5, s)
    k = o.nq - 1          # one level down, where the plan squares (rescale drops a 40-bit prime)
    out = o.square(np.ascontiguousarray(ct[:, :k]), rlk)
    assert out.shape == (2, k - 1, o.n)
    dec = o.decrypt_decode(s, out, o.scale * o.scale / o.q[k - 1]).real
    assert np.max(np.abs(dec - z * z)) < 2.0 ** -20


# ------------------------------------------------------------------ the dense layer (Eq. (1))
@pytest.mark.parametrize("n_in,n_out,t1", [(64, 64, 64), (512, 128, 32), (128, 128, 16), (20, 12, 4)])
def test_bsgs_identity_in_slots(n_in, n_out, t1):
    """FP64 slot-level evaluation of Eq. (1) with the oracle's diagonal plaintexts and [x|x]
    layout gives [Mx | 0] in every block."""
    o = CKKSOracle(13, (40, 40), 60, 30)
    plan = o.plan([(n_in, n_out, t1)])
    layer = plan.layers[0]
    rng = np.random.default_rng(n_in + n_out)
    w = rng.normal(0, 0.1, (n_out, n_in))
    x = rng.uniform(-1, 1, (plan.items, n_in))
    z = o.input_slots(plan, x)
    acc = np.zeros_like(z)
    for k2 in range(layer.t2):
        inner = np.zeros_like(z)
        for j in range(layer.t1):
            inner += o.diag_slots(plan, layer, w, k2 * layer.t1 + j) * np.roll(z, -j)
        acc += np.roll(inner, -k2 * layer.t1)
    for b in range(plan.items):
        blk = acc[b * plan.block: (b + 1) * plan.block]
        assert np.allclose(blk[:n_out], w @ x[b], atol=1e-12)
        assert np.allclose(blk[n_out:], 0, atol=1e-12)


def test_rotation_counts_and_layout():
    """t1 + t2 - 2 rotations per dense layer (Section 3.1, Dense-Layer) and the Table 2 packing."""
    o = CKKSOracle.for_workload(W.LARGE)
    plan = o.plan([(l.n_in, l.n_out, l.t1) for l in W.LARGE.layers])
    for layer in plan.layers:
        rots = list(range(1, layer.t1)) + [k2 * layer.t1 for k2 in range(1, layer.t2)]
        assert len(rots) == layer.t1 + layer.t2 - 2
    assert plan.layers[0].t1 + plan.layers[0].t2 - 2 == 74          # 768 = 64 x 12 (the split's reading)
    spec = json.load(open(os.path.join(GOLDEN, "table2_layout.json")))
    for case in spec["cases"]:
        o2 = CKKSOracle(int(math.log2(case["n"])), (40, 40), 60, 30)
        p = o2.plan([(spec["neurons"], spec["neurons"], 32)])
        assert p.items == case["p"]


@pytest.mark.parametrize("name,tol_log2", [("small", -12), ("mid", -20), ("large", -20)])
def test_forward_matches_fp64(name, tol_log2):
    """Decrypted encrypted forward pass vs the plain FP64 forward pass, normwise."""
    w = W.WORKLOADS[name]
    o = CKKSOracle.for_workload(w)
    plan = o.plan([(l.n_in, l.n_out, l.t1) for l in w.layers])
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    keys = o.keygen_rotations(w.seed_keys, s, plan.rotations)
    rlk = o.keygen_relin(w.seed_keys, s)
    ws = W.weights(w)
    x = W.inputs(w, 1, plan.items)[0]
    ct = o.encrypt(pk, o.encode(o.input_slots(plan, x), o.scale), w.seed_encrypt)
    banks = [o.bank_ntt(o.layer_bank(plan, li, ws[li]), plan.layers[li].k) for li in range(len(ws))]
    out = o.forward(plan, ct, banks, keys, rlk)
    assert out.shape == (2, plan.k_out, o.n)
    y = o.output_slots(plan, o.decrypt_decode(s, out, plan.scales[-1]))
    err = normwise_error(y, o.forward_fp64(ws, x))
    assert err < 2.0 ** tol_log2


# ------------------------------------------------------------------ single-ModDown giant steps
@pytest.mark.parametrize("name", ["small", "mid"])
def test_lazy_giant_steps_differ_only_by_rounding(name):
    """One ModDown of the summed giant-step key products vs one per giant step: before the final
    rescale each coefficient of each ciphertext polynomial differs by at most t2 - 1 (the per-step
    roundings to nearest, at most 1/2 each, against one rounding of the sum); after the rescale the
    decrypted coefficients differ by at most one; with t2 = 1 the variants are the same computation."""
    w = W.WORKLOADS[name]
    o = CKKSOracle.for_workload(w)
    plan = o.plan([(l.n_in, l.n_out, l.t1) for l in w.layers])
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    keys = o.keygen_rotations(w.seed_keys, s, plan.rotations)
    layer = plan.layers[0]
    bank = W.raw_plaintexts(5, layer.t, o.n, bound_bits=40)
    pts = o.bank_ntt(bank, layer.k)
    ct = o.encrypt(pk, W.raw_plaintexts(6, 1, o.n)[0], 7)
    a = o.dense(ct, pts, layer.t1, keys, lazy=False)
    b = o.dense(ct, pts, layer.t1, keys, lazy=True)
    if layer.t2 == 1:
        assert np.array_equal(a, b)
        return
    da = o.compose(o.decrypt(s, a))
    db = o.compose(o.decrypt(s, b))
    assert max(abs(x - y) for x, y in zip(da, db)) <= 1
    # before the rescale: the sums themselves
    a0 = o.dense(ct, pts, layer.t1, keys, lazy=False, rescale=False)
    b0 = o.dense(ct, pts, layer.t1, keys, lazy=True, rescale=False)
    assert not np.array_equal(a0, b0)
    for poly in range(2):
        diff = np.stack([o.ntt((a0[poly, i] + (o.q[i] - b0[poly, i])) % np.uint64(o.q[i]), i, inverse=True)
                         for i in range(layer.k)])
        d = o.compose(diff)
        assert max(abs(v) for v in d) <= layer.t2 - 1


@pytest.mark.parametrize("name,tol_log2", [("mid", -20), ("large", -20)])
def test_forward_lazy_giant_matches_fp64(name, tol_log2):
    w = W.WORKLOADS[name]
    o = CKKSOracle.for_workload(w)
    plan = o.plan([(l.n_in, l.n_out, l.t1) for l in w.layers], lazy=True)
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    keys = o.keygen_rotations(w.seed_keys, s, plan.rotations)
    rlk = o.keygen_relin(w.seed_keys, s)
    ws = W.weights(w)
    x = W.inputs(w, 1, plan.items)[0]
    ct = o.encrypt(pk, o.encode(o.input_slots(plan, x), o.scale), w.seed_encrypt)
    banks = [o.bank_ntt(o.layer_bank(plan, li, ws[li]), plan.layers[li].k) for li in range(len(ws))]
    out = o.forward(plan, ct, banks, keys, rlk)
    y = o.output_slots(plan, o.decrypt_decode(s, out, plan.scales[-1]))
    assert normwise_error(y, o.forward_fp64(ws, x)) < 2.0 ** tol_log2


# ------------------------------------------------------------------ baby steps over Q*P
def _qp_setup(rots):
    o = CKKSOracle.for_workload(W.SMALL)
    s = o.keygen_secret(41)
    pk = o.keygen_public(41, s)
    keys = o.keygen_rotations(41, s, rots)
    ct = o.encrypt(pk, W.raw_plaintexts(42, 1, o.n)[0], 43)
    return o, s, keys, ct


def test_qp_baby_steps_without_baby_rotations_equal_lazy():
    """t1 = 1: the only baby term is P ct, whose ModDown is ct exactly, so every giant step sees
    the same c1 and the final ModDown absorbs the P multiples exactly: the Q*P variant must equal
    the single-ModDown variant bit for bit (a check of its giant steps and final sum)."""
    t = 8
    o, s, keys, ct = _qp_setup(list(range(1, t)))
    bank = W.raw_plaintexts(44, t, o.n, bound_bits=40)
    k = o.nq
    for rescale in (False, True):
        a = o.dense(ct, o.bank_ntt(bank, k), 1, keys, lazy=True, rescale=rescale)
        b = o.dense(ct, o.bank_ntt(bank, k, ext=True), 1, keys, rescale=rescale, qp=True)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("j", [0, 1, 5, 7])
def test_qp_unit_diagonal_selects_one_rotation(j):
    """t2 = 1 and every plaintext zero except pt_j = 1: the output before the rescale is
    ModDown(ct~_j), which must be the rotation rot_j(ct) computed by the plain (unhoisted) key
    switch, bit for bit (ModDown of P sigma(c0) is sigma(c0) exactly); j = 0 gives ct itself."""
    t1 = 8
    o, s, keys, ct = _qp_setup(list(range(1, t1)))
    k = o.nq
    raw = np.zeros((t1, o.n), dtype=np.int64)
    raw[j, 0] = 1
    out = o.dense(ct, o.bank_ntt(raw, k, ext=True), t1, keys, rescale=False, qp=True)
    if j == 0:
        assert np.array_equal(out, ct)
    else:
        g = o.galois_elt(j)
        assert np.array_equal(out, o.rotate(ct, keys[g], g))


@pytest.mark.parametrize("name,tol_log2", [("mid", -20), ("large", -20)])
def test_forward_qp_baby_steps_matches_fp64(name, tol_log2):
    w = W.WORKLOADS[name]
    o = CKKSOracle.for_workload(w)
    plan = o.plan([(l.n_in, l.n_out, l.t1) for l in w.layers], lazy=True, qp=True)
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    keys = o.keygen_rotations(w.seed_keys, s, plan.rotations)
    rlk = o.keygen_relin(w.seed_keys, s)
    ws = W.weights(w)
    x = W.inputs(w, 1, plan.items)[0]
    ct = o.encrypt(pk, o.encode(o.input_slots(plan, x), o.scale), w.seed_encrypt)
    banks = [o.bank_ntt(o.layer_bank(plan, li, ws[li]), plan.layers[li].k, ext=True) for li in range(len(ws))]
    out = o.forward(plan, ct, banks, keys, rlk)
    y = o.output_slots(plan, o.decrypt_decode(s, out, plan.scales[-1]))
    assert normwise_error(y, o.forward_fp64(ws, x)) < 2.0 ** tol_log2


def test_seeded_symmetric_encryption():
    """(-a s + e + m, a): decryption returns m + e exactly with |e| within the Gaussian's tail cut,
    and c1 is the uniform stream of the seed (its first prime's row equals the sampler's output)."""
    o = CKKSOracle(12, (40, 30, 30), 40, 30)
    s = o.keygen_secret(5)
    m = np.random.default_rng(1).integers(-2 ** 35, 2 ** 35, o.n)
    ct = o.encrypt_sym(s, m, 99)
    e = np.array([int(c) - int(x) for c, x in zip(o.compose(o.decrypt(s, ct)), m)])
    assert np.max(np.abs(e)) <= 19 and 2.5 < e.std() < 4.0
    assert np.array_equal(np.asarray(o.sample(99, 11, 0, 2, o.q[0], o.n), dtype=np.uint64), ct[1, 0])
    assert np.array_equal(o.encrypt_sym(s, m, 99)[1], ct[1])          # c1 depends on the seed only
    assert not np.array_equal(o.encrypt_sym(s, m, 100)[1], ct[1])
