"""Property tests of the oracle (hypothesis): random ring sizes, prime sizes and residues, with the
edge values 0, 1, q-1 and the centered-lift boundaries (q-1)/2, (q+1)/2 forced in, checked against
Python big-integer definitions; and the output noise of an encrypted dense layer against the
heuristic estimate (fresh encryption noise in slots scaled by the weight rows)."""
import math

import numpy as np
from hypothesis import given, settings, strategies as st

import workloads as W
from oracle import CKKSOracle, bigint

_CTX = {}


def _oracle(logn, bits):
    key = (logn, bits)
    if key not in _CTX:
        _CTX[key] = CKKSOracle(logn, bits, 61, 20)
    return _CTX[key]


def _residues(data, q, n):
    edge = [0, 1, q - 1, (q - 1) // 2, (q + 1) // 2]
    vals = data.draw(st.lists(st.integers(0, q - 1), min_size=n, max_size=n))
    for i, e in enumerate(data.draw(st.permutations(edge))[: min(5, n)]):
        vals[(i * 7) % n] = e
    return np.array(vals, dtype=np.uint64)


_BITS = st.sampled_from([(30, 40), (40, 60), (25, 50, 60), (34, 25)])


@settings(max_examples=25, deadline=None)
@given(logn=st.integers(2, 7), bits=_BITS, data=st.data())
def test_ntt_is_the_negacyclic_convolution_transform(logn, bits, data):
    o = _oracle(logn, bits)
    for pi, q in enumerate(o.primes):
        a, b = _residues(data, q, o.n), _residues(data, q, o.n)
        assert np.array_equal(o.ntt(o.ntt(a, pi), pi, inverse=True), a)
        lhs = [(int(x) * int(y)) % q for x, y in zip(o.ntt(a, pi), o.ntt(b, pi))]
        prod = bigint.negacyclic_product([int(x) for x in a], [int(x) for x in b], q)
        assert lhs == [int(x) for x in o.ntt(np.array(prod, dtype=np.uint64), pi)]


@settings(max_examples=20, deadline=None)
@given(logn=st.integers(2, 6), bits=st.sampled_from([(30, 40, 60), (40, 40, 25), (60, 50, 34)]), data=st.data())
def test_rescale_is_rounded_division_at_edges(logn, bits, data):
    o = _oracle(logn, bits)
    k = o.nq
    coef = np.stack([np.stack([_residues(data, q, o.n) for q in o.q]) for _ in range(2)])
    ct = np.stack([np.stack([o.ntt(coef[p, i], i) for i in range(k)]) for p in range(2)])
    got = o.rescale(ct)
    for p in range(2):
        res = np.stack([o.ntt(got[p, i], i, inverse=True) for i in range(k - 1)])
        for x in range(o.n):
            X = bigint.crt([int(coef[p, i, x]) for i in range(k)], o.q)
            want = bigint.round_div(X, o.q[k - 1])
            assert [int(res[i, x]) for i in range(k - 1)] == [want % q for q in o.q[: k - 1]]


@settings(max_examples=20, deadline=None)
@given(logn=st.integers(3, 7), bits=_BITS, g_idx=st.integers(0, 10 ** 6), h_idx=st.integers(0, 10 ** 6),
       data=st.data())
def test_automorphisms_compose(logn, bits, g_idx, h_idx, data):
    o = _oracle(logn, bits)
    two_n = 2 * o.n
    g, h = 2 * (g_idx % o.n) + 1, 2 * (h_idx % o.n) + 1
    for pi, q in enumerate(o.primes):
        a = _residues(data, q, o.n)
        lhs = o.automorph_coef(o.automorph_coef(a, pi, h), pi, g)
        assert np.array_equal(lhs, o.automorph_coef(a, pi, g * h % two_n))
        assert [int(x) for x in o.automorph_coef(a, pi, g)] == bigint.automorph_definition(
            [int(x) for x in a], g, q)


def test_dense_layer_noise_matches_the_estimate():
    """Small workload (N = 2^12, Delta = 2^30, one 64 -> 64 layer, U[-1,1] weights): the output
    error std is within 2x of sigma_f * rms row norm, sigma_f = sqrt(N/2 sigma^2 (4N/3 + 1)) / Delta
    the fresh encryption noise of one slot (rescale and key-switching noise are far smaller)."""
    w = W.SMALL
    o = CKKSOracle.for_workload(w)
    plan = o.plan([(l.n_in, l.n_out, l.t1) for l in w.layers])
    s = o.keygen_secret(w.seed_keys)
    pk = o.keygen_public(w.seed_keys, s)
    keys = o.keygen_rotations(w.seed_keys, s, plan.rotations)
    rlk = o.keygen_relin(w.seed_keys, s)
    ws = W.weights(w)
    banks = [o.bank_ntt(o.layer_bank(plan, 0, ws[0]), plan.layers[0].k)]
    errs = []
    x = W.inputs(w, 3, plan.items, stream=11)
    for i in range(3):
        ct = o.encrypt(pk, o.encode(o.input_slots(plan, x[i]), o.scale), 7000 + i)
        out = o.forward(plan, ct, banks, keys, rlk)
        y = o.output_slots(plan, o.decrypt_decode(s, out, plan.scales[-1]))
        errs.append((y - x[i] @ ws[0].T).ravel())
    measured = float(np.std(np.concatenate(errs)))
    n = o.n
    sigma_f = math.sqrt(n / 2 * w.sigma ** 2 * (4 * n / 3 + 1)) / o.scale
    estimate = sigma_f * math.sqrt(np.mean(np.sum(ws[0] ** 2, axis=1)))
    assert 0.5 < measured / estimate < 2.0, (measured, estimate)
