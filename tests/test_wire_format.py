"""Wire format of the client-server messages (host only, no device): round trips at both of the
paper's parameter sets, the exact bit layout against a packer written here from the format's
description, message sizes against Table 2, and rejection of malformed input."""
import numpy as np
import pytest

import paper_2205_11935_amd as ctl
import workloads as W

SETS = {"p1": W.CNN_P1, "p2": W.CNN_P2}


def _rand_ct(w, n_poly, k, seed):
    primes = ctl.params_primes(w.log2n, w.q_bits, w.p_bits)
    g = np.random.Generator(np.random.PCG64(seed))
    ct = np.zeros((n_poly, k, w.n), dtype=np.uint64)
    for i in range(k):
        ct[:, i] = g.integers(0, primes[i], size=(n_poly, w.n), dtype=np.uint64)
    return ct, primes


def _reference_pack(ct, primes, log2n, k, n_poly, seed):
    """The format restated: 24-byte header, then residues LSB-first at bits(q_i) bits each."""
    d = 1469598103934665603
    for q in primes:
        for b in range(8):
            d ^= (q >> (8 * b)) & 0xFF
            d = (d * 1099511628211) & (2 ** 64 - 1)
    head = b"CTL1" + bytes([1, log2n, k, n_poly]) + d.to_bytes(8, "little") + \
        (seed if n_poly == 1 else 0).to_bytes(8, "little")
    acc, nbits = 0, 0
    for p in range(n_poly):
        for i in range(k):
            b = int(primes[i]).bit_length()
            for v in ct[p, i]:
                acc |= int(v) << nbits
                nbits += b
    return head + acc.to_bytes((nbits + 7) // 8, "little")


@pytest.mark.parametrize("name", ["p1", "p2"])
@pytest.mark.parametrize("n_poly,k", [(1, 7), (2, 7), (2, 1), (2, 3)])
def test_round_trip(name, n_poly, k):
    w = SETS[name]
    ct, _ = _rand_ct(w, n_poly, k, 7 * k + n_poly)
    data = ctl.ct_pack(w.log2n, w.q_bits, w.p_bits, ct, seed=12345)
    back, seed = ctl.ct_unpack(w.log2n, w.q_bits, w.p_bits, data)
    assert np.array_equal(back, ct)
    assert seed == (12345 if n_poly == 1 else 0)


def test_layout_matches_the_description():
    w = W.SMALL
    for n_poly, k in ((1, 3), (2, 2)):
        ct, primes = _rand_ct(w, n_poly, k, 3)
        data = ctl.ct_pack(w.log2n, w.q_bits, w.p_bits, ct, seed=99)
        assert data == _reference_pack(ct, primes, w.log2n, k, n_poly, 99)


def test_sizes_against_table2():
    """Section 4.2: the client sends log2(q) N bits, the server 2 log2(q_0) N bits. Table 2 lists
    SEAL's compressed sizes (235.3 / 82.4 kB at p1, 838.1 / 262.3 kB at p2); exact bit packing
    needs less, and the seeded upload carries one polynomial."""
    for w, up_kb, down_kb in ((W.CNN_P1, 235.3, 82.4), (W.CNN_P2, 838.1, 262.3)):
        nq = len(w.q_bits)
        up = ctl.ct_packed_bytes(w.log2n, w.q_bits, w.p_bits, nq, 1)
        down = ctl.ct_packed_bytes(w.log2n, w.q_bits, w.p_bits, 1, 2)
        assert up == 24 + w.n * sum(w.q_bits) // 8
        assert down == 24 + 2 * w.n * w.q_bits[0] // 8
        assert up / 1000 < up_kb and down / 1000 < down_kb
        assert up / 1000 > 0.75 * up_kb and down / 1000 > 0.75 * down_kb


def test_rejects_malformed_input():
    w = W.SMALL
    ct, primes = _rand_ct(w, 2, 3, 5)
    data = ctl.ct_pack(w.log2n, w.q_bits, w.p_bits, ct)
    bad = bytearray(data)
    bad[0] = ord("X")
    with pytest.raises(ctl.CtlError):
        ctl.ct_unpack(w.log2n, w.q_bits, w.p_bits, bytes(bad))
    with pytest.raises(ctl.CtlError):
        ctl.ct_unpack(w.log2n, w.q_bits, w.p_bits, data[:-1])
    with pytest.raises(ctl.CtlError):                       # another parameter set
        ctl.ct_unpack(w.log2n, (40, 30, 41), w.p_bits, data)
    bad = bytearray(data)                                   # first residue of q_0 set to all ones (>= q_0)
    b0 = int(primes[0]).bit_length()
    for j in range(b0):
        bad[24 + (j >> 3)] |= 1 << (j & 7)
    with pytest.raises(ctl.CtlError):
        ctl.ct_unpack(w.log2n, w.q_bits, w.p_bits, bytes(bad))
    ct2 = ct.copy()
    ct2[1, 2, 5] = primes[2]
    with pytest.raises(ctl.CtlError):
        ctl.ct_pack(w.log2n, w.q_bits, w.p_bits, ct2)
