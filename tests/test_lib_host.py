"""Host-side checks of libcryptotl that need no GPU: the library loads, exports every symbol its
header declares, and its host logic (prime chain, Galois elements, ChaCha20 samplers) agrees
bit for bit with the independently written CPU oracle. No compute call touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
import paper_2205_11935_amd as ctl
from oracle import CKKSOracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "ctl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ctl_[a-z0-9_]+)\s*\(", src)) - {"ctl_alloc_fn", "ctl_free_fn"})


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ctl.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps exactly the declared calls
    assert set(names) == set(ctl._SIGS)


def test_error_reporting_without_device():
    with pytest.raises(ctl.CtlError) as ei:
        ctl.params_primes(11, [40], 60)
    assert ei.value.code == -7 and "log2n" in str(ei.value)
    with pytest.raises(ctl.CtlError) as ei:
        ctl.params_primes(12, [70], 60)
    assert ei.value.code == -7


@pytest.mark.parametrize("name", ["small", "mid", "large"])
def test_primes_match_oracle(name):
    w = W.WORKLOADS[name]
    o = CKKSOracle.for_workload(w)
    assert ctl.params_primes(w.log2n, w.q_bits, w.p_bits) == o.primes


@pytest.mark.parametrize("log2n", [12, 13, 14])
def test_galois_elements_match_oracle(log2n):
    o = CKKSOracle(log2n, (40,), 60, 30)
    for r in [0, 1, 2, 7, 31, 32, 768, -1, -256, -768, (1 << (log2n - 1)) + 3]:
        assert ctl.galois_elt(log2n, r) == o.galois_elt(r)


@pytest.mark.parametrize("name", ["small", "large"])
def test_samplers_match_oracle(name):
    w = W.WORKLOADS[name]
    o = CKKSOracle.for_workload(w)
    n = 5000
    for seed, tag, index in [(1, 1, 0), (2024, 3, 5), (7, 4, 64 * 5 + 3), (2 ** 63 + 11, 10, 2 ** 40)]:
        for kind, mod in [(0, 0), (1, 0), (2, o.primes[0]), (2, o.primes[1]), (2, o.P)]:
            a = ctl.sample(w.log2n, w.q_bits, w.p_bits, seed, tag, index, kind, mod, n)
            b = o.sample(seed, tag, index, kind, mod, n)
            assert np.array_equal(a, b), (seed, tag, index, kind)


def test_gaussian_sampler_moments():
    e = ctl.sample(12, [40], 60, 99, 9, 0, 1, 0, 200000)
    assert e.min() >= -19 and e.max() <= 19
    assert abs(e.var() / 3.2 ** 2 - 1) < 0.02
