"""Seeded synthetic workloads shared by the CPU oracle tests, the GPU tests and the benchmark.

This module holds parameter-set descriptions and seeded random draws only. It contains none of
the method's arithmetic: no primes, no modular reduction, no encoding, no slot layout. Both the
oracle and the GPU library receive what is drawn here and do all of the CKKS work themselves.

Workloads (the paper evaluates frozen dense layers on 768-d sentence embeddings, Section 4.1;
the embeddings and trained weights are not available, so these synthetic stand-ins keep the
shape, dimensionality and value ranges):

* ``small``  N=2^12, ciphertext primes {40,30,40} bits, scale 2^30; one 64->64 dense layer by
  the plain diagonal method (t1 = t = 64, 63 rotations); weights and inputs U[-1,1].
* ``mid``    N=2^13, primes {60,40,40,60}, scale 2^40; 512->128->128 with x^2 between;
  weights N(0, 0.05^2), inputs U[-1,1].
* ``large``  N=2^14, primes {60,40,40,40,40,60}, scale 2^40; 768->256->64 with x^2 between;
  weights N(0, 0.05^2), inputs N(0,1) clipped to [-3,3]; batches of 64 ciphertexts.

Every workload adds one 60-bit special prime for key switching and uses error sigma = 3.2.

The BSGS split t = t1 * t2 of a dense layer is not fixed by the paper (Eq. (1) gives t only). With
the baby steps hoisted and kept over Q*P a baby rotation costs one key product, a giant rotation a
full key switch (ModDown, ModUp, key product), measured about 5x more at N = 2^14; t1 near
sqrt(5 t) balances them: 768 = 64 x 12, 512 = 64 x 8, 256 = 32 x 8, 128 = 32 x 4 (t1 <= 64, the
largest rotation count one key-product launch takes). The small workload keeps t1 = t = 64.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Layer:
    n_in: int
    n_out: int
    t1: int          # baby-step count of the BSGS split (t = t1 * t2)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    log2n: int
    q_bits: Tuple[int, ...]      # ciphertext primes q_0..q_L, in chain order
    p_bits: int                  # special key-switching prime
    log2_scale: int
    sigma: float
    layers: Tuple[Layer, ...]
    weight_dist: str             # "uniform1" or "normal005"
    input_dist: str              # "uniform1" or "clipnormal3"
    batch: int                   # ciphertexts per launch sequence
    seed_base: int

    @property
    def n(self) -> int:
        return 1 << self.log2n

    # seeds: base + {1 weights, 2 inputs, 3 keys, 4 encryption}
    @property
    def seed_weights(self) -> int:
        return self.seed_base + 1

    @property
    def seed_inputs(self) -> int:
        return self.seed_base + 2

    @property
    def seed_keys(self) -> int:
        return self.seed_base + 3

    @property
    def seed_encrypt(self) -> int:
        return self.seed_base + 4


SMALL = Workload("small", 12, (40, 30, 40), 60, 30, 3.2,
                 (Layer(64, 64, 64),), "uniform1", "uniform1", 1, 1000)
MID = Workload("mid", 13, (60, 40, 40, 60), 60, 40, 3.2,
               (Layer(512, 128, 64), Layer(128, 128, 32)), "normal005", "uniform1", 1, 2000)
LARGE = Workload("large", 14, (60, 40, 40, 40, 40, 60), 60, 40, 3.2,
                 (Layer(768, 256, 64), Layer(256, 64, 32)), "normal005", "clipnormal3", 64, 3000)

WORKLOADS = {w.name: w for w in (SMALL, MID, LARGE)}


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, stream]))


def weights(w: Workload) -> List[np.ndarray]:
    """One float64 matrix [n_out][n_in] per layer."""
    out = []
    for li, layer in enumerate(w.layers):
        g = _rng(w.seed_weights, li)
        if w.weight_dist == "uniform1":
            m = g.uniform(-1.0, 1.0, size=(layer.n_out, layer.n_in))
        elif w.weight_dist == "normal005":
            m = g.normal(0.0, 0.05, size=(layer.n_out, layer.n_in))
        else:
            raise ValueError(w.weight_dist)
        out.append(np.ascontiguousarray(m, dtype=np.float64))
    return out


def inputs(w: Workload, n_ct: int, items: int, stream: int = 0) -> np.ndarray:
    """float64 array [n_ct][items][n_in] of client feature vectors."""
    g = _rng(w.seed_inputs, stream)
    shape = (n_ct, items, w.layers[0].n_in)
    if w.input_dist == "uniform1":
        x = g.uniform(-1.0, 1.0, size=shape)
    elif w.input_dist == "clipnormal3":
        x = np.clip(g.normal(0.0, 1.0, size=shape), -3.0, 3.0)
    else:
        raise ValueError(w.input_dist)
    return np.ascontiguousarray(x, dtype=np.float64)


def raw_plaintexts(seed: int, count: int, n: int, bound_bits: int = 40, stream: int = 0) -> np.ndarray:
    """int64 array [count][n] of signed plaintext coefficients, uniform in [-2^b, 2^b].

    Used by the bit-exact tests: both sides take these integers as already-encoded
    plaintexts, so the comparison covers only exact modular arithmetic.
    """
    g = _rng(seed, 1000 + stream)
    lim = 1 << bound_bits
    return np.ascontiguousarray(g.integers(-lim, lim, size=(count, n), endpoint=True, dtype=np.int64))


def residues(seed: int, count: int, n: int, bits: int = 64, stream: int = 0) -> np.ndarray:
    """uint64 array [count][n] of raw random words (each side reduces them mod its primes)."""
    g = _rng(seed, 2000 + stream)
    return np.ascontiguousarray(g.integers(0, 1 << bits, size=(count, n), dtype=np.uint64,
                                           endpoint=False))


# ---------------------------------------------------------------------------------------------
# Batched mix of layer widths: 512 independent queries on the large workload's chain, each with
# d ~ U{1,2,3} dense layers and widths w_0..w_d ~ U{128,256,512,768}; x^2 between layers; weights
# drawn per (position, w_in, w_out) and shared by every query with that shape; one slot layout for
# all queries (block stride 1536 = 2 * 768, 5 items per ciphertext).
MIX_WIDTHS = (128, 256, 512, 768)
MIX_T1 = {128: 32, 256: 32, 512: 64, 768: 64}      # BSGS split of each padded width
MIX_BLOCK = 1536
MIX_SEED = 4000


@dataclasses.dataclass(frozen=True)
class Query:
    widths: Tuple[int, ...]          # w_0 .. w_d

    @property
    def depth(self) -> int:
        return len(self.widths) - 1


def mix_queries(n: int = 512, seed: int = MIX_SEED, widths=MIX_WIDTHS, max_depth: int = 3) -> List[Query]:
    g = _rng(seed, 5)
    out = []
    for _ in range(n):
        d = int(g.integers(1, max_depth + 1))
        out.append(Query(tuple(int(widths[i]) for i in g.integers(0, len(widths), size=d + 1))))
    return out


def mix_weights(pos: int, w_in: int, w_out: int, seed: int = MIX_SEED) -> np.ndarray:
    g = _rng(seed + 1, pos * 1_000_000 + w_in * 1000 + w_out)
    return np.ascontiguousarray(g.normal(0.0, 0.05, size=(w_out, w_in)), dtype=np.float64)


def mix_inputs(queries: List[Query], items: int, seed: int = MIX_SEED) -> List[np.ndarray]:
    g = _rng(seed + 2, 0)
    return [np.ascontiguousarray(np.clip(g.normal(0.0, 1.0, size=(items, q.widths[0])), -3.0, 3.0))
            for q in queries]


# ---------------------------------------------------------------------------------------------
# The paper's frozen server layers (Section 4.1 server CNN; its first four layers are frozen):
# Conv1D (f = 9, 'same' padding, one channel, 768 -> 768), Dense 768 with the degree-3 ReLU
# approximation, AveragePooling (size 3, stride 1, 768 -> 766), Dense 766. Parameter sets of
# Table 2 with q_0 and P of log2(Delta) + 9 or + 10 bits: CryptoTL_p1 (N = 2^13, log2 q = 218,
# Delta = 2^25, p = 2 items) and CryptoTL_p2 (N = 2^14, log2 q = 420, Delta = 2^50, p = 5).
# Trained weights are not available: taps N(0, 1/9), dense weights N(0, 0.03^2) and N(0, 0.05^2),
# inputs N(0,1) clipped to [-3, 3] (the encoder features' stand-in).
@dataclasses.dataclass(frozen=True)
class CnnWorkload:
    name: str
    log2n: int
    q_bits: Tuple[int, ...]
    p_bits: int
    log2_scale: int
    seed_base: int
    batch: int
    sigma: float = 3.2
    width: int = 768
    f_conv: int = 9
    f_pool: int = 3
    t1: int = 64                     # BSGS split of both dense layers (t = 768 = 64 x 12)

    @property
    def n(self) -> int:
        return 1 << self.log2n

    @property
    def pooled(self) -> int:
        return self.width - self.f_pool + 1

    @property
    def seed_keys(self) -> int:
        return self.seed_base + 3


CNN_P1 = CnnWorkload("cnn_p1", 13, (34,) + (25,) * 6, 34, 25, 5000, 64)
CNN_P2 = CnnWorkload("cnn_p2", 14, (60,) + (50,) * 6, 60, 50, 6000, 64)
CNN_WORKLOADS = {w.name: w for w in (CNN_P1, CNN_P2)}

# The degree-3 ReLU approximation as printed in Section 3.1, coefficients of z^0 .. z^3.
RELU3_COEF = (0.49383, 0.59259, 0.092593, -0.0061728)


def cnn_weights(w: CnnWorkload):
    """(taps [f_conv], W1 [width][width], W2 [pooled][pooled]) as float64."""
    g = _rng(w.seed_base + 1, 0)
    taps = g.normal(0.0, 1.0 / 3.0, size=w.f_conv)
    w1 = g.normal(0.0, 0.03, size=(w.width, w.width))
    w2 = g.normal(0.0, 0.05, size=(w.pooled, w.pooled))
    return (np.ascontiguousarray(taps), np.ascontiguousarray(w1), np.ascontiguousarray(w2))


def cnn_inputs(w: CnnWorkload, n_ct: int, items: int, stream: int = 0) -> np.ndarray:
    g = _rng(w.seed_base + 2, stream)
    return np.ascontiguousarray(np.clip(g.normal(0.0, 1.0, size=(n_ct, items, w.width)), -3.0, 3.0))
