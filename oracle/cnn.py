"""Oracle of the paper's frozen CNN layers (TEST INFRASTRUCTURE ONLY, like the rest of oracle/).

The server network of Section 4.1 starts with four frozen layers: a 1D convolution with filter
size 9, a dense layer of 768 units with the degree-3 ReLU approximation, average pooling of size
3 and a dense layer of 766 units. Section 3.1 gives the encrypted algorithms: packed single-channel
convolution (f plaintext products, f - 1 rotations), average pooling (f - 1 rotations rot_{-i},
one plaintext product), the BSGS diagonal dense layer (Eq. (1)) and the polynomial activation;
"Multiplicative Depth" counts 6 rescales. Readings used here:

* Conv1D: 'same' zero padding and one channel, output y[s] = sum_i w_i x[s + i - 4]; computed on
  both halves of each item block, so [x | x] in gives [y | y] out and the dense layer that follows
  needs no replicate.
* AvgPool: the printed sum runs to f, yet f - 1 rotations are counted; the sum here has f terms
  rot_{-i}, i = 0..f-1, so output slot s holds the mean of x[s-2..s] and the 766 valid outputs sit
  at slots 2..767 of each block; the pooling plaintext is 1/f there and 0 elsewhere (it also clears
  the activation's value at the zero half of the block). The next dense layer reads its input at
  offset 2: its padded 768 x 768 matrix holds W2 in rows 0..765, columns 2..767.
* ReLU approximation: c0 + c1 z + c2 z^2 + c3 z^3 with the printed coefficients, depth 2, by the
  constant-product schedule of ``CKKSOracle.poly3`` (constants rounded at the scales it names).
* Levels: conv (n_q -> n_q - 1), dense, activation (-2), pool, replicate, dense: 6 rescales, so 7
  ciphertext primes; each plaintext is encoded at the scale of the prime its layer drops.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence

import numpy as np

from . import CKKSOracle, LayerPlan, ModelPlan


@dataclasses.dataclass
class CnnPlan:
    width: int
    f_conv: int
    f_pool: int
    t1: int
    block: int
    items: int
    k_conv: int
    k_dense1: int
    k_act: int
    k_pool: int
    k_dense2: int
    k_out: int
    scale_in: float
    scale_act_out: float
    rotations: List[int]


def plan(o: CKKSOracle, width: int, f_conv: int, f_pool: int, t1: int, coef: Sequence[float]) -> CnnPlan:
    block = 2 * width
    items = (o.n // 2) // block
    k = o.nq
    if k < 7:
        raise ValueError("the frozen stack needs 7 ciphertext primes")
    h = (f_conv - 1) // 2
    t2 = width // t1
    rots = [r for r in range(-h, h + 1) if r != 0]
    rots += list(range(1, t1)) + [k2 * t1 for k2 in range(1, t2)]
    rots += [-i for i in range(1, f_pool)] + [-width]
    uniq = list(dict.fromkeys(rots))
    S = o.scale
    _, s3 = o.poly3_consts(k - 2, S, coef)
    return CnnPlan(width, f_conv, f_pool, t1, block, items, k, k - 1, k - 2, k - 4, k - 5, k - 6, S, s3, uniq)


def input_slots(p: CnnPlan, o: CKKSOracle, x: np.ndarray) -> np.ndarray:
    """[x | x] per item block. x: [items][width]."""
    z = np.zeros(o.n // 2)
    for b in range(x.shape[0]):
        base = b * p.block
        z[base: base + p.width] = x[b]
        z[base + p.width: base + 2 * p.width] = x[b]
    return z


def conv_tap_slots(p: CnnPlan, o: CKKSOracle, taps: np.ndarray, i: int) -> np.ndarray:
    """Tap i multiplies rot_{i-h}(x): slot s of either half holds w_i where x[s + i - h] exists."""
    h = (p.f_conv - 1) // 2
    r = i - h
    s = np.arange(p.width)
    half = np.where((s + r >= 0) & (s + r < p.width), taps[i], 0.0)
    z = np.zeros(o.n // 2)
    for b in range(p.items):
        base = b * p.block
        z[base: base + p.width] = half
        z[base + p.width: base + 2 * p.width] = half
    return z


def pool_slots(p: CnnPlan, o: CKKSOracle) -> np.ndarray:
    z = np.zeros(o.n // 2)
    for b in range(p.items):
        base = b * p.block
        z[base + p.f_pool - 1: base + p.width] = 1.0 / p.f_pool
    return z


def _dense_plan(p: CnnPlan, k: int) -> ModelPlan:
    layer = LayerPlan(p.width, p.width, p.width, p.t1, p.width // p.t1, k, False, 0)
    return ModelPlan(p.block, p.items, [layer], k - 1, [], [])


def dense2_matrix(p: CnnPlan, w2: np.ndarray) -> np.ndarray:
    """The second dense layer as a width x width matrix reading the pooled values at slots
    f_pool - 1 .. width - 1."""
    m = np.zeros((p.width, p.width))
    off = p.f_pool - 1
    m[: w2.shape[0], off: off + w2.shape[1]] = w2
    return m


def banks(p: CnnPlan, o: CKKSOracle, taps, w1, w2) -> Dict[str, np.ndarray]:
    """int64 encoded plaintexts: conv [f][N], dense1 [t][N], pool [N], dense2 [t][N]."""
    sc = lambda k: float(o.q[k - 1])           # noqa: E731 -- the prime the layer's rescale drops
    conv = np.stack([o.encode(conv_tap_slots(p, o, taps, i), sc(p.k_conv)) for i in range(p.f_conv)])
    pd1, pd2 = _dense_plan(p, p.k_dense1), _dense_plan(p, p.k_dense2)
    d1 = np.stack([o.encode(o.diag_slots(pd1, pd1.layers[0], w1, i), sc(p.k_dense1)) for i in range(p.width)])
    m2 = dense2_matrix(p, w2)
    d2 = np.stack([o.encode(o.diag_slots(pd2, pd2.layers[0], m2, i), sc(p.k_dense2)) for i in range(p.width)])
    pool = o.encode(pool_slots(p, o), sc(p.k_pool))
    return {"conv": conv, "dense1": d1, "pool": pool, "dense2": d2}


def forward(p: CnnPlan, o: CKKSOracle, ct: np.ndarray, raw: Dict[str, np.ndarray], keys, rlk,
            coef: Sequence[float], qp: bool = False) -> np.ndarray:
    """The encrypted frozen stack on one top-level ciphertext; raw: int64 plaintexts (see banks).
    Dense layers with single-ModDown giant steps; qp: every hoisted rotation (dense baby steps,
    convolution, pool) kept over Q*P with one ModDown per sum."""
    conv = np.stack([o.plaintext(m, p.k_conv, ext=qp) for m in raw["conv"]])
    ct = o.conv1d(ct, conv, keys, qp=qp)
    ct = o.dense(ct, o.bank_ntt(raw["dense1"], p.k_dense1, ext=qp), p.t1, keys, lazy=True, qp=qp)
    ct, _ = o.poly3(ct, p.scale_in, coef, rlk)
    ct = o.avgpool(ct, o.plaintext(raw["pool"], p.k_pool, ext=qp), p.f_pool, keys, qp=qp)
    ct = o.replicate(ct, p.width, keys)
    return o.dense(ct, o.bank_ntt(raw["dense2"], p.k_dense2, ext=qp), p.t1, keys, lazy=True, qp=qp)


def forward_fp64(x: np.ndarray, taps, w1, w2, coef: Sequence[float], f_pool: int) -> np.ndarray:
    """Plain FP64 frozen stack on one item x [width] (loops written out, no library kernels)."""
    n, f = x.shape[0], taps.shape[0]
    h = (f - 1) // 2
    y = np.zeros(n)
    for s in range(n):
        for i in range(f):
            if 0 <= s + i - h < n:
                y[s] += taps[i] * x[s + i - h]
    z = w1 @ y
    a = coef[0] + coef[1] * z + coef[2] * z ** 2 + coef[3] * z ** 3
    pooled = np.array([a[j: j + f_pool].sum() / f_pool for j in range(n - f_pool + 1)])
    return w2 @ pooled


def output_values(p: CnnPlan, z: np.ndarray, n_out: int) -> np.ndarray:
    return np.stack([z[b * p.block: b * p.block + n_out].real for b in range(p.items)])
