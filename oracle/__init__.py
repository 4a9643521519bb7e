"""CPU oracle of the encrypted frozen-layer forward pass (RNS-CKKS), for tests only.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the benchmark's
CPU-baseline leg, never by the GPU library. It shares no code with the GPU library.

The integer work lives in ``ckks_oracle.c`` (plain loops, 128-bit products). This module wraps it
with ctypes and adds the parts that are plainly defined in floating point or big integers:

* encode / decode (canonical embedding; slot j <-> zeta^{5^j}, zeta = exp(i pi / N)), done with a
  library FFT of length 2N as one step;
* centered CRT composition of decrypted residues with Python integers;
* the layer plan: padded width t, the BSGS split t = t1 t2 (Eq. (1)), slot layout with block
  stride B = 2 t_max and p = floor((N/2) / B) items per ciphertext ("Multiple Predictions"),
  levels and scales;
* the diagonal plaintexts diag'_i of Eq. (1) placed on their support in every item block.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Dict, List, Sequence

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)


def _lib():
    global _LIB
    if _LIB is None:
        # CTL_ORACLE_LIB: another build of the same source (the sanitizer run of the tests)
        path = os.environ.get("CTL_ORACLE_LIB") or _build.build(force=False)
        lib = ctypes.CDLL(path)
        lib.or_ctx_new.restype = ctypes.c_void_p
        lib.or_ctx_new.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                   ctypes.c_int, ctypes.c_double]
        lib.or_ctx_free.argtypes = [ctypes.c_void_p]
        lib.or_galois_elt.restype = ctypes.c_uint64
        lib.or_galois_elt.argtypes = [ctypes.c_void_p, ctypes.c_long]
        lib.or_min_psi.restype = ctypes.c_uint64
        lib.or_min_psi.argtypes = [ctypes.c_uint64, ctypes.c_int]
        lib.or_find_primes.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, u64p]
        lib.or_affine.restype = None
        lib.or_affine.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, u64p, ctypes.c_int64,
                                  ctypes.c_int64, u64p]
        lib.or_poly3_consts.restype = ctypes.c_double
        lib.or_poly3_consts.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_double), i64p]
        lib.or_poly3.restype = ctypes.c_double
        lib.or_poly3.argtypes = [ctypes.c_void_p, ctypes.c_int, u64p, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double), u64p, u64p]
        _LIB = lib
    return _LIB


def _p(a: np.ndarray):
    if a.dtype == np.uint64:
        return a.ctypes.data_as(u64p)
    if a.dtype == np.int64:
        return a.ctypes.data_as(i64p)
    if a.dtype == np.uint8:
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    if a.dtype == np.uint32:
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    raise TypeError(a.dtype)


def find_primes(logn: int, bits: Sequence[int]) -> List[int]:
    arr = (ctypes.c_int * len(bits))(*bits)
    out = np.zeros(len(bits), dtype=np.uint64)
    rc = _lib().or_find_primes(logn, arr, len(bits), _p(out))
    if rc != 0:
        raise ValueError("no prime found")
    return [int(x) for x in out]


def min_psi(q: int, logn: int) -> int:
    return int(_lib().or_min_psi(q, logn))


def chacha20_block(key_words: Sequence[int], counter: int, nonce_words: Sequence[int]) -> bytes:
    key = np.array(key_words, dtype=np.uint32)
    nonce = np.array(nonce_words, dtype=np.uint32)
    out = np.zeros(64, dtype=np.uint8)
    _lib().or_chacha20_block(_p(key), ctypes.c_uint32(counter), _p(nonce), _p(out))
    return out.tobytes()


@dataclasses.dataclass
class LayerPlan:
    n_in: int
    n_out: int
    t: int
    t1: int
    t2: int
    k: int              # live primes at the layer input
    square_after: bool
    next_t: int         # padded width of the next layer (replicate distance), 0 if last
    lazy: bool = False  # giant steps lowered by one ModDown of their summed key products
    qp: bool = False    # baby steps kept over Q*P (implies one final ModDown of the giant steps)


@dataclasses.dataclass
class ModelPlan:
    block: int          # B = 2 t_max
    items: int          # p
    layers: List[LayerPlan]
    k_out: int
    scales: List[float]  # scale at each layer input, then the output scale
    rotations: List[int]  # every left-rotation amount the model needs


class CKKSOracle:
    """One parameter set: ring degree 2^logn, ciphertext primes of the given bit sizes, one
    special prime of p_bits, error sigma."""

    def __init__(self, logn: int, q_bits: Sequence[int], p_bits: int, log2_scale: int,
                 sigma: float = 3.2):
        self.lib = _lib()
        arr = (ctypes.c_int * len(q_bits))(*q_bits)
        self.ctx = self.lib.or_ctx_new(logn, len(q_bits), arr, p_bits, sigma)
        if not self.ctx:
            raise ValueError("oracle context creation failed")
        self.logn = logn
        self.n = 1 << logn
        self.nq = len(q_bits)
        self.np = self.nq + 1
        self.log2_scale = log2_scale
        self.scale = float(2.0 ** log2_scale)
        pr = np.zeros(self.np, dtype=np.uint64)
        self.lib.or_ctx_primes(ctypes.c_void_p(self.ctx), _p(pr))
        self.primes = [int(x) for x in pr]
        self.q = self.primes[: self.nq]
        self.P = self.primes[self.nq]
        ps = np.zeros(self.np, dtype=np.uint64)
        self.lib.or_ctx_psis(ctypes.c_void_p(self.ctx), _p(ps))
        self.psis = [int(x) for x in ps]

    @classmethod
    def for_workload(cls, w) -> "CKKSOracle":
        return cls(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma)

    def __del__(self):
        if getattr(self, "ctx", None):
            self.lib.or_ctx_free(ctypes.c_void_p(self.ctx))
            self.ctx = None

    @property
    def c(self):
        return ctypes.c_void_p(self.ctx)

    # ------------------------------------------------------------ primitives
    def cdt(self) -> np.ndarray:
        out = np.zeros(39, dtype=np.uint64)
        self.lib.or_ctx_cdt(self.c, _p(out))
        return out

    def ntt(self, a: np.ndarray, prime_index: int, inverse: bool = False) -> np.ndarray:
        x = np.ascontiguousarray(a, dtype=np.uint64).copy()
        self.lib.or_ntt(self.c, prime_index, _p(x), int(inverse))
        return x

    def galois_elt(self, r: int) -> int:
        return int(self.lib.or_galois_elt(self.c, r))

    def automorph_ntt(self, a: np.ndarray, g: int) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        out = np.zeros_like(a)
        self.lib.or_automorph_ntt(self.c, ctypes.c_uint64(g), _p(a), _p(out))
        return out

    def automorph_coef(self, a: np.ndarray, prime_index: int, g: int) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        out = np.zeros_like(a)
        self.lib.or_automorph_coef(self.c, prime_index, ctypes.c_uint64(g), _p(a), _p(out))
        return out

    def sample(self, seed: int, tag: int, index: int, kind: int, modulus: int, n: int) -> np.ndarray:
        out = np.zeros(n, dtype=np.int64)
        self.lib.or_sample(self.c, ctypes.c_uint64(seed), ctypes.c_uint32(tag),
                           ctypes.c_uint64(index), kind, ctypes.c_uint64(modulus), n, _p(out))
        return out

    # ------------------------------------------------------------ keys
    def keygen_secret(self, seed: int) -> np.ndarray:
        s = np.zeros(self.n, dtype=np.int64)
        self.lib.or_keygen_secret(self.c, ctypes.c_uint64(seed), _p(s))
        return s

    def keygen_public(self, seed: int, s: np.ndarray) -> np.ndarray:
        pk = np.zeros((2, self.nq, self.n), dtype=np.uint64)
        self.lib.or_keygen_public(self.c, ctypes.c_uint64(seed), _p(s), _p(pk))
        return pk

    def keygen_galois(self, seed: int, s: np.ndarray, g: int) -> np.ndarray:
        key = np.zeros((self.nq, 2, self.np, self.n), dtype=np.uint64)
        self.lib.or_keygen_galois(self.c, ctypes.c_uint64(seed), _p(s), ctypes.c_uint64(g), _p(key))
        return key

    def keygen_relin(self, seed: int, s: np.ndarray) -> np.ndarray:
        key = np.zeros((self.nq, 2, self.np, self.n), dtype=np.uint64)
        self.lib.or_keygen_relin(self.c, ctypes.c_uint64(seed), _p(s), _p(key))
        return key

    def keygen_rotations(self, seed: int, s: np.ndarray, rotations: Sequence[int]) -> Dict[int, np.ndarray]:
        keys = {}
        for r in rotations:
            g = self.galois_elt(r)
            if g not in keys:
                keys[g] = self.keygen_galois(seed, s, g)
        return keys

    # ------------------------------------------------------------ encrypt / decrypt
    def plaintext(self, m: np.ndarray, k: int, ext: bool = False) -> np.ndarray:
        """[k][N] NTT form over q_0..q_{k-1}; with ext a last row mod P ([k+1][N])."""
        m = np.ascontiguousarray(m, dtype=np.int64)
        pt = np.zeros((k + (1 if ext else 0), self.n), dtype=np.uint64)
        (self.lib.or_plaintext_ext if ext else self.lib.or_plaintext)(self.c, _p(m), k, _p(pt))
        return pt

    def encrypt(self, pk: np.ndarray, m: np.ndarray, seed: int) -> np.ndarray:
        m = np.ascontiguousarray(m, dtype=np.int64)
        ct = np.zeros((2, self.nq, self.n), dtype=np.uint64)
        self.lib.or_encrypt(self.c, _p(pk), _p(m), ctypes.c_uint64(seed), _p(ct))
        return ct

    def encrypt_sym(self, s: np.ndarray, m: np.ndarray, seed: int) -> np.ndarray:
        """Seeded secret-key encryption (-a s + e + m, a); a depends on the seed only."""
        m = np.ascontiguousarray(m, dtype=np.int64)
        ct = np.zeros((2, self.nq, self.n), dtype=np.uint64)
        self.lib.or_encrypt_sym(self.c, _p(np.ascontiguousarray(s, dtype=np.int64)), _p(m),
                                ctypes.c_uint64(seed), _p(ct))
        return ct

    def decrypt(self, s: np.ndarray, ct: np.ndarray) -> np.ndarray:
        """Coefficient-form residues of c0 + c1 s, [k][N]."""
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        k = ct.shape[1]
        out = np.zeros((k, self.n), dtype=np.uint64)
        self.lib.or_decrypt(self.c, _p(s), _p(ct), k, _p(out))
        return out

    def compose(self, residues: np.ndarray) -> List[int]:
        """Centered CRT composition of [k][N] coefficient residues, as Python integers."""
        k = residues.shape[0]
        mods = self.q[:k]
        Q = 1
        for m in mods:
            Q *= m
        coeffs = [0] * self.n
        for i, m in enumerate(mods):
            mh = Q // m
            f = mh * pow(mh, -1, m)
            col = residues[i].tolist()
            for x in range(self.n):
                coeffs[x] += col[x] * f
        half = (Q - 1) // 2
        out = []
        for v in coeffs:
            v %= Q
            out.append(v - Q if v > half else v)
        return out

    # ------------------------------------------------------------ homomorphic operations
    def modup(self, d: np.ndarray) -> np.ndarray:
        k = d.shape[0]
        out = np.zeros((k, k + 1, self.n), dtype=np.uint64)
        self.lib.or_modup(self.c, k, _p(np.ascontiguousarray(d)), _p(out))
        return out

    def moddown(self, u: np.ndarray) -> np.ndarray:
        k = u.shape[1] - 1
        out = np.zeros((2, k, self.n), dtype=np.uint64)
        self.lib.or_moddown(self.c, k, _p(np.ascontiguousarray(u)), _p(out))
        return out

    def keyswitch(self, d: np.ndarray, key: np.ndarray) -> np.ndarray:
        k = d.shape[0]
        out = np.zeros((2, k, self.n), dtype=np.uint64)
        self.lib.or_keyswitch(self.c, k, _p(np.ascontiguousarray(d)), _p(key), _p(out))
        return out

    def rotate(self, ct: np.ndarray, key: np.ndarray, g: int) -> np.ndarray:
        k = ct.shape[1]
        out = np.zeros_like(ct)
        self.lib.or_rotate(self.c, k, _p(np.ascontiguousarray(ct)), _p(key), ctypes.c_uint64(g), _p(out))
        return out

    def rotate_hoisted(self, ct: np.ndarray, digits: np.ndarray, key: np.ndarray, g: int) -> np.ndarray:
        k = ct.shape[1]
        out = np.zeros_like(ct)
        self.lib.or_rotate_hoisted(self.c, k, _p(np.ascontiguousarray(ct)), _p(digits), _p(key),
                                   ctypes.c_uint64(g), _p(out))
        return out

    def rescale(self, ct: np.ndarray) -> np.ndarray:
        k = ct.shape[1]
        out = np.zeros((2, k - 1, self.n), dtype=np.uint64)
        self.lib.or_rescale(self.c, k, _p(np.ascontiguousarray(ct)), _p(out))
        return out

    def square(self, ct: np.ndarray, rlk: np.ndarray) -> np.ndarray:
        k = ct.shape[1]
        out = np.zeros((2, k - 1, self.n), dtype=np.uint64)
        rc = self.lib.or_square(self.c, k, _p(np.ascontiguousarray(ct)), _p(rlk), _p(out))
        if rc:
            raise RuntimeError(rc)
        return out

    def _keyset(self, keys: Dict[int, np.ndarray]):
        gs = np.array(sorted(keys), dtype=np.uint64)
        arr = (u64p * len(gs))(*[_p(keys[int(g)]) for g in gs])
        return gs, arr

    def dense(self, ct: np.ndarray, pts: np.ndarray, t1: int, keys: Dict[int, np.ndarray],
              lazy: bool = False, rescale: bool = True, qp: bool = False) -> np.ndarray:
        """qp: baby steps over Q*P (pts then [t][k+1][N], see bank_ntt(ext=True))."""
        k = ct.shape[1]
        t = pts.shape[0]
        if pts.shape[1] != k + (1 if qp else 0):
            raise ValueError("plaintext rows do not match the variant")
        out = np.zeros((2, k - 1 if rescale else k, self.n), dtype=np.uint64)
        gs, arr = self._keyset(keys)
        flags = (1 if lazy else 0) | (0 if rescale else 2) | (4 if qp else 0)
        rc = self.lib.or_dense(self.c, k, _p(np.ascontiguousarray(ct)), _p(np.ascontiguousarray(pts)),
                               t, t1, flags, len(gs), _p(gs), arr, _p(out))
        if rc:
            raise RuntimeError("or_dense failed: %d" % rc)
        return out

    def replicate(self, ct: np.ndarray, w: int, keys: Dict[int, np.ndarray]) -> np.ndarray:
        k = ct.shape[1]
        out = np.zeros_like(ct)
        gs, arr = self._keyset(keys)
        rc = self.lib.or_replicate(self.c, k, _p(np.ascontiguousarray(ct)), w, len(gs), _p(gs), arr, _p(out))
        if rc:
            raise RuntimeError("or_replicate failed: %d" % rc)
        return out

    # ------------------------------------------------------------ layers of the paper's CNN
    def mul(self, a: np.ndarray, b: np.ndarray, rlk: np.ndarray) -> np.ndarray:
        """Ciphertext product with relinearization and rescale: [2][k][N] -> [2][k-1][N]."""
        k = a.shape[1]
        out = np.zeros((2, k - 1, self.n), dtype=np.uint64)
        self.lib.or_mul(self.c, k, _p(np.ascontiguousarray(a)), _p(np.ascontiguousarray(b)),
                        _p(np.ascontiguousarray(rlk)), _p(out))
        return out

    def affine(self, ct: np.ndarray, mul: int, add: int, k_out: int = 0) -> np.ndarray:
        """ct * mul + add (signed integer constants; add goes to c0), keeping the first k_out primes."""
        k = ct.shape[1]
        k_out = k_out or k
        out = np.zeros((2, k_out, self.n), dtype=np.uint64)
        self.lib.or_affine(self.c, k, k_out, _p(np.ascontiguousarray(ct)), mul, add, _p(out))
        return out

    def conv1d(self, ct: np.ndarray, pts: np.ndarray, keys: Dict[int, np.ndarray], qp: bool = False) -> np.ndarray:
        """sum_i pts_i * rot_{i - (f-1)/2}(ct), rescaled. pts: [f][k][N] NTT form; qp: the rotations
        kept over Q*P with one ModDown of the sum (pts then [f][k+1][N])."""
        k = ct.shape[1]
        if pts.shape[1] != k + (1 if qp else 0):
            raise ValueError("plaintext rows do not match the variant")
        out = np.zeros((2, k - 1, self.n), dtype=np.uint64)
        gs, arr = self._keyset(keys)
        fn = self.lib.or_conv1d_qp if qp else self.lib.or_conv1d
        rc = fn(self.c, k, _p(np.ascontiguousarray(ct)), _p(np.ascontiguousarray(pts)),
                pts.shape[0], len(gs), _p(gs), arr, _p(out))
        if rc:
            raise RuntimeError("or_conv1d failed: %d" % rc)
        return out

    def avgpool(self, ct: np.ndarray, pt: np.ndarray, f: int, keys: Dict[int, np.ndarray],
                qp: bool = False) -> np.ndarray:
        """pt * sum_{i < f} rot_{-i}(ct), rescaled. pt: [k][N] NTT form; qp: the rotations kept over
        Q*P with one ModDown of the sum (pt then [k+1][N])."""
        k = ct.shape[1]
        if pt.shape[0] != k + (1 if qp else 0):
            raise ValueError("plaintext rows do not match the variant")
        out = np.zeros((2, k - 1, self.n), dtype=np.uint64)
        gs, arr = self._keyset(keys)
        fn = self.lib.or_avgpool_qp if qp else self.lib.or_avgpool
        rc = fn(self.c, k, _p(np.ascontiguousarray(ct)), _p(np.ascontiguousarray(pt)), f,
                len(gs), _p(gs), arr, _p(out))
        if rc:
            raise RuntimeError("or_avgpool failed: %d" % rc)
        return out

    def poly3_consts(self, k: int, scale: float, coef: Sequence[float]):
        """Integer constants (C0..C3) and output scale of the degree-3 activation at k primes."""
        cf = (ctypes.c_double * 4)(*coef)
        C = np.zeros(4, dtype=np.int64)
        s3 = self.lib.or_poly3_consts(self.c, k, scale, cf, _p(C))
        return [int(x) for x in C], float(s3)

    def poly3(self, ct: np.ndarray, scale: float, coef: Sequence[float], rlk: np.ndarray):
        """c0 + c1 z + c2 z^2 + c3 z^3 with depth 2: returns ([2][k-2][N], output scale)."""
        k = ct.shape[1]
        out = np.zeros((2, k - 2, self.n), dtype=np.uint64)
        cf = (ctypes.c_double * 4)(*coef)
        s3 = self.lib.or_poly3(self.c, k, _p(np.ascontiguousarray(ct)), scale, cf,
                               _p(np.ascontiguousarray(rlk)), _p(out))
        return out, float(s3)

    # ------------------------------------------------------------ encoding (canonical embedding)
    def slot_exponents(self) -> np.ndarray:
        """e_j = 5^j mod 2N for the N/2 slots."""
        two_n = 2 * self.n
        out = np.zeros(self.n // 2, dtype=np.int64)
        e = 1
        for j in range(self.n // 2):
            out[j] = e
            e = e * 5 % two_n
        return out

    def encode_real(self, z: np.ndarray) -> np.ndarray:
        """Unrounded coefficients m with m(zeta^{5^j}) = z_j: m_k = (1/N) sum_e w_e zeta^{-e k}
        over the odd exponents e, w_{5^j} = z_j, w_{-5^j} = conj(z_j)."""
        n = self.n
        e = self.slot_exponents()
        w = np.zeros(2 * n, dtype=np.complex128)
        zc = np.asarray(z, dtype=np.complex128)
        w[e] = zc
        w[(2 * n - e) % (2 * n)] = np.conj(zc)
        return (np.fft.fft(w)[:n] / n).real

    def encode(self, z: np.ndarray, scale: float) -> np.ndarray:
        """Integer plaintext coefficients rint(scale * m) (round half to even)."""
        v = np.rint(scale * self.encode_real(z))
        if np.max(np.abs(v)) >= 2.0 ** 62:
            raise OverflowError("encoded coefficient exceeds 2^62")
        return v.astype(np.int64)

    def decode_coeffs(self, coeffs: Sequence, scale: float) -> np.ndarray:
        """Slots z_j = sum_k (m_k / scale) zeta^{5^j k}."""
        n = self.n
        m = np.array([float(c) for c in coeffs], dtype=np.float64) / scale
        pad = np.zeros(2 * n, dtype=np.complex128)
        pad[:n] = m
        v = np.fft.ifft(pad) * (2 * n)
        return v[self.slot_exponents()]

    def decrypt_decode(self, s: np.ndarray, ct: np.ndarray, scale: float) -> np.ndarray:
        return self.decode_coeffs(self.compose(self.decrypt(s, ct)), scale)

    # ------------------------------------------------------------ model plan
    def plan(self, layers, lazy: bool = False, qp: bool = False) -> ModelPlan:
        """layers: sequence of (n_in, n_out, t1); lazy selects the single-ModDown giant steps, qp
        the baby steps over Q*P."""
        ts = [max(a, b) for (a, b, _) in layers]
        block = 2 * max(ts)
        items = (self.n // 2) // block
        if items < 1:
            raise ValueError("layer wider than half the slots")
        k = self.nq
        scale = self.scale
        plans, scales, rots = [], [], []
        for li, (n_in, n_out, t1) in enumerate(layers):
            t = ts[li]
            if t % t1:
                raise ValueError("t1 must divide t")
            last = li == len(layers) - 1
            nxt = 0 if last else ts[li + 1]
            plans.append(LayerPlan(n_in, n_out, t, t1, t // t1, k, not last, nxt, lazy, qp))
            scales.append(scale)
            rots += list(range(1, t1)) + [k2 * t1 for k2 in range(1, t // t1)]
            k -= 1                                    # dense rescale; scale preserved
            if not last:
                scale = scale * scale / self.q[k - 1]  # square, then rescale by q_{k-1}
                k -= 1
                rots.append(-nxt)
            if k < 1:
                raise ValueError("modulus chain exhausted")
        scales.append(scale)
        seen, uniq = set(), []
        for r in rots:
            if r not in seen:
                seen.add(r)
                uniq.append(r)
        return ModelPlan(block, items, plans, k, scales, uniq)

    def input_slots(self, plan: ModelPlan, x: np.ndarray) -> np.ndarray:
        """[x | x] per item block (x zero-padded to the first layer's t). x: [items][n_in]."""
        z = np.zeros(self.n // 2)
        t = plan.layers[0].t
        for b in range(x.shape[0]):
            base = b * plan.block
            z[base: base + x.shape[1]] = x[b]
            z[base + t: base + t + x.shape[1]] = x[b]
        return z

    def diag_slots(self, plan: ModelPlan, layer: LayerPlan, w: np.ndarray, i: int) -> np.ndarray:
        """Slot vector of plaintext i = k2 t1 + j: in every block, slot k2 t1 + s holds
        diag_i[s] = M[s][(s + i) mod t] for s in [0, t) (M = w zero-padded to t x t)."""
        t, t1 = layer.t, layer.t1
        k2 = i // t1
        m = np.zeros((t, t))
        m[: w.shape[0], : w.shape[1]] = w
        rows = np.arange(t)
        diag = m[rows, (rows + i) % t]
        z = np.zeros(self.n // 2)
        for b in range(plan.items):
            base = b * plan.block + k2 * t1
            z[base: base + t] = diag
        return z

    def layer_bank(self, plan: ModelPlan, li: int, w: np.ndarray) -> np.ndarray:
        """int64 [t][N] encoded diagonal plaintexts at scale q_{k-1} (the prime this layer's
        rescale drops)."""
        layer = plan.layers[li]
        sc = float(self.q[layer.k - 1])
        return np.stack([self.encode(self.diag_slots(plan, layer, w, i), sc) for i in range(layer.t)])

    def bank_ntt(self, bank: np.ndarray, k: int, ext: bool = False) -> np.ndarray:
        return np.stack([self.plaintext(bank[i], k, ext) for i in range(bank.shape[0])])

    def forward(self, plan: ModelPlan, ct: np.ndarray, banks_ntt: List[np.ndarray],
                keys: Dict[int, np.ndarray], rlk: np.ndarray) -> np.ndarray:
        for li, layer in enumerate(plan.layers):
            ct = self.dense(ct, banks_ntt[li], layer.t1, keys, layer.lazy, qp=layer.qp)
            if layer.square_after:
                ct = self.square(ct, rlk)
                ct = self.replicate(ct, layer.next_t, keys)
        return ct

    @staticmethod
    def forward_fp64(weights: List[np.ndarray], x: np.ndarray) -> np.ndarray:
        """Plain FP64 reference: y = W_d (... (W_1 x)^2 ...), x^2 between consecutive layers."""
        y = x
        for li, w in enumerate(weights):
            y = y @ w.T
            if li + 1 < len(weights):
                y = y * y
        return y

    def output_slots(self, plan: ModelPlan, z: np.ndarray) -> np.ndarray:
        n_out = plan.layers[-1].n_out
        return np.stack([z[b * plan.block: b * plan.block + n_out].real for b in range(plan.items)])


def normwise_error(dec: np.ndarray, ref: np.ndarray) -> float:
    """max |dec - ref| / max |ref| over the valid output slots."""
    return float(np.max(np.abs(dec - ref)) / np.max(np.abs(ref)))


def log2_or_inf(x: float) -> float:
    return math.log2(x) if x > 0 else -math.inf
