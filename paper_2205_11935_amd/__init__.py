"""Python binding of libcryptotl (CryptoTL's encrypted frozen-layer forward pass on MI355X).

Argument marshalling only: every step of the path runs in the HIP kernels of the shared library.
PyTorch supplies device memory (ciphertext buffers and, through the allocator hook, the library's
workspace and banks) and streams. If the library is not built, importing the binding works but
creating a Context raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import weakref
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CTL_LIB_PATH: another build of the same sources (the sanitizer run of the host tests)
LIB_PATH = os.environ.get("CTL_LIB_PATH") or os.path.join(_HERE, "libcryptotl.so")

CTL_ACT_NONE = 0
CTL_ACT_SQUARE = 1
CTL_ACT_POLY3 = 2
CTL_LAYER_LAZY_GIANT = 1
CTL_LAYER_BABY_QP = 2
CTL_KNOB_MAC_CHUNK = 0
CTL_KNOB_MAC_CTS = 1
CTL_KNOB_KEYIP_XCD = 2
CTL_KNOB_MAC_DIRECT = 3
CTL_KNOB_NTT_XCD = 4
CTL_KNOB_MAC_LIMB = 5
CTL_KNOB_KEYIP_RR = 6
CTL_KNOB_NTT_SPLIT = 7
CTL_KNOB_NTT_LOOP = 8
CTL_KNOB_FUSE_RESCALE = 9
KNOBS = {"mac_chunk": CTL_KNOB_MAC_CHUNK, "mac_cts": CTL_KNOB_MAC_CTS, "keyip_xcd": CTL_KNOB_KEYIP_XCD,
         "mac_direct": CTL_KNOB_MAC_DIRECT, "ntt_xcd": CTL_KNOB_NTT_XCD, "mac_limb": CTL_KNOB_MAC_LIMB,
         "keyip_rr": CTL_KNOB_KEYIP_RR, "ntt_split": CTL_KNOB_NTT_SPLIT,
         "ntt_loop": CTL_KNOB_NTT_LOOP, "fuse_rescale": CTL_KNOB_FUSE_RESCALE}
CTL_FORM_NTT = 0
CTL_FORM_COEFF = 1
CTL_LAYER_DENSE = 0
CTL_LAYER_CONV1D = 1
CTL_LAYER_AVGPOOL = 2
MAX_PRIMES = 8

ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "ELEVEL", -4: "ESCALE", -5: "EKEY", -6: "EHIP", -7: "EPARAM"}

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
i32p = ctypes.POINTER(ctypes.c_int32)
f64p = ctypes.POINTER(ctypes.c_double)


class CtlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("log2n", ctypes.c_int), ("n_q", ctypes.c_int), ("q_bits", ctypes.c_int * MAX_PRIMES),
                ("p_bits", ctypes.c_int), ("log2_scale", ctypes.c_int), ("sigma", ctypes.c_double)]


class _LayerDesc(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int), ("n_out", ctypes.c_int), ("t1", ctypes.c_int), ("act", ctypes.c_int),
                ("flags", ctypes.c_int), ("kind", ctypes.c_int), ("f", ctypes.c_int),
                ("coef", ctypes.c_double * 4)]


@dataclasses.dataclass
class Layer:
    """One layer descriptor (ctl_layer_desc). Plain (n_in, n_out, t1[, act]) tuples stand for dense
    layers with x^2 between them."""
    kind: int
    n_in: int
    n_out: int
    t1: int = 0
    f: int = 0
    act: int = CTL_ACT_NONE
    coef: Sequence[float] = (0.0, 0.0, 0.0, 0.0)

    @staticmethod
    def dense(n_in, n_out, t1, act=CTL_ACT_NONE, coef=(0.0, 0.0, 0.0, 0.0)):
        return Layer(CTL_LAYER_DENSE, n_in, n_out, t1=t1, act=act, coef=coef)

    @staticmethod
    def conv1d(width, f, act=CTL_ACT_NONE, coef=(0.0, 0.0, 0.0, 0.0)):
        return Layer(CTL_LAYER_CONV1D, width, width, f=f, act=act, coef=coef)

    @staticmethod
    def avgpool(width, f, act=CTL_ACT_NONE, coef=(0.0, 0.0, 0.0, 0.0)):
        return Layer(CTL_LAYER_AVGPOOL, width, width - f + 1, f=f, act=act, coef=coef)


class _ModelOpts(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("k_in", ctypes.c_int), ("scale_in", ctypes.c_double)]


class _ModelInfo(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int), ("block", ctypes.c_int), ("items", ctypes.c_int),
                ("k_in", ctypes.c_int), ("k_out", ctypes.c_int), ("n_in", ctypes.c_int), ("n_out", ctypes.c_int),
                ("n_rotations", ctypes.c_int), ("scale_in", ctypes.c_double), ("scale_out", ctypes.c_double),
                ("layer_k", ctypes.c_int * 8), ("layer_t", ctypes.c_int * 8)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

# every symbol the header declares, with its ctypes signature
_SIGS = {
    "ctl_last_error": (ctypes.c_char_p, []),
    "ctl_params_primes": (ctypes.c_int, [ctypes.POINTER(_Params), u64p, ctypes.POINTER(ctypes.c_int)]),
    "ctl_galois_elt": (ctypes.c_int, [ctypes.POINTER(_Params), ctypes.c_int, u64p]),
    "ctl_sample": (ctypes.c_int, [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_int, ctypes.c_uint64, ctypes.c_int, i64p]),
    "ctl_ctx_create": (ctypes.c_int, [ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "ctl_ctx_free": (ctypes.c_int, [ctypes.c_void_p]),
    "ctl_ctx_primes": (ctypes.c_int, [ctypes.c_void_p, u64p, ctypes.POINTER(ctypes.c_int)]),
    "ctl_set_allocator": (ctypes.c_int, [ctypes.c_void_p, _ALLOC_FN, _FREE_FN, ctypes.c_void_p]),
    "ctl_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, u64p]),
    "ctl_ntt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, i32p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_ct_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     u64p, ctypes.c_void_p]),
    "ctl_ct_import": (ctypes.c_int, [ctypes.c_void_p, u64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "ctl_pt_import": (ctypes.c_int, [ctypes.c_void_p, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "ctl_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ctl_profile_families": (ctypes.c_int, []),
    "ctl_profile_family_name": (ctypes.c_char_p, [ctypes.c_int]),
    "ctl_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "ctl_profile_read_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "ctl_profile_launches": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "ctl_profile_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_char_p)]),
    "ctl_probe_valu": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                      ctypes.c_void_p]),
    "ctl_keygen": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, i32p, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.POINTER(ctypes.c_void_p)]),
    "ctl_sk_free": (ctypes.c_int, [ctypes.c_void_p]),
    "ctl_pk_free": (ctypes.c_int, [ctypes.c_void_p]),
    "ctl_evk_free": (ctypes.c_int, [ctypes.c_void_p]),
    "ctl_sk_export": (ctypes.c_int, [ctypes.c_void_p, i64p]),
    "ctl_pk_export": (ctypes.c_int, [ctypes.c_void_p, u64p]),
    "ctl_evk_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, u64p]),
    "ctl_evk_galois": (ctypes.c_int, [ctypes.c_void_p, u64p, ctypes.POINTER(ctypes.c_int)]),
    "ctl_evk_import": (ctypes.c_int, [ctypes.c_void_p, u64p, ctypes.c_int, ctypes.POINTER(u64p),
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "ctl_evk_bytes": (ctypes.c_int, [ctypes.c_void_p, u64p]),
    "ctl_model_bytes": (ctypes.c_int, [ctypes.c_void_p, u64p]),
    "ctl_model_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_LayerDesc), ctypes.c_int,
                                      ctypes.POINTER(f64p), ctypes.POINTER(ctypes.c_void_p)]),
    "ctl_model_load_raw": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_LayerDesc), ctypes.c_int,
                                          ctypes.POINTER(i64p), ctypes.POINTER(ctypes.c_void_p)]),
    "ctl_model_load_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_LayerDesc), ctypes.c_int,
                                         ctypes.POINTER(f64p), ctypes.POINTER(i64p), ctypes.POINTER(_ModelOpts),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "ctl_workspace_freeze": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ctl_knob_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "ctl_knob_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "ctl_model_free": (ctypes.c_int, [ctypes.c_void_p]),
    "ctl_model_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_ModelInfo)]),
    "ctl_model_rotations": (ctypes.c_int, [ctypes.c_void_p, i32p, ctypes.POINTER(ctypes.c_int)]),
    "ctl_encode": (ctypes.c_int, [ctypes.c_void_p, f64p, ctypes.c_double, i64p]),
    "ctl_encode_items": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, f64p, ctypes.c_int, i64p]),
    "ctl_encrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, i64p, ctypes.c_uint64, ctypes.c_void_p,
                                   ctypes.c_void_p]),
    "ctl_encrypt_sym": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, i64p, ctypes.c_uint64, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "ctl_expand_seeded": (ctypes.c_int, [ctypes.c_void_p, u64p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "ctl_ct_packed_bytes": (ctypes.c_int, [ctypes.POINTER(_Params), ctypes.c_int, ctypes.c_int, u64p]),
    "ctl_ct_pack": (ctypes.c_int, [ctypes.POINTER(_Params), u64p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                   ctypes.POINTER(ctypes.c_uint8), ctypes.c_uint64, u64p]),
    "ctl_ct_unpack": (ctypes.c_int, [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_uint8), ctypes.c_uint64, u64p,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), u64p]),
    "ctl_decrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, u64p,
                                   ctypes.c_void_p]),
    "ctl_decode": (ctypes.c_int, [ctypes.c_void_p, u64p, ctypes.c_int, ctypes.c_double, f64p]),
    "ctl_decode_items": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, u64p, f64p]),
    "ctl_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_forward_multi": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_dense": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_dense_groups": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int),
                                        ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "ctl_square": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_square_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_mul": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_poly3": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double, f64p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_double)]),
    "ctl_replicate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_rotate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "ctl_rescale": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int, ctypes.c_void_p]),
}

_LIB = None


def lib():
    """Load the shared library (raises if it is not built: there is no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcryptotl.so is not built (run paper_2205_11935_amd/build.py)")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _LIB = l
    return _LIB


def _check(rc: int):
    if rc != 0:
        raise CtlError(rc, (lib().ctl_last_error() or b"").decode())


def _params(log2n, q_bits, p_bits, log2_scale, sigma) -> _Params:
    if len(q_bits) > MAX_PRIMES:
        raise ValueError("at most %d ciphertext primes" % MAX_PRIMES)
    p = _Params()
    p.log2n, p.n_q, p.p_bits, p.log2_scale, p.sigma = log2n, len(q_bits), p_bits, log2_scale, sigma
    for i, b in enumerate(q_bits):
        p.q_bits[i] = b
    return p


def params_primes(log2n, q_bits, p_bits, log2_scale=40, sigma=3.2) -> List[int]:
    p = _params(log2n, q_bits, p_bits, log2_scale, sigma)
    out = (ctypes.c_uint64 * (len(q_bits) + 1))()
    n = ctypes.c_int()
    _check(lib().ctl_params_primes(ctypes.byref(p), out, ctypes.byref(n)))
    return [int(out[i]) for i in range(n.value)]


def galois_elt(log2n: int, rotation: int) -> int:
    p = _params(log2n, [40], 60, 40, 3.2)
    g = ctypes.c_uint64()
    _check(lib().ctl_galois_elt(ctypes.byref(p), rotation, ctypes.byref(g)))
    return int(g.value)


def sample(log2n, q_bits, p_bits, seed, tag, index, kind, modulus, n, sigma=3.2) -> np.ndarray:
    p = _params(log2n, q_bits, p_bits, 40, sigma)
    out = np.zeros(n, dtype=np.int64)
    _check(lib().ctl_sample(ctypes.byref(p), seed, tag, index, kind, modulus, n, out.ctypes.data_as(i64p)))
    return out


def _stream(stream) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def check_tensor(t, shape, device: int, what: str):
    """Check a device buffer before its address crosses the C ABI, which takes only sizes and a
    pointer: the tensor must be a contiguous torch.int64 tensor of exactly `shape` on cuda:`device`.
    Raises TypeError / ValueError naming `what` otherwise. Returns the pointer."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s: expected a torch.Tensor, got %s" % (what, type(t).__name__))
    if t.dtype != torch.int64:
        raise ValueError("%s: dtype %s, expected torch.int64 (uint64 residues)" % (what, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s: shape %s, expected %s" % (what, tuple(t.shape), tuple(shape)))
    if not t.is_contiguous():
        raise ValueError("%s: tensor is not contiguous" % what)
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError("%s: tensor on %s, expected cuda:%d" % (what, t.device, device))
    return _ptr(t)


def check_disjoint(a, b, what: str):
    """The library's outputs must not overlap its inputs."""
    a0, b0 = a.data_ptr(), b.data_ptr()
    a1, b1 = a0 + a.numel() * a.element_size(), b0 + b.numel() * b.element_size()
    if a0 < b1 and b0 < a1:
        raise ValueError("%s: output overlaps the input" % what)


def _batch_dims(t, what: str):
    """(n_ct, k) of a ciphertext batch [n_ct][2][k][N]."""
    if getattr(t, "dim", None) is None or t.dim() != 4 or t.shape[1] != 2:
        raise ValueError("%s: expected a ciphertext batch [n_ct][2][k][N], got shape %s"
                         % (what, tuple(getattr(t, "shape", ()))))
    return int(t.shape[0]), int(t.shape[2])


@dataclasses.dataclass
class ModelInfo:
    n_layers: int
    block: int
    items: int
    k_in: int
    k_out: int
    n_in: int
    n_out: int
    scale_in: float
    scale_out: float
    layer_k: List[int]
    layer_t: List[int]
    rotations: List[int]


class Keys:
    def __init__(self, ctx: "Context", sk, pk, evk):
        self.ctx, self.sk, self.pk, self.evk = ctx, sk, pk, evk
        ctx._handles.add(self)

    def secret(self) -> np.ndarray:
        s = np.zeros(self.ctx.n, dtype=np.int64)
        _check(lib().ctl_sk_export(self.sk, s.ctypes.data_as(i64p)))
        return s

    def public(self) -> np.ndarray:
        out = np.zeros((2, self.ctx.nq, self.ctx.n), dtype=np.uint64)
        _check(lib().ctl_pk_export(self.pk, out.ctypes.data_as(u64p)))
        return out

    def galois_key(self, g: int) -> np.ndarray:
        out = np.zeros((self.ctx.nq, 2, self.ctx.nq + 1, self.ctx.n), dtype=np.uint64)
        _check(lib().ctl_evk_export(self.evk, g, out.ctypes.data_as(u64p)))
        return out

    def galois_elements(self) -> List[int]:
        n = ctypes.c_int()
        _check(lib().ctl_evk_galois(self.evk, None, ctypes.byref(n)))
        out = (ctypes.c_uint64 * max(n.value, 1))()
        _check(lib().ctl_evk_galois(self.evk, out, ctypes.byref(n)))
        return [int(out[i]) for i in range(n.value)]

    def evaluation_keys(self) -> Dict[int, np.ndarray]:
        """Every evaluation key (Galois element -> [n_q][2][n_q+1][N]), as a client would send them."""
        return {g: self.galois_key(g) for g in self.galois_elements()}

    def nbytes(self) -> int:
        b = ctypes.c_uint64()
        _check(lib().ctl_evk_bytes(self.evk, ctypes.byref(b)))
        return int(b.value)

    def free(self):
        """Release the key handles (also done by the context's close(): a handle must not outlive
        the context it was made on)."""
        if _LIB is not None:
            for f, h in (("ctl_sk_free", self.sk), ("ctl_pk_free", self.pk), ("ctl_evk_free", self.evk)):
                if h:
                    getattr(_LIB, f)(h)
        self.sk = self.pk = self.evk = None

    def __del__(self):
        self.free()


class Model:
    def __init__(self, ctx: "Context", handle):
        self.ctx, self.handle = ctx, handle
        ctx._handles.add(self)
        info = _ModelInfo()
        _check(lib().ctl_model_get_info(handle, ctypes.byref(info)))
        rots = (ctypes.c_int32 * max(info.n_rotations, 1))()
        n = ctypes.c_int()
        _check(lib().ctl_model_rotations(handle, rots, ctypes.byref(n)))
        self.info = ModelInfo(info.n_layers, info.block, info.items, info.k_in, info.k_out, info.n_in,
                              info.n_out, info.scale_in, info.scale_out, list(info.layer_k)[: info.n_layers],
                              list(info.layer_t)[: info.n_layers], [int(rots[i]) for i in range(n.value)])

    def nbytes(self) -> int:
        b = ctypes.c_uint64()
        _check(lib().ctl_model_bytes(self.handle, ctypes.byref(b)))
        return int(b.value)

    def free(self):
        """Release the plaintext banks (also done by the context's close())."""
        if _LIB is not None and self.handle:
            _LIB.ctl_model_free(self.handle)
        self.handle = None

    def __del__(self):
        self.free()


class Context:
    """One CKKS parameter set on one GPU."""

    def __init__(self, log2n: int, q_bits: Sequence[int], p_bits: int, log2_scale: int, sigma: float = 3.2,
                 device: int = 0, torch_allocator: bool = True):
        import torch
        self._torch = torch
        self._handles = weakref.WeakSet()          # keys and models made on this context
        self.log2n, self.n, self.nq = log2n, 1 << log2n, len(q_bits)
        self.device = device
        self.scale = float(2.0 ** log2_scale)
        self._params = _params(log2n, q_bits, p_bits, log2_scale, sigma)
        h = ctypes.c_void_p()
        torch.cuda.init()
        _check(lib().ctl_ctx_create(ctypes.byref(self._params), device, ctypes.byref(h)))
        self.handle = h
        self._hooks = None
        if torch_allocator:
            dev = device

            def _alloc(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
                except Exception:       # noqa: BLE001 -- report failure to the library as NULL
                    return None

            def _free(ptr, stream, user):
                torch.cuda.caching_allocator_delete(ptr)

            self._hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))
            _check(lib().ctl_set_allocator(self.handle, self._hooks[0], self._hooks[1], None))
        pr = (ctypes.c_uint64 * (self.nq + 1))()
        n = ctypes.c_int()
        _check(lib().ctl_ctx_primes(self.handle, pr, ctypes.byref(n)))
        self.primes = [int(pr[i]) for i in range(n.value)]

    def set_allocator(self, alloc, free):
        """Install a device allocator for the context's workspace, keys and banks (before anything
        is allocated): alloc(nbytes, stream, user) -> device pointer or None (the library then
        fails with CTL_ENOMEM), free(ptr, stream, user). The ctypes thunks are kept on the context,
        so they live as long as it and the handles made on it do."""
        hooks = (_ALLOC_FN(alloc), _FREE_FN(free))
        _check(lib().ctl_set_allocator(self.handle, hooks[0], hooks[1], None))
        self._hooks = hooks

    @classmethod
    def for_workload(cls, w, **kw) -> "Context":
        return cls(w.log2n, w.q_bits, w.p_bits, w.log2_scale, w.sigma, **kw)

    def close(self):
        """Free the context, after the keys and models made on it (which may still be referenced,
        e.g. from a traceback; they become empty)."""
        if getattr(self, "handle", None):
            self._torch.cuda.synchronize()
            for h in list(self._handles):
                h.free()
            lib().ctl_ctx_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001 -- interpreter shutdown
            pass

    # ------------------------------------------------------------ buffers
    def empty_ct(self, n_ct: int, k: int):
        return self._torch.empty((n_ct, 2, k, self.n), dtype=self._torch.int64, device="cuda:%d" % self.device)

    def _dev(self, t, shape, what: str) -> ctypes.c_void_p:
        return check_tensor(t, shape, self.device, what)

    def _level(self, t, k_min: int, what: str):
        """(n_ct, k) of a ciphertext batch whose level this context holds, k >= k_min."""
        n_ct, k = _batch_dims(t, what)
        if not k_min <= k <= self.nq:
            raise ValueError("%s: %d primes, this call takes %d..%d" % (what, k, k_min, self.nq))
        return n_ct, k

    def _coeffs(self, m: np.ndarray, what: str):
        if m.shape != (self.n,):
            raise ValueError("%s: shape %s, expected (%d,)" % (what, m.shape, self.n))

    def workspace_bytes(self) -> int:
        b = ctypes.c_uint64()
        _check(lib().ctl_workspace_bytes(self.handle, ctypes.byref(b)))
        return int(b.value)

    # ------------------------------------------------------------ instrumentation
    def profile_enable(self, on: bool = True):
        _check(lib().ctl_profile_enable(self.handle, int(on)))

    def profile_read(self):
        """{kernel family: (launches, summed milliseconds, algorithmic work, work on FP64 primes)}
        since profiling was enabled (work: residue transforms or modular products, see ctl.h)."""
        out = {}
        for f in range(lib().ctl_profile_families()):
            n, ms, wk, fw = ctypes.c_int(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            _check(lib().ctl_profile_read(self.handle, f, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(wk),
                                          ctypes.byref(fw)))
            out[lib().ctl_profile_family_name(f).decode()] = (n.value, ms.value, wk.value, fw.value)
        return out

    def profile_bytes(self):
        """{kernel family: algorithmic HBM bytes of its recorded launches} (0 where not modelled)."""
        out = {}
        for f in range(lib().ctl_profile_families()):
            b = ctypes.c_double()
            _check(lib().ctl_profile_read_bytes(self.handle, f, ctypes.byref(b)))
            out[lib().ctl_profile_family_name(f).decode()] = b.value
        return out

    def profile_launches(self):
        """Every launch record since profiling was enabled, in launch order: dicts with the
        kernel family, milliseconds, work, FP64 work, algorithmic bytes, layer and phase."""
        n = ctypes.c_int()
        _check(lib().ctl_profile_launches(self.handle, ctypes.byref(n)))
        names = [lib().ctl_profile_family_name(f).decode() for f in range(lib().ctl_profile_families())]
        out = []
        for i in range(n.value):
            fam, layer = ctypes.c_int(), ctypes.c_int()
            ms, wk, fw, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            ph = ctypes.c_char_p()
            _check(lib().ctl_profile_launch(self.handle, i, ctypes.byref(fam), ctypes.byref(ms), ctypes.byref(wk),
                                            ctypes.byref(fw), ctypes.byref(by), ctypes.byref(layer), ctypes.byref(ph)))
            out.append({"family": names[fam.value], "ms": ms.value, "work": wk.value, "fp_work": fw.value,
                        "bytes": by.value, "layer": layer.value, "phase": (ph.value or b"").decode()})
        return out

    PROBES = {"add32": 0, "mul32": 1, "mad64": 2, "fma64": 3}

    def probe_valu(self, kind: str, iters: int = 4096, stream=None) -> float:
        """Measured vector-ALU lane operations per second of one instruction class (ctl_probe_valu)."""
        v = ctypes.c_double()
        _check(lib().ctl_probe_valu(self.handle, self.PROBES[kind], iters, ctypes.byref(v), _stream(stream)))
        return v.value

    # ------------------------------------------------------------ parity hook
    def ntt(self, buf, prime_idx: Sequence[int], inverse: bool = False, stream=None):
        idx = (ctypes.c_int32 * len(prime_idx))(*prime_idx)
        if buf.numel() != len(prime_idx) * self.n:
            raise ValueError("ntt: %d residues of %d words need %d elements, the buffer has %d"
                             % (len(prime_idx), self.n, len(prime_idx) * self.n, buf.numel()))
        p = self._dev(buf, tuple(buf.shape), "ntt buffer")
        _check(lib().ctl_ntt(self.handle, p, len(prime_idx), idx, int(inverse), _stream(stream)))

    def ct_export(self, ct, coeff: bool = False, stream=None) -> np.ndarray:
        """Device residues [..][k][N] in NTT form -> host uint64 array of the same shape, in NTT or
        coefficient form (ctl_ct_export)."""
        if ct.dim() < 2 or ct.shape[-1] != self.n:
            raise ValueError("ct_export: expected [..][k][N], got %s" % (tuple(ct.shape),))
        k = int(ct.shape[-2])
        n_poly = ct.numel() // (k * self.n)
        p = self._dev(ct, tuple(ct.shape), "ct_export input")
        out = np.zeros(tuple(ct.shape), dtype=np.uint64)
        _check(lib().ctl_ct_export(self.handle, p, k, n_poly, CTL_FORM_COEFF if coeff else CTL_FORM_NTT,
                                   out.ctypes.data_as(u64p), _stream(stream)))
        return out

    def ct_import(self, host: np.ndarray, coeff: bool = False, out=None, stream=None):
        """Host residues [..][k][N] (NTT or coefficient form) -> device tensor in NTT form (ctl_ct_import)."""
        h = np.ascontiguousarray(host, dtype=np.uint64)
        if h.ndim < 2 or h.shape[-1] != self.n:
            raise ValueError("ct_import: expected [..][k][N], got %s" % (h.shape,))
        k = int(h.shape[-2])
        if out is None:
            out = self._torch.empty(h.shape, dtype=self._torch.int64, device="cuda:%d" % self.device)
        p = self._dev(out, h.shape, "ct_import output")
        _check(lib().ctl_ct_import(self.handle, h.ctypes.data_as(u64p), k, h.size // (k * self.n),
                                   CTL_FORM_COEFF if coeff else CTL_FORM_NTT, p, _stream(stream)))
        return out

    def pt_import(self, coeffs: np.ndarray, k: int, ext: bool = False, out=None, stream=None):
        """Signed integer plaintexts [n_pt][N] -> device [n_pt][k (+1 with ext)][N] NTT form (ctl_pt_import)."""
        m = np.ascontiguousarray(coeffs, dtype=np.int64)
        if m.ndim != 2 or m.shape[1] != self.n:
            raise ValueError("pt_import: expected [n_pt][N], got %s" % (m.shape,))
        shape = (m.shape[0], k + (1 if ext else 0), self.n)
        if out is None:
            out = self._torch.empty(shape, dtype=self._torch.int64, device="cuda:%d" % self.device)
        p = self._dev(out, shape, "pt_import output")
        _check(lib().ctl_pt_import(self.handle, m.ctypes.data_as(i64p), m.shape[0], k, int(ext), p, _stream(stream)))
        return out

    # ------------------------------------------------------------ client side
    def keygen(self, seed: int, rotations: Sequence[int], relin: bool = True) -> Keys:
        rots = (ctypes.c_int32 * max(len(rotations), 1))(*rotations)
        sk, pk, evk = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().ctl_keygen(self.handle, seed, rots, len(rotations), int(relin), ctypes.byref(sk),
                                ctypes.byref(pk), ctypes.byref(evk)))
        return Keys(self, sk, pk, evk)

    def import_keys(self, keys: Dict[int, np.ndarray]) -> Keys:
        """Evaluation keys received from a client (Galois element -> [n_q][2][n_q+1][N] uint64)."""
        gs = sorted(keys)
        arrs = [np.ascontiguousarray(keys[g], dtype=np.uint64) for g in gs]
        for a in arrs:
            if a.shape != (self.nq, 2, self.nq + 1, self.n):
                raise ValueError("key shape %s, expected %s" % (a.shape, (self.nq, 2, self.nq + 1, self.n)))
        elts = (ctypes.c_uint64 * max(len(gs), 1))(*gs)
        ptrs = (u64p * max(len(arrs), 1))(*[a.ctypes.data_as(u64p) for a in arrs])
        h = ctypes.c_void_p()
        _check(lib().ctl_evk_import(self.handle, elts, len(gs), ptrs, ctypes.byref(h)))
        return Keys(self, None, None, h)

    def encode(self, slots: np.ndarray, scale: float) -> np.ndarray:
        z = np.ascontiguousarray(slots, dtype=np.float64)
        out = np.zeros(self.n, dtype=np.int64)
        _check(lib().ctl_encode(self.handle, z.ctypes.data_as(f64p), scale, out.ctypes.data_as(i64p)))
        return out

    def encode_items(self, model: Model, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(self.n, dtype=np.int64)
        _check(lib().ctl_encode_items(self.handle, model.handle, x.ctypes.data_as(f64p), x.shape[0],
                                      out.ctypes.data_as(i64p)))
        return out

    def encrypt(self, keys: Keys, coeffs: np.ndarray, seed: int, out=None, stream=None):
        m = np.ascontiguousarray(coeffs, dtype=np.int64)
        self._coeffs(m, "plaintext")
        if out is None:
            out = self.empty_ct(1, self.nq)[0]
        p = self._dev(out, (2, self.nq, self.n), "encrypt output")
        _check(lib().ctl_encrypt(self.handle, keys.pk, m.ctypes.data_as(i64p), seed, p, _stream(stream)))
        return out

    def encrypt_sym(self, keys: Keys, coeffs: np.ndarray, seed: int, out=None, stream=None):
        m = np.ascontiguousarray(coeffs, dtype=np.int64)
        self._coeffs(m, "plaintext")
        if out is None:
            out = self.empty_ct(1, self.nq)[0]
        p = self._dev(out, (2, self.nq, self.n), "encrypt output")
        _check(lib().ctl_encrypt_sym(self.handle, keys.sk, m.ctypes.data_as(i64p), seed, p, _stream(stream)))
        return out

    def expand_seeded(self, c0: np.ndarray, seed: int, out=None, stream=None):
        c0 = np.ascontiguousarray(c0, dtype=np.uint64)
        if c0.size != self.nq * self.n:
            raise ValueError("c0: %d words, expected %d" % (c0.size, self.nq * self.n))
        if out is None:
            out = self.empty_ct(1, self.nq)[0]
        p = self._dev(out, (2, self.nq, self.n), "expanded ciphertext")
        _check(lib().ctl_expand_seeded(self.handle, c0.ctypes.data_as(u64p), seed, p, _stream(stream)))
        return out

    def decrypt(self, keys: Keys, ct, k: int, stream=None) -> np.ndarray:
        p = self._dev(ct, (2, k, self.n), "ciphertext")
        out = np.zeros((k, self.n), dtype=np.uint64)
        _check(lib().ctl_decrypt(self.handle, keys.sk, p, k, out.ctypes.data_as(u64p), _stream(stream)))
        return out

    def decode(self, residues: np.ndarray, scale: float) -> np.ndarray:
        r = np.ascontiguousarray(residues, dtype=np.uint64)
        if r.ndim != 2 or r.shape[1] != self.n or not 1 <= r.shape[0] <= self.nq:
            raise ValueError("residues: shape %s, expected (k, %d) with 1 <= k <= %d" % (r.shape, self.n, self.nq))
        out = np.zeros(self.n // 2, dtype=np.float64)
        _check(lib().ctl_decode(self.handle, r.ctypes.data_as(u64p), r.shape[0], scale, out.ctypes.data_as(f64p)))
        return out

    def decode_items(self, model: Model, residues: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(residues, dtype=np.uint64)
        if r.shape != (model.info.k_out, self.n):
            raise ValueError("residues: shape %s, expected %s" % (r.shape, (model.info.k_out, self.n)))
        out = np.zeros((model.info.items, model.info.n_out), dtype=np.float64)
        _check(lib().ctl_decode_items(self.handle, model.handle, r.ctypes.data_as(u64p), out.ctypes.data_as(f64p)))
        return out

    # ------------------------------------------------------------ server side
    @staticmethod
    def _descs(layers, lazy: bool, qp: bool = False):
        arr = (_LayerDesc * len(layers))()
        for i, l in enumerate(layers):
            if isinstance(l, Layer):
                arr[i].kind, arr[i].n_in, arr[i].n_out, arr[i].t1, arr[i].f = l.kind, l.n_in, l.n_out, l.t1, l.f
                arr[i].act = l.act
                for j in range(4):
                    arr[i].coef[j] = float(l.coef[j])
                lazy_ok = l.kind == CTL_LAYER_DENSE
                qp_ok = True                       # every kind has hoisted rotations
            else:
                arr[i].n_in, arr[i].n_out, arr[i].t1 = l[0], l[1], l[2]
                arr[i].act = l[3] if len(l) > 3 else (CTL_ACT_SQUARE if i + 1 < len(layers) else CTL_ACT_NONE)
                lazy_ok = qp_ok = True
            arr[i].flags = (CTL_LAYER_BABY_QP if (qp and qp_ok) else
                            CTL_LAYER_LAZY_GIANT if (lazy and lazy_ok) else 0)
        return arr

    @staticmethod
    def _f64_ptrs(weights):
        """(arrays kept alive, double* array); None entries (average pools) become NULL."""
        ws = [None if w is None else np.ascontiguousarray(w, dtype=np.float64) for w in weights]
        return ws, (f64p * len(ws))(*[None if w is None else w.ctypes.data_as(f64p) for w in ws])

    def load_model(self, layers, weights: Sequence[np.ndarray], lazy: bool = False, qp: bool = False) -> Model:
        """layers: Layer descriptors or (n_in, n_out, t1[, act]) dense tuples; weights per layer:
        float64 [n_out][n_in] (dense), [f] taps (convolution), None (average pool);
        lazy: single-ModDown giant steps (CTL_LAYER_LAZY_GIANT) on every dense layer; qp: baby
        steps over Q*P as well (CTL_LAYER_BABY_QP)."""
        ws, ptrs = self._f64_ptrs(weights)
        h = ctypes.c_void_p()
        _check(lib().ctl_model_load(self.handle, self._descs(layers, lazy, qp), len(layers), ptrs, ctypes.byref(h)))
        return Model(self, h)

    def load_model_raw(self, layers, pts: Sequence[np.ndarray], lazy: bool = False, qp: bool = False) -> Model:
        """pts: int64 [t][N] encoded diagonal plaintexts per layer."""
        ps = [np.ascontiguousarray(p, dtype=np.int64) for p in pts]
        ptrs = (i64p * len(ps))(*[p.ctypes.data_as(i64p) for p in ps])
        h = ctypes.c_void_p()
        _check(lib().ctl_model_load_raw(self.handle, self._descs(layers, lazy, qp), len(layers), ptrs,
                                        ctypes.byref(h)))
        return Model(self, h)

    def load_model_ex(self, layers, weights=None, pts=None, lazy: bool = False, block: int = 0, k_in: int = 0,
                      scale_in: float = 0.0, qp: bool = False) -> Model:
        """One of weights (float64 [n_out][n_in] per layer) or pts (int64 [t][N] per layer), with plan
        overrides: a shared slot stride `block`, the starting level `k_in`, the input scale."""
        opts = _ModelOpts(block, k_in, scale_in)
        h = ctypes.c_void_p()
        wp = pp = None
        if weights is not None:
            ws, wp = self._f64_ptrs(weights)
        if pts is not None:
            ps = [np.ascontiguousarray(p, dtype=np.int64) for p in pts]
            pp = (i64p * len(ps))(*[p.ctypes.data_as(i64p) for p in ps])
        _check(lib().ctl_model_load_ex(self.handle, self._descs(layers, lazy, qp), len(layers), wp, pp,
                                       ctypes.byref(opts), ctypes.byref(h)))
        return Model(self, h)

    def knob(self, name: str, value: Optional[int] = None) -> int:
        """Read (value None) or set a launch knob (the names of KNOBS: "mac_chunk", "mac_cts", "keyip_xcd",
        "mac_direct", "ntt_xcd", "mac_limb", "keyip_rr", "ntt_split", "ntt_loop", "fuse_rescale"; ranges
        in ctl.h)."""
        if value is not None:
            _check(lib().ctl_knob_set(self.handle, KNOBS[name], int(value)))
        v = ctypes.c_int()
        _check(lib().ctl_knob_get(self.handle, KNOBS[name], ctypes.byref(v)))
        return v.value

    def workspace_freeze(self, frozen: bool = True):
        _check(lib().ctl_workspace_freeze(self.handle, int(frozen)))

    def forward(self, model: Model, keys: Keys, ct, out=None, stream=None):
        n_ct, _ = _batch_dims(ct, "forward input")
        pi = self._dev(ct, (n_ct, 2, model.info.k_in, self.n), "forward input")
        if out is None:
            out = self.empty_ct(n_ct, model.info.k_out)
        po = self._dev(out, (n_ct, 2, model.info.k_out, self.n), "forward output")
        check_disjoint(ct, out, "forward")
        _check(lib().ctl_forward(self.handle, model.handle, keys.evk, pi, po, n_ct, _stream(stream)))
        return out

    def forward_multi(self, model: Model, keys: Sequence[Keys], ct, out=None, stream=None):
        """forward on a batch mixing clients: ciphertext b is evaluated with keys[b]. Key products
        run once per run of consecutive ciphertexts with the same Keys object."""
        n_ct, _ = _batch_dims(ct, "forward input")
        if len(keys) != n_ct:
            raise ValueError("one Keys per ciphertext")
        pi = self._dev(ct, (n_ct, 2, model.info.k_in, self.n), "forward input")
        if out is None:
            out = self.empty_ct(n_ct, model.info.k_out)
        po = self._dev(out, (n_ct, 2, model.info.k_out, self.n), "forward output")
        check_disjoint(ct, out, "forward_multi")
        arr = (ctypes.c_void_p * n_ct)(*[kk.evk for kk in keys])
        _check(lib().ctl_forward_multi(self.handle, model.handle, arr, pi, po, n_ct, _stream(stream)))
        return out

    def dense(self, model: Model, layer: int, keys: Keys, ct, out=None, stream=None):
        n_ct, _ = _batch_dims(ct, "dense input")
        if not 0 <= layer < model.info.n_layers:
            raise ValueError("layer %d out of range" % layer)
        k = model.info.layer_k[layer]
        pi = self._dev(ct, (n_ct, 2, k, self.n), "dense input")
        if out is None:
            out = self.empty_ct(n_ct, k - 1)
        po = self._dev(out, (n_ct, 2, k - 1, self.n), "dense output")
        check_disjoint(ct, out, "dense")
        _check(lib().ctl_dense(self.handle, model.handle, layer, keys.evk, pi, po, n_ct, _stream(stream)))
        return out

    def dense_groups(self, models: Sequence[Model], counts: Sequence[int], keys: Keys, ct, layer: int = 0,
                     out=None, stream=None):
        """Layer `layer` of models[g] on counts[g] consecutive ciphertexts of ct, for every g, in
        one call (ctl_dense_groups: the ModUps, the final ModDown and the rescale shared)."""
        n_ct, _ = _batch_dims(ct, "dense_groups input")
        if len(models) != len(counts) or not models:
            raise ValueError("one count per model")
        if sum(counts) != n_ct or min(counts) < 1:
            raise ValueError("counts must be positive and add up to the batch (%d)" % n_ct)
        k = models[0].info.layer_k[layer]
        pi = self._dev(ct, (n_ct, 2, k, self.n), "dense_groups input")
        if out is None:
            out = self.empty_ct(n_ct, k - 1)
        po = self._dev(out, (n_ct, 2, k - 1, self.n), "dense_groups output")
        check_disjoint(ct, out, "dense_groups")
        ms = (ctypes.c_void_p * len(models))(*[m.handle for m in models])
        cs = (ctypes.c_int * len(counts))(*[int(x) for x in counts])
        _check(lib().ctl_dense_groups(self.handle, ms, cs, len(models), layer, keys.evk, pi, po, _stream(stream)))
        return out

    def mul(self, keys: Keys, a, b, out=None, stream=None):
        n_ct, k = self._level(a, 2, "mul operand a")
        pa = self._dev(a, (n_ct, 2, k, self.n), "mul operand a")
        pb = self._dev(b, (n_ct, 2, k, self.n), "mul operand b")
        if out is None:
            out = self.empty_ct(n_ct, k - 1)
        po = self._dev(out, (n_ct, 2, k - 1, self.n), "mul output")
        check_disjoint(a, out, "mul")
        check_disjoint(b, out, "mul")
        _check(lib().ctl_mul(self.handle, keys.evk, k, pa, pb, po, n_ct, _stream(stream)))
        return out

    def poly3(self, keys: Keys, ct, scale: float, coef: Sequence[float], out=None, stream=None):
        """Degree-3 activation; returns (output [n][2][k-2][N], output scale)."""
        n_ct, k = self._level(ct, 3, "poly3 input")
        pi = self._dev(ct, (n_ct, 2, k, self.n), "poly3 input")
        if out is None:
            out = self.empty_ct(n_ct, k - 2)
        po = self._dev(out, (n_ct, 2, k - 2, self.n), "poly3 output")
        check_disjoint(ct, out, "poly3")
        cf = (ctypes.c_double * 4)(*[float(c) for c in coef])
        so = ctypes.c_double()
        _check(lib().ctl_poly3(self.handle, keys.evk, k, scale, cf, pi, po, n_ct, _stream(stream), ctypes.byref(so)))
        return out, so.value

    def square(self, keys: Keys, ct, out=None, stream=None):
        n_ct, k = self._level(ct, 2, "square input")
        pi = self._dev(ct, (n_ct, 2, k, self.n), "square input")
        if out is None:
            out = self.empty_ct(n_ct, k - 1)
        po = self._dev(out, (n_ct, 2, k - 1, self.n), "square output")
        check_disjoint(ct, out, "square")
        _check(lib().ctl_square(self.handle, keys.evk, k, pi, po, n_ct, _stream(stream)))
        return out

    def square_noalloc(self, keys: Keys, ct, out, stream=None):
        """ctl_square without any device allocation (the library's fixed per-GPU scratch array);
        `out` must be given, since allocating it here would defeat the purpose."""
        n_ct, k = self._level(ct, 2, "square input")
        pi = self._dev(ct, (n_ct, 2, k, self.n), "square input")
        po = self._dev(out, (n_ct, 2, k - 1, self.n), "square output")
        check_disjoint(ct, out, "square_noalloc")
        _check(lib().ctl_square_noalloc(self.handle, keys.evk, k, pi, po, n_ct, _stream(stream)))
        return out

    def replicate(self, keys: Keys, ct, width: int, out=None, stream=None):
        n_ct, k = self._level(ct, 1, "replicate input")
        pi = self._dev(ct, (n_ct, 2, k, self.n), "replicate input")
        if out is None:
            out = self.empty_ct(n_ct, k)
        po = self._dev(out, (n_ct, 2, k, self.n), "replicate output")
        check_disjoint(ct, out, "replicate")
        _check(lib().ctl_replicate(self.handle, keys.evk, k, width, pi, po, n_ct, _stream(stream)))
        return out

    def rotate(self, keys: Keys, ct, rotation: int, out=None, stream=None):
        n_ct, k = self._level(ct, 1, "rotate input")
        pi = self._dev(ct, (n_ct, 2, k, self.n), "rotate input")
        if out is None:
            out = self.empty_ct(n_ct, k)
        po = self._dev(out, (n_ct, 2, k, self.n), "rotate output")
        check_disjoint(ct, out, "rotate")
        _check(lib().ctl_rotate(self.handle, keys.evk, k, rotation, pi, po, n_ct, _stream(stream)))
        return out

    def rescale(self, ct, out=None, stream=None):
        n_ct, k = self._level(ct, 2, "rescale input")
        pi = self._dev(ct, (n_ct, 2, k, self.n), "rescale input")
        if out is None:
            out = self.empty_ct(n_ct, k - 1)
        po = self._dev(out, (n_ct, 2, k - 1, self.n), "rescale output")
        check_disjoint(ct, out, "rescale")
        _check(lib().ctl_rescale(self.handle, k, pi, po, n_ct, _stream(stream)))
        return out


def ct_packed_bytes(log2n, q_bits, p_bits, k: int, n_poly: int) -> int:
    b = ctypes.c_uint64()
    _check(lib().ctl_ct_packed_bytes(ctypes.byref(_params(log2n, q_bits, p_bits, 40, 3.2)), k, n_poly, ctypes.byref(b)))
    return int(b.value)


def ct_pack(log2n, q_bits, p_bits, ct: np.ndarray, seed: int = 0) -> bytes:
    """Serialize host residues [n_poly][k][N] (n_poly = 1: c0 of a seeded upload, with its seed)."""
    ct = np.ascontiguousarray(ct, dtype=np.uint64)
    n_poly, k = ct.shape[0], ct.shape[1]
    prm = _params(log2n, q_bits, p_bits, 40, 3.2)
    size = ct_packed_bytes(log2n, q_bits, p_bits, k, n_poly)
    out = np.zeros(size, dtype=np.uint8)
    ln = ctypes.c_uint64()
    _check(lib().ctl_ct_pack(ctypes.byref(prm), ct.ctypes.data_as(u64p), k, n_poly, seed,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), size, ctypes.byref(ln)))
    return out[: ln.value].tobytes()


def ct_unpack(log2n, q_bits, p_bits, data: bytes):
    """-> (residues [n_poly][k][N] uint64, seed)."""
    buf = np.frombuffer(data, dtype=np.uint8).copy()
    out = np.zeros(2 * len(q_bits) << log2n, dtype=np.uint64)
    k, npl, seed = ctypes.c_int(), ctypes.c_int(), ctypes.c_uint64()
    _check(lib().ctl_ct_unpack(ctypes.byref(_params(log2n, q_bits, p_bits, 40, 3.2)),
                               buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), len(data),
                               out.ctypes.data_as(u64p), ctypes.byref(k), ctypes.byref(npl), ctypes.byref(seed)))
    n = 1 << log2n
    return out[: npl.value * k.value * n].reshape(npl.value, k.value, n), int(seed.value)


def to_numpy_u64(t) -> np.ndarray:
    """Device int64 tensor of residues -> host uint64 array (bit reinterpretation)."""
    return t.detach().cpu().numpy().view(np.uint64)


def from_numpy_u64(a: np.ndarray, device: int = 0):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to("cuda:%d" % device)
