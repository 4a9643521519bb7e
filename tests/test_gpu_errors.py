"""Error paths of the C ABI on the GPU: each failing call returns its CTL_E* code, writes nothing
to its outputs and leaves its inputs as they were. CTL_ENOMEM comes from an allocator hook that
refuses on request; CTL_ELEVEL from a model deeper than the chain and from calls below the level
they need; CTL_ESCALE from values that do not fit the integer range of an encoding."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ENOMEM, ELEVEL, ESCALE = -2, -3, -4
SENTINEL = 0x5A5A5A5A5A5A5A5


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _filled(c, n_ct, k):
    t = c.empty_ct(n_ct, k)
    t.fill_(SENTINEL)
    return t


class _Hook:
    """A device allocator for the library that can be told to refuse (returns NULL). Installed
    with Context.set_allocator, which keeps its ctypes thunks alive as long as the context."""

    def __init__(self, ctl, c):
        self.refuse = False
        self.calls = 0
        dev = c.device

        def alloc(nbytes, stream, user):
            self.calls += 1
            if self.refuse:
                return None
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)

        def free(ptr, stream, user):
            torch.cuda.caching_allocator_delete(ptr)

        c.set_allocator(alloc, free)


def _small_setup(ctl, hook=False):
    w = W.SMALL
    c = ctl.Context.for_workload(w, torch_allocator=not hook)
    h = _Hook(ctl, c) if hook else None
    layers = [(l.n_in, l.n_out, l.t1) for l in w.layers]
    m = c.load_model(layers, W.weights(w), lazy=True, qp=True)
    keys = c.keygen(w.seed_keys, m.info.rotations, relin=True)
    x = W.inputs(w, 2, m.info.items)
    ct = c.empty_ct(2, c.nq)
    for i in range(2):
        c.encrypt(keys, c.encode_items(m, x[i]), 40 + i, out=ct[i])
    torch.cuda.synchronize()
    return w, c, h, m, keys, ct


def test_enomem_leaves_outputs_unchanged():
    _need_gpu()
    import paper_2205_11935_amd as ctl
    w, c, h, m, keys, ct = _small_setup(ctl, hook=True)
    assert h.calls > 0                                  # keys, banks and workspace come through the hook
    ct_before = ct.clone()
    out = _filled(c, 2, m.info.k_out)
    h.refuse = True
    with pytest.raises(ctl.CtlError) as ei:
        c.forward(m, keys, ct, out=out)
    assert ei.value.code == ENOMEM
    torch.cuda.synchronize()
    assert torch.all(out == SENTINEL)
    assert torch.equal(ct, ct_before)
    with pytest.raises(ctl.CtlError) as ei:             # a bank that cannot be allocated
        c.load_model([(l.n_in, l.n_out, l.t1) for l in w.layers], W.weights(w), lazy=True, qp=True)
    assert ei.value.code == ENOMEM
    # once the hook allocates again the same call succeeds and equals a context without the hook
    h.refuse = False
    c.forward(m, keys, ct, out=out)
    ref_c = ctl.Context.for_workload(w)
    ref_m = ref_c.load_model([(l.n_in, l.n_out, l.t1) for l in w.layers], W.weights(w), lazy=True, qp=True)
    ref_k = ref_c.keygen(w.seed_keys, ref_m.info.rotations, relin=True)
    ref_ct = ref_c.empty_ct(2, ref_c.nq)
    ref_ct.copy_(ct)
    assert torch.equal(ref_c.forward(ref_m, ref_k, ref_ct), out)
    # a frozen workspace that would have to grow fails the same way
    c.workspace_freeze(True)
    try:
        big = c.empty_ct(8, c.nq)
        big.zero_()
        out8 = _filled(c, 8, m.info.k_out)
        with pytest.raises(ctl.CtlError) as ei:
            c.forward(m, keys, big, out=out8)
        assert ei.value.code == ENOMEM
        torch.cuda.synchronize()
        assert torch.all(out8 == SENTINEL)
    finally:
        c.workspace_freeze(False)


def test_enomem_frozen_workspace():
    """A frozen workspace that would have to grow gives CTL_ENOMEM and leaves the output and
    the input as they were; unfrozen, the same call succeeds."""
    _need_gpu()
    import paper_2205_11935_amd as ctl
    w, c, _, m, keys, ct = _small_setup(ctl)
    c.forward(m, keys, ct)                      # the workspace now fits batches of 2
    big = c.empty_ct(8, c.nq)
    big.zero_()
    before = big.clone()
    out8 = _filled(c, 8, m.info.k_out)
    c.workspace_freeze(True)
    try:
        with pytest.raises(ctl.CtlError) as ei:
            c.forward(m, keys, big, out=out8)
        assert ei.value.code == ENOMEM
        torch.cuda.synchronize()
        assert torch.all(out8 == SENTINEL) and torch.equal(big, before)
    finally:
        c.workspace_freeze(False)
    c.forward(m, keys, big, out=out8)
    torch.cuda.synchronize()
    assert not torch.all(out8 == SENTINEL)


def test_elevel():
    _need_gpu()
    import paper_2205_11935_amd as ctl
    w, c, _, m, keys, ct = _small_setup(ctl)
    # the small chain has 3 primes: dense (3 -> 2), x^2 (2 -> 1), then no level for a second layer
    with pytest.raises(ctl.CtlError) as ei:
        c.load_model([(64, 64, 64), (64, 64, 64)], [np.eye(64), np.eye(64)], lazy=True, qp=True)
    assert ei.value.code == ELEVEL
    with pytest.raises(ctl.CtlError) as ei:
        c.load_model_ex([(64, 64, 64)], weights=[np.eye(64)], k_in=1)
    assert ei.value.code == ELEVEL
    lib = ctl.lib()
    one = ct[:, :, :1].contiguous()
    two = ct[:, :, :2].contiguous()
    before = (one.clone(), two.clone())
    out = _filled(c, 2, 1)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())        # noqa: E731
    # rescale, square and the cubic below the primes they consume, straight through the C ABI
    assert lib.ctl_rescale(c.handle, 1, p(one), p(out), 2, st) == ELEVEL
    assert lib.ctl_square(c.handle, keys.evk, 1, p(one), p(out), 2, st) == ELEVEL
    coef = (ctypes.c_double * 4)(0.1, 0.2, 0.3, 0.4)
    assert lib.ctl_poly3(c.handle, keys.evk, 2, c.scale, coef, p(two), p(out), 2, st, None) == ELEVEL
    assert lib.ctl_rescale(c.handle, c.nq + 1, p(ct), p(out), 2, st) == ELEVEL
    torch.cuda.synchronize()
    assert torch.all(out == SENTINEL)
    assert torch.equal(one, before[0]) and torch.equal(two, before[1])


def test_escale():
    _need_gpu()
    import paper_2205_11935_amd as ctl
    w, c, _, m, keys, ct = _small_setup(ctl)
    big = np.full(c.n // 2, 1e11)                       # constant slots: coefficient 0 = 1e11 * 2^30 > 2^62
    with pytest.raises(ctl.CtlError) as ei:
        c.encode(big, c.scale)
    assert ei.value.code == ESCALE
    with pytest.raises(ctl.CtlError) as ei:
        c.load_model([(64, 64, 64)], [np.full((64, 64), 1e12)], lazy=True, qp=True)
    assert ei.value.code == ESCALE
    bad = np.zeros((64, c.n), dtype=np.int64)
    bad[3, 5] = 1 << 62
    with pytest.raises(ctl.CtlError) as ei:
        c.load_model_raw([(64, 64, 64)], [bad], lazy=True, qp=True)
    assert ei.value.code == ESCALE
    out1 = _filled(c, 1, c.nq)
    msg = np.zeros(c.n, dtype=np.int64)
    msg[0] = -(1 << 62)
    with pytest.raises(ctl.CtlError) as ei:
        c.encrypt(keys, msg, 1, out=out1[0])
    assert ei.value.code == ESCALE
    # a cubic whose constants overflow the 62-bit range at this scale
    before = ct.clone()
    out = _filled(c, 2, c.nq - 2)
    with pytest.raises(ctl.CtlError) as ei:
        c.poly3(keys, ct, c.scale, (1e30, 0.0, 0.0, 0.0), out=out)
    assert ei.value.code == ESCALE
    torch.cuda.synchronize()
    assert torch.all(out == SENTINEL) and torch.all(out1 == SENTINEL)
    assert torch.equal(ct, before)
