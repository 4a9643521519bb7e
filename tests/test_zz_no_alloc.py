"""The entry point that allocates nothing (ctl_square_noalloc, the library's fixed per-GPU scratch
array): through the C ABI it gives ctl_square's result bit for bit on two calls in a row, the
second with a smaller input, makes no allocation through the context's allocator hook and leaves
the context's workspace as it was; a batch beyond the scratch array is rejected before anything
runs."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_square_noalloc_equals_square():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_11935_amd as ctl
    w = W.LARGE
    c = ctl.Context.for_workload(w, torch_allocator=False)
    calls = {"n": 0}

    def alloc(nbytes, stream, user):
        calls["n"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream or 0)

    def free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    c.set_allocator(alloc, free)
    keys = c.keygen(w.seed_keys, [1], relin=True)
    msgs = W.raw_plaintexts(123, 4, c.n, bound_bits=40)
    ct = c.empty_ct(4, c.nq)
    for i in range(4):
        c.encrypt(keys, msgs[i], 4200 + i, out=ct[i])
    torch.cuda.synchronize()

    for n_ct, k in ((4, c.nq), (2, c.nq - 2)):           # the second call is smaller
        x = ct[:n_ct, :, :k].contiguous()
        want = c.square(keys, x)
        torch.cuda.synchronize()
        ws, before = c.workspace_bytes(), calls["n"]
        got = c.empty_ct(n_ct, k - 1)
        got.fill_(-1)
        c.square_noalloc(keys, x, got)
        torch.cuda.synchronize()
        assert calls["n"] == before and c.workspace_bytes() == ws
        assert torch.equal(got, want), (n_ct, k)

    # 6 ciphertexts at N = 2^14, k = 6 need 6 x 12 MiB: more than the 64 MiB array
    big = c.empty_ct(6, c.nq)
    big.zero_()
    out = c.empty_ct(6, c.nq - 1)
    out.fill_(7)
    with pytest.raises(ctl.CtlError) as ei:
        c.square_noalloc(keys, big, out)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7)
    # closing the context frees the handles made on it first, even those still referenced (here
    # through the traceback that pytest.raises keeps)
    c.close()
    assert keys.evk is None
