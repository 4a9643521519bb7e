"""The binding's checks of device buffers, on the CPU: the C ABI takes a pointer and counts only,
so a tensor of the wrong dtype, shape, layout or device must be rejected in Python before its
address reaches a kernel."""
import pytest
import torch

import paper_2205_11935_amd as ctl


def test_rejects_wrong_dtype():
    t = torch.zeros((2, 2, 3, 16), dtype=torch.int32)
    with pytest.raises(ValueError, match="dtype"):
        ctl.check_tensor(t, (2, 2, 3, 16), 0, "x")


def test_rejects_wrong_shape():
    t = torch.zeros((2, 2, 3, 16), dtype=torch.int64)
    for shape in [(2, 2, 4, 16), (3, 2, 3, 16), (2, 2, 3, 32), (2, 2, 3)]:
        with pytest.raises(ValueError, match="shape"):
            ctl.check_tensor(t, shape, 0, "x")


def test_rejects_non_contiguous():
    t = torch.zeros((2, 2, 6, 16), dtype=torch.int64)[:, :, ::2]
    assert tuple(t.shape) == (2, 2, 3, 16)
    with pytest.raises(ValueError, match="contiguous"):
        ctl.check_tensor(t, (2, 2, 3, 16), 0, "x")


def test_rejects_host_tensor_and_non_tensor():
    t = torch.zeros((1, 2, 3, 16), dtype=torch.int64)
    with pytest.raises(ValueError, match="cuda:0"):
        ctl.check_tensor(t, (1, 2, 3, 16), 0, "x")
    with pytest.raises(TypeError):
        ctl.check_tensor(t.numpy(), (1, 2, 3, 16), 0, "x")


def test_batch_dims():
    assert ctl._batch_dims(torch.zeros((5, 2, 3, 8), dtype=torch.int64), "x") == (5, 3)
    for shape in [(2, 3, 8), (5, 3, 3, 8), (5, 2, 3, 8, 1)]:
        with pytest.raises(ValueError, match="ciphertext batch"):
            ctl._batch_dims(torch.zeros(shape, dtype=torch.int64), "x")


def test_overlap():
    base = torch.zeros((4, 2, 3, 8), dtype=torch.int64)
    ctl.check_disjoint(base[:2], base[2:], "x")
    with pytest.raises(ValueError, match="overlaps"):
        ctl.check_disjoint(base[:3], base[2:], "x")
    with pytest.raises(ValueError, match="overlaps"):
        ctl.check_disjoint(base, base, "x")
