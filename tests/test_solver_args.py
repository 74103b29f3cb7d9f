"""Host-side argument checks of the torch layer (no GPU needed): every
tensor handed to the C entry points must be FP64 (or the stated dtype),
contiguous, on the expected device and of the expected size, else
ValueError before any call."""
import pytest
import torch

from paper_1504_08340_amd.solver import check_tensor


def test_accepts_a_matching_tensor():
    t = torch.zeros(12, dtype=torch.float64)
    assert check_tensor("x", t, 12, "cpu") is t


@pytest.mark.parametrize("t,match", [
    (torch.zeros(12, dtype=torch.float32), "dtype"),
    (torch.zeros(11, dtype=torch.float64), "elements"),
    (torch.zeros(24, dtype=torch.float64)[::2], "contiguous"),
    ([0.0] * 12, "torch.Tensor"),
])
def test_rejects(t, match):
    with pytest.raises(ValueError, match=match):
        check_tensor("x", t, 12, "cpu")


def test_rejects_wrong_device():
    with pytest.raises(ValueError, match="expected cuda:0"):
        check_tensor("x", torch.zeros(12, dtype=torch.float64), 12, "cuda:0")
