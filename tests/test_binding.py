"""Host-side checks of the Python binding (no GPU needed): device fields
handed to the library as bare pointers are validated first, so that a tensor
on the wrong device, of the wrong type or of the wrong size is refused before
any kernel could read or write outside it."""
import numpy as np
import pytest
import torch

from paper_1712_05145_amd import ffth

N = (4, 6, 8)


def test_check_field_accepts_exact_tensor():
    t = torch.zeros((2, 6) + N, dtype=torch.float64)
    assert ffth.check_field(t, "cpu", (2, 6) + N, "out") is t


@pytest.mark.parametrize("bad,why", [
    (lambda: torch.zeros((2, 6) + N, dtype=torch.float32), "dtype"),
    (lambda: torch.zeros((1, 6) + N, dtype=torch.float64), "shape"),          # too few loads
    (lambda: torch.zeros((2, 6) + N[::-1], dtype=torch.float64), "shape"),    # transposed grid
    (lambda: torch.zeros((2, 6) + N + (2,), dtype=torch.float64)[..., 0], "contiguous"),
    (lambda: np.zeros((2, 6) + N), "torch tensor"),
])
def test_check_field_refuses(bad, why):
    with pytest.raises(ffth.FFTHError) as e:
        ffth.check_field(bad(), "cpu", (2, 6) + N, "out")
    assert e.value.status == ffth.FFTH_ERR_INVALID
    assert why in str(e.value)


def test_check_field_refuses_other_device():
    """A host tensor given to a plan on the GPU is refused (its address would
    be read as a device address)."""
    t = torch.zeros((6,) + N, dtype=torch.float64)
    with pytest.raises(ffth.FFTHError) as e:
        ffth.check_field(t, torch.device("cuda", 0), (6,) + N, "tau")
    assert e.value.status == ffth.FFTH_ERR_INVALID and "cuda" in str(e.value)
