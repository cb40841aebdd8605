"""Host-side checks of the Python binding's argument marshalling (no GPU):
request operands that are not float64 GPU tensors are refused before any
pointer reaches the library."""
import pytest
import torch

from paper_1608_00044_amd import spchol


def test_request_operands_refuse_host_tensors():
    b = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(TypeError):
        spchol.request_operands(8, 8, None, b, b.clone())
    with pytest.raises(TypeError):
        spchol.request_operands(8, 8, torch.zeros(8, dtype=torch.float64), b, b.clone())


def test_request_operands_refuse_float32():
    b = torch.zeros(8, dtype=torch.float32)
    with pytest.raises(TypeError):
        spchol.request_operands(8, 8, None, b, b.clone())


def test_request_operands_refuse_non_tensors():
    import numpy as np

    with pytest.raises(TypeError):
        spchol.request_operands(4, 4, None, np.zeros(4), np.zeros(4))
