"""Host-side checks of the tensors the Python binding hands to the kernels: a buffer too
small, of the wrong type, on the host or on another GPU is refused before any launch."""
import types

import pytest
import torch

from paper_1809_03606_amd import binding


class FakeGpuTensor:
    """What the checks read of a torch tensor, for a machine without a GPU."""

    def __init__(self, n, dtype, index=0, contiguous=True):
        self.is_cuda = True
        self.device = types.SimpleNamespace(index=index)
        self.dtype = dtype
        self._n = n
        self._contiguous = contiguous

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._contiguous


def test_device_buffer_accepts_a_fitting_tensor():
    binding._device_buffer(FakeGpuTensor(64, torch.uint8), "status", (torch.uint8,), 64, 0)


@pytest.mark.parametrize("t,exc", [
    (None, ValueError),
    (torch.zeros(64, dtype=torch.uint8), ValueError),             # host memory
    (FakeGpuTensor(64, torch.uint8, index=1), ValueError),        # another GPU
    (FakeGpuTensor(64, torch.uint8, contiguous=False), ValueError),
    (FakeGpuTensor(64, torch.int16), TypeError),
    (FakeGpuTensor(63, torch.uint8), ValueError),                 # one element short
])
def test_device_buffer_refuses(t, exc):
    with pytest.raises(exc):
        binding._device_buffer(t, "status", (torch.uint8,), 64, 0)


def test_decode_refuses_a_short_payload_before_launching():
    ctx = types.SimpleNamespace(device=0)
    code = types.SimpleNamespace(N=8, payload_bits=4)
    llr = FakeGpuTensor(8 * 10, torch.float32)
    ok_status = FakeGpuTensor(10, torch.uint8)
    with pytest.raises(ValueError, match="payload"):
        binding.ScsContext._frames(ctx, code, llr, FakeGpuTensor(39, torch.uint8), ok_status, None)
    with pytest.raises(ValueError, match="multiple of N"):
        binding.ScsContext._frames(ctx, code, FakeGpuTensor(81, torch.float32),
                                   FakeGpuTensor(40, torch.uint8), ok_status, None)
    with pytest.raises(ValueError, match="stats"):
        binding.ScsContext._frames(ctx, code, llr, FakeGpuTensor(40, torch.uint8), ok_status,
                                   FakeGpuTensor(79, torch.int32))
    assert binding.ScsContext._frames(ctx, code, llr, FakeGpuTensor(40, torch.uint8), ok_status,
                                      FakeGpuTensor(80, torch.int32)) == (binding.SCS_LLR_F32, 10)
