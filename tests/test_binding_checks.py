"""Host-side checks of the tensors the Python binding hands to the kernels: a buffer too
small, of the wrong type, on the host or on another GPU is refused before any launch."""
import types

import numpy as np

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


def _plan(n_codes_frames):
    plan = np.zeros(len(n_codes_frames), binding.FRAME_DTYPE)
    off = out = 0
    for f, (c, N, kp) in enumerate(n_codes_frames):
        plan[f] = (c, 8, 8, 0, off, out)
        off += N
        out += kp
    return plan, off, out


def test_mixed_plans_are_checked_against_the_tensors():
    """scs_decode_mixed, its no-allocation variant and scs_mixed_launch refuse tensors that a
    descriptor would read or write past, before the library is called."""
    codes = [binding.PolarCode(128, 64, 16), binding.PolarCode(256, 128, 16)]
    handles = [c.handle for c in codes]
    plan, n_llr, n_out = _plan([(0, 128, 48), (1, 256, 112), (0, 128, 48)])
    ok = dict(llr=FakeGpuTensor(n_llr, torch.float32), pay=FakeGpuTensor(n_out, torch.uint8),
              st=FakeGpuTensor(3, torch.uint8))
    bad = [("llr", FakeGpuTensor(n_llr - 1, torch.float32), "llr"),
           ("llr", FakeGpuTensor(n_llr, torch.int8), "llr"),
           ("pay", FakeGpuTensor(n_out - 1, torch.uint8), "payload"),
           ("st", FakeGpuTensor(2, torch.uint8), "status")]
    for fn in (binding.scs_decode_mixed, binding.scs_decode_mixed_noalloc):
        for key, t, name in bad:
            args = dict(ok)
            args[key] = t
            with pytest.raises((ValueError, TypeError), match=name):
                fn(0, handles, plan, binding.SCS_LLR_F32, args["llr"], args["pay"], args["st"])
        with pytest.raises(ValueError, match="stats"):
            fn(0, handles, plan, binding.SCS_LLR_F32, ok["llr"], ok["pay"], ok["st"],
               FakeGpuTensor(3 * 8 - 1, torch.int32))
    # a plan recorded at prepare time checks the launch's tensors
    binding._PLANS[12345] = binding._plan_extent(handles, plan)
    with pytest.raises(ValueError, match="payload"):
        binding.scs_mixed_launch(12345, binding.SCS_LLR_F32, ok["llr"],
                                 FakeGpuTensor(n_out - 1, torch.uint8), ok["st"])
    del binding._PLANS[12345]
    # a descriptor whose code index is out of range is left to the library's own check
    assert binding._plan_extent(handles, _plan([(2, 128, 48)])[0]) is None
