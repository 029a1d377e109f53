"""The no-allocation mixed decoder (scs_decode_mixed_noalloc) against scs_decode_mixed: two
calls in a row on one context and stream, the second with a smaller batch over a subset of
the codes, each compared byte for byte with the allocating entry point (payload, status,
statistics) and with the oracle; requests beyond the fixed scratch capacity are refused
before anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest

from test_gpu_mixed import build_mixed

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _subset(codes, frames, flat, want, keep):
    """The frames whose code is in `keep`, re-indexed to a code list of `keep` only, with
    their LLRs packed anew and their payload offsets recomputed."""
    from paper_1809_03606_amd.binding import FRAME_DTYPE

    remap = {c: j for j, c in enumerate(keep)}
    sel = [f for f in range(len(frames)) if frames["code"][f] in remap]
    out = np.zeros(len(sel), FRAME_DTYPE)
    parts, w, off, oo = [], {}, 0, 0
    for j, f in enumerate(sel):
        c = int(frames["code"][f])
        N, K = codes[c]
        lo = int(frames["llr_off"][f])
        parts.append(flat[lo:lo + N])
        out[j] = (remap[c], frames["D"][f], frames["L"][f], 0, off, oo)
        w[j] = want[f]
        off += N
        oo += K - 16
    return [codes[c] for c in keep], out, np.concatenate(parts), w, oo


def _run(cuda, fn, handles, frames, flat, total_out, stream):
    from paper_1809_03606_amd import binding

    x = cuda.from_numpy(flat).cuda()
    pay = cuda.full((max(total_out, 1),), 0xEE, dtype=cuda.uint8, device="cuda")
    st = cuda.full((len(frames),), 0xEE, dtype=cuda.uint8, device="cuda")
    sts = cuda.zeros((len(frames), 8), dtype=cuda.int32, device="cuda")
    cuda.cuda.synchronize()
    fn(handles, frames, binding.SCS_LLR_F32, x, pay, st, sts, stream)
    stream.synchronize()
    return pay.cpu().numpy(), st.cpu().numpy(), sts.cpu().numpy()


def test_gpu_noalloc_matches_mixed_on_two_calls(cuda):
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import PolarCode

    codes, frames, flat, _, want, total_out = build_mixed(600, seed=61)
    pcs = [PolarCode(N, K, 16, 2.0) for (N, K) in codes]
    ctx = binding.ScsContext(0)
    stream = cuda.cuda.Stream()

    def noalloc(h, fr, dt, x, p, s, st, strm):
        binding.scs_decode_mixed_noalloc(ctx.handle, h, fr, dt, x, p, s, st, strm)

    def alloc(h, fr, dt, x, p, s, st, strm):
        binding.scs_decode_mixed(ctx.handle, h, fr, dt, x, p, s, st, strm)

    keep = [3, 7, 12, 20, 24]  # the second call: fewer frames over five of the codes
    sub_codes, sub_frames, sub_flat, sub_want, sub_out = _subset(codes, frames, flat, want, keep)
    calls = [("first call, %d frames, %d codes" % (len(frames), len(codes)),
              codes, [p.handle for p in pcs], frames, flat, want, total_out),
             ("second call, %d frames, %d codes" % (len(sub_frames), len(keep)),
              sub_codes, [pcs[c].handle for c in keep], sub_frames, sub_flat, sub_want, sub_out)]
    assert len(sub_frames) < len(frames)
    for name, cl, handles, fr, fl, wt, tout in calls:
        _say("gpu: no-allocation mixed decoder, " + name)
        got = _run(cuda, noalloc, handles, fr, fl, tout, stream)
        _say("gpu: allocating mixed decoder, " + name)
        ref = _run(cuda, alloc, handles, fr, fl, tout, stream)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), name
        pay, st, _ = got
        for f in range(len(fr)):
            kp = cl[fr["code"][f]][1] - 16
            o = fr["out_off"][f]
            assert (pay[o:o + kp] == wt[f][0]).all() and st[f] == wt[f][1], (name, f)
    assert binding.scs_ctx_last_error(ctx.handle) == 0


def test_gpu_noalloc_refuses_beyond_capacity(cuda):
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import FRAME_DTYPE, PolarCode

    pc = PolarCode(128, 64, 16)
    ctx = binding.ScsContext(0)
    x = cuda.zeros((256,), device="cuda")
    pay = cuda.zeros((128,), dtype=cuda.uint8, device="cuda")
    st = cuda.zeros((2,), dtype=cuda.uint8, device="cuda")
    lib = binding.lib()

    def raw(handles, frames):
        # the C entry point itself (the Python wrapper would refuse these small buffers first)
        arr = (ctypes.c_void_p * len(handles))(*handles)
        return lib.scs_decode_mixed_noalloc(ctx.handle, ctypes.cast(arr, ctypes.c_void_p),
                                            len(handles), frames.ctypes.data, len(frames),
                                            binding.SCS_LLR_F32, x.data_ptr(), pay.data_ptr(),
                                            st.data_ptr(), None, None)

    # more descriptors than the scratch array holds (24 bytes each)
    n = binding.NOALLOC_SCRATCH_BYTES // 24 + 1
    big = np.zeros(n, FRAME_DTYPE)
    big["D"], big["L"] = 8, 8
    assert raw([pc.handle], big) == binding.POLAR_ETOOLARGE
    # more codes than the fixed table holds
    few = np.zeros(2, FRAME_DTYPE)
    few["D"], few["L"] = 8, 8
    few[1]["llr_off"] = 128
    assert raw([pc.handle] * (binding.NOALLOC_MAX_CODES + 1), few) == binding.POLAR_ETOOLARGE
    # a bad descriptor is an argument error, as for scs_decode_mixed
    bad = few.copy()
    bad[1]["D"] = 65
    assert raw([pc.handle], bad) == binding.POLAR_EINVAL
    cuda.cuda.synchronize()
    assert binding.scs_ctx_last_error(ctx.handle) == 0
