"""Systematic codes on the GPU (Section 2.2.2, last paragraph; Section 4): the device encoder
of a systematic twin equals the oracle's systematic encoder, and the three decoders read the
payload from (and check the CRC on) the codeword estimate exactly as the oracle's
systematic mode does: payload, status and every search counter."""
import sys

import numpy as np
import pytest

import oracle
from cases import THREADS, assert_parity, gpu_decode
from paper_1809_03606_amd import channel

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _frames(N, K, crc, eb, B, seed, dtype):
    info = oracle.construct(N, K, 2.0)
    pay = channel.payload_bits(seed, 7, 0, B, K - crc)
    cw = oracle.encode_batch(info, crc, pay, systematic=True)
    nz = channel.noise(seed, 7, 0, B, N)
    if dtype == "f32":
        return info, pay, channel.bpsk_awgn_llr(cw, nz, eb, K / N)
    return info, pay, channel.bpsk_awgn_i8(cw, nz, eb, K / N)


@pytest.mark.parametrize("N,K,crc", [(8, 4, 0), (128, 64, 16), (1024, 512, 16), (2048, 853, 16)])
def test_gpu_systematic_device_encoder(cuda, N, K, crc):
    from paper_1809_03606_amd.binding import PolarCode

    code = PolarCode(N, K, crc, 2.0).make_systematic()
    info = oracle.construct(N, K, 2.0)
    pay = channel.payload_bits(9, N, 0, 300, K - crc)
    p = cuda.from_numpy(pay).cuda()
    cw = cuda.zeros((300, N), dtype=cuda.uint8, device="cuda")
    _say("gpu: systematic device encoder N=%d K=%d" % (N, K))
    code.encode_device(p, cw)
    cuda.cuda.synchronize()
    assert (cw.cpu().numpy() == oracle.encode_batch(info, crc, pay, systematic=True)).all()


CASES = [(64, 32, 0, 8, 8, 2.0), (128, 64, 16, 16, 8, 1.5), (512, 256, 16, 32, 8, 2.0),
         (1024, 512, 16, 32, 8, 2.0), (2048, 1024, 16, 64, 8, 2.5)]


@pytest.mark.parametrize("decoder", ["scs", "fsscs", "scl"])
@pytest.mark.parametrize("dtype", ["f32", "i8"])
@pytest.mark.parametrize("N,K,crc,D,L,eb", CASES)
def test_gpu_systematic_decoders_match_oracle(cuda, N, K, crc, D, L, eb, dtype, decoder):
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import PolarCode

    B = 60 if N >= 1024 else 150
    info, pay, llr = _frames(N, K, crc, eb, B, 100 + N, dtype)
    code = PolarCode(N, K, crc, 2.0).make_systematic()
    mode = oracle.F32 if dtype == "f32" else oracle.FIX
    label = "systematic %s N=%d K=%d crc=%d D=%d L=%d %s" % (decoder, N, K, crc, D, L, dtype)
    if decoder == "scl":
        lsize = 4
        ref = oracle.scl_decode_batch(mode, info, crc, lsize, llr, threads=THREADS,
                                      systematic=True)
        _say("gpu: " + label)
        ctx = binding.ScsContext(0)
        x = cuda.from_numpy(llr).cuda()
        p = cuda.full((B, K - crc), 0xEE, dtype=cuda.uint8, device="cuda")
        s = cuda.full((B,), 0xEE, dtype=cuda.uint8, device="cuda")
        ctx.decode_list(code, lsize, x, p, s)
        cuda.cuda.synchronize()
        assert (p.cpu().numpy() == ref[0]).all() and (s.cpu().numpy() == ref[1]).all(), label
    else:
        fn = oracle.fsscs_decode_batch if decoder == "fsscs" else oracle.scs_decode_batch
        ref = fn(mode, info, crc, D, L, llr, threads=THREADS, systematic=True)
        _say("gpu: " + label)
        got = gpu_decode(cuda, code, D, L, llr, fast=decoder == "fsscs")
        assert_parity(got, ref, label)
    # most frames come back as the sent payload (the decoder really reads the codeword)
    assert (ref[0] == pay).all(axis=1).mean() > 0.5


def test_gpu_mixed_plan_with_systematic_and_plain_codes(cuda):
    """One persistent launch over frames of a systematic code and of the plain code of the
    same parameters: each frame equals the oracle in its own mode."""
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import FRAME_DTYPE, PolarCode

    N, K, crc, B = 256, 128, 16, 200
    plain = PolarCode(N, K, crc, 2.0)
    sysc = plain.make_systematic()
    info = oracle.construct(N, K, 2.0)
    llrs, refs = [], []
    for c, sys_mode in ((0, False), (1, True)):
        pay = channel.payload_bits(12 + c, 8, 0, B, K - crc)
        cw = oracle.encode_batch(info, crc, pay, systematic=sys_mode)
        llr = channel.bpsk_awgn_llr(cw, channel.noise(12 + c, 8, 0, B, N), 2.0, K / N)
        llrs.append(llr)
        refs.append(oracle.scs_decode_batch(oracle.F32, info, crc, 16, 8, llr, threads=THREADS,
                                            systematic=sys_mode))
    frames = np.zeros(2 * B, FRAME_DTYPE)
    kp = K - crc
    for f in range(2 * B):
        frames[f] = (f % 2, 16, 8, 0, f * N, f * kp)  # interleaved codes
    flat = np.empty((2 * B, N), np.float32)
    flat[0::2], flat[1::2] = llrs[0], llrs[1]
    x = cuda.from_numpy(flat.reshape(-1)).cuda()
    p = cuda.full((2 * B * kp,), 0xEE, dtype=cuda.uint8, device="cuda")
    s = cuda.full((2 * B,), 0xEE, dtype=cuda.uint8, device="cuda")
    ctx = binding.ScsContext(0)
    _say("gpu: mixed plan with a systematic and a plain code")
    binding.scs_decode_mixed(ctx.handle, [plain.handle, sysc.handle], frames, binding.SCS_LLR_F32,
                             x, p, s)
    cuda.cuda.synchronize()
    pp, ss = p.cpu().numpy().reshape(2 * B, kp), s.cpu().numpy()
    for c in (0, 1):
        assert (pp[c::2] == refs[c][0]).all() and (ss[c::2] == refs[c][1]).all(), c
