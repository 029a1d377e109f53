"""Non-finite channel LLRs: the output is unspecified, but every decoder must finish the
batch without a device error and write a status byte from its documented set (the stack
decoders stop after at most L N + L extensions; the list decoder runs N leaves)."""
import sys

import numpy as np
import pytest

from cases import make_frames

pytestmark = pytest.mark.gpu

VALID_STATUS = {0, 1, 2, 6}  # 0: the iteration budget ran out


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _poisoned(N, K, crc, B, seed):
    info, pay, llr = make_frames(N, K, crc, 2.0, B, seed)
    llr = np.array(llr, dtype=np.float32)
    rng = np.random.default_rng(seed)
    special = np.array([np.nan, np.inf, -np.inf, -np.nan], dtype=np.float32)
    # frames 0-3: all NaN / +Inf / -Inf / mixed; the rest: 10 % of positions poisoned
    llr[0, :] = np.nan
    llr[1, :] = np.inf
    llr[2, :] = -np.inf
    llr[3, :] = special[rng.integers(0, 4, N)]
    mask = rng.random(llr[4:].shape) < 0.1
    llr[4:][mask] = special[rng.integers(0, 4, int(mask.sum()))]
    return llr


@pytest.mark.parametrize("N,K,crc", [(64, 32, 0), (1024, 512, 16)])
@pytest.mark.parametrize("decoder,D,L", [("scs", 32, 8), ("scs", 128, 8), ("scs", 256, 4),
                                         ("fsscs", 32, 8), ("fsscs", 200, 8),
                                         ("scl", 0, 8), ("scl", 0, 1)])
def test_nonfinite_llrs_terminate(cuda, N, K, crc, decoder, D, L):
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import PolarCode, ScsContext

    B = 67
    llr = _poisoned(N, K, crc, B, seed=N + D + L)
    code = PolarCode(N, K, crc, 2.0)
    ctx = ScsContext(0)
    x = cuda.from_numpy(llr).to("cuda")
    pay = cuda.zeros((B, code.payload_bits), dtype=cuda.uint8, device="cuda")
    st = cuda.full((B,), 255, dtype=cuda.uint8, device="cuda")
    _say("gpu: non-finite LLRs %s N=%d D=%d L=%d" % (decoder, N, D, L))
    if decoder == "scl":
        ctx.decode_list(code, L, x, pay, st)
    else:
        ctx.decode(code, D, L, x, pay, st, fast=decoder == "fsscs")
    cuda.cuda.synchronize()
    assert binding.scs_ctx_last_error(ctx.handle) == 0
    status = set(st.cpu().numpy().tolist())
    assert status <= VALID_STATUS, status
    assert set(np.unique(pay.cpu().numpy()).tolist()) <= {0, 1}
