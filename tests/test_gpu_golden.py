"""The hand-worked stack-search cases of tests/golden/ (tie order, full stack, fallback after
CRC failures, REP sum order) and the fixed-point saturation input, decoded by the HIP
library: payload, status and every search counter must equal the values worked out in the
fixtures (and the oracle's)."""
import sys

import numpy as np
import pytest

import oracle
from test_oracle_golden_search import STACK_FIXTURES, load_saturation_input, read_cases

pytestmark = pytest.mark.gpu

COUNTERS = ("iterations", "switches", "completions", "evictions", "drops", "prunes")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _decode(cuda, code, D, L, x, fast):
    from paper_1809_03606_amd import binding

    n = x.shape[0]
    ctx = binding.ScsContext(0)
    xd = cuda.from_numpy(x).cuda()
    pay = cuda.full((n, max(code.payload_bits, 1)), 0xEE, dtype=cuda.uint8, device="cuda")
    st = cuda.full((n,), 0xEE, dtype=cuda.uint8, device="cuda")
    sts = cuda.zeros((n, 8), dtype=cuda.int32, device="cuda")
    ctx.decode(code, D, L, xd, pay[:, :code.payload_bits] if code.payload_bits else None, st,
               sts, fast=fast)
    cuda.cuda.synchronize()
    stats = sts.cpu().numpy().view(np.uint32)
    fields = binding.STATS_FIELDS
    return (pay.cpu().numpy()[:, :code.payload_bits], st.cpu().numpy(),
            [{k: int(stats[f, fields.index(k)]) for k in COUNTERS} for f in range(n)])


def golden_params():
    out = []
    for f in STACK_FIXTURES:
        for c in read_cases(f):
            out.append(pytest.param(c, id="%s:%s" % (f, c["name"])))
    return out


@pytest.mark.parametrize("case", golden_params())
def test_gpu_hand_worked_case(cuda, case):
    from paper_1809_03606_amd.binding import PolarCode

    N, crc = int(case["N"]), int(case["crc"])
    mask = np.zeros(N, np.uint8)
    mask[[int(v) for v in case["info"].split()]] = 1
    code = PolarCode.from_set(mask, crc)
    y = np.array([float(v) for v in case["llr"].split()], np.float32)[None, :]
    u = np.array([int(b) for b in case["u"]], np.uint8)
    want_pay = u[mask == 1][:code.payload_bits]
    _say("gpu: golden case %s (N=%d D=%s L=%s)" % (case["name"], N, case["D"], case["L"]))
    pay, st, stats = _decode(cuda, code, int(case["D"]), int(case["L"]), y,
                             case["decoder"] == "fsscs")
    assert (pay[0] == want_pay).all() and st[0] == int(case["status"])
    want = dict(kv.split("=") for kv in case["stats"].split())
    for k in COUNTERS:
        assert stats[0][k] == int(want[k]), k


@pytest.mark.parametrize("K,D,L", [(1, 1, 1), (16, 8, 8), (32, 16, 8)])
def test_gpu_fixed_point_metric_saturation(cuda, K, D, L):
    """Paths whose int16 metric saturates at 32767 (from leaf 1905 of the stored input on):
    the GPU's saturated metrics must order the search exactly as the oracle's."""
    from paper_1809_03606_amd.binding import PolarCode

    y = load_saturation_input()
    # the stored frame and two seeded perturbations of it (a few hundred values redrawn)
    rng = np.random.default_rng(7)
    x = np.stack([y, y, y]).astype(np.int8)
    for f in (1, 2):
        j = rng.choice(2048, 100 * f, replace=False)
        x[f, j] = rng.integers(-127, 128, j.size)
    code = PolarCode(2048, K, 0, 2.0)
    info = oracle.construct(2048, K, 2.0)
    rp, rs, rstats = oracle.scs_decode_batch(oracle.FIX, info, 0, D, L, x)
    pops = oracle.scs_trace(oracle.FIX, info, 0, D, L, y, cap=8192)[4]
    assert any(p[2] == 32767.0 for p in pops)  # the first frame's search does saturate
    _say("gpu: saturated fixed-point metric, K=%d D=%d L=%d" % (K, D, L))
    pay, st, stats = _decode(cuda, code, D, L, x, False)
    assert (pay == rp).all() and (st == rs).all()
    for f in range(x.shape[0]):
        for k in COUNTERS:
            assert stats[f][k] == int(rstats[f][k]), (f, k)
