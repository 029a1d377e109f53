"""Hand-worked pins of the stack-search rules that the special cases (D = 1, L = 1,
unbounded search) leave open: the order of equal metrics (reading R11), the full-stack rule
(R12), the output after L CRC failures (R15), the binary32 order of the fast simplified
node sums and candidates (F2-F5), and the saturation of the fixed-point path metric (R18).

Each fixture under tests/golden/ carries its derivation; the oracle must reproduce every
path it takes off the stack (creation number, length, metric), its output, status, metric
and counters."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
STACK_FIXTURES = ("scs_tie_order_n2.txt", "scs_full_stack_n4.txt", "scs_fallback_n32.txt",
                  "fsscs_rep_sum_n4.txt")
MODES = {"f32": oracle.F32, "f64": oracle.F64, "fix": oracle.FIX}
NODE_CLASS = {"R0": oracle.NODE_R0, "R1": oracle.NODE_R1, "REP": oracle.NODE_REP,
              "SPC": oracle.NODE_SPC}


def read_cases(name):
    cases, cur = [], None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, _, rest = line.partition(" ")
        if key == "case":
            cur = {"name": rest, "decoder": "scs"}
            cases.append(cur)
        else:
            cur[key] = rest
    return cases


def stack_cases():
    out = []
    for f in STACK_FIXTURES:
        for c in read_cases(f):
            out.append(pytest.param(c, id="%s:%s" % (f, c["name"])))
    return out


def run_case(c):
    mode = MODES[c["mode"]]
    N = int(c["N"])
    info = np.zeros(N, np.uint8)
    info[[int(v) for v in c["info"].split()]] = 1
    dt = {oracle.F32: np.float32, oracle.F64: np.float64, oracle.FIX: np.int8}[mode]
    y = np.array([float(v) for v in c["llr"].split()]).astype(dt)
    fn = oracle.fsscs_trace if c["decoder"] == "fsscs" else oracle.scs_trace
    return fn(mode, info, int(c["crc"]), int(c["D"]), int(c["L"]), y)


@pytest.mark.parametrize("case", stack_cases())
def test_hand_worked_stack_trace(case):
    u, status, pm, stats, pops, n = run_case(case)
    want_pops = [tuple(float(x) for x in t.split(":")) for t in case["pops"].split()]
    assert n == len(want_pops)
    assert [(float(a), float(b), c) for a, b, c in pops] == want_pops
    assert "".join(str(int(b)) for b in u) == case["u"]
    assert status == int(case["status"])
    assert pm == float(case["pm"])
    for kv in case["stats"].split():
        k, v = kv.split("=")
        assert stats[k] == int(v), k


def test_hand_worked_node_candidates_binary32():
    nodes, cur = [], None
    for line in open(os.path.join(GOLDEN, "fsscs_node_f32.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        t = line.split()
        if t[0] == "node":
            cur = {"cls": NODE_CLASS[t[1]], "pm": float(t[3]),
                   "alpha": [float(v) for v in t[5:]], "cands": []}
            nodes.append(cur)
        else:
            cur["cands"].append((t[1], float(t[2])))
    assert len(nodes) == 5
    for nd in nodes:
        got = oracle.node_candidates(oracle.F32, nd["cls"], nd["alpha"], nd["pm"])
        assert [("".join(str(int(b)) for b in bits), m) for bits, m in got] == nd["cands"], nd


def load_saturation_input():
    vals = []
    for line in open(os.path.join(GOLDEN, "fixed_saturation_n2048.txt")):
        if not line.startswith("#"):
            vals += [int(v) for v in line.split()]
    y = np.array(vals, np.int8)
    assert y.size == 2048 and y.min() >= -127
    return y


def test_fixed_point_metric_saturates_at_int16_max():
    """Reading R18: the metric is min(PM + |alpha|, 32767).  On the stored input the penalties
    of the forced (all-frozen) SC path, summed exactly from the oracle's leaf LLRs, exceed
    32767 from leaf 1905 on; the decoder's metric must stop at 32767 (no wrap, no overflow,
    no other cap)."""
    y = load_saturation_input()
    info1 = oracle.construct(2048, 1, 2.0)
    _, leaf = oracle.sc_decode(oracle.FIX, info1, y)
    pen = np.maximum(0, -leaf.astype(np.int64))
    pen[info1 == 1] = 0
    total = int(pen.sum())
    assert total > 32767 + 127 * 16
    first = int(np.argmax(np.cumsum(pen) >= 32767))
    assert first == 1905
    # SC (D = 1): the metric of the only path is the capped sum
    u, st, pm, stats = oracle.scs_decode(oracle.FIX, info1, 0, 1, 1, y)
    assert st == oracle.ST_OK and pm == 32767.0 and stats["iterations"] == 2048


def test_fixed_point_saturated_ties_drive_the_search():
    """With K = 16 (information positions 1983 and above) every path of the stack search is
    saturated once it passes leaf 1905, so equal metrics of 32767 are ordered by length and
    creation number: the search never leaves the hard-decision chain (2048 iterations) and
    flips compete for the full stack only through the tie rule (9 evictions)."""
    y = load_saturation_input()
    info = oracle.construct(2048, 16, 2.0)
    assert np.nonzero(info)[0][0] == 1983
    u, st, pm, stats, pops, n = oracle.scs_trace(oracle.FIX, info, 0, 8, 8, y, cap=4096)
    assert st == oracle.ST_OK and pm == 32767.0
    assert stats["iterations"] == 2048 and stats["switches"] == 1 and stats["evictions"] == 9
    sat = [p for p in pops if p[2] == 32767.0]
    assert len(sat) == 2049 - 1905 - 1
    assert [p[1] for p in sat] == list(range(1906, 2049))
