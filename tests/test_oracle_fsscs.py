"""Pins of the oracle's fast simplified stack decoder (FSSCS-RM, Section 4) to facts fixed
outside it: the schedule printed in the paper, the node rules of Section 2.2.2 / 2.2.4
against brute force over the node's words, the node metrics against the leaf-by-leaf path
metric of eq. (PMupd), and special cases that reduce to SCS, SC or ML decoding."""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from paper_1809_03606_amd import channel

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NAMES = {"R-0": O.NODE_R0, "R-1": O.NODE_R1, "REP": O.NODE_REP, "SPC": O.NODE_SPC}


def test_schedule_reproduces_paper_pc8_4():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "pc8_4_fssc_schedule.txt"))
             if l.strip() and l[0] != "#"]
    info = np.zeros(8, np.uint8)
    info[[int(x) for x in lines[0][1:]]] = 1
    want = [(int(phi) << int(lam), int(lam), NAMES[c]) for _, lam, phi, c in lines[1:]]
    assert O.fssc_schedule(info) == want


def _class_of(block):
    """Class of a block of leaves by the definitions of Section 2.2.2 (None: no class)."""
    k, n = int(block.sum()), block.size
    if k == 0:
        return O.NODE_R0
    if k == n:
        return O.NODE_R1
    if n >= 2 and k == 1 and block[-1]:
        return O.NODE_REP
    if n >= 4 and k == n - 1 and not block[0]:
        return O.NODE_SPC
    return None


@pytest.mark.parametrize("N", [2, 8, 32, 128, 1024])
def test_schedule_is_an_ordered_maximal_partition(N):
    rng = np.random.default_rng(N)
    for _ in range(20):
        info = O.construct(N, int(rng.integers(1, N + 1)), float(rng.uniform(0, 4)))
        nodes = O.fssc_schedule(info)
        pos = 0
        for start, lam, t in nodes:
            size = 1 << lam
            assert start == pos and start % size == 0
            assert _class_of(info[start:start + size]) == t
            if lam < int(np.log2(N)):  # the enclosing block has no class (else it is the node)
                ps = start & ~(2 * size - 1)
                assert _class_of(info[ps:ps + 2 * size]) is None
            pos += size
        assert pos == N


def _flip_sets(cls, a):
    """Allowed flip positions of the node rules: the least reliable positions by |alpha|
    (stable order), two for R-1 (one for a single leaf), four for SPC, all for R-0/REP."""
    order = list(np.argsort(np.abs(a), kind="stable"))
    if cls == O.NODE_R1:
        return set(order[:2 if a.size >= 2 else 1])
    if cls == O.NODE_SPC:
        return set(order[:4])
    return set(range(a.size))


def _node_words(cls, n):
    for w in itertools.product((0, 1), repeat=n):
        w = np.array(w, np.uint8)
        if cls == O.NODE_R0 and w.any():
            continue
        if cls == O.NODE_REP and not (w.all() or not w.any()):
            continue
        if cls == O.NODE_SPC and int(w.sum()) % 2:
            continue
        yield w


@pytest.mark.parametrize("cls,lam", [(O.NODE_R0, 0), (O.NODE_R0, 3), (O.NODE_REP, 1),
                                     (O.NODE_REP, 3), (O.NODE_R1, 0), (O.NODE_R1, 1),
                                     (O.NODE_R1, 3), (O.NODE_SPC, 2), (O.NODE_SPC, 3),
                                     (O.NODE_SPC, 4)])
def test_node_candidates_match_brute_force(cls, lam):
    """The candidates are exactly the node's words whose disagreements with HD(alpha) lie
    in the allowed flip positions, each with metric pm + sum of |alpha| over the
    disagreements (the node discrepancy); the best of them is the ML word of the node's
    code (checked over all its words)."""
    rng = np.random.default_rng(100 * cls + lam)
    for _ in range(25):
        a = rng.normal(0, 2, 1 << lam)
        hd = (a < 0).astype(np.uint8)
        pm0 = float(rng.uniform(0, 5))
        cands = O.node_candidates(O.F64, cls, a, pm0)
        allowed = _flip_sets(cls, a)
        want = {}
        for w in _node_words(cls, a.size):
            flips = set(np.nonzero(w != hd)[0])
            if cls in (O.NODE_R1, O.NODE_SPC) and not flips <= allowed:
                continue
            want[w.tobytes()] = pm0 + float(np.abs(a)[list(flips)].sum()) if flips else pm0
        got = {b.tobytes(): m for b, m in cands}
        assert len(got) == len(cands) == len(want)
        assert got.keys() == want.keys()
        for k in want:
            assert abs(got[k] - want[k]) < 1e-9
        best = min(pm0 + float(np.where(w != hd, np.abs(a), 0).sum())
                   for w in _node_words(cls, a.size))
        assert abs(min(got.values()) - best) < 1e-9
        # first candidate as listed in Section 2.2.4: HD for R-1, all-zero for R-0/REP
        if cls == O.NODE_R1:
            assert (cands[0][0] == hd).all() and cands[0][1] == pm0
        if cls in (O.NODE_R0, O.NODE_REP):
            assert not cands[0][0].any()


@pytest.mark.parametrize("cls,lam", [(O.NODE_REP, 2), (O.NODE_R1, 3), (O.NODE_SPC, 3),
                                     (O.NODE_R0, 2)])
def test_node_metric_equals_leaf_by_leaf_metric(cls, lam):
    """For every candidate the node metric equals the path metric of eq. (PMupd)
    accumulated leaf by leaf by SC on the node's own code (its LLRs as channel, its
    bits u = the candidate re-encoded)."""
    rng = np.random.default_rng(7 + cls)
    n = 1 << lam
    for _ in range(20):
        a = rng.normal(0, 2, n)
        for beta, m in O.node_candidates(O.F64, cls, a, 0.0):
            u = O.polar_transform(beta)
            pm = 0.0
            for i in range(n):
                leaf = O.leaf_llr(O.F64, a, u, i)
                if u[i] != (1 if leaf < 0 else 0):
                    pm += abs(leaf)
            assert abs(pm - m) < 1e-9, (cls, beta, pm, m)


def _frames(N, K, crc, eb, B, seed, dtype="f32"):
    info = O.construct(N, K, 2.0)
    pay = channel.payload_bits(seed, N, 0, B, K - crc)
    cw = O.encode_batch(info, crc, pay)
    n = channel.noise(seed, N, 0, B, N)
    if dtype == "f64":
        s2 = channel.sigma2(eb, K / N)
        llr = (2.0 * ((1.0 - 2.0 * cw) + np.sqrt(s2) * n) / s2)
    elif dtype == "i8":
        llr = channel.bpsk_awgn_i8(cw, n, eb, K / N)
    else:
        llr = channel.bpsk_awgn_llr(cw, n, eb, K / N)
    return info, pay, llr


@pytest.mark.parametrize("N,K,crc,D,L,eb,mode", [
    (16, 8, 0, 4, 4, 1.0, "f32"), (32, 24, 16, 8, 8, 2.0, "f32"), (64, 32, 0, 8, 8, 2.0, "f32"),
    (128, 64, 16, 16, 4, 1.5, "f32"), (256, 128, 16, 32, 8, 1.5, "i8"), (64, 20, 0, 1, 3, 0.5, "f32"),
    (128, 100, 16, 64, 255, 2.5, "f32")])
def test_leaf_schedule_equals_scs(N, K, crc, D, L, eb, mode):
    """With every node a single leaf the fast decoder is the SCS decoder: same outputs,
    same search."""
    info, pay, llr = _frames(N, K, crc, eb, 60, seed=N + D)
    m = O.FIX if mode == "i8" else O.F32
    if mode == "i8":
        _, _, llr = _frames(N, K, crc, eb, 60, seed=N + D, dtype="i8")
    p1, s1, t1 = O.scs_decode_batch(m, info, crc, D, L, llr)
    p2, s2, t2 = O.fsscs_decode_batch(m, info, crc, D, L, llr, types=0)
    assert np.array_equal(p1, p2) and np.array_equal(s1, s2)
    for f in ("iterations", "completions", "evictions", "drops", "prunes", "sc_elems"):
        assert np.array_equal(t1[f], t2[f]), f


@pytest.mark.parametrize("N,K", [(16, 8), (64, 32), (128, 50), (256, 200), (1024, 512)])
def test_fssc_without_spc_equals_sc(N, K):
    """D = 1 keeps only the best candidate of every node: with R-0, R-1 and REP nodes that
    is SC decoding (min-sum SC decodes a rate-1 node to the hard decision of its LLRs and a
    repetition node to the sign of their sum), bit for bit, on binary64 channel LLRs."""
    info, pay, llr = _frames(N, K, 0, 1.0, 30, seed=3 * N, dtype="f64")
    types = (1 << O.NODE_R0) | (1 << O.NODE_R1) | (1 << O.NODE_REP)
    assert any(t != O.NODE_R0 and lam > 0 for _, lam, t in O.fssc_schedule(info, types)) or N < 64
    for b in range(llr.shape[0]):
        u_sc, _ = O.sc_decode(O.F64, info, llr[b])
        u_f, st, _, _ = O.fsscs_decode(O.F64, info, 0, 1, 1, llr[b], types=types)
        assert st == O.ST_OK
        assert np.array_equal(u_sc, u_f), b


@pytest.mark.parametrize("N,K", [(8, 4), (16, 6), (16, 10), (16, 12)])
def test_unbounded_fsscs_with_complete_nodes_is_ml(N, K):
    """With only node classes whose candidate lists are complete (R-0, REP, one-leaf R-1)
    and no limit from D or L, the best-first search returns an ML word."""
    rng = np.random.default_rng(N * K)
    info = O.construct(N, K, 2.0)
    types = (1 << O.NODE_R0) | (1 << O.NODE_REP)
    for _ in range(40):
        llr = rng.normal(0.5, 1.5, N)
        u, st, pm, _ = O.fsscs_decode(O.F64, info, 0, 1 << 20, 1 << 20, llr, types=types)
        dmin, _, _ = O.ml_decode(info, llr)
        c = O.polar_transform(u)
        d = float(np.where(c != (llr < 0), np.abs(llr), 0).sum())
        assert abs(d - dmin) < 1e-9 and abs(pm - d) < 1e-9


@pytest.mark.parametrize("N,K,crc", [(64, 32, 0), (256, 128, 16), (1024, 512, 16), (2048, 1024, 16)])
def test_noiseless_recovery_all_node_classes(N, K, crc):
    info = O.construct(N, K, 2.0)
    pay = channel.payload_bits(5, N, 0, 8, K - crc)
    cw = O.encode_batch(info, crc, pay)
    llr = channel.noiseless_llr(cw)
    got, st, stats = O.fsscs_decode_batch(O.F32, info, crc, 8, 8, llr)
    assert np.array_equal(got, pay) and (st == O.ST_OK).all()
    assert (stats["iterations"] == len(O.fssc_schedule(info))).all()


def test_invariants_on_noisy_frames():
    N, K, crc, D, L = 256, 128, 16, 16, 8
    info, pay, llr = _frames(N, K, crc, 1.0, 120, seed=9)
    nodes = len(O.fssc_schedule(info))
    pos = np.nonzero(info)[0]
    for b in range(llr.shape[0]):
        u, st, pm, stats = O.fsscs_decode(O.F32, info, crc, D, L, llr[b])
        assert stats["iterations"] <= L * nodes
        assert st in (O.ST_OK, O.ST_FALLBACK, O.ST_FALLBACK | O.ST_EXHAUSTED)
        assert not u[info == 0].any()  # frozen positions stay 0 through every node class
        if st == O.ST_OK:  # an accepted output satisfies the CRC
            bits = u[pos]
            r = O.crc16(bits[:K - crc])
            assert [(r >> (15 - j)) & 1 for j in range(16)] == list(bits[K - crc:])
