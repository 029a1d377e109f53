"""Pins of the CPU oracle to facts the paper and the mathematics fix on their own.

Nothing here re-types the oracle's formulas: each check compares the oracle with an
independent definition (dense Kronecker matrix, GF(2) long division, brute-force
max-log over all completions, brute-force ML), a value printed in the paper, or a
special case that must reduce to another decoder.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from paper_1809_03606_amd import channel

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def kron_matrix(N):
    F = np.array([[1, 0], [1, 1]], dtype=np.int64)
    G = np.array([[1]], dtype=np.int64)
    while G.shape[0] < N:
        G = np.kron(G, F)
    return G


def disc(c, llr):
    """sum of |llr_j| over the positions where c disagrees with the hard decision."""
    hd = (llr < 0).astype(np.int64)
    return np.where(c != hd, np.abs(llr), 0.0).sum(axis=-1)


def rand_code(rng, N):
    K = int(rng.integers(1, N + 1))
    return K, O.construct(N, K, float(rng.uniform(0.0, 4.0)))


# -- construction --------------------------------------------------------------------

def test_construction_reproduces_paper_pc8_4():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "pc8_4_encoder.txt")) if l[0] != "#"]
    info_set = [int(x) for x in lines[0][1:]]
    assert list(np.nonzero(O.construct(8, 4, 2.0))[0]) == info_set


@pytest.mark.parametrize("N,K", [(16, 8), (64, 32), (256, 100), (1024, 512), (2048, 1024)])
def test_construction_is_closed_under_bit_dominance(N, K):
    # Replacing an f (0) step by a g (1) step can only lower the parameter, so the set
    # must contain every index whose bits cover those of a member.
    info = O.construct(N, K, 2.0)
    members = np.nonzero(info)[0]
    for i in members:
        for j in range(N):
            if (j & i) == i:
                assert info[j], (i, j)


@pytest.mark.parametrize("N", [4, 8, 16, 32, 64])
def test_construction_matches_direct_bhattacharyya(N):
    # Evaluate z directly (not in the log domain) and rank it with numpy.
    for K in range(1, N + 1, max(1, N // 8)):
        R = K / N
        z = np.array([np.exp(-R * 10 ** 0.2)])
        for _ in range(int(np.log2(N))):
            z = np.stack([2 * z - z * z, z * z], axis=1).reshape(-1)
        order = sorted(range(N), key=lambda j: (z[j], -j))
        srt = np.sort(z)
        if K < N and np.isclose(srt[K - 1], srt[K], rtol=1e-12, atol=0):
            continue  # a numerical tie at the cut: the ranking is not pinned by z
        want = np.zeros(N, np.uint8)
        want[order[:K]] = 1
        assert (O.construct(N, K, 2.0) == want).all(), (N, K)


# -- CRC-16 --------------------------------------------------------------------------

def test_crc16_catalogue_check_value():
    fx = dict(l.split() for l in open(os.path.join(GOLDEN, "crc16_check.txt")) if l[0] != "#")
    bits = np.unpackbits(np.frombuffer(fx["message"].encode(), np.uint8))
    assert O.crc16(bits) == int(fx["check"], 16)


def _gf2_remainder(bits):
    """Remainder of m(x) * x^16 modulo x^16 + x^12 + x^5 + 1 by long division."""
    g = [1] + [0] * 3 + [1] + [0] * 6 + [1] + [0] * 4 + [1]  # x^16 .. x^0
    r = list(bits) + [0] * 16
    for k in range(len(bits)):
        if r[k]:
            for t in range(17):
                r[k + t] ^= g[t]
    return int("".join(map(str, r[-16:])), 2)


def test_crc16_equals_polynomial_division_and_zero_remainder():
    rng = np.random.default_rng(5)
    for n in [0, 1, 7, 8, 9, 31, 496, 1000]:
        m = rng.integers(0, 2, n).astype(np.uint8)
        c = O.crc16(m)
        assert c == _gf2_remainder(m)
        appended = np.concatenate([m, [(c >> (15 - b)) & 1 for b in range(16)]]).astype(np.uint8)
        assert O.crc16(appended) == 0


# -- encoder -------------------------------------------------------------------------

@pytest.mark.parametrize("N", [2, 4, 8, 16, 32, 64, 128])
def test_encoder_equals_kronecker_power(N):
    G = kron_matrix(N)
    rng = np.random.default_rng(N)
    for _ in range(20):
        u = rng.integers(0, 2, N).astype(np.uint8)
        assert (O.polar_transform(u) == (u.astype(np.int64) @ G) % 2).all()


def test_encoder_follows_paper_xor_tree():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "pc8_4_encoder.txt")) if l[0] != "#"]
    info_set = [int(x) for x in lines[0][1:]]
    stages = [[tuple(map(int, op.split("^="))) for op in l[1:]] for l in lines[1:]]
    info = O.construct(8, 4, 2.0)
    for m in itertools.product([0, 1], repeat=4):
        u = np.zeros(8, np.uint8)
        u[info_set] = m
        x = u.copy()
        for ops in stages:
            for t, s in ops:
                x[t] ^= x[s]
        assert (O.polar_transform(u) == x).all()
        assert (O.encode_batch(info, 0, np.array([m], np.uint8))[0] == x).all()


def test_encoder_is_an_involution():
    rng = np.random.default_rng(1)
    for N in [2, 16, 256, 2048]:
        u = rng.integers(0, 2, N).astype(np.uint8)
        assert (O.polar_transform(O.polar_transform(u)) == u).all()


def test_encode_batch_places_payload_and_crc():
    rng = np.random.default_rng(2)
    N, K, r = 64, 40, 16
    info = O.construct(N, K, 2.0)
    pay = rng.integers(0, 2, (5, K - r)).astype(np.uint8)
    cw = O.encode_batch(info, r, pay)
    G = kron_matrix(N)
    for b in range(5):
        u = (cw[b].astype(np.int64) @ G) % 2  # G is its own inverse over GF(2)
        assert (u[info == 0] == 0).all()
        msg = u[info == 1]
        assert (msg[:K - r] == pay[b]).all()
        assert int("".join(map(str, msg[K - r:])), 2) == _gf2_remainder(pay[b])


# -- the SC tree: f, g, HD and the leaf LLRs -------------------------------------------

def test_two_bit_kernel_by_hand():
    # N = 2: c0 = u0 xor u1, c1 = u1.  Leaf 0 sees u0 through c0 = u0 ^ u1 with u1
    # unknown (box-plus, min-sum: sign(a) sign(b) min|.|); leaf 1 sees u1 directly in c1
    # and, given u0, in c0: LLR = L1 + (-1)^u0 L0.
    for L0, L1 in [(1.5, -0.5), (-2.0, -3.0), (0.25, 4.0), (-1.0, 1.0)]:
        llr = np.array([L0, L1])
        m = min(abs(L0), abs(L1)) * np.sign(L0) * np.sign(L1)
        assert O.leaf_llr(O.F64, llr, [], 0) == m
        assert O.leaf_llr(O.F64, llr, [0], 1) == L1 + L0
        assert O.leaf_llr(O.F64, llr, [1], 1) == L1 - L0
    # hard decision of a zero: neither +0 nor -0 decides 1
    info = np.array([1, 1], np.uint8)
    for z in (0.0, -0.0):
        u, _ = O.sc_decode(O.F64, info, np.array([z, 1.0]))
        assert u[0] == 0


def _maxlog_bruteforce(llr, prefix, i):
    """min over completions with u_i = 1 minus min with u_i = 0 of disc(uG)."""
    N = llr.size
    G = kron_matrix(N)
    tail = N - i - 1
    comp = np.array(list(itertools.product([0, 1], repeat=tail)), dtype=np.int64).reshape(2 ** tail, tail)
    best = []
    for ui in (0, 1):
        U = np.zeros((comp.shape[0], N), np.int64)
        U[:, :i] = prefix[:i]
        U[:, i] = ui
        U[:, i + 1:] = comp
        best.append(disc((U @ G) % 2, llr).min())
    return best[1] - best[0]


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_leaf_llr_is_maxlog_of_all_completions(N):
    rng = np.random.default_rng(100 + N)
    for _ in range(25):
        llr = rng.normal(0, 2.0, N)
        prefix = rng.integers(0, 2, N).astype(np.uint8)
        for i in range(N):
            assert abs(O.leaf_llr(O.F64, llr, prefix, i) - _maxlog_bruteforce(llr, prefix, i)) < 1e-9


@pytest.mark.parametrize("N", [4, 8, 16])
def test_sc_leaf_llrs_and_decisions(N):
    rng = np.random.default_rng(200 + N)
    for _ in range(20):
        K, info = rand_code(rng, N)
        llr = rng.normal(0, 2.0, N)
        u, lf = O.sc_decode(O.F64, info, llr)
        for i in range(N):
            assert abs(lf[i] - _maxlog_bruteforce(llr, u, i)) < 1e-9
            assert u[i] == (int(lf[i] < 0) if info[i] else 0)


# -- SC / SCS special cases ----------------------------------------------------------

@pytest.mark.parametrize("N,K,crc", [(16, 8, 0), (64, 32, 0), (256, 128, 16), (1024, 512, 16)])
def test_noiseless_channel_recovers_payload(N, K, crc):
    info = O.construct(N, K, 2.0)
    pay = channel.payload_bits(8, N, 0, 30, K - crc)
    llr = channel.noiseless_llr(O.encode_batch(info, crc, pay))
    for frame, p in zip(llr, pay):
        u, _ = O.sc_decode(O.F32, info, frame)
        assert (u[info == 1][:K - crc] == p).all()
    got, st, stats = O.scs_decode_batch(O.F32, info, crc, 8, 8, llr)
    assert (got == pay).all() and (st == O.ST_OK).all()
    assert (stats["iterations"] == N).all() and (stats["switches"] == 1).all()


def _sc_payload(info, crc, llr, mode=O.F32):
    u = np.array([O.sc_decode(mode, info, f)[0] for f in llr])
    k = int(info.sum()) - crc
    return u[:, info == 1][:, :k]


@pytest.mark.parametrize("N", [8, 16, 64, 256, 1024])
def test_scs_with_one_path_or_list_one_is_sc(N):
    rng = np.random.default_rng(N)
    for trial in range(4 if N >= 256 else 12):
        K, info = rand_code(rng, N)
        llr = channel.bpsk_awgn_llr(rng.integers(0, 2, (40, N)).astype(np.uint8),
                                    rng.normal(size=(40, N)), float(rng.uniform(-1, 3)), 0.5)
        want = _sc_payload(info, 0, llr)
        for D, L in [(1, 8), (64, 1), (1, 1)]:
            got, st, _ = O.scs_decode_batch(O.F32, info, 0, D, L, llr)
            assert (got == want).all(), (N, K, D, L)
            assert (st == O.ST_OK).all()


@pytest.mark.parametrize("N", [4, 8, 16])
def test_unbounded_scs_is_maximum_likelihood(N):
    rng = np.random.default_rng(300 + N)
    G = kron_matrix(N)
    for _ in range(40):
        K, info = rand_code(rng, N)
        llr = rng.normal(0, 1.5, N)
        dmin, mins, nmin = O.ml_decode(info, llr, max_out=4)
        u, st, pm, _ = O.scs_decode(O.F64, info, 0, 1 << 20, 1 << 20, llr)
        c = (u.astype(np.int64) @ G) % 2
        assert st == O.ST_OK
        assert (u[info == 0] == 0).all()
        assert abs(disc(c, llr) - dmin) < 1e-9
        assert abs(pm - dmin) < 1e-9
        if nmin == 1:
            assert (u == mins[0]).all()


@pytest.mark.parametrize("N", [8, 16, 64])
def test_path_metric_is_discrepancy_of_output(N):
    # PM of a complete path = sum over decided bits of [u_i != HD(alpha_i)] |alpha_i|
    #                       = disc(u G) (closed form, exact for integer LLRs).
    rng = np.random.default_rng(400 + N)
    G = kron_matrix(N)
    for _ in range(30):
        K, info = rand_code(rng, N)
        llr = rng.integers(-3, 4, N).astype(np.int8)
        u, st, pm, _ = O.scs_decode(O.FIX, info, 0, 8, 4, llr)
        assert pm == disc((u.astype(np.int64) @ G) % 2, llr.astype(np.float64))
        llr64 = rng.normal(0, 2.0, N)
        u, st, pm, _ = O.scs_decode(O.F64, info, 0, 8, 4, llr64)
        assert abs(pm - disc((u.astype(np.int64) @ G) % 2, llr64)) < 1e-9


def test_fixed_point_equals_float_without_saturation():
    # |L| <= 7 and N = 16 keep every |alpha| <= 16 * 7 < 127 and PM far below 32767, so
    # the saturating integer decoder must agree with binary32 on every frame.
    rng = np.random.default_rng(7)
    for _ in range(60):
        K, info = rand_code(rng, 16)
        llr = rng.integers(-7, 8, (20, 16)).astype(np.int8)
        for D, L, crc in [(4, 3, 0), (16, 8, 0), (64, 255, 0)]:
            a = O.scs_decode_batch(O.FIX, info, crc, D, L, llr)
            b = O.scs_decode_batch(O.F32, info, crc, D, L, llr.astype(np.float32))
            assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
            for f in O.STATS_FIELDS:
                if f not in ("f_ops", "g_ops"):
                    assert (a[2][f] == b[2][f]).all(), f


def test_fixed_point_saturates():
    info = np.array([0, 1], np.uint8)
    # g = L1 + L0 = 200 saturates to 127 at leaf 1
    u, lf = O.sc_decode(O.FIX, info, np.array([100, 100], np.int8))
    assert lf[1] == 127


@pytest.mark.parametrize("N,K", [(64, 40), (256, 128), (1024, 512)])
def test_scs_invariants_with_crc(N, K):
    crc, D, L = 16, 32, 8
    info = O.construct(N, K, 2.0)
    pay = channel.payload_bits(6, N, 0, 60, K - crc)
    cw = O.encode_batch(info, crc, pay)
    llr = channel.bpsk_awgn_llr(cw, channel.noise(6, N, 0, 60, N), 1.0, K / N)
    got, st, stats = O.scs_decode_batch(O.F32, info, crc, D, L, llr)
    assert set(np.unique(st)) <= {O.ST_OK, O.ST_FALLBACK, O.ST_FALLBACK | O.ST_EXHAUSTED}
    assert (stats["iterations"] <= L * N).all()
    assert (stats["completions"] <= L).all()
    assert ((st == O.ST_FALLBACK) == (stats["completions"] == L)).all()
    for b in np.nonzero(st == O.ST_OK)[0]:
        # accepted output: re-encode the payload with the CRC and decode the codeword
        # again noiselessly; the CRC of an accepted path holds by construction
        msg_crc = _gf2_remainder(got[b])
        u, s2, _, _ = O.scs_decode(O.F32, info, crc, D, L,
                                   channel.noiseless_llr(O.encode_batch(info, crc, got[b:b + 1]))[0])
        assert s2 == O.ST_OK
        assert int("".join(map(str, u[info == 1][K - crc:])), 2) == msg_crc


def test_fer_improves_from_sc_to_scs():
    # statistical sanity only (not a pin): at 1.5 dB on PC(256,128) SCS with D=32, L=8
    # must not do worse than SC on the same frames
    N, K = 256, 128
    info = O.construct(N, K, 2.0)
    pay = channel.payload_bits(12, 0, 0, 400, K)
    llr = channel.bpsk_awgn_llr(O.encode_batch(info, 0, pay), channel.noise(12, 0, 0, 400, N), 1.5, 0.5)
    sc = (_sc_payload(info, 0, llr) != pay).any(axis=1).sum()
    scs = (O.scs_decode_batch(O.F32, info, 0, 32, 8, llr)[0] != pay).any(axis=1).sum()
    assert scs <= sc
