"""Systematic encoding (Section 2.2.2, last paragraph; Section 4): the oracle's encoder
puts the message (payload, then CRC) into the codeword itself at the information
positions, and its decoders in systematic mode check the CRC on, and read the payload from,
the codeword estimate.  Pinned by the hand-worked PC(8,4) table, the defining property, and
round trips through every decoder."""
import os

import numpy as np
import pytest

import oracle
from paper_1809_03606_amd import channel

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_pc8_4_systematic_codewords_by_hand():
    info = np.zeros(8, np.uint8)
    info[[3, 5, 6, 7]] = 1
    rows = []
    for line in open(os.path.join(GOLDEN, "pc8_4_systematic.txt")):
        if line.startswith("message"):
            t = line.split()
            rows.append(([int(b) for b in t[1]], [int(b) for b in t[3]]))
    assert len(rows) == 6
    msg = np.array([m for m, _ in rows], np.uint8)
    want = np.array([c for _, c in rows], np.uint8)
    assert (oracle.encode_batch(info, 0, msg, systematic=True) == want).all()


@pytest.mark.parametrize("N,K,crc", [(8, 4, 0), (16, 9, 0), (64, 32, 16), (256, 77, 16),
                                     (1024, 512, 16), (2048, 1707, 16)])
def test_systematic_codeword_carries_the_message(N, K, crc):
    """x at the information positions is the message (payload, then its CRC), and x is a
    codeword: its transform u = x F^(x)n is zero at every frozen position."""
    info = oracle.construct(N, K, 2.0)
    pay = channel.payload_bits(3, N, 0, 40, K - crc)
    x = oracle.encode_batch(info, crc, pay, systematic=True)
    pos = np.nonzero(info)[0]
    for b in range(pay.shape[0]):
        msg = list(pay[b])
        if crc:
            c = oracle.crc16(pay[b])
            msg += [(c >> (15 - j)) & 1 for j in range(16)]
        assert list(x[b][pos]) == msg
        u = oracle.polar_transform(x[b])
        assert not u[info == 0].any()


def test_systematic_encoding_is_a_bijection_small_codes():
    """Brute force over every message of small codes: distinct messages give distinct
    codewords, and the systematic and non-systematic codebooks are the same set."""
    for N, K in [(4, 2), (8, 4), (16, 6), (16, 11)]:
        info = oracle.construct(N, K, 2.0)
        msgs = np.array([[(m >> j) & 1 for j in range(K)] for m in range(1 << K)], np.uint8)
        xs = oracle.encode_batch(info, 0, msgs, systematic=True)
        xn = oracle.encode_batch(info, 0, msgs)
        assert len({x.tobytes() for x in xs}) == 1 << K
        assert {x.tobytes() for x in xs} == {x.tobytes() for x in xn}


DECODERS = [
    ("scs", lambda m, info, crc, llr, sys: oracle.scs_decode_batch(m, info, crc, 8, 8, llr,
                                                                   systematic=sys)),
    ("fsscs", lambda m, info, crc, llr, sys: oracle.fsscs_decode_batch(m, info, crc, 8, 8, llr,
                                                                       systematic=sys)),
    ("scl", lambda m, info, crc, llr, sys: oracle.scl_decode_batch(m, info, crc, 4, llr,
                                                                   systematic=sys)),
]


@pytest.mark.parametrize("name,dec", DECODERS)
@pytest.mark.parametrize("N,K,crc", [(64, 32, 0), (128, 64, 16), (256, 128, 16)])
def test_noiseless_round_trip(name, dec, N, K, crc):
    info = oracle.construct(N, K, 2.0)
    pay = channel.payload_bits(4, N, 0, 25, K - crc)
    x = oracle.encode_batch(info, crc, pay, systematic=True)
    llr = channel.noiseless_llr(x)
    p, s, _ = dec(oracle.F32, info, crc, llr, True)
    assert (p == pay).all() and (s == oracle.ST_OK).all()


@pytest.mark.parametrize("name,dec", DECODERS)
def test_without_crc_the_codeword_estimate_is_the_same(name, dec):
    """Without a CRC the search does not depend on the encoding: the systematic payload is
    the non-systematic estimate re-encoded and read at the information positions."""
    N, K = 256, 128
    info = oracle.construct(N, K, 2.0)
    pay = channel.payload_bits(5, N, 0, 60, K)
    x = oracle.encode_batch(info, 0, pay, systematic=True)
    llr = channel.bpsk_awgn_llr(x, channel.noise(5, N, 0, 60, N), 1.5, K / N)
    p_ns, s_ns, _ = dec(oracle.F32, info, 0, llr, False)
    p_s, s_s, _ = dec(oracle.F32, info, 0, llr, True)
    xhat = oracle.encode_batch(info, 0, p_ns)
    assert (p_s == xhat[:, info == 1]).all() and (s_s == s_ns).all()
    assert (p_s != pay).any(axis=1).mean() < 0.5  # mostly decoded


@pytest.mark.parametrize("name,dec", DECODERS)
def test_crc_accepted_outputs_satisfy_the_crc(name, dec):
    """With CRC-16: an accepted systematic output path shows payload and a matching CRC in
    its codeword estimate (checked on single frames through u_hat)."""
    N, K, crc = 128, 64, 16
    info = oracle.construct(N, K, 2.0)
    pay = channel.payload_bits(6, N, 0, 40, K - crc)
    x = oracle.encode_batch(info, crc, pay, systematic=True)
    llr = channel.bpsk_awgn_llr(x, channel.noise(6, N, 0, 40, N), 1.0, K / N)
    single = {"scs": lambda y: oracle.scs_decode(oracle.F32, info, crc, 8, 8, y, systematic=True),
              "fsscs": lambda y: oracle.fsscs_decode(oracle.F32, info, crc, 8, 8, y,
                                                     systematic=True),
              "scl": lambda y: oracle.scl_decode(oracle.F32, info, crc, 4, y, systematic=True)}
    p, s, _ = dec(oracle.F32, info, crc, llr, True)
    ok = 0
    for b in range(llr.shape[0]):
        u, st, _, _ = single[name](llr[b])
        xh = oracle.polar_transform(u)[info == 1]
        assert st == s[b] and (xh[:K - crc] == p[b]).all()
        if st == oracle.ST_OK:
            ok += 1
            c = oracle.crc16(xh[:K - crc])
            assert list(xh[K - crc:]) == [(c >> (15 - j)) & 1 for j in range(16)]
    assert ok > 20
