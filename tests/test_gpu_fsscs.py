"""GPU parity of the fast simplified stack decoder (FSSCS-RM, Section 4) with the oracle,
frame by frame: payload bits, status and the search itself (node extensions, switches,
completions, SC-schedule work, evictions, drops, prunes)."""
import sys

import numpy as np
import pytest

import oracle
from cases import THREADS, assert_parity, gpu_decode, make_frames

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(cuda, N, K, crc, D, L, eb, B, seed, dtype="f32"):
    from paper_1809_03606_amd.binding import PolarCode

    label = "FSSCS N=%d K=%d crc=%d D=%d L=%d Eb/N0=%.1f B=%d seed=%d %s" % (
        N, K, crc, D, L, eb, B, seed, dtype)
    info, pay, llr = make_frames(N, K, crc, eb, B, seed, dtype=dtype)
    code = PolarCode(N, K, crc, 2.0)
    assert (code.info_mask == info).all()
    mode = oracle.F32 if dtype == "f32" else oracle.FIX
    ref = oracle.fsscs_decode_batch(mode, info, crc, D, L, llr, threads=THREADS)
    _say("gpu: " + label)
    got = gpu_decode(cuda, code, D, L, llr, fast=True)
    assert_parity(got, ref, label)
    return got, ref, pay


# every length; CRC on and off; D 1..64, L 1..255; degenerate codes whose root is a node
# (K = 1: REP, K = N - 1: SPC, K = N: R-1); batches not a multiple of the workgroup size
CASES = [
    (2, 1, 0, 1, 1, 1.0), (2, 2, 0, 4, 8, 0.0), (4, 3, 0, 4, 8, 1.0), (8, 4, 0, 8, 8, 0.5),
    (16, 8, 0, 64, 255, 0.0), (16, 15, 0, 5, 3, 1.0), (32, 24, 16, 16, 8, 2.0),
    (32, 1, 0, 3, 2, 0.0), (64, 32, 0, 8, 8, 2.0), (64, 64, 0, 8, 4, 3.0),
    (64, 48, 16, 32, 4, 1.0), (128, 64, 16, 64, 8, 1.5), (128, 127, 0, 8, 8, 2.0),
    (256, 128, 16, 32, 8, 1.5), (256, 1, 0, 4, 4, 0.0), (512, 256, 16, 64, 8, 1.5),
    (512, 511, 0, 8, 8, 3.0), (1024, 512, 16, 32, 8, 1.5), (1024, 853, 16, 64, 16, 2.5),
    (1024, 1024, 0, 8, 8, 4.0), (2048, 1024, 16, 32, 8, 1.5), (2048, 1707, 16, 64, 8, 3.0),
    (2048, 2047, 0, 4, 4, 4.0), (2048, 1, 0, 4, 4, 0.0),
]


@pytest.mark.parametrize("N,K,crc,D,L,eb", CASES)
def test_fsscs_matches_oracle_f32(cuda, N, K, crc, D, L, eb):
    B = 37 if N >= 1024 else 101
    _run(cuda, N, K, crc, D, L, eb, B, seed=31 + N)


@pytest.mark.parametrize("N,K,crc,D,L,eb", CASES[::2])
def test_fsscs_matches_oracle_i8(cuda, N, K, crc, D, L, eb):
    B = 37 if N >= 1024 else 101
    _run(cuda, N, K, crc, D, L, eb, B, seed=41 + N, dtype="i8")


# stacks deeper than one 64-slot bank (D up to 256), filled by low Eb/N0 and large L
DEEP = [
    (16, 8, 0, 256, 255, 0.0), (64, 32, 0, 65, 8, 1.0), (128, 64, 16, 100, 8, 1.0),
    (256, 128, 16, 128, 16, 1.0), (512, 256, 16, 200, 16, 1.0), (1024, 512, 16, 256, 8, 1.0),
    (1024, 512, 16, 129, 8, 2.0), (1024, 853, 16, 192, 64, 2.0), (2048, 1024, 16, 256, 8, 1.5),
]


@pytest.mark.parametrize("N,K,crc,D,L,eb", DEEP)
def test_fsscs_deep_stack_matches_oracle_f32(cuda, N, K, crc, D, L, eb):
    B = 37 if N >= 1024 else 101
    _run(cuda, N, K, crc, D, L, eb, B, seed=71 + N + D)


@pytest.mark.parametrize("N,K,crc,D,L,eb", DEEP[1::2])
def test_fsscs_deep_stack_matches_oracle_i8(cuda, N, K, crc, D, L, eb):
    B = 37 if N >= 1024 else 101
    _run(cuda, N, K, crc, D, L, eb, B, seed=81 + N + D, dtype="i8")


@pytest.mark.parametrize("eb", [1.0, 2.0, 3.0])
def test_fsscs_n1024_crc16_points(cuda, eb):
    """PC(1024,512)+CRC-16, D = 32, L = 8 at three Eb/N0 points, 400 frames each."""
    got, ref, pay = _run(cuda, 1024, 512, 16, 32, 8, eb, 400, seed=int(eb * 10))


# FSSC: the fast simplified decoder with D = 1 and L = 1 (Section 2.2.2 nodes on the schedule
# of Section 3, no stack), at realistic lengths whose schedules hold R-0, R-1, REP and SPC
# nodes, with and without CRC
FSSC = [(64, 32, 0, 2.0), (128, 64, 16, 1.5), (256, 128, 0, 2.0), (512, 256, 16, 2.0),
        (1024, 512, 16, 2.0), (1024, 853, 0, 3.0), (2048, 1024, 16, 2.0), (2048, 512, 0, 1.0)]


@pytest.mark.parametrize("dtype", ["f32", "i8"])
@pytest.mark.parametrize("N,K,crc,eb", FSSC)
def test_fssc_matches_oracle(cuda, N, K, crc, eb, dtype):
    classes = {t for (_, lam, t) in oracle.fssc_schedule(oracle.construct(N, K, 2.0)) if lam > 0}
    assert {oracle.NODE_R1, oracle.NODE_REP, oracle.NODE_SPC} <= classes, classes
    B = 150 if N >= 1024 else 301
    _run(cuda, N, K, crc, 1, 1, eb, B, seed=91 + N + K, dtype=dtype)
