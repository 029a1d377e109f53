"""The C-ABI library on the host: it loads without a GPU, exports every entry point that
include/polarscs.h declares, and its host-side calls (construction, encoding, argument
checks) behave as documented.  No decoding runs here."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1809_03606_amd import binding, channel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polarscs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.library_path()):
        pytest.fail("libpolarscs.so is not built (run __graft_entry__.build())")
    return binding.lib()


def test_library_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 12, names
    raw = ctypes.CDLL(binding.library_path())
    for n in names:
        assert hasattr(raw, n), n
    assert set(binding.EXPORTS) == set(names)


@pytest.mark.parametrize("N,K,crc,db", [(2, 1, 0, 2.0), (8, 4, 0, 2.0), (64, 32, 0, 2.0),
                                        (128, 32, 16, 2.0), (1024, 512, 16, 2.0),
                                        (2048, 1707, 16, 2.0), (512, 427, 16, 0.0)])
def test_construction_and_encoder_match_oracle(lib, N, K, crc, db):
    code = binding.PolarCode(N, K, crc, db)
    assert (code.N, code.K, code.crc_bits) == (N, K, crc)
    assert (code.info_mask == oracle.construct(N, K, db)).all()
    pay = channel.payload_bits(21, N, 0, 64, K - crc)
    assert (code.encode(pay) == oracle.encode_batch(code.info_mask, crc, pay)).all()


def test_construct_rejects_bad_arguments(lib):
    h = ctypes.c_void_p()
    for args in [(3, 1, 0), (4096, 8, 0), (1, 1, 0), (64, 0, 0), (64, 65, 0), (64, 32, 8),
                 (64, 16, 16), (0, 0, 0)]:
        rc = lib.polar_construct(args[0], args[1], args[2], 2.0, ctypes.byref(h))
        assert rc == binding.POLAR_EINVAL, args
    assert lib.polar_construct(64, 32, 0, float("nan"), ctypes.byref(h)) == binding.POLAR_EINVAL
    assert lib.polar_construct(64, 32, 0, 2.0, None) == binding.POLAR_EINVAL


def test_encode_and_decode_reject_bad_arguments(lib):
    code = binding.PolarCode(64, 32, 0)
    assert lib.polar_encode(None, None, None, 1) == binding.POLAR_EINVAL
    assert lib.polar_encode(code.handle, None, None, 1) == binding.POLAR_EINVAL
    assert lib.polar_encode(code.handle, None, None, 0) == binding.POLAR_OK
    assert lib.polar_encode(code.handle, None, None, -1) == binding.POLAR_EINVAL
    # every argument error is caught on the host before any device work
    assert lib.scs_decode_batch(None, code.handle, 8, 8, 0, None, 1, None, None, None,
                                None) == binding.POLAR_EINVAL
    assert lib.scs_ctx_last_error(None) == binding.POLAR_EINVAL
    assert lib.polar_code_query(None, None, None, None, None) == binding.POLAR_EINVAL
    assert lib.polar_strerror(binding.POLAR_EINVAL) == b"invalid argument"


def test_query_roundtrip(lib):
    code = binding.PolarCode(256, 100, 16, 1.5)
    N, K, r, mask = binding.polar_code_query(code.handle)
    assert (N, K, r) == (256, 100, 16) and mask.sum() == 100


def test_channel_generator_is_seeded_and_chunk_independent():
    a = channel.noise(5, 7, 0, 70000, 8)
    b = channel.noise(5, 7, 65530, 100, 8)
    assert np.array_equal(a[65530:65630], b)
    p = channel.payload_bits(5, 7, 100, 10, 33)
    assert np.array_equal(channel.payload_bits(5, 7, 0, 200, 33)[100:110], p)
    assert not np.array_equal(channel.noise(5, 8, 0, 4, 8), channel.noise(5, 7, 0, 4, 8))


def test_channel_llr_formula():
    cw = np.array([[0, 1, 0, 1]], np.uint8)
    n = np.array([[0.0, 0.0, 0.5, -0.5]])
    s2 = channel.sigma2(2.0, 0.5)
    llr = channel.bpsk_awgn_llr(cw, n, 2.0, 0.5)
    y = np.array([1.0, -1.0, 1 + 0.5 * np.sqrt(s2), -1 - 0.5 * np.sqrt(s2)])
    assert np.allclose(llr[0], 2 * y / s2, rtol=1e-6)
    q = channel.bpsk_awgn_i8(cw, n, 2.0, 0.5, 8.0)
    assert q.dtype == np.int8 and list(q[0][:2]) == [8, -8]


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_waves_per_block_knob_rejects_bad_arguments(lib):
    assert lib.scs_ctx_set_waves_per_block(None, 2) == binding.POLAR_EINVAL


def test_tune_cache_roundtrip(tmp_path):
    from paper_1809_03606_amd import tune

    code = binding.PolarCode(1024, 512, 16)
    k = tune.key("gfx950", code, 32, 8, "f32")
    assert k == "gfx950:N1024:K512:crc16:D32:L8:f32"
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load(path) == {}
    tune.save({k: {"waves_per_block": 2}}, path)
    assert tune.load(path)[k]["waves_per_block"] == 2
    assert sorted(tune.CANDIDATES) == [1, 2, 4]
    # the list decoder: no stack depth in its key, workgroup sizes only
    assert tune.key("gfx950", code, 32, 4, "f32", "scl") == tune.key("gfx950", code, 0, 4, "f32", "scl")
    assert tune.key("gfx950", code, 32, 4, "f32", "scl").endswith(":D0:L4:f32:scl")
    assert tune.candidates("scl") == [4, 2, 1]


def test_library_shares_pytorchs_hip_runtime():
    """Loading the library before PyTorch must not map a second HIP runtime (device buffers
    of one runtime are not usable by the other)."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1809_03606_amd import binding\n"
            "binding.lib()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len(set(l.split()[-1] for l in maps if 'libamdhip64' in l)))\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"


@pytest.mark.parametrize("N", [2, 4, 8, 64, 256, 1024, 2048])
def test_library_schedule_matches_oracle(lib, N):
    """The fast decoder's node table, built by the library, equals the oracle's schedule,
    including the degenerate codes whose root is a node (K = 1, N - 1, N)."""
    rng = np.random.default_rng(N)
    Ks = sorted({1, max(1, N - 1), N, N // 2, int(rng.integers(1, N + 1))})
    for K in Ks:
        crc = 16 if K > 16 and N >= 64 else 0
        code = binding.PolarCode(N, K, crc, 2.0)
        assert binding.polar_code_schedule(code.handle) == oracle.fssc_schedule(code.info_mask), (N, K)


def test_fsscs_rejects_bad_arguments(lib):
    code = binding.PolarCode(64, 32, 0)
    assert lib.fsscs_decode_batch(None, code.handle, 8, 8, 0, None, 1, None, None, None,
                                  None) == binding.POLAR_EINVAL
    assert lib.polar_code_schedule(None, None) == binding.POLAR_EINVAL


def test_scl_rejects_bad_arguments(lib):
    code = binding.PolarCode(64, 32, 0)
    assert lib.scl_decode_batch(None, code.handle, 8, 0, None, 1, None, None, None,
                                None) == binding.POLAR_EINVAL


def test_construct_from_an_explicit_set(lib):
    """polar_construct_set keeps the given information set; the encoder, CRC placement and
    schedule follow it exactly as for a constructed code."""
    rng = np.random.default_rng(5)
    for N, K, crc in [(2, 1, 0), (4, 3, 0), (32, 17, 16), (256, 100, 16), (2048, 700, 16)]:
        mask = np.zeros(N, np.uint8)
        mask[rng.choice(N, K, replace=False)] = 1
        code = binding.PolarCode.from_set(mask, crc)
        assert (code.N, code.K, code.crc_bits) == (N, K, crc)
        assert (code.info_mask == mask).all()
        pay = channel.payload_bits(23, N, 0, 16, K - crc)
        assert (code.encode(pay) == oracle.encode_batch(mask, crc, pay)).all()
        assert binding.polar_code_schedule(code.handle) == [
            (s, lam, t) for (s, lam, t) in oracle.fssc_schedule(mask)]
    h = ctypes.c_void_p()
    ok = np.ones(8, np.uint8)
    for N, m, crc in [(6, ok, 0), (8, np.zeros(8, np.uint8), 0), (8, ok * 2, 0), (8, ok, 8),
                      (32, np.r_[np.ones(16, np.uint8), np.zeros(16, np.uint8)], 16)]:
        m = np.ascontiguousarray(m, dtype=np.uint8)
        assert lib.polar_construct_set(N, m.ctypes.data, crc, ctypes.byref(h)) == binding.POLAR_EINVAL
    assert lib.polar_construct_set(8, None, 0, ctypes.byref(h)) == binding.POLAR_EINVAL
    assert lib.polar_construct_set(8, ok.ctypes.data, 0, None) == binding.POLAR_EINVAL


@pytest.mark.parametrize("N,K,crc", [(2, 1, 0), (8, 4, 0), (64, 32, 16), (256, 77, 16),
                                     (1024, 512, 16), (2048, 1707, 16)])
def test_systematic_twin_encodes_like_the_oracle(lib, N, K, crc):
    code = binding.PolarCode(N, K, crc, 2.0)
    twin = code.make_systematic()
    assert twin.systematic and not code.systematic
    assert (twin.N, twin.K, twin.crc_bits) == (N, K, crc) and (twin.info_mask == code.info_mask).all()
    pay = channel.payload_bits(31, N, 0, 32, K - crc)
    assert (twin.encode(pay) == oracle.encode_batch(code.info_mask, crc, pay, systematic=True)).all()
    assert (code.encode(pay) == oracle.encode_batch(code.info_mask, crc, pay)).all()


def test_systematic_twin_needs_a_set_that_shows_the_message(lib):
    """PC(4,3) with set {0, 1, 3}: the unit message at 3 encodes (by hand: v = e3,
    u = v F = 1111, cleared at 2: 1101, x = 1011) to a codeword reading (1, 0, 1) at the
    set, not (0, 0, 1): refused.  The set {1, 7} of N = 8 is not contiguous in the subset
    order but does show every message, and is accepted; both agree with the oracle."""
    bad = np.array([1, 1, 0, 1], np.uint8)
    assert (oracle.encode_batch(bad, 0, np.array([[0, 0, 1]], np.uint8), systematic=True)
            == np.array([[1, 0, 1, 1]], np.uint8)).all()
    with pytest.raises(binding.PolarError) as e:
        binding.PolarCode.from_set(bad, 0).make_systematic()
    assert e.value.code == binding.POLAR_EUNSUPPORTED
    good = np.zeros(8, np.uint8)
    good[[1, 7]] = 1
    msgs = np.array([[1, 0], [0, 1], [1, 1]], np.uint8)
    twin = binding.PolarCode.from_set(good, 0).make_systematic()
    assert (twin.encode(msgs) == oracle.encode_batch(good, 0, msgs, systematic=True)).all()
    assert (twin.encode(msgs)[:, [1, 7]] == msgs).all()
    # random upward-closed sets (constructed) are accepted
    for N, K in [(32, 5), (512, 300)]:
        binding.PolarCode(N, K, 0, 1.0).make_systematic()
    assert lib.polar_code_is_systematic(None) == binding.POLAR_EINVAL
    assert lib.polar_code_systematic(None, None) == binding.POLAR_EINVAL
