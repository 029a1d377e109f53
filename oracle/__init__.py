"""Python access to the plain CPU oracle (``polar_oracle.cpp``).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously-correct reference that the
HIP decoder is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product package never
does, and the two share no code (the seeded input generator in
``paper_1809_03606_amd.channel`` is the only module both sides consume, and it holds
none of the decoder's arithmetic).

Each function names the passage of the paper (Aurora & Gross, "Towards Practical
Software Stack Decoding of Polar Codes") it follows; the C++ source carries the details.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "polar_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

F32, F64, FIX = 0, 1, 2
ST_OK, ST_FALLBACK, ST_EXHAUSTED = 1, 2, 4

STATS_FIELDS = ("iterations", "switches", "completions", "f_ops", "g_ops", "sc_elems",
                "evictions", "drops", "prunes")
STATS_DTYPE = np.dtype([(f, np.uint64) for f in STATS_FIELDS])


class _Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in STATS_FIELDS]


def build(force: bool = True) -> str:
    """Compile the oracle with plain IEEE arithmetic (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lock = threading.Lock()


def lib():
    """The compiled oracle.  POLAR_ORACLE_LIB names another build of the same source (the
    mutation tests load deliberately broken copies this way, in child processes)."""
    global _lib
    with _lock:
        if _lib is None:
            path = os.environ.get("POLAR_ORACLE_LIB") or _LIB
            if path == _LIB and not os.path.exists(_LIB):
                build(force=False)
            L = ctypes.CDLL(path)
            vp, u8p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8)
            L.orc_construct.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, vp]
            L.orc_bhattacharyya_log.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, vp]
            L.orc_crc16_bits.argtypes = [vp, ctypes.c_int]
            L.orc_crc16_bits.restype = ctypes.c_uint16
            L.orc_polar_transform.argtypes = [ctypes.c_int, vp, vp]
            L.orc_encode_batch.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int64, vp]
            L.orc_sc_decode.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp, vp]
            L.orc_leaf_llr.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int]
            L.orc_leaf_llr.restype = ctypes.c_double
            L.orc_scs_decode.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_int]
            L.orc_scs_decode_batch.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64,
                                               vp, vp, vp, ctypes.c_int]
            L.orc_encode_systematic_batch.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp,
                                                      ctypes.c_int64, vp]
            L.orc_ml_decode.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_int64]
            L.orc_fssc_schedule.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, ctypes.c_int]
            L.orc_node_candidates.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                              ctypes.c_double, vp, vp, ctypes.c_int]
            L.orc_fsscs_decode.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp,
                                           ctypes.c_int]
            L.orc_fsscs_decode_batch.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                                 ctypes.c_int64, vp, vp, vp, ctypes.c_int]
            L.orc_scs_trace.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int,
                                        ctypes.c_int]
            L.orc_fsscs_trace.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                          vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int]
            L.orc_scl_decode.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int,
                                         vp, vp, vp, vp, vp, ctypes.c_int]
            L.orc_scl_decode_batch.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int,
                                               ctypes.c_int, vp, ctypes.c_int64, vp, vp, vp,
                                               ctypes.c_int]
            for name in ("orc_construct", "orc_bhattacharyya_log", "orc_polar_transform",
                         "orc_encode_batch", "orc_sc_decode", "orc_scs_decode",
                         "orc_scs_decode_batch", "orc_ml_decode", "orc_fssc_schedule",
                         "orc_node_candidates", "orc_fsscs_decode", "orc_fsscs_decode_batch",
                         "orc_scl_decode", "orc_scl_decode_batch", "orc_scs_trace",
                         "orc_fsscs_trace", "orc_encode_systematic_batch"):
                getattr(L, name).restype = ctypes.c_int
            del u8p
            _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc):
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)


def _llr_array(mode: int, llr) -> np.ndarray:
    dt = {F32: np.float32, F64: np.float64, FIX: np.int8}[mode]
    a = np.ascontiguousarray(llr)
    if a.dtype != dt:
        raise TypeError("mode %d expects %s LLRs, got %s" % (mode, np.dtype(dt), a.dtype))
    return a


# -- construction, CRC, encoding (Section 2.1) --------------------------------------

def construct(N: int, K: int, design_db: float = 2.0) -> np.ndarray:
    """Bhattacharyya information set; returns info_mask[N] (1 = information)."""
    m = np.zeros(N, np.uint8)
    _check(lib().orc_construct(N, K, float(design_db), _p(m)))
    return m


def bhattacharyya_log(N: int, rate: float, design_db: float = 2.0) -> np.ndarray:
    z = np.zeros(N, np.float64)
    _check(lib().orc_bhattacharyya_log(N, float(rate), float(design_db), _p(z)))
    return z


def crc16(bits) -> int:
    b = np.ascontiguousarray(bits, dtype=np.uint8)
    return int(lib().orc_crc16_bits(_p(b), int(b.size)))


def polar_transform(u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.uint8)
    c = np.zeros_like(u)
    _check(lib().orc_polar_transform(int(u.size), _p(u), _p(c)))
    return c


def encode_batch(info_mask: np.ndarray, crc_bits: int, payload: np.ndarray,
                 systematic: bool = False) -> np.ndarray:
    """Codewords of B payloads (CRC appended): u F^(x)n with the message at the information
    positions of u, or with systematic=True the codeword that shows the message at the
    information positions (Section 2.2.2, last paragraph; Section 4)."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    pay = np.ascontiguousarray(payload, dtype=np.uint8)
    B = pay.shape[0]
    cw = np.zeros((B, info.size), np.uint8)
    fn = lib().orc_encode_systematic_batch if systematic else lib().orc_encode_batch
    _check(fn(int(info.size), _p(info), int(crc_bits), _p(pay), B, _p(cw)))
    return cw


# -- decoders ----------------------------------------------------------------------

def sc_decode(mode: int, info_mask: np.ndarray, llr):
    """SC decoding (Section 2.2.1, Algorithms 1-2).  Returns (u_hat[N], leaf_llr[N])."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = _llr_array(mode, llr)
    u = np.zeros(info.size, np.uint8)
    lf = np.zeros(info.size, np.float64)
    _check(lib().orc_sc_decode(mode, int(info.size), _p(info), _p(a), _p(u), _p(lf)))
    return u, lf


def leaf_llr(mode: int, llr, prefix, i: int) -> float:
    """alpha at leaf i for a given decided prefix (Algorithms 3-4)."""
    a = _llr_array(mode, llr)
    pre = np.zeros(a.size, np.uint8)
    pre[:i] = np.asarray(prefix, dtype=np.uint8)[:i]
    return float(lib().orc_leaf_llr(mode, int(a.size), _p(a), _p(pre), int(i)))


def scs_decode(mode: int, info_mask: np.ndarray, crc_bits: int, D: int, L: int, llr,
               systematic: bool = False):
    """SCS decoding of one frame (Section 2.2.5 with Section 3.3's reduced memory).

    Returns (u_hat[N], status, path_metric, stats dict)."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = _llr_array(mode, llr)
    u = np.zeros(info.size, np.uint8)
    st = ctypes.c_uint8(0)
    pm = ctypes.c_double(0.0)
    s = _Stats()
    _check(lib().orc_scs_decode(mode, int(info.size), _p(info), int(crc_bits), int(D), int(L),
                                _p(a), _p(u), ctypes.byref(st), ctypes.byref(pm), ctypes.byref(s),
                                int(bool(systematic))))
    return u, int(st.value), float(pm.value), {f: int(getattr(s, f)) for f in STATS_FIELDS}


def _trace(fn, mode, info_mask, head, llr, cap, systematic=False):
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = _llr_array(mode, llr)
    u = np.zeros(info.size, np.uint8)
    st = ctypes.c_uint8(0)
    pm = ctypes.c_double(0.0)
    s = _Stats()
    seq = np.zeros(cap, np.uint32)
    pl = np.zeros(cap, np.int32)
    tpm = np.zeros(cap, np.float64)
    n = fn(mode, int(info.size), _p(info), *head, _p(a), _p(u), ctypes.byref(st),
           ctypes.byref(pm), ctypes.byref(s), _p(seq), _p(pl), _p(tpm), int(cap),
           int(bool(systematic)))
    _check(min(n, 0))
    pops = [(int(seq[q]), int(pl[q]), float(tpm[q])) for q in range(min(n, cap))]
    return (u, int(st.value), float(pm.value), {f: int(getattr(s, f)) for f in STATS_FIELDS},
            pops, n)


def scs_trace(mode: int, info_mask: np.ndarray, crc_bits: int, D: int, L: int, llr,
              cap: int = 4096, systematic: bool = False):
    """scs_decode plus the paths taken off the stack in order, as (creation number, length,
    metric); returns (u_hat, status, pm, stats, pops, number of pops)."""
    return _trace(lib().orc_scs_trace, mode, info_mask, (int(crc_bits), int(D), int(L)), llr,
                  cap, systematic)


def fsscs_trace(mode: int, info_mask: np.ndarray, crc_bits: int, D: int, L: int, llr,
                types: int = 0xF, cap: int = 4096, systematic: bool = False):
    """fsscs_decode plus the paths taken off the stack in order (as scs_trace)."""
    return _trace(lib().orc_fsscs_trace, mode, info_mask,
                  (int(crc_bits), int(D), int(L), int(types)), llr, cap, systematic)


def scs_decode_batch(mode: int, info_mask: np.ndarray, crc_bits: int, D: int, L: int, llr,
                     threads: int = 1, systematic: bool = False):
    """Decode frames llr[B][N]; returns (payload[B][K-r], status[B], stats[B]).

    With threads > 1 the frames are split into contiguous chunks decoded concurrently
    (the C call releases the GIL); the result does not depend on the split."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = _llr_array(mode, llr)
    N = int(info.size)
    a = a.reshape(-1, N)
    B = a.shape[0]
    k = int(info.sum()) - int(crc_bits)
    pay = np.zeros((B, k), np.uint8)
    status = np.zeros(B, np.uint8)
    stats = np.zeros(B, STATS_DTYPE)
    L_ = lib()

    def run(lo, hi):
        if hi <= lo:
            return 0
        return L_.orc_scs_decode_batch(mode, N, _p(info), int(crc_bits), int(D), int(L),
                                       _p(a[lo:hi]), hi - lo, _p(pay[lo:hi]), _p(status[lo:hi]),
                                       _p(stats[lo:hi]), int(bool(systematic)))

    threads = max(1, min(int(threads), B if B else 1))
    if threads == 1:
        _check(run(0, B))
    else:
        edges = np.linspace(0, B, threads + 1).astype(int)
        with ThreadPoolExecutor(threads) as ex:
            for rc in ex.map(lambda t: run(edges[t], edges[t + 1]), range(threads)):
                _check(rc)
    return pay, status, stats


NODE_R0, NODE_R1, NODE_REP, NODE_SPC = 0, 1, 2, 3
NODE_NAMES = ("R-0", "R-1", "REP", "SPC")
TYPES_ALL = 0xF


def fssc_schedule(info_mask: np.ndarray, types: int = TYPES_ALL):
    """FSSC schedule (Section 3): list of (first leaf, lambda, class) in decoding order."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    N = int(info.size)
    st, lam, ty = (np.zeros(N, np.int32) for _ in range(3))
    cnt = lib().orc_fssc_schedule(N, _p(info), int(types), _p(st), _p(lam), _p(ty), N)
    _check(min(cnt, 0))
    return [(int(st[q]), int(lam[q]), int(ty[q])) for q in range(cnt)]


def node_candidates(mode: int, node_type: int, alpha, pm: float = 0.0):
    """FSSCL candidates of one node (Section 2.2.4): list of (estimates, metric)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    lam = int(a.size).bit_length() - 1
    beta = np.zeros((16, a.size), np.uint8)
    pms = np.zeros(16, np.float64)
    cnt = lib().orc_node_candidates(mode, int(node_type), lam, _p(a), float(pm), _p(beta),
                                    _p(pms), 16)
    _check(min(cnt, 0))
    return [(beta[q].copy(), float(pms[q])) for q in range(cnt)]


def fsscs_decode(mode: int, info_mask: np.ndarray, crc_bits: int, D: int, L: int, llr,
                 types: int = TYPES_ALL, systematic: bool = False):
    """FSSCS-RM decoding of one frame (Section 4).  Returns (u_hat, status, pm, stats)."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = _llr_array(mode, llr)
    u = np.zeros(info.size, np.uint8)
    st = ctypes.c_uint8(0)
    pm = ctypes.c_double(0.0)
    s = _Stats()
    _check(lib().orc_fsscs_decode(mode, int(info.size), _p(info), int(crc_bits), int(D), int(L),
                                  int(types), _p(a), _p(u), ctypes.byref(st), ctypes.byref(pm),
                                  ctypes.byref(s), int(bool(systematic))))
    return u, int(st.value), float(pm.value), {f: int(getattr(s, f)) for f in STATS_FIELDS}


def fsscs_decode_batch(mode: int, info_mask: np.ndarray, crc_bits: int, D: int, L: int, llr,
                       threads: int = 1, types: int = TYPES_ALL, systematic: bool = False):
    """Decode frames llr[B][N] with FSSCS-RM; returns (payload[B][K-r], status[B], stats[B])."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = _llr_array(mode, llr)
    N = int(info.size)
    a = a.reshape(-1, N)
    B = a.shape[0]
    k = int(info.sum()) - int(crc_bits)
    pay = np.zeros((B, k), np.uint8)
    status = np.zeros(B, np.uint8)
    stats = np.zeros(B, STATS_DTYPE)
    L_ = lib()

    def run(lo, hi):
        if hi <= lo:
            return 0
        return L_.orc_fsscs_decode_batch(mode, N, _p(info), int(crc_bits), int(D), int(L),
                                         int(types), _p(a[lo:hi]), hi - lo, _p(pay[lo:hi]),
                                         _p(status[lo:hi]), _p(stats[lo:hi]),
                                         int(bool(systematic)))

    threads = max(1, min(int(threads), B if B else 1))
    if threads == 1:
        _check(run(0, B))
    else:
        edges = np.linspace(0, B, threads + 1).astype(int)
        with ThreadPoolExecutor(threads) as ex:
            for rc in ex.map(lambda t: run(edges[t], edges[t + 1]), range(threads)):
                _check(rc)
    return pay, status, stats


def scl_decode(mode: int, info_mask: np.ndarray, crc_bits: int, L: int, llr,
               systematic: bool = False):
    """CA-SCL decoding of one frame (Section 2.2.3).  Returns (u_hat, status, pm, stats)."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = _llr_array(mode, llr)
    u = np.zeros(info.size, np.uint8)
    st = ctypes.c_uint8(0)
    pm = ctypes.c_double(0.0)
    s = _Stats()
    _check(lib().orc_scl_decode(mode, int(info.size), _p(info), int(crc_bits), int(L), _p(a),
                                _p(u), ctypes.byref(st), ctypes.byref(pm), ctypes.byref(s),
                                int(bool(systematic))))
    return u, int(st.value), float(pm.value), {f: int(getattr(s, f)) for f in STATS_FIELDS}


def scl_decode_batch(mode: int, info_mask: np.ndarray, crc_bits: int, L: int, llr,
                     threads: int = 1, systematic: bool = False):
    """Decode frames llr[B][N] with CA-SCL; returns (payload[B][K-r], status[B], stats[B])."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = _llr_array(mode, llr)
    N = int(info.size)
    a = a.reshape(-1, N)
    B = a.shape[0]
    k = int(info.sum()) - int(crc_bits)
    pay = np.zeros((B, k), np.uint8)
    status = np.zeros(B, np.uint8)
    stats = np.zeros(B, STATS_DTYPE)
    L_ = lib()

    def run(lo, hi):
        if hi <= lo:
            return 0
        return L_.orc_scl_decode_batch(mode, N, _p(info), int(crc_bits), int(L), _p(a[lo:hi]),
                                       hi - lo, _p(pay[lo:hi]), _p(status[lo:hi]),
                                       _p(stats[lo:hi]), int(bool(systematic)))

    threads = max(1, min(int(threads), B if B else 1))
    if threads == 1:
        _check(run(0, B))
    else:
        edges = np.linspace(0, B, threads + 1).astype(int)
        with ThreadPoolExecutor(threads) as ex:
            for rc in ex.map(lambda t: run(edges[t], edges[t + 1]), range(threads)):
                _check(rc)
    return pay, status, stats


def ml_decode(info_mask: np.ndarray, llr, max_out: int = 64):
    """Brute-force ML over all 2^K information words; returns (disc_min, [u minimisers])."""
    info = np.ascontiguousarray(info_mask, dtype=np.uint8)
    a = np.ascontiguousarray(llr, dtype=np.float64)
    N = int(info.size)
    mins = np.zeros((max_out, N), np.uint8)
    dmin = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().orc_ml_decode(N, _p(info), _p(a), ctypes.byref(dmin), ctypes.byref(cnt),
                               _p(mins), int(max_out)))
    return float(dmin.value), mins[:min(int(cnt.value), max_out)], int(cnt.value)
