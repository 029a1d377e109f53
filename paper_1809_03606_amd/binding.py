"""Thin ctypes binding of ``libpolarscs.so`` (argument marshalling only).

Every decoding step runs in the library's HIP kernels; this module only converts
arguments (numpy arrays for host buffers, torch tensors or raw addresses for device
buffers, torch streams for ``hip_stream``).  If the library has not been built the first
call raises: there is no fallback path.

The functions keep the C names (``polar_construct``, ``polar_encode``,
``scs_decode_batch``, ...); ``PolarCode`` and ``ScsContext`` wrap the opaque handles.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpolarscs.so")

POLAR_OK, POLAR_EINVAL, POLAR_ENOMEM, POLAR_EDEVICE, POLAR_EUNSUPPORTED = 0, -1, -2, -3, -4
POLAR_ETOOLARGE = -5
NOALLOC_SCRATCH_BYTES, NOALLOC_MAX_CODES = 16 << 20, 64
SCS_STATUS_OK, SCS_STATUS_FALLBACK, SCS_STATUS_EXHAUSTED = 1, 2, 4
SCS_LLR_F32, SCS_LLR_I8 = 0, 1

EXPORTS = ("polar_construct", "polar_construct_set", "polar_code_systematic",
           "polar_code_is_systematic", "polar_code_query", "polar_code_free", "polar_encode",
           "polar_encode_device", "scs_ctx_create", "scs_ctx_destroy", "scs_decode_batch",
           "scs_decode_mixed", "scs_mixed_prepare", "scs_mixed_launch",
           "scs_decode_mixed_noalloc", "scs_ctx_set_waves_per_block", "scs_ctx_set_grid_cus",
           "scs_ctx_last_error", "polar_strerror",
           "polar_code_schedule", "fsscs_decode_batch", "scl_decode_batch")

STATS_FIELDS = ("iterations", "switches", "completions", "sc_elems", "fg_elems", "evictions",
                "drops", "prunes")
STATS_DTYPE = np.dtype([(f, np.uint32) for f in STATS_FIELDS])

FRAME_DTYPE = np.dtype([("code", np.int32), ("D", np.int32), ("L", np.int32), ("_pad", np.int32),
                        ("llr_off", np.int64), ("out_off", np.int64)])


class ScsFrame(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("D", ctypes.c_int32), ("L", ctypes.c_int32),
                ("_pad", ctypes.c_int32), ("llr_off", ctypes.c_int64), ("out_off", ctypes.c_int64)]


class PolarError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))
        self.code = code


_lib = None
_lock = threading.Lock()


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load the HIP library; raises if it is missing (build it first)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError("libpolarscs.so is not built: run `python -m "
                                   "paper_1809_03606_amd.build` (no CPU fallback exists)")
            # PyTorch ships its own HIP runtime and asks for it by an unversioned name, so
            # loading this library first would put a second runtime into the process (device
            # buffers of one are not usable by the other).  Loaded after torch, the library's
            # libamdhip64.so.7 resolves to the copy torch already mapped.
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = ctypes.CDLL(_LIB_PATH)
            vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
            L.polar_construct.argtypes = [i32, i32, i32, dbl, ctypes.POINTER(vp)]
            L.polar_construct_set.argtypes = [i32, vp, i32, ctypes.POINTER(vp)]
            L.polar_code_systematic.argtypes = [vp, ctypes.POINTER(vp)]
            L.polar_code_is_systematic.argtypes = [vp]
            L.polar_code_query.argtypes = [vp, vp, vp, vp, vp]
            L.polar_code_free.argtypes = [vp]
            L.polar_code_free.restype = None
            L.polar_encode.argtypes = [vp, vp, vp, i64]
            L.polar_encode_device.argtypes = [vp, vp, vp, i64, vp]
            L.scs_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
            L.scs_ctx_destroy.argtypes = [vp]
            L.scs_ctx_destroy.restype = None
            L.scs_decode_batch.argtypes = [vp, vp, i32, i32, i32, vp, i64, vp, vp, vp, vp]
            L.scs_decode_mixed.argtypes = [vp, vp, i32, vp, i64, i32, vp, vp, vp, vp, vp]
            L.scs_decode_mixed_noalloc.argtypes = [vp, vp, i32, vp, i64, i32, vp, vp, vp, vp, vp]
            L.scs_mixed_prepare.argtypes = [vp, vp, i32, vp, i64, vp]
            L.scs_mixed_launch.argtypes = [vp, i32, vp, vp, vp, vp, vp]
            L.scs_ctx_last_error.argtypes = [vp]
            L.scs_ctx_set_waves_per_block.argtypes = [vp, i32]
            L.scs_ctx_set_grid_cus.argtypes = [vp, i32]
            L.polar_code_schedule.argtypes = [vp, vp]
            L.fsscs_decode_batch.argtypes = [vp, vp, i32, i32, i32, vp, i64, vp, vp, vp, vp]
            L.scl_decode_batch.argtypes = [vp, vp, i32, i32, vp, i64, vp, vp, vp, vp]
            L.polar_strerror.argtypes = [ctypes.c_int]
            L.polar_strerror.restype = ctypes.c_char_p
            for n in ("polar_construct", "polar_construct_set", "polar_code_systematic",
                      "polar_code_is_systematic", "polar_code_query", "polar_encode", "polar_encode_device",
                      "scs_ctx_create", "scs_decode_batch", "scs_decode_mixed",
                      "scs_decode_mixed_noalloc",
                      "scs_mixed_prepare", "scs_mixed_launch",
                      "scs_ctx_set_waves_per_block", "scs_ctx_set_grid_cus",
                      "scs_ctx_last_error",
                      "polar_code_schedule", "fsscs_decode_batch", "scl_decode_batch"):
                getattr(L, n).restype = ctypes.c_int
            _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().polar_strerror(int(code)).decode()
    except Exception:  # the library itself may be what is missing
        return "status %d" % code


def _check(rc: int, what: str):
    if rc != POLAR_OK:
        raise PolarError(rc, what)


def _addr(x) -> int | None:
    """Device or host address of a torch tensor / numpy array / int (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return int(x.data_ptr())


def _device_buffer(t, name: str, dtypes, min_elems: int, device: int | None):
    """Check a torch tensor handed to a kernel: on the expected GPU, contiguous, of one of
    `dtypes`, with at least `min_elems` elements (so the kernel stays inside it)."""
    if t is None:
        raise ValueError("%s is required" % name)
    if not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a GPU tensor" % name)
    if device is not None and t.device.index != device:
        raise ValueError("%s is on cuda:%s, the context on cuda:%d" % (name, t.device.index, device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s; expected one of %s" % (name, t.dtype, dtypes))
    if t.numel() < min_elems:
        raise ValueError("%s holds %d elements; at least %d needed" % (name, t.numel(), min_elems))


def _stream(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)  # torch.cuda.Stream


# -- raw C-ABI names ----------------------------------------------------------------

def polar_construct(N: int, K: int, crc_bits: int, design_ebn0_db: float) -> int:
    h = ctypes.c_void_p()
    _check(lib().polar_construct(N, K, crc_bits, float(design_ebn0_db), ctypes.byref(h)),
           "polar_construct")
    return h.value


def polar_construct_set(info_mask: np.ndarray, crc_bits: int) -> int:
    m = np.ascontiguousarray(info_mask, dtype=np.uint8)
    h = ctypes.c_void_p()
    _check(lib().polar_construct_set(int(m.size), m.ctypes.data, int(crc_bits), ctypes.byref(h)),
           "polar_construct_set")
    return h.value


def polar_code_systematic(handle: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().polar_code_systematic(handle, ctypes.byref(h)), "polar_code_systematic")
    return h.value


def polar_code_is_systematic(handle: int) -> bool:
    rc = lib().polar_code_is_systematic(handle)
    if rc < 0:
        _check(rc, "polar_code_is_systematic")
    return rc == 1


def polar_code_query(handle: int):
    N, K, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().polar_code_query(handle, ctypes.byref(N), ctypes.byref(K), ctypes.byref(r), None),
           "polar_code_query")
    mask = np.zeros(N.value, np.uint8)
    _check(lib().polar_code_query(handle, None, None, None, mask.ctypes.data), "polar_code_query")
    return N.value, K.value, r.value, mask


def polar_code_free(handle: int):
    lib().polar_code_free(handle)


def polar_encode(handle: int, payload: np.ndarray, codeword: np.ndarray):
    assert payload.flags.c_contiguous and codeword.flags.c_contiguous
    assert payload.dtype == np.uint8 and codeword.dtype == np.uint8
    _check(lib().polar_encode(handle, _addr(payload), _addr(codeword), int(codeword.shape[0])),
           "polar_encode")


def polar_encode_device(handle: int, payload_dev, codeword_dev, B: int, stream=None):
    _check(lib().polar_encode_device(handle, _addr(payload_dev), _addr(codeword_dev), int(B),
                                     _stream(stream)), "polar_encode_device")


def scs_ctx_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().scs_ctx_create(int(device), ctypes.byref(h)), "scs_ctx_create")
    return h.value


def scs_ctx_destroy(ctx: int):
    _PLANS.pop(ctx, None)
    lib().scs_ctx_destroy(ctx)


def scs_decode_batch(ctx: int, code: int, D: int, L: int, llr_dtype: int, llr_dev, n_frames: int,
                     payload_dev, status_dev, stats_dev=None, stream=None):
    _check(lib().scs_decode_batch(ctx, code, int(D), int(L), int(llr_dtype), _addr(llr_dev),
                                  int(n_frames), _addr(payload_dev), _addr(status_dev),
                                  _addr(stats_dev), _stream(stream)), "scs_decode_batch")


def fsscs_decode_batch(ctx: int, code: int, D: int, L: int, llr_dtype: int, llr_dev, n_frames: int,
                       payload_dev, status_dev, stats_dev=None, stream=None):
    _check(lib().fsscs_decode_batch(ctx, code, int(D), int(L), int(llr_dtype), _addr(llr_dev),
                                    int(n_frames), _addr(payload_dev), _addr(status_dev),
                                    _addr(stats_dev), _stream(stream)), "fsscs_decode_batch")


def scl_decode_batch(ctx: int, code: int, L: int, llr_dtype: int, llr_dev, n_frames: int,
                     payload_dev, status_dev, stats_dev=None, stream=None):
    _check(lib().scl_decode_batch(ctx, code, int(L), int(llr_dtype), _addr(llr_dev),
                                  int(n_frames), _addr(payload_dev), _addr(status_dev),
                                  _addr(stats_dev), _stream(stream)), "scl_decode_batch")


def polar_code_schedule(handle: int) -> list:
    """The code's fast simplified schedule: [(first leaf, lambda, class)] in order."""
    N, _, _, _ = polar_code_query(handle)
    raw = np.zeros(N, np.uint8)
    _check(lib().polar_code_schedule(handle, raw.ctypes.data), "polar_code_schedule")
    return [(int(j), int(v) & 15, int(v) >> 4) for j, v in enumerate(raw) if v != 0xFF]


_PLANS = {}  # context handle -> extent of its prepared mixed plan (see _plan_extent)


def _plan_extent(codes, fr):
    """(LLR elements, payload bytes, frames) that the buffers of a mixed plan must hold, or
    None when a descriptor names no code (the library refuses such a plan itself)."""
    n = int(fr.shape[0])
    if n == 0:
        return (0, 0, 0)
    shapes = []
    for h in codes:
        N, K, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().polar_code_query(h, ctypes.byref(N), ctypes.byref(K), ctypes.byref(r), None),
               "polar_code_query")
        shapes.append((N.value, K.value - r.value))
    c = fr["code"].astype(np.int64)
    if len(shapes) == 0 or c.min() < 0 or c.max() >= len(shapes):
        return None
    Ns = np.array([a for a, _ in shapes], np.int64)[c]
    kps = np.array([b for _, b in shapes], np.int64)[c]
    return int((fr["llr_off"] + Ns).max()), int((fr["out_off"] + kps).max()), n


def _check_plan_buffers(extent, llr_dtype, llr_dev, payload_dev, status_dev, stats_dev):
    """Check torch tensors against a plan's extent (raw addresses cannot be checked)."""
    if extent is None:
        return
    need_llr, need_out, n = extent
    import torch

    def tensor(t):
        return t is not None and not isinstance(t, int) and hasattr(t, "is_cuda")

    if tensor(llr_dev):
        _device_buffer(llr_dev, "llr", (torch.float32,) if llr_dtype == SCS_LLR_F32 else
                       (torch.int8,), need_llr, None)
    dev = llr_dev.device.index if tensor(llr_dev) else None
    if tensor(payload_dev):
        _device_buffer(payload_dev, "payload", (torch.uint8,), need_out, dev)
    if tensor(status_dev):
        _device_buffer(status_dev, "status", (torch.uint8,), n, dev)
    if tensor(stats_dev):
        _device_buffer(stats_dev, "stats", (torch.int32, torch.uint32), n * len(STATS_FIELDS), dev)


def scs_decode_mixed(ctx: int, codes, frames: np.ndarray, llr_dtype: int, llr_dev, payload_dev,
                     status_dev, stats_dev=None, stream=None):
    arr = (ctypes.c_void_p * max(1, len(codes)))(*codes)
    fr = np.ascontiguousarray(frames, dtype=FRAME_DTYPE)
    _check_plan_buffers(_plan_extent(codes, fr), llr_dtype, llr_dev, payload_dev, status_dev,
                        stats_dev)
    _check(lib().scs_decode_mixed(ctx, ctypes.cast(arr, ctypes.c_void_p), len(codes),
                                  fr.ctypes.data, int(fr.shape[0]), int(llr_dtype),
                                  _addr(llr_dev), _addr(payload_dev), _addr(status_dev),
                                  _addr(stats_dev), _stream(stream)), "scs_decode_mixed")


def scs_decode_mixed_noalloc(ctx: int, codes, frames: np.ndarray, llr_dtype: int, llr_dev,
                             payload_dev, status_dev, stats_dev=None, stream=None):
    """scs_decode_mixed with the batch plan in the library's fixed per-device scratch array
    (no device allocation); raises PolarError(POLAR_ETOOLARGE) beyond its capacity."""
    arr = (ctypes.c_void_p * max(1, len(codes)))(*codes)
    fr = np.ascontiguousarray(frames, dtype=FRAME_DTYPE)
    _check_plan_buffers(_plan_extent(codes, fr), llr_dtype, llr_dev, payload_dev, status_dev,
                        stats_dev)
    _check(lib().scs_decode_mixed_noalloc(ctx, ctypes.cast(arr, ctypes.c_void_p), len(codes),
                                          fr.ctypes.data, int(fr.shape[0]), int(llr_dtype),
                                          _addr(llr_dev), _addr(payload_dev), _addr(status_dev),
                                          _addr(stats_dev), _stream(stream)),
           "scs_decode_mixed_noalloc")


def scs_mixed_prepare(ctx: int, codes, frames: np.ndarray, stream=None):
    arr = (ctypes.c_void_p * max(1, len(codes)))(*codes)
    fr = np.ascontiguousarray(frames, dtype=FRAME_DTYPE)
    extent = _plan_extent(codes, fr)
    _check(lib().scs_mixed_prepare(ctx, ctypes.cast(arr, ctypes.c_void_p), len(codes),
                                   fr.ctypes.data, int(fr.shape[0]), _stream(stream)),
           "scs_mixed_prepare")
    _PLANS[ctx] = extent


def scs_mixed_launch(ctx: int, llr_dtype: int, llr_dev, payload_dev, status_dev, stats_dev=None,
                     stream=None):
    """Launch the plan last prepared on ctx; torch tensors are checked against that plan."""
    _check_plan_buffers(_PLANS.get(ctx), llr_dtype, llr_dev, payload_dev, status_dev, stats_dev)
    _check(lib().scs_mixed_launch(ctx, int(llr_dtype), _addr(llr_dev), _addr(payload_dev),
                                  _addr(status_dev), _addr(stats_dev), _stream(stream)),
           "scs_mixed_launch")


def scs_ctx_set_waves_per_block(ctx: int, waves_per_block: int):
    _check(lib().scs_ctx_set_waves_per_block(ctx, int(waves_per_block)),
           "scs_ctx_set_waves_per_block")


def scs_ctx_set_grid_cus(ctx: int, cus: int):
    _check(lib().scs_ctx_set_grid_cus(ctx, int(cus)), "scs_ctx_set_grid_cus")


def scs_ctx_last_error(ctx: int) -> int:
    return int(lib().scs_ctx_last_error(ctx))


# -- handle wrappers -----------------------------------------------------------------

class PolarCode:
    """A constructed PC(N, K) (Bhattacharyya set at design_db), CRC bits inside K."""

    def __init__(self, N: int, K: int, crc_bits: int = 0, design_db: float = 2.0,
                 info_mask=None):
        """info_mask (N bytes, 1 = information position) replaces the construction: the code
        then has that information set (polar_construct_set) and K must be its size."""
        if info_mask is None:
            self.handle = polar_construct(N, K, crc_bits, design_db)
        else:
            m = np.asarray(info_mask, dtype=np.uint8)
            if m.size != N or int(m.sum()) != K:
                raise ValueError("info_mask must have N = %d entries and K = %d ones" % (N, K))
            self.handle = polar_construct_set(m, crc_bits)
        self.N, self.K, self.crc_bits, self.info_mask = polar_code_query(self.handle)
        self.design_db = design_db
        self.systematic = False

    def make_systematic(self) -> "PolarCode":
        """The systematic twin of this code (polar_code_systematic): a new PolarCode."""
        twin = PolarCode.__new__(PolarCode)
        twin.handle = polar_code_systematic(self.handle)
        twin.N, twin.K, twin.crc_bits, twin.info_mask = polar_code_query(twin.handle)
        twin.design_db = self.design_db
        twin.systematic = polar_code_is_systematic(twin.handle)
        return twin

    @classmethod
    def from_set(cls, info_mask, crc_bits: int = 0) -> "PolarCode":
        m = np.asarray(info_mask, dtype=np.uint8)
        return cls(int(m.size), int(m.sum()), crc_bits, float("nan"), info_mask=m)

    @property
    def payload_bits(self) -> int:
        return self.K - self.crc_bits

    @property
    def rate(self) -> float:
        return self.K / self.N

    def encode(self, payload: np.ndarray) -> np.ndarray:
        payload = np.ascontiguousarray(payload, dtype=np.uint8).reshape(-1, self.payload_bits)
        cw = np.zeros((payload.shape[0], self.N), np.uint8)
        polar_encode(self.handle, payload, cw)
        return cw

    def encode_device(self, payload_dev, codeword_dev, stream=None):
        """Encode frames x payload_bits uint8 payloads into frames x N uint8 codewords."""
        import torch

        n = payload_dev.shape[0]
        _device_buffer(payload_dev, "payload", (torch.uint8,), n * self.payload_bits, None)
        _device_buffer(codeword_dev, "codewords", (torch.uint8,), n * self.N,
                       payload_dev.device.index)
        polar_encode_device(self.handle, payload_dev, codeword_dev, n, stream)

    def close(self):
        if self.handle:
            polar_code_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ScsContext:
    def __init__(self, device: int = 0, waves_per_block: int = 0):
        self.handle = scs_ctx_create(device)
        self.device = device
        if waves_per_block:
            scs_ctx_set_waves_per_block(self.handle, waves_per_block)

    def configure(self, waves_per_block: int = 0):
        scs_ctx_set_waves_per_block(self.handle, waves_per_block)

    def set_grid_cus(self, cus: int = 0):
        """CUs' worth of workgroups of this context's persistent mixed launches (0: all)."""
        scs_ctx_set_grid_cus(self.handle, cus)

    def _frames(self, code: PolarCode, llr_dev, payload_dev, status_dev, stats_dev):
        """Check the buffers of one batch; returns (LLR dtype code, frames)."""
        import torch  # device buffers are torch tensors here

        if llr_dev.numel() % code.N:
            raise ValueError("LLRs hold %d values, not a multiple of N = %d" % (llr_dev.numel(),
                                                                               code.N))
        n = llr_dev.numel() // code.N
        _device_buffer(llr_dev, "llr", (torch.float32, torch.int8), n * code.N, self.device)
        if code.payload_bits > 0 or payload_dev is not None:
            _device_buffer(payload_dev, "payload", (torch.uint8,), n * code.payload_bits,
                           self.device)
        _device_buffer(status_dev, "status", (torch.uint8,), n, self.device)
        if stats_dev is not None:
            _device_buffer(stats_dev, "stats", (torch.int32, torch.uint32), n * len(STATS_FIELDS),
                           self.device)
        return (SCS_LLR_F32 if llr_dev.dtype == torch.float32 else SCS_LLR_I8), n

    def decode(self, code: PolarCode, D: int, L: int, llr_dev, payload_dev, status_dev,
               stats_dev=None, stream=None, fast: bool = False):
        """SCS decoding of llr_dev (frames x N); fast=True: FSSCS-RM (fsscs_decode_batch)."""
        dtype, n = self._frames(code, llr_dev, payload_dev, status_dev, stats_dev)
        fn = fsscs_decode_batch if fast else scs_decode_batch
        fn(self.handle, code.handle, D, L, dtype, llr_dev, n, payload_dev, status_dev, stats_dev,
           stream)

    def decode_list(self, code: PolarCode, L: int, llr_dev, payload_dev, status_dev,
                    stats_dev=None, stream=None):
        """CA-SCL decoding of llr_dev (frames x N) with a list of L paths."""
        dtype, n = self._frames(code, llr_dev, payload_dev, status_dev, stats_dev)
        scl_decode_batch(self.handle, code.handle, L, dtype, llr_dev, n, payload_dev, status_dev,
                         stats_dev, stream)

    def close(self):
        if self.handle:
            scs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
