"""Seeded synthetic inputs: random payloads, BPSK over AWGN, int8 quantisation.

This module is the one input generator that both the HIP path and the CPU oracle
consume.  It holds none of the decoder's arithmetic: no construction, no encoding, no
tree, no CRC.  Codewords are produced elsewhere (by the library's encoder for the
product path, by the oracle's encoder in tests) and handed in.

Channel (the paper fixes none, it only plots against Eb/N0): BPSK maps bit c to
x = 1 - 2c, AWGN adds sigma * n with sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)) and R = K / N
(CRC bits counted in K), and the channel LLR is 2 y / sigma^2.  All of it is computed in
binary64 and rounded once to binary32.  The fixed-point variant quantises y itself:
q = clamp(rint(T * y), -127, 127); min-sum decisions are invariant to a common positive
scale of the LLRs, so q is an integer approximation of LLR * T sigma^2 / 2.

Random numbers come from numpy's Philox4x32-10 counter-based generator (host) keyed by
(seed, stream, chunk, kind), so any frame range can be regenerated on its own; the
device helpers use torch's CUDA generator for large batches and are not bit-identical
to the host ones.
"""
from __future__ import annotations

import math

import numpy as np

CHUNK = 1 << 16  # frames per independently keyed block of the host generator


def sigma2(ebn0_db: float, rate: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def _gen(seed: int, stream: int, chunk: int, kind: int) -> np.random.Generator:
    key = [int(seed) & 0xFFFFFFFFFFFFFFFF,
           ((int(stream) & 0xFFFFFFFF) << 32) | ((int(chunk) & 0x7FFFFFFF) << 1) | (kind & 1)]
    return np.random.Generator(np.random.Philox(key=key))


def _chunked(seed, stream, f0, B, kind, draw):
    out = []
    f = f0
    end = f0 + B
    while f < end:
        c = f // CHUNK
        lo = f - c * CHUNK
        hi = min(CHUNK, end - c * CHUNK)
        block = draw(_gen(seed, stream, c, kind), hi)  # always draw from the chunk start
        out.append(block[lo:hi])
        f = c * CHUNK + hi
    return np.concatenate(out, axis=0) if out else draw(_gen(seed, stream, 0, kind), 0)


def payload_bits(seed: int, stream: int, f0: int, B: int, k: int) -> np.ndarray:
    """Uniform random payload bits for frames [f0, f0 + B): uint8[B][k]."""
    return _chunked(seed, stream, f0, B, 0,
                    lambda g, n: g.integers(0, 2, size=(n, k), dtype=np.uint8))


def noise(seed: int, stream: int, f0: int, B: int, N: int) -> np.ndarray:
    """Standard normal samples for frames [f0, f0 + B): float64[B][N]."""
    return _chunked(seed, stream, f0, B, 1, lambda g, n: g.standard_normal((n, N)))


def bpsk_awgn_llr(codeword: np.ndarray, n: np.ndarray, ebn0_db: float, rate: float) -> np.ndarray:
    """float32 channel LLRs 2y/sigma^2 for y = (1 - 2c) + sigma * n."""
    s2 = sigma2(ebn0_db, rate)
    s = math.sqrt(s2)
    x = 1.0 - 2.0 * codeword.astype(np.float64)
    y = x + s * n
    return ((2.0 * y) / s2).astype(np.float32)


def bpsk_awgn_i8(codeword: np.ndarray, n: np.ndarray, ebn0_db: float, rate: float,
                 scale: float = 8.0) -> np.ndarray:
    """int8 channel values clamp(rint(scale * y), -127, 127)."""
    s = math.sqrt(sigma2(ebn0_db, rate))
    y = (1.0 - 2.0 * codeword.astype(np.float64)) + s * n
    return np.clip(np.rint(scale * y), -127, 127).astype(np.int8)


def noiseless_llr(codeword: np.ndarray, magnitude: float = 4.0) -> np.ndarray:
    """Channel with no noise: LLR = +magnitude for bit 0, -magnitude for bit 1."""
    return (magnitude * (1.0 - 2.0 * codeword.astype(np.float64))).astype(np.float32)


# -- device helpers (large batches; torch is used only as an RNG and elementwise map) --

def device_payload(torch, gen, B: int, k: int, device):
    return torch.randint(0, 2, (B, k), generator=gen, dtype=torch.uint8, device=device)


def device_llr(torch, gen, codeword, ebn0_db: float, rate: float, dtype: str = "f32",
               scale: float = 8.0):
    """LLRs for a device codeword tensor uint8[B][N], same formulas as the host helpers."""
    B, N = codeword.shape
    n = torch.randn((B, N), generator=gen, dtype=torch.float64, device=codeword.device)
    s2 = sigma2(ebn0_db, rate)
    x = 1.0 - 2.0 * codeword.to(torch.float64)
    y = x + math.sqrt(s2) * n
    del n, x
    if dtype == "f32":
        return ((2.0 * y) / s2).to(torch.float32)
    return torch.clamp(torch.round(scale * y), -127, 127).to(torch.int8)


# -- mixed batches -------------------------------------------------------------------

MIXED_N = (128, 256, 512, 1024, 2048)
MIXED_RATES = ((1, 4), (1, 3), (1, 2), (2, 3), (5, 6))
MIXED_D = (8, 32, 64)


def mixed_codes():
    """The 25 (N, K) pairs of the mixed workload, K = floor(N p / q + 1/2) (CRC inside K)."""
    return [(n, (n * p + q // 2) // q) for n in MIXED_N for (p, q) in MIXED_RATES]


def mixed_draw(seed: int, B: int):
    """Per-frame code index (into mixed_codes()), stack depth and Eb/N0 ~ U[1.5, 3.5]."""
    g = np.random.Generator(np.random.Philox(key=[int(seed), 0x6D6978]))
    code = g.integers(0, len(MIXED_N) * len(MIXED_RATES), size=B)
    D = np.asarray(MIXED_D)[g.integers(0, len(MIXED_D), size=B)]
    ebn0 = g.uniform(1.5, 3.5, size=B)
    return code.astype(np.int32), D.astype(np.int32), ebn0


def device_llr_per_frame(torch, gen, codeword, ebn0_db, rate: float):
    """As device_llr (binary32) with one Eb/N0 per frame (a float64 tensor of length B)."""
    B, N = codeword.shape
    n = torch.randn((B, N), generator=gen, dtype=torch.float64, device=codeword.device)
    s2 = 1.0 / (2.0 * rate * torch.pow(10.0, ebn0_db / 10.0))
    x = 1.0 - 2.0 * codeword.to(torch.float64)
    y = x + torch.sqrt(s2)[:, None] * n
    del n, x
    return ((2.0 * y) / s2[:, None]).to(torch.float32)


def device_noise(torch, gen, B: int, N: int, device):
    return torch.randn((B, N), generator=gen, dtype=torch.float64, device=device)


def device_llr_from_noise(torch, codeword, n, ebn0_db: float, rate: float, dtype: str = "f32",
                          scale: float = 8.0):
    """Same arithmetic as bpsk_awgn_llr / bpsk_awgn_i8 on device tensors (binary64, rounded
    once), so that host and device give identical values for identical noise."""
    s2 = sigma2(ebn0_db, rate)
    x = 1.0 - 2.0 * codeword.to(torch.float64)
    y = x + math.sqrt(s2) * n
    if dtype == "f32":
        return ((2.0 * y) / s2).to(torch.float32)
    return torch.clamp(torch.round(scale * y), -127, 127).to(torch.int8)


def _per_frame_sigma(ebn0_db, rate: float):
    """sigma and sigma^2 of every frame (binary64, host), for per-frame Eb/N0."""
    s2 = 1.0 / (2.0 * rate * np.power(10.0, np.asarray(ebn0_db, dtype=np.float64) / 10.0))
    return np.sqrt(s2), s2


def bpsk_awgn_llr_per_frame(codeword: np.ndarray, n: np.ndarray, ebn0_db, rate: float) -> np.ndarray:
    """bpsk_awgn_llr with one Eb/N0 per frame (row)."""
    s, s2 = _per_frame_sigma(ebn0_db, rate)
    x = 1.0 - 2.0 * codeword.astype(np.float64)
    y = x + s[:, None] * n
    return ((2.0 * y) / s2[:, None]).astype(np.float32)


def device_llr_from_noise_per_frame(torch, codeword, n, ebn0_db, rate: float):
    """bpsk_awgn_llr_per_frame on device tensors, with sigma and sigma^2 computed on the host
    (so the two agree bit for bit: the device does only IEEE multiply, add and divide)."""
    s, s2 = _per_frame_sigma(ebn0_db, rate)
    dev = codeword.device
    s = torch.from_numpy(s).to(dev)
    s2 = torch.from_numpy(s2).to(dev)
    x = 1.0 - 2.0 * codeword.to(torch.float64)
    y = x + s[:, None] * n
    return ((2.0 * y) / s2[:, None]).to(torch.float32)
