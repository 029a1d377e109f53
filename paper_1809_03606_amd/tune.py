"""Launch-shape autotuner for the SCS decoder.

For one (code, D, L, LLR type) it times every launch shape the library offers -- lanes per
frame (64: one frame per wavefront; 32 / 16: two / four frames per wavefront) times
wavefronts per workgroup (1, 2, 4) -- on a sample batch of noisy frames at a
representative Eb/N0, and keeps the fastest.  Results go to a JSON cache keyed by device
architecture, N, K, CRC bits, D, L and LLR type (default file: $POLARSCS_TUNE_CACHE or
~/.cache/polarscs/tune.json), and ``apply`` configures a decoder context from it.  The
decoded bits do not depend on the launch shape; only the time does.
"""
from __future__ import annotations

import json
import os
import time

from . import binding, channel

CANDIDATES = [(lanes, wpb) for lanes in (64, 32, 16) for wpb in (4, 2, 1)]


def cache_path() -> str:
    return os.environ.get("POLARSCS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "polarscs", "tune.json"))


def _arch(torch) -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def key(arch: str, code, D: int, L: int, dtype: str) -> str:
    return "%s:N%d:K%d:crc%d:D%d:L%d:%s" % (arch, code.N, code.K, code.crc_bits, D, L, dtype)


def load(path: str | None = None) -> dict:
    try:
        with open(path or cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save(entries: dict, path: str | None = None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(entries, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(code, D: int, L: int, dtype: str = "f32", ebn0_db: float = 2.0, frames: int = 65536,
         reps: int = 2, seed: int = 7, path: str | None = None, verbose: bool = False) -> dict:
    """Time every launch shape on `frames` noisy frames; store and return the best."""
    import torch

    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    pay = channel.device_payload(torch, gen, frames, code.payload_bits, dev)
    cw = torch.empty((frames, code.N), dtype=torch.uint8, device=dev)
    code.encode_device(pay, cw)
    llr = channel.device_llr(torch, gen, cw, ebn0_db, code.rate, dtype)
    del cw
    out = torch.empty((frames, code.payload_bits), dtype=torch.uint8, device=dev)
    st = torch.empty((frames,), dtype=torch.uint8, device=dev)
    ctx = binding.ScsContext(0)
    stream = torch.cuda.Stream(device=dev)
    times = {}
    ref = None
    for lanes, wpb in CANDIDATES:
        ctx.configure(lanes, wpb)
        ms = []
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.decode(code, D, L, llr, out, st, None, stream)
            b.record(stream)
            stream.synchronize()
            if r:
                ms.append(a.elapsed_time(b))
        if ref is None:
            ref = (out.clone(), st.clone())
        elif not (torch.equal(ref[0], out) and torch.equal(ref[1], st)):
            raise RuntimeError("launch shape %s changed the decoded bits" % ((lanes, wpb),))
        times["%d/%d" % (lanes, wpb)] = min(ms)
        if verbose:
            print("tune %s lanes=%d wpb=%d: %.2f ms" % (key("", code, D, L, dtype), lanes, wpb, min(ms)))
    best = min(times, key=times.get)
    lanes, wpb = (int(x) for x in best.split("/"))
    entry = {"lanes_per_frame": lanes, "waves_per_block": wpb, "ms": times[best],
             "candidates_ms": times, "frames": frames, "ebn0_db": ebn0_db,
             "tuned_at": time.strftime("%Y-%m-%dT%H:%M:%S")}
    entries = load(path)
    entries[key(_arch(torch), code, D, L, dtype)] = entry
    save(entries, path)
    ctx.close()
    return entry


def apply(ctx, code, D: int, L: int, dtype: str = "f32", path: str | None = None) -> dict | None:
    """Configure `ctx` with the cached best launch shape, if any; returns the entry."""
    import torch

    entry = load(path).get(key(_arch(torch), code, D, L, dtype))
    if entry:
        ctx.configure(entry["lanes_per_frame"], entry["waves_per_block"])
    return entry
