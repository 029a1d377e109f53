"""Launch-shape autotuner for the decoders.

For one (code, D, L, LLR type) it times every launch shape the library offers --
wavefronts per workgroup (1, 2, 4) -- on a sample batch of noisy frames at a
representative Eb/N0, and keeps the fastest.  For a mixed batch (several codes, depths and
list sizes in one persistent launch) it times the same sizes on a sample of the caller's
own plan, keyed by the plan's set of configurations.  The list decoder packs 8 / L frames into a
wavefront at L <= 4 by itself and ignores D.  Results go to a JSON cache keyed by device
architecture, N, K, CRC bits, D, L and LLR type (default file: $POLARSCS_TUNE_CACHE or
~/.cache/polarscs/tune.json), and ``apply`` configures a decoder context from it.  Entries
shipped with the package (``tuned.json``, written by this module's command line on an
MI355X) answer when the user cache has none.  The decoded bits do not depend on the launch
shape; only the time does.

    python -m paper_1809_03606_amd.tune --N 1024 --K 512 --crc 16 --D 32 --L 8 --dtype f32
"""
from __future__ import annotations

import json
import os
import time

from . import binding, channel

CANDIDATES = [4, 2, 1]  # wavefronts per workgroup
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def cache_path() -> str:
    return os.environ.get("POLARSCS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "polarscs", "tune.json"))


def _arch(torch) -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def key(arch: str, code, D: int, L: int, dtype: str, decoder: str = "scs") -> str:
    if decoder == "scl":
        D = 0  # the list decoder has no stack
    k = "%s:N%d:K%d:crc%d:D%d:L%d:%s" % (arch, code.N, code.K, code.crc_bits, D, L, dtype)
    return k if decoder == "scs" else k + ":" + decoder


def candidates(decoder: str = "scs"):
    """Launch shapes (wavefronts per workgroup); the same for every decoder."""
    return list(CANDIDATES)


def _read(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def load(path: str | None = None) -> dict:
    """Entries of `path`, or of the user cache over the shipped entries."""
    if path:
        return _read(path)
    entries = _read(SHIPPED)
    entries.update(_read(cache_path()))
    return entries


def save(entries: dict, path: str | None = None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(entries, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(code, D: int, L: int, dtype: str = "f32", ebn0_db: float = 2.0, frames: int = 262144,
         reps: int = 2, seed: int = 7, path: str | None = None, verbose: bool = False,
         decoder: str = "scs") -> dict:
    """Time every launch shape on `frames` noisy frames (for the list decoder at L < 8,
    8 / L times as many: the same number of wavefronts); store and return the best."""
    import torch

    if decoder == "scl" and L < 8:
        frames *= 8 // L

    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    pay = channel.device_payload(torch, gen, frames, code.payload_bits, dev)
    cw = torch.empty((frames, code.N), dtype=torch.uint8, device=dev)
    code.encode_device(pay, cw)
    llr = channel.device_llr(torch, gen, cw, ebn0_db, code.rate, dtype)
    del cw
    torch.cuda.synchronize()  # the LLRs are written on the default stream, decoded on another
    out = torch.empty((frames, code.payload_bits), dtype=torch.uint8, device=dev)
    st = torch.empty((frames,), dtype=torch.uint8, device=dev)
    ctx = binding.ScsContext(0)
    stream = torch.cuda.Stream(device=dev)
    times = {}
    ref = None
    fast = decoder == "fsscs"
    for wpb in candidates(decoder):
        ctx.configure(wpb)
        ms = []
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            if decoder == "scl":
                ctx.decode_list(code, L, llr, out, st, None, stream)
            else:
                ctx.decode(code, D, L, llr, out, st, None, stream, fast=fast)
            b.record(stream)
            stream.synchronize()
            if r:
                ms.append(a.elapsed_time(b))
        if ref is None:
            ref = (out.clone(), st.clone())
        elif not (torch.equal(ref[0], out) and torch.equal(ref[1], st)):
            raise RuntimeError("launch shape wpb=%d changed the decoded bits" % wpb)
        times[str(wpb)] = min(ms)
        if verbose:
            print("tune %s wpb=%d: %.2f ms" % (key("", code, D, L, dtype, decoder), wpb, min(ms)))
    best = min(times, key=times.get)
    entry = {"waves_per_block": int(best), "ms": times[best],
             "candidates_ms": times, "frames": frames, "ebn0_db": ebn0_db,
             "tuned_at": time.strftime("%Y-%m-%dT%H:%M:%S")}
    entries = _read(path or cache_path())
    entries[key(_arch(torch), code, D, L, dtype, decoder)] = entry
    save(entries, path)
    ctx.close()
    return entry


def apply(ctx, code, D: int, L: int, dtype: str = "f32", path: str | None = None,
          decoder: str = "scs") -> dict | None:
    """Configure `ctx` with the cached best launch shape, if any; returns the entry."""
    import torch

    entry = load(path).get(key(_arch(torch), code, D, L, dtype, decoder))
    if entry:
        ctx.configure(entry["waves_per_block"])
    return entry


def mixed_key(arch: str, codes, frames, dtype: str = "f32") -> str:
    """Cache key of a mixed plan: the sorted set of (N, K, CRC, D, L) configurations it
    holds (not the frame count or order)."""
    import hashlib

    import numpy as np

    confs = sorted({(codes[int(c)].N, codes[int(c)].K, codes[int(c)].crc_bits, int(d), int(l))
                    for c, d, l in np.unique(np.stack([frames["code"], frames["D"],
                                                       frames["L"]], 1), axis=0)})
    h = hashlib.sha1(repr(confs).encode()).hexdigest()[:12]
    return "%s:mixed:%dconf:%s:%s" % (arch, len(confs), h, dtype)


def tune_mixed(ctx, codes, frames, llr, payload, status, stream, dtype: str = "f32",
               sample: int = 262144, reps: int = 2, path: str | None = None,
               verbose: bool = False) -> dict:
    """Time the persistent mixed launch (scs_mixed_prepare + scs_mixed_launch) at every
    workgroup size on the first `sample` descriptors of the caller's plan, over the caller's
    device buffers (LLRs, payload, status sized for the whole plan); check that every size
    gives the same bytes; store the fastest under mixed_key and configure ctx with it."""
    import numpy as np
    import torch

    sub = np.ascontiguousarray(frames[:sample])
    handles = [c.handle for c in codes]
    dt = binding.SCS_LLR_F32 if dtype == "f32" else binding.SCS_LLR_I8
    binding.scs_mixed_prepare(ctx.handle, handles, sub, stream)
    stream.synchronize()
    idx = torch.from_numpy(np.arange(len(sub))).to(status.device)
    times, ref = {}, None
    for wpb in CANDIDATES:
        ctx.configure(wpb)
        ms = []
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            binding.scs_mixed_launch(ctx.handle, dt, llr, payload, status, None, stream)
            b.record(stream)
            stream.synchronize()
            if r:
                ms.append(a.elapsed_time(b))
        got = (payload.clone(), status[idx].clone())
        if ref is None:
            ref = got
        elif not (torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])):
            raise RuntimeError("mixed launch at wpb=%d changed the decoded bits" % wpb)
        times[str(wpb)] = min(ms)
        if verbose:
            print("tune mixed wpb=%d: %.2f ms" % (wpb, min(ms)))
    best = min(times, key=times.get)
    entry = {"waves_per_block": int(best), "ms": times[best], "candidates_ms": times,
             "frames": int(len(sub)), "tuned_at": time.strftime("%Y-%m-%dT%H:%M:%S")}
    entries = _read(path or cache_path())
    entries[mixed_key(_arch(torch), codes, frames, dtype)] = entry
    save(entries, path)
    ctx.configure(int(best))
    binding.scs_mixed_prepare(ctx.handle, handles, frames, stream)  # the whole plan again
    stream.synchronize()
    return entry


def apply_mixed(ctx, codes, frames, dtype: str = "f32", path: str | None = None) -> dict | None:
    """Configure ctx with the cached workgroup size of this mixed plan, if any."""
    import torch

    entry = load(path).get(mixed_key(_arch(torch), codes, frames, dtype))
    if entry:
        ctx.configure(entry["waves_per_block"])
    return entry


def main(argv=None):
    import argparse

    from . import binding

    ap = argparse.ArgumentParser(description="time the decoder's launch shapes, keep the best")
    ap.add_argument("--N", type=int, required=True)
    ap.add_argument("--K", type=int, required=True)
    ap.add_argument("--crc", type=int, default=16)
    ap.add_argument("--D", type=int, default=32, help="stack depth (not used by the list decoder)")
    ap.add_argument("--L", type=int, default=8)
    ap.add_argument("--dtype", choices=("f32", "i8"), default="f32")
    ap.add_argument("--ebn0", type=float, default=2.0)
    ap.add_argument("--frames", type=int, default=262144)
    ap.add_argument("--decoder", choices=("scs", "fsscs", "scl"), default="scs")
    ap.add_argument("--out", default=None, help="cache file (default: the user cache)")
    a = ap.parse_args(argv)
    code = binding.PolarCode(a.N, a.K, a.crc, 2.0)
    entry = tune(code, a.D, a.L, a.dtype, ebn0_db=a.ebn0, frames=a.frames, path=a.out,
                 verbose=True, decoder=a.decoder)
    print(json.dumps(entry))


if __name__ == "__main__":
    main()
