#!/usr/bin/env python3
"""Throughput of batched SCS decoding on one MI355X.

Workload: PC(1024, 512) with CRC-16 (496 payload bits), Bhattacharyya set at 2 dB, stack
depth D = 32, list parameter L = 8, BPSK over AWGN at Eb/N0 = 1.0, 1.5, 2.0, 2.5, 3.0 dB,
1,000,000 seeded frames per point held in HBM, one decoder launch per point.  One step is
the whole sweep (5 launches, 5,000,000 frames).  ``value`` is payload Mbit/s over the
timed steps.

Prints one JSON line (rank 0).  Extra objects: ``roofline`` for the decoder kernel (ALU
bound, algorithmic lane-operations from the kernel's own per-frame work counters, peak
from 256 CUs x 64 lanes x 2.4 GHz) and ``cpu_baseline`` (the CPU oracle on a bounded
sample of the same frames, all host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, K, CRC, D, L = 1024, 512, 16, 32, 8
POINTS = (1.0, 1.5, 2.0, 2.5, 3.0)
SEED = 2
PEAK_LANE_OPS = 256 * 64 * 2.4e9  # 32-bit VALU lane-operations per second
# Algorithmic lane-operations (see the design notes): 3 per f/g element of the SC
# schedule, and per path extension 4 D for the best/worst-path searches over the stack
# plus 8 for the leaf decision, metric, CRC register and counters.
OPS_PER_ELEM = 3
OPS_PER_ITER_FIXED = 8


def ops_per_iteration(d: int) -> int:
    return 4 * d + OPS_PER_ITER_FIXED


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=1_000_000, help="frames per Eb/N0 point")
    ap.add_argument("--points", type=str, default=",".join(str(p) for p in POINTS))
    ap.add_argument("--dtype", choices=("f32", "i8"), default="f32")
    ap.add_argument("--cpu-sample", type=int, default=2000,
                    help="frames per point decoded by the CPU oracle for cpu_baseline (0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0: all usable host cores (max 16)")
    ap.add_argument("--lanes", type=int, default=0, choices=(0, 16, 32, 64),
                    help="lanes per frame (0: the library's choice)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter calibration)")
    return ap.parse_args()


KERNEL_SOURCES = ("paper_1809_03606_amd/csrc/scs_decode.hip", "paper_1809_03606_amd/csrc/scs_device.h",
                  "paper_1809_03606_amd/csrc/scs_rows.hip")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "decoder_traffic_n1024.json")


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(frames_per_launch: int):
    """HBM bytes per launch from the recorded FETCH_SIZE / WRITE_SIZE counters, or None when
    the record is missing or was taken on different kernel sources."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec["hbm_bytes_per_frame"] * frames_per_launch


def calibrate_copy(nbytes: int):
    import torch

    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}))


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print("bench.py: this build decodes on one GPU; --gpus %d is not supported (frames are "
              "independent, see the design notes for how the batch would shard)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1809_03606_amd import binding, channel

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    points = [float(x) for x in args.points.split(",")]
    B = args.frames
    kp = K - CRC

    code = binding.PolarCode(N, K, CRC, 2.0)
    ctx = binding.ScsContext(0, args.lanes)
    stream = torch.cuda.Stream(device=dev)
    llr_dtype = binding.SCS_LLR_F32 if args.dtype == "f32" else binding.SCS_LLR_I8

    # -- inputs: generated on the device, resident in HBM before timing --------------
    t0 = time.time()
    data = []
    with torch.cuda.stream(stream):
        for pi, eb in enumerate(points):
            gen = torch.Generator(device=dev)
            gen.manual_seed(SEED * 1000 + pi)
            pay = channel.device_payload(torch, gen, B, kp, dev)
            llr = torch.empty((B, N), dtype=torch.float32 if args.dtype == "f32" else torch.int8,
                              device=dev)
            chunk = 1 << 17
            for lo in range(0, B, chunk):
                hi = min(B, lo + chunk)
                cw = torch.empty((hi - lo, N), dtype=torch.uint8, device=dev)
                code.encode_device(pay[lo:hi], cw, stream)
                llr[lo:hi] = channel.device_llr(torch, gen, cw, eb, K / N, args.dtype)
                del cw
            data.append((eb, pay, llr))
            stream.synchronize()
            log("inputs ready: Eb/N0 %.1f dB, %d frames" % (eb, B))
    stream.synchronize()
    gen_s = time.time() - t0

    out_pay = torch.empty((B, kp), dtype=torch.uint8, device=dev)
    out_st = torch.empty((B,), dtype=torch.uint8, device=dev)
    stats = torch.zeros((B, 8), dtype=torch.int32, device=dev)

    def launch(llr, with_stats=False):
        binding.scs_decode_batch(ctx.handle, code.handle, D, L, llr_dtype, llr, B, out_pay,
                                 out_st, stats if with_stats else None, stream)

    # -- per-point work counters and FER (untimed) ------------------------------------
    per_point = {}
    work_ops = {}
    for eb, pay, llr in data:
        launch(llr, with_stats=True)
        stream.synchronize()
        s = stats.cpu().numpy().view(np.uint32).astype(np.int64)
        it, sc = s[:, 0].sum(), s[:, 3].sum()
        work_ops[eb] = OPS_PER_ELEM * sc + ops_per_iteration(D) * it
        fer = float((out_pay != pay).any(dim=1).float().mean().item())
        log("work counters: Eb/N0 %.1f dB, FER %.2e, %.0f iterations/frame" % (eb, fer, it / B))
        per_point[eb] = {"fer": fer, "mean_iterations": float(it / B),
                         "mean_switches": float(s[:, 1].mean()),
                         "mean_fg_elems": float(s[:, 4].mean()),
                         "status_counts": {str(k): int(v) for k, v in
                                           zip(*np.unique(out_st.cpu().numpy(), return_counts=True))}}

    # -- timed region --------------------------------------------------------------
    for _ in range(args.warmup):
        for eb, pay, llr in data:
            launch(llr)
    stream.synchronize()
    torch.cuda.synchronize()

    ev = []
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t_start.record(stream)
    for step in range(args.steps):
        for eb, pay, llr in data:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            launch(llr)
            b.record(stream)
            ev.append((eb, a, b))
    t_end.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    log("timed region done: %d steps in %.2f s" % (args.steps, wall))
    total_ms = t_start.elapsed_time(t_end)
    err = binding.scs_ctx_last_error(ctx.handle)
    if err:
        raise RuntimeError("decoder reported %s" % binding.strerror(err))

    launch_ms = {eb: [] for eb in points}
    for eb, a, b in ev:
        launch_ms[eb].append(a.elapsed_time(b))
    all_ms = np.array([m for v in launch_ms.values() for m in v])
    frames_timed = args.steps * len(points) * B
    value = frames_timed * kp / (total_ms * 1e-3) / 1e6
    for eb in points:
        ms = float(np.mean(launch_ms[eb]))
        per_point[eb].update({"launch_ms": ms, "payload_mbps": B * kp / (ms * 1e-3) / 1e6})

    # roofline of the decoder kernel: algorithmic lane-ops per launch / mean launch time
    ops_per_launch = float(np.mean([work_ops[eb] for eb in points]))
    mean_launch_s = float(all_ms.mean()) * 1e-3
    achieved = ops_per_launch / mean_launch_s / 1e12
    peak = PEAK_LANE_OPS / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tlane-op/s",
                "frac": achieved / peak, "traffic": measured_traffic(B),
                "kernel": "scs_uniform_kernel<10,f32>" if args.dtype == "f32" else
                          "scs_uniform_kernel<10,i8>",
                "mean_launch_ms": float(all_ms.mean()), "ops_per_launch": ops_per_launch}

    # -- CPU oracle on a bounded sample of the same frames -----------------------------
    cpu = None
    if args.cpu_sample > 0:
        import oracle

        thr = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
        info = code.info_mask
        mode = oracle.F32 if args.dtype == "f32" else oracle.FIX
        n = min(args.cpu_sample, B)
        t = 0.0
        match = True
        for eb, pay, llr in data:
            x = llr[:n].contiguous()
            c0 = time.perf_counter()
            rp, rs, _ = oracle.scs_decode_batch(mode, info, CRC, D, L, x.cpu().numpy(), threads=thr)
            t += time.perf_counter() - c0
            # the same sample on the GPU must give the same bits
            binding.scs_decode_batch(ctx.handle, code.handle, D, L, llr_dtype, x, n, out_pay,
                                     out_st, None, stream)
            stream.synchronize()
            match &= bool(np.array_equal(out_pay[:n].cpu().numpy(), rp) and
                          np.array_equal(out_st[:n].cpu().numpy(), rs))
            log("cpu oracle sample: Eb/N0 %.1f dB done (%.1f s so far)" % (eb, t))
        cpu = {"value": len(points) * n * kp / t / 1e6, "unit": "Mbit/s", "cores": thr,
               "kind": "oracle",
               "sample": "first %d frames of each of the %d Eb/N0 points (%d frames), %d threads"
                         % (n, len(points), n * len(points), thr),
               "seconds": t, "gpu_matches_oracle_on_sample": match}

    line = {
        "metric": "info Mbit/s decoded (N=1024,K=512,D=32) at oracle-matched FER; p99 latency",
        "value": value, "unit": "Mbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic: seeded BPSK/AWGN frames generated on the device",
        "config": {"workload": "SCS sweep PC(1024,512)+CRC16 D=32 L=8 Eb/N0 1.0-3.0 dB",
                   "N": N, "K": K, "crc_bits": CRC, "D": D, "L": L,
                   "ebn0_db": points, "frames_per_point": B, "global_batch": B * len(points),
                   "launches_per_step": len(points), "parallelism": "single GPU"},
        "latency": {"launch_ms_p50": float(np.percentile(all_ms, 50)),
                    "launch_ms_p99": float(np.percentile(all_ms, 99))},
        "per_point": {str(k): v for k, v in per_point.items()},
        "wall_s": wall, "input_generation_s": gen_s,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
