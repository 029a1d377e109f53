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
HEADLINE_DL = (D, L)


def sweep_config(d, l):
    """Another stack depth / L for the sweep workload (the other workloads keep theirs)."""
    global D, L
    if not (1 <= d <= 256 and 1 <= l <= 255):
        raise SystemExit("bench.py: D must be in [1, 256] and L in [1, 255]")
    D, L = d, l
POINTS = (1.0, 1.5, 2.0, 2.5, 3.0)
SEED = 2
PEAK_LANE_OPS = 256 * 64 * 2.4e9  # 32-bit VALU lane-operations per second

# The paper's own throughput at Eb/N0 = POINTS (Section 5, throughput figure), Mbit/s of
# information bits per thread of a six-thread AMD Ryzen 5 1600 at 3.2 GHz, for PC(1024,512)
# with the 5G information set, CRC-24C, L = 8 and D = 8192: context only (another machine,
# code set, CRC and stack depth).
PAPER_TP_MBPS = {
    "scs": ("SCS-RM", (0.0346253, 0.0518958, 0.0721866, 0.110722, 0.232370)),
    "fsscs": ("FSSCS-RM", (0.232408, 0.342818, 0.448689, 0.619550, 0.925226)),
    "scl": ("SCL", (0.290247, 0.280185, 0.290871, 0.309693, 0.314545)),
}
# Algorithmic lane-operations, the cost model the measurement plan fixes: f = 4 and g = 2
# operations per value (3 on average over the SC schedule, which evaluates as many f as g
# values), and per path extension 2 for the hard decision and the path metric and 8 for the
# stack (6 DPP steps and 2 ballots of one best-path search).  Earlier versions charged the
# stack 4 D per extension (both searches over every slot), which overstated the work.
OPS_PER_ELEM = 3
OPS_PER_ITER_FIXED = 10


def ops_per_iteration(d: int) -> int:
    return OPS_PER_ITER_FIXED


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
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="frames per point decoded by the CPU oracle for cpu_baseline (0: skip; "
                         "default 40000, 8000 for the list decoder, whose oracle is slower)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0: all usable host cores (max 16)")
    ap.add_argument("--wpb", type=int, default=0, choices=(0, 1, 2, 4),
                    help="wavefronts per workgroup (0: the autotuner's choice)")
    ap.add_argument("--decoder", choices=("scs", "fsscs", "fssc", "scl"), default="scs",
                    help="scs: successive-cancellation stack decoding (the headline); fsscs: "
                         "fast simplified stack decoding (FSSCS-RM); fssc: fast simplified SC "
                         "(the FSSCS-RM kernel with D = 1, L = 1); scl: CA-SCL with a list "
                         "of L paths; all on the same frames")
    ap.add_argument("--D", type=int, default=D,
                    help="stack depth of the sweep (1..256; the headline is D = 32)")
    ap.add_argument("--L", type=int, default=L,
                    help="L of the sweep: the stack decoders' path-length counter (1..255) or "
                         "the list size of CA-SCL (1, 2, 4, 8); the headline is L = 8")
    ap.add_argument("--tune", choices=("auto", "force", "off"), default="auto",
                    help="launch-shape autotuner: use the cached choice or tune once (auto), "
                         "always re-tune (force), or use the library's defaults (off)")
    ap.add_argument("--workload", choices=("sweep", "mixed", "serve", "fixed", "depth"),
                    default="sweep",
                    help="sweep: PC(1024,512) headline; mixed: 25 codes / 3 depths in one launch; "
                         "serve: Poisson requests through the continuous-batching server")
    ap.add_argument("--latency-requests", type=int, default=300,
                    help="closed-loop requests timed for the latency percentiles of the sweep")
    ap.add_argument("--e2e-reps", type=int, default=None,
                    help="repetitions of the end-to-end run from pinned host memory (0: off; "
                         "default 3, or 0 with --latency-requests 0, as the profile records run)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load as a fraction of the mixed batch's sustained frame rate "
                         "(measured in the same run)")
    ap.add_argument("--serve-rate-frames", type=int, default=500_000,
                    help="frames of the i.i.d. mixed batch that measures that rate")
    ap.add_argument("--serve-pool", type=int, default=4096,
                    help="distinct requests generated for the serving run (replayed)")
    ap.add_argument("--mixed-frames", type=int, default=2_000_000)
    ap.add_argument("--traffic-record", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the HBM traffic record from four rocprofv3 --pmc output folders "
                         "(decoder FETCH_SIZE, decoder WRITE_SIZE, 1 GiB copy FETCH_SIZE and "
                         "WRITE_SIZE) and exit; runs on the CPU")
    ap.add_argument("--counters-record", nargs=2, metavar=("SQ_DIR", "BENCH_JSON"),
                    help="write the SCS instruction-count record from a rocprofv3 --pmc SQ_* folder "
                         "and that run's JSON line, and exit; runs on the CPU")
    ap.add_argument("--trace-summary", nargs=3, metavar=("TRACE_DIR", "BENCH_JSON", "OUT_MD"),
                    help="summarise a rocprofv3 --kernel-trace --stats folder of a bench run "
                         "into markdown and exit; runs on the CPU")
    ap.add_argument("--util-record", nargs=4, metavar=("LDS_DIR", "BUSY_DIR", "BENCH_JSON", "PEAK_JSON"),
                    help="write the LDS and ALU utilisation record from two rocprofv3 --pmc "
                         "folders (LDS bandwidth counters; busy and bank-conflict metrics), "
                         "that run's JSON line and a --lds-peak JSON line, and exit; runs on "
                         "the CPU")
    ap.add_argument("--lds-peak", action="store_true",
                    help="only measure the chip's LDS read bandwidth (project microbenchmark)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter calibration)")
    a = ap.parse_args()
    if a.cpu_sample is None:
        a.cpu_sample = 8000 if a.decoder == "scl" else 40000
    return a


KERNEL_SOURCES = ("paper_1809_03606_amd/csrc/scs_decode.hip", "paper_1809_03606_amd/csrc/scs_device.h",
                  "paper_1809_03606_amd/csrc/scs_tree.h", "paper_1809_03606_amd/csrc/scs_stack.h",
                  "paper_1809_03606_amd/build.py")  # the compiler flags shape the kernel too
# the other decoders' sources (their kernels share the device headers and the flags)
_SHARED_SOURCES = ("paper_1809_03606_amd/csrc/scs_device.h", "paper_1809_03606_amd/csrc/scs_tree.h",
                   "paper_1809_03606_amd/build.py")
OTHER_SOURCES = {
    "fsscs": ("paper_1809_03606_amd/csrc/fsscs_decode.hip",
              "paper_1809_03606_amd/csrc/scs_stack.h") + _SHARED_SOURCES,
    "scl": ("paper_1809_03606_amd/csrc/scl_decode.hip",) + _SHARED_SOURCES,
}
DECODER_KERNELS = {"scs": "scs_uniform_kernel", "fsscs": "fsscs_uniform_kernel",
                   "scl": "scl_uniform_kernel"}
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "decoder_traffic_n1024.json")
COUNTERS_RECORD = os.path.join(ROOT, "profiles", "decoder_counters_n1024.json")
UTIL_RECORD = os.path.join(ROOT, "profiles", "decoder_utilization_n1024.json")
# LDS: 128 bytes per clock per CU (the data sheet's figure), 256 CUs at 2.4 GHz
LDS_PEAK_BYTES_PER_S = 128 * 256 * 2.4e9
CU_CYCLES_PER_S = 256 * 2.4e9  # MI355X: 256 CUs at 2.4 GHz


def kernel_source_hash(decoder: str = "scs") -> str:
    """Hash of a decoder's sources with comments and blank lines removed, so that a record
    of counters stays valid through comment edits and only a change of code voids it."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in (KERNEL_SOURCES if decoder == "scs" else OTHER_SOURCES[decoder]):
        with open(os.path.join(ROOT, f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def traffic_record_path(decoder: str = "scs") -> str:
    if decoder == "scs":
        return TRAFFIC_RECORD
    return os.path.join(ROOT, "profiles", "%s_traffic_n1024.json" % decoder)


def measured_traffic(frames_per_launch: int, decoder: str = "scs"):
    """HBM bytes per launch from the recorded FETCH_SIZE / WRITE_SIZE counters, or None when
    the record is missing or was taken on different kernel sources."""
    try:
        with open(traffic_record_path(decoder)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash(decoder):
        return None
    return rec["hbm_bytes_per_frame"] * frames_per_launch


def issue_bound(per_point, frames):
    """The SCS kernel against its binding resource, scalar instruction issue (one per CU per
    cycle): recorded scalar instructions per path extension (SQ_INSTS_SALU of the 2 dB point)
    over the CU-cycles per extension of this run at 2 dB.  None without a record taken on the
    current kernel sources or without a 2 dB point."""
    try:
        with open(COUNTERS_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash() or 2.0 not in per_point:
        return None
    p = per_point[2.0]
    if not frames or not p.get("mean_iterations"):
        return None
    cycles = p["launch_ms"] * 1e-3 * CU_CYCLES_PER_S / (frames * p["mean_iterations"])
    salu = rec["per_extension"]["SQ_INSTS_SALU"]
    return {"bound": "scalar issue (1 instruction per CU per cycle)",
            "scalar_insts_per_extension": salu,
            "vector_insts_per_extension": rec["per_extension"]["SQ_INSTS_VALU"],
            "cu_cycles_per_extension": cycles, "frac": salu / cycles, "at_ebn0_db": 2.0}


def lds_peak():
    """The LDS read rate of the whole chip with conflict-free 16-byte and 4-byte reads per
    lane (libldspeak.so, a microbenchmark built beside the decoder library)."""
    import ctypes

    from paper_1809_03606_amd import build

    if not os.path.exists(build.LDS_PEAK_LIB):
        raise SystemExit("bench.py: %s is not built (python -m paper_1809_03606_amd.build)"
                         % build.LDS_PEAK_LIB)
    lib = ctypes.CDLL(build.LDS_PEAK_LIB)
    lib.lds_peak_measure.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    res = {}
    for width in (16, 4):
        bps, ms = ctypes.c_double(), ctypes.c_double()
        rc = lib.lds_peak_measure(width, 5, ctypes.byref(bps), ctypes.byref(ms))
        if rc != 0:
            raise SystemExit("bench.py: lds_peak_measure(%d) failed: %d" % (width, rc))
        res["read_%dB_per_lane" % width] = {"bytes_per_s": bps.value, "launch_ms": ms.value}
        log("LDS reads of %d B per lane: %.2f TB/s (%.3f ms per launch)"
            % (width, bps.value / 1e12, ms.value))
    res["nominal_bytes_per_s"] = LDS_PEAK_BYTES_PER_S
    print(json.dumps({"lds_peak": res}))


def _counter_totals(folder: str, exclude: str = ", true"):
    """Per-counter values of the timed decoder launch in a rocprofv3 --pmc folder: raw
    counters summed over their rows, derived metrics (one row per dispatch) averaged."""
    tot, rows = {}, {}
    for r in _csv_rows(folder, "counter_collection.csv"):
        name = r["Kernel_Name"]
        if DECODER in name and exclude not in name:
            c = r["Counter_Name"]
            tot[c] = tot.get(c, 0.0) + float(r["Counter_Value"])
            rows[c] = rows.get(c, 0) + 1
    return tot, rows


def write_util_record(lds_dir, busy_dir, bench_json, peak_json):
    """LDS bytes per path extension (SQ_INSTS_LDS_{LOAD,STORE,ATOMIC}_BANDWIDTH, 64-byte
    units), LDS, vector and scalar busy fractions and vector lane use of the timed 2 dB SCS
    launch of `bench.py --frames 100000 --points 2.0 --steps 1 --warmup 0 --cpu-sample 0
    --latency-requests 0`,
    beside the LDS rate measured by `bench.py --lds-peak`."""
    with open(bench_json) as fh:
        b = json.loads([ln for ln in fh.read().splitlines() if ln.startswith("{")][-1])
    with open(peak_json) as fh:
        pk = json.loads([ln for ln in fh.read().splitlines() if ln.startswith("{")][-1])["lds_peak"]
    lds, _ = _counter_totals(lds_dir)
    busy, nrows = _counter_totals(busy_dir)
    derived = {k: busy[k] / nrows[k] for k in ("VALUBusy", "SALUBusy", "VALUUtilization",
                                               "LDSBankConflict") if k in busy}
    if "LdsUtil" in lds:
        _, lrows = _counter_totals(lds_dir)
        derived["LdsUtil"] = lds["LdsUtil"] / lrows["LdsUtil"]
    p = b["per_point"]["2.0"]
    ext = p["mean_iterations"] * b["config"]["frames_per_point"]
    parts = {k: lds.get("SQ_INSTS_LDS_%s_BANDWIDTH" % k, 0.0) * 64.0
             for k in ("LOAD", "STORE", "ATOMIC")}
    total = sum(parts.values())
    secs = p["launch_ms"] * 1e-3
    rec = {
        "kernel": DECODER + "<10,f32> (64 lanes per frame, one stack bank)",
        "kernel_source_hash": kernel_source_hash(),
        "workload": "PC(1024,512)+CRC16, D=32, L=8, Eb/N0 2.0 dB, %d frames"
                    % b["config"]["frames_per_point"],
        "commands": [
            "rocprofv3 --pmc SQ_INSTS_LDS_LOAD_BANDWIDTH SQ_INSTS_LDS_STORE_BANDWIDTH "
            "SQ_INSTS_LDS_ATOMIC_BANDWIDTH LdsUtil --output-format csv -d <dir> -o run -- python "
            "bench.py --frames 100000 --points 2.0 --steps 1 --warmup 0 --cpu-sample 0 "
            "--latency-requests 0",
            "rocprofv3 --pmc VALUBusy SALUBusy VALUUtilization LDSBankConflict --output-format csv "
            "-d <dir> -o run -- python bench.py --frames 100000 --points 2.0 --steps 1 --warmup 0 "
            "--cpu-sample 0 --latency-requests 0",
            "python bench.py --lds-peak",
            "python bench.py --util-record <lds dir> <busy dir> <bench json> <lds-peak json>"],
        "extensions": ext,
        "lds_bytes": parts,
        "lds_bytes_per_extension": total / ext,
        "lds_bytes_per_s_in_profiled_run": total / secs,
        "profiled_launch_ms": p["launch_ms"],
        "derived_pct": derived,
        "lds_peak": pk,
    }
    with open(UTIL_RECORD, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({"util_record": UTIL_RECORD, "lds_bytes_per_extension": rec["lds_bytes_per_extension"],
                      "derived_pct": derived}))


def rocprof_use(per_point, frames):
    """The SCS kernel at 2 dB against the chip's vector-ALU and LDS peaks, from the recorded
    counters (vector instructions per path extension and their lane use; LDS bytes per
    extension) times this run's path extensions per second.  The LDS peak is the one
    `bench.py --lds-peak` measured.  None without both records taken on the current kernel
    sources or without a 2 dB point."""
    recs = []
    for path in (COUNTERS_RECORD, UTIL_RECORD):
        try:
            with open(path) as fh:
                recs.append(json.load(fh))
        except (OSError, ValueError):
            return None
    if any(r.get("kernel_source_hash") != kernel_source_hash() for r in recs) or 2.0 not in per_point:
        return None
    sq, util = recs
    p = per_point[2.0]
    if not frames or not p.get("mean_iterations"):
        return None
    ext_per_s = frames * p["mean_iterations"] / (p["launch_ms"] * 1e-3)
    lanes = util["derived_pct"]["VALUUtilization"] / 100.0 * 64.0
    valu = sq["per_extension"]["SQ_INSTS_VALU"] * lanes * ext_per_s
    lds = util["lds_bytes_per_extension"] * ext_per_s
    meas = util["lds_peak"]["read_16B_per_lane"]["bytes_per_s"]
    return {"at_ebn0_db": 2.0, "extensions_per_s": ext_per_s,
            "valu_lane_ops_per_s": valu, "valu_peak": PEAK_LANE_OPS, "valu_frac": valu / PEAK_LANE_OPS,
            "valu_insts_per_extension": sq["per_extension"]["SQ_INSTS_VALU"],
            "valu_active_lanes": lanes,
            "lds_bytes_per_s": lds, "lds_bytes_per_extension": util["lds_bytes_per_extension"],
            "lds_peak_measured": meas, "lds_frac_measured": lds / meas,
            "lds_peak_nominal": LDS_PEAK_BYTES_PER_S, "busy_pct": util["derived_pct"]}


def write_counters_record(sq_dir, bench_json):
    """Instructions per path extension of the timed SCS launch from a rocprofv3 --pmc SQ_*
    folder of `bench.py --frames 100000 --points 2.0 --steps 1 --warmup 0 --cpu-sample 0
    --latency-requests 0`."""
    with open(bench_json) as fh:
        b = json.loads([ln for ln in fh.read().splitlines() if ln.startswith("{")][-1])
    agg = {}
    for r in _csv_rows(sq_dir, "counter_collection.csv"):
        name = r["Kernel_Name"]
        if DECODER in name and ", true" not in name:
            agg[r["Counter_Name"]] = agg.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    p = b["per_point"]["2.0"]
    ext = p["mean_iterations"] * b["config"]["frames_per_point"]
    rec = {
        "kernel": DECODER + "<10,f32> (64 lanes per frame, one stack bank)",
        "kernel_source_hash": kernel_source_hash(),
        "workload": "PC(1024,512)+CRC16, D=32, L=8, Eb/N0 2.0 dB, %d frames"
                    % b["config"]["frames_per_point"],
        "command": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS "
                   "SQ_INSTS_SMEM SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_INSTS_BRANCH --output-format csv "
                   "-d <dir> -o run -- python bench.py --frames 100000 --points 2.0 --steps 1 "
                   "--warmup 0 --cpu-sample 0 --latency-requests 0",
        "extensions": ext,
        "totals": agg,
        "per_extension": {k: v / ext for k, v in agg.items()},
    }
    with open(COUNTERS_RECORD, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({"counters_record": COUNTERS_RECORD, "per_extension": rec["per_extension"]}))


COPY_BYTES = 1 << 30
DECODER = "scs_uniform_kernel"


def _csv_rows(folder: str, suffix: str):
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(os.path.join(folder, "**", "*" + suffix), recursive=True)):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _counter_kib(folder: str, counter: str, kernel: str, exclude: str = "\0"):
    """Per-dispatch values (KiB) of `counter` for the dispatches whose name contains
    `kernel` and not `exclude`, summed over the counter's instances."""
    per = {}
    for r in _csv_rows(folder, "counter_collection.csv"):
        name = r["Kernel_Name"]
        if kernel in name and exclude not in name and r["Counter_Name"] == counter:
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return [per[k] for k in sorted(per, key=int)]


def write_traffic_record(fetch_dir, write_dir, cfetch_dir, cwrite_dir, frames=1_000_000,
                         decoder: str = "scs"):
    """HBM bytes per decoder launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each
    scaled by what the same counter reads for a device copy of COPY_BYTES."""
    kernel = DECODER_KERNELS[decoder]
    # the timed launch only: the counter launch (the ", true" variant) also writes statistics
    dec_f = _counter_kib(fetch_dir, "FETCH_SIZE", kernel, ", true")
    dec_w = _counter_kib(write_dir, "WRITE_SIZE", kernel, ", true")
    cp_f = max(_counter_kib(cfetch_dir, "FETCH_SIZE", "copyBuffer"))  # the device copy
    cp_w = max(_counter_kib(cwrite_dir, "WRITE_SIZE", "copyBuffer"))
    ff = COPY_BYTES / (cp_f * 1024.0)
    wf = COPY_BYTES / (cp_w * 1024.0)
    rd = float(np.mean(dec_f)) * 1024.0 * ff
    wr = float(np.mean(dec_w)) * 1024.0 * wf
    flag = "" if decoder == "scs" else "--decoder %s " % decoder
    rec = {
        "kernel": kernel + "<10,f32> (64 lanes per frame)",
        "kernel_source_hash": kernel_source_hash(decoder),
        "workload": "PC(1024,512)+CRC16, %s, Eb/N0 2.0 dB, %d frames per launch"
                    % ("list L=8" if decoder == "scl" else "D=32, L=8", frames),
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- python bench.py "
            "%s--points 2.0 --steps 1 --warmup 0 --cpu-sample 0 --latency-requests 0" % flag,
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- python bench.py "
            "%s--points 2.0 --steps 1 --warmup 0 --cpu-sample 0 --latency-requests 0" % flag,
            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- python bench.py "
            "--calibrate-copy %d" % COPY_BYTES,
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- python bench.py "
            "--calibrate-copy %d" % COPY_BYTES,
            "python bench.py %s--traffic-record <fetch> <write> <copy fetch> <copy write>" % flag],
        "raw_kib_per_dispatch": {"decoder_fetch_size": dec_f, "decoder_write_size": dec_w,
                                 "copy_1GiB_fetch_size": cp_f, "copy_1GiB_write_size": cp_w},
        "calibration": {"fetch_factor": ff, "write_factor": wf,
                        "note": "a 1 GiB device copy reads 1 GiB and writes 1 GiB; each counter "
                                "is scaled by the ratio of that to what it reports for the copy"},
        "hbm_read_bytes_per_launch": rd,
        "hbm_write_bytes_per_launch": wr,
        "hbm_bytes_per_frame": (rd + wr) / frames,
        "algorithmic_bytes_per_frame": 4 * N + (K - CRC) + 1,
    }
    path = traffic_record_path(decoder)
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({"traffic_record": path, "hbm_bytes_per_frame": rec["hbm_bytes_per_frame"]}))


def write_workload_trace_summary(trace_dir, bench_json, out_md):
    """Markdown summary of a kernel trace of `python bench.py --workload mixed|serve`: the
    kernels by GPU time, and for the persistent mixed launches their number, durations and
    how many ran at once on average (the sum of their durations over the span they cover)."""
    rows = _csv_rows(trace_dir, "kernel_trace.csv")
    with open(bench_json) as fh:
        b = json.loads([ln for ln in fh.read().splitlines() if ln.startswith("{")][-1])
    serve = "latency_ms" in b
    per, mixed = {}, []
    for r in rows:
        name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
        short = name.split("(")[0].strip()[:90]
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        per.setdefault(short, []).append((t1 - t0) * 1e-6)
        if short.startswith("scs_mixed_kernel"):
            mixed.append((t0, t1))
    total = sum(sum(v) for v in per.values())
    cmd = "--workload serve" if serve else "--workload mixed"
    lines = ["# Kernel trace: %s workload" % ("serving" if serve else "mixed-batch"), "",
             "Command (from the repository root on one MI355X):", "",
             "    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- "
             "python bench.py %s" % cmd, "",
             "Workload: %s.  Bench line of the same run: %.1f Mbit/s%s." % (
                 b["config"]["workload"], b["value"],
                 (", %.0f frames/s offered, %.0f sustained, request latency p50 %.1f ms, p99 %.1f ms"
                  % (b["config"]["offered_frames_per_s"], b["sustained_frames_per_s"],
                     b["latency_ms"]["p50"], b["latency_ms"]["p99"])) if serve else
                 (", %.0f frames/s, %.2fx the one-launch-per-configuration form"
                  % (b["frames_per_s"], b["mixed_over_plain"]))), "",
             "| kernel | calls | average ms | min ms | max ms | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:8]:
        lines.append("| %s | %d | %.3f | %.3f | %.3f | %.2f%% |" % (
            k, len(v), np.mean(v), min(v), max(v), 100.0 * sum(v) / total))
    if serve and mixed:
        # the serving phase is the run's last: keep the launches of its span only
        t_end = max(t1 for _, t1 in mixed)
        mixed = [(t0, t1) for t0, t1 in mixed if t0 >= t_end - b["ms_per_step"] * 1e6]
    if mixed:
        mixed.sort()
        busy = sum(t1 - t0 for t0, t1 in mixed)
        span, cur0, cur1 = 0, mixed[0][0], mixed[0][1]
        for t0, t1 in mixed[1:]:
            if t0 > cur1:
                span += cur1 - cur0
                cur0, cur1 = t0, t1
            else:
                cur1 = max(cur1, t1)
        span += cur1 - cur0
        lines += ["", "Persistent mixed launches%s: %d, mean %.3f ms; on average %.2f of them "
                  "ran at once over the %.1f s they cover." % (
                      " of the serving span" if serve else "", len(mixed),
                      busy * 1e-6 / len(mixed), busy / max(span, 1), span * 1e-9)]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def write_trace_summary(trace_dir, bench_json, out_md):
    """Markdown summary of a kernel trace of `python bench.py --cpu-sample 0
    --latency-requests 0`: per-kernel statistics, and the decoder's mean duration beside
    bench.py's own HIP-event mean."""
    rows = _csv_rows(trace_dir, "kernel_trace.csv")
    with open(bench_json) as fh:
        b = json.loads([ln for ln in fh.read().splitlines() if ln.startswith("{")][-1])
    decoder = b["roofline"]["kernel"].split("<")[0]
    per = {}
    for r in rows:
        name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
        short = name.split("(")[0].strip()
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
        per.setdefault(short[:90], []).append(d)
    total = sum(sum(v) for v in per.values())
    title = ("FSSCS-RM" if decoder.startswith("fsscs") else
             "CA-SCL" if decoder.startswith("scl") else "SCS")
    extra = (" --decoder fsscs" if decoder.startswith("fsscs") else
             " --decoder scl" if decoder.startswith("scl") else "")
    cfg = b["config"]
    if not decoder.startswith("scl") and cfg["D"] != HEADLINE_DL[0]:
        extra += " --D %d" % cfg["D"]
    if cfg["L"] != HEADLINE_DL[1]:
        extra += " --L %d" % cfg["L"]
    lines = ["# Kernel trace: %s decoder, PC(1024,512)+CRC-16 sweep" % title, "",
             "Command (from the repository root on one MI355X):", "",
             "    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- "
             "python bench.py%s --cpu-sample 0 --latency-requests 0" % extra, "",
             "Workload: N=1024, K=512 (496 payload + 16 CRC), %s, Eb/N0 1.0/1.5/2.0/2.5/3.0 "
             "dB, %d frames per point, launch shape %s.  Decoder launches: one counter launch "
             "per point (stats variant), %d warmup and %d timed steps of one launch per point.  "
             "The CPU-oracle sample and the request-latency probe are off so that their small "
             "launches do not enter the average."
             % (("list of L=%d" % b["config"]["L"]) if decoder.startswith("scl") else
                ("D=%d, L=%d" % (b["config"]["D"], b["config"]["L"])),
                b["config"]["frames_per_point"], b["config"].get("launch_shape"), b["warmup"],
                b["steps"]), "",
             "| kernel | calls | average ms | min ms | max ms | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:8]:
        lines.append("| %s | %d | %.3f | %.3f | %.3f | %.2f%% |" % (
            k, len(v), np.mean(v), min(v), max(v), 100.0 * sum(v) / total))
    dec = [d for k, v in per.items() if k.startswith(decoder) for d in v]
    timed = [d for k, v in per.items() if k.startswith(decoder) and ", true" not in k for d in v]
    lines += ["", "Decoder mean over all %d launches (points mixed): %.1f ms.  Without the counter "
              "launches (%d warmup + timed launches): %.1f ms.  bench.py's HIP-event mean over its "
              "timed launches: %.1f ms (`roofline.mean_launch_ms`); bench value %.1f Mbit/s." % (
                  len(dec), np.mean(dec), len(timed), np.mean(timed) if timed else float("nan"),
                  b["roofline"]["mean_launch_ms"], b["value"]),
              "", "Per point (bench.py, HIP events): " + ", ".join(
                  "%s dB %.0f ms" % (k, v["launch_ms"]) for k, v in b["per_point"].items()) + "."]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


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
    if args.traffic_record:
        if args.decoder == "fssc":
            raise SystemExit("bench.py: traffic records are taken for scs, fsscs and scl")
        write_traffic_record(*args.traffic_record, decoder=args.decoder)
        return
    if args.util_record:
        write_util_record(*args.util_record)
        return
    if args.lds_peak:
        lds_peak()
        return
    if args.counters_record:
        write_counters_record(*args.counters_record)
        return
    if args.trace_summary:
        with open(args.trace_summary[1]) as fh:
            line = [ln for ln in fh.read().splitlines() if ln.startswith("{")][-1]
        if "roofline" in json.loads(line):
            write_trace_summary(*args.trace_summary)
        else:
            write_workload_trace_summary(*args.trace_summary)
        return
    if args.workload == "serve":
        # The serving slots run their batches side by side only from separate hardware queues:
        # HIP maps streams beyond its queue count (GPU_MAX_HW_QUEUES, 4 by default) onto shared
        # queues, whose launches run one after another.  Four slots plus the default and the
        # input-generation streams need more than 4 (set before HIP starts).
        if int(os.environ.get("GPU_MAX_HW_QUEUES") or 4) < 8:
            os.environ["GPU_MAX_HW_QUEUES"] = "8"
    if args.workload in ("mixed", "serve"):
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        {"mixed": run_mixed, "serve": run_serve}[args.workload](args)
        return
    if args.workload in ("fixed", "depth"):
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        {"fixed": run_fixed, "depth": run_depth}[args.workload](args)
        return
    if args.decoder == "fssc":
        sweep_config(1, 1)  # fast simplified SC: no stack, no second path
    elif args.workload == "sweep" and (args.D, args.L) != (D, L):
        sweep_config(args.D, args.L)
    if args.gpus != 1:
        print("bench.py: the library decodes on one GPU; --gpus %d is not supported (frames are "
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
    ctx = binding.ScsContext(0, args.wpb)
    launch_shape = {"waves_per_block": args.wpb, "source": "flags"}
    if not args.wpb and args.tune != "off":
        from paper_1809_03606_amd import tune

        dec = "fsscs" if args.decoder == "fssc" else args.decoder
        entry = None if args.tune == "force" else tune.apply(ctx, code, D, L, args.dtype, decoder=dec)
        source = "cache"
        if entry is None:
            t0 = time.time()
            entry = tune.tune(code, D, L, args.dtype, decoder=dec)
            tune.apply(ctx, code, D, L, args.dtype, decoder=dec)
            source = "tuned in %.1f s" % (time.time() - t0)
        launch_shape = {"waves_per_block": entry["waves_per_block"], "source": source,
                        "candidates_ms": entry["candidates_ms"]}
        log("launch shape: %s" % launch_shape)
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

    fast = args.decoder in ("fsscs", "fssc")
    fssc = args.decoder == "fssc"
    scl = args.decoder == "scl"
    if scl:
        def decode_fn(ctx_h, code_h, D_, L_, dt, x, n, p_, s_, st_, strm):
            binding.scl_decode_batch(ctx_h, code_h, L_, dt, x, n, p_, s_, st_, strm)
    else:
        decode_fn = binding.fsscs_decode_batch if fast else binding.scs_decode_batch

    def launch(llr, with_stats=False):
        decode_fn(ctx.handle, code.handle, D, L, llr_dtype, llr, B, out_pay,
                                 out_st, stats if with_stats else None, stream)

    # -- per-point work counters and FER (untimed) ------------------------------------
    per_point = {}
    work_ops = {}
    for eb, pay, llr in data:
        launch(llr, with_stats=True)
        stream.synchronize()
        s = stats.cpu().numpy().view(np.uint32).astype(np.int64)
        it, sc = s[:, 0].sum(), s[:, 3].sum()
        if scl:  # every list entry runs the SC schedule: N log2 N f/g values per entry
            work_ops[eb] = OPS_PER_ELEM * (it / N) * N * int(np.log2(N)) + OPS_PER_ITER_FIXED * it
        else:
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

    # -- request latency: closed-loop requests of 1..256 frames on this code and decoder, one
    # in flight at a time, host clock from submission to completion (untimed for `value`) --
    lat_eb = 2.0 if 2.0 in points else points[len(points) // 2]
    lat_llr = [llr for eb, _, llr in data if eb == lat_eb][0]
    rng = np.random.default_rng(11)
    req_ms = []
    for r in range(args.latency_requests):
        m = int(rng.integers(1, 257))
        lo = int(rng.integers(0, B - m + 1))
        stream.synchronize()
        t0 = time.perf_counter()
        decode_fn(ctx.handle, code.handle, D, L, llr_dtype, lat_llr[lo:lo + m], m, out_pay,
                  out_st, None, stream)
        stream.synchronize()
        req_ms.append((time.perf_counter() - t0) * 1e3)
    req_ms = np.array(req_ms) if req_ms else np.zeros(1)

    # -- end to end from host memory (untimed for `value`): the point's LLRs in pinned host
    # memory are copied in, decoded and their payload and status copied back, in eight chunks
    # alternating over two streams so that one chunk's copies overlap another's decoding --
    e2e = None
    e2e_reps = args.e2e_reps if args.e2e_reps is not None else (3 if args.latency_requests else 0)
    if e2e_reps > 0:
        h_llr = torch.empty(lat_llr.shape, dtype=lat_llr.dtype, pin_memory=True)
        h_llr.copy_(lat_llr)
        h_pay = torch.empty((B, kp), dtype=torch.uint8, pin_memory=True)
        h_st = torch.empty((B,), dtype=torch.uint8, pin_memory=True)
        d_llr = torch.empty_like(lat_llr)
        launch(lat_llr)
        stream.synchronize()
        ref_pay, ref_st = out_pay.cpu(), out_st.cpu()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):  # the host-to-device copy alone
            a.record(stream)
            d_llr.copy_(h_llr, non_blocking=True)
            b.record(stream)
        stream.synchronize()
        h2d_ms = a.elapsed_time(b)
        streams = [stream, torch.cuda.Stream(device=dev)]
        chunk = (B + 7) // 8
        e2e_ms = []
        for _ in range(e2e_reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c, lo in enumerate(range(0, B, chunk)):
                hi = min(B, lo + chunk)
                s = streams[c % 2]
                with torch.cuda.stream(s):
                    d_llr[lo:hi].copy_(h_llr[lo:hi], non_blocking=True)
                    decode_fn(ctx.handle, code.handle, D, L, llr_dtype, d_llr[lo:hi], hi - lo,
                              out_pay[lo:hi], out_st[lo:hi], None, s)
                    h_pay[lo:hi].copy_(out_pay[lo:hi], non_blocking=True)
                    h_st[lo:hi].copy_(out_st[lo:hi], non_blocking=True)
            for s in streams:
                s.synchronize()
            e2e_ms.append((time.perf_counter() - t0) * 1e3)
        ms_e = float(np.mean(e2e_ms))
        e2e = {"ebn0_db": lat_eb, "frames": B, "chunks": (B + chunk - 1) // chunk, "streams": 2,
               "ms": ms_e, "payload_mbps": B * kp / (ms_e * 1e-3) / 1e6,
               "h2d_bytes": h_llr.numel() * h_llr.element_size(), "h2d_ms": h2d_ms,
               "h2d_gbps": h_llr.numel() * h_llr.element_size() / (h2d_ms * 1e-3) / 1e9,
               "equals_device_resident": bool(torch.equal(h_pay, ref_pay) and
                                              torch.equal(h_st, ref_st)),
               "note": "LLRs from pinned host memory and results back to it, host clock, "
                       "mean of %d runs; not the bench value" % e2e_reps}
        log("end to end from host memory: %.1f ms, %.0f Mbit/s" % (ms_e, e2e["payload_mbps"]))
        del h_llr, h_pay, h_st, d_llr, ref_pay, ref_st

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
    # the counter records were taken on the binary32 kernels on the headline configuration
    # (traffic: each decoder; instruction and LDS counts: the SCS kernel)
    headline = args.dtype == "f32" and (D, L) == HEADLINE_DL
    recorded = headline and not fast and not scl
    dec_name = "scl" if scl else "fsscs" if fast else "scs"
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tlane-op/s",
                "frac": achieved / peak,
                "traffic": measured_traffic(B, dec_name) if headline else None,
                "kernel": ("fsscs_uniform_kernel" if fast else "scl_uniform_kernel" if scl else
                           "scs_uniform_kernel")
                          + ("<10,f32>" if args.dtype == "f32" else "<10,i8>"),
                "mean_launch_ms": float(all_ms.mean()), "ops_per_launch": ops_per_launch,
                "issue": issue_bound(per_point, B) if recorded else None,
                "rocprof": rocprof_use(per_point, B) if recorded else None}

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
            if scl:
                rp, rs, _ = oracle.scl_decode_batch(mode, info, CRC, L, x.cpu().numpy(), threads=thr)
            else:
                ofn = oracle.fsscs_decode_batch if fast else oracle.scs_decode_batch
                rp, rs, _ = ofn(mode, info, CRC, D, L, x.cpu().numpy(), threads=thr)
            t += time.perf_counter() - c0
            # the same sample on the GPU must give the same bits
            decode_fn(ctx.handle, code.handle, D, L, llr_dtype, x, n, out_pay,
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
        "metric": "info Mbit/s decoded (N=1024,K=512,D=32) at oracle-matched FER; p99 latency"
                  + ("; FSSC decoder" if fssc else "; FSSCS-RM decoder" if fast else
                     "; CA-SCL decoder, list %d" % L if scl else "")
                  + ("; D=%d, L=%d" % (D, L) if not scl and (D, L) != HEADLINE_DL else ""),
        "value": value, "unit": "Mbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic: seeded BPSK/AWGN frames generated on the device",
        "config": {"workload": ("FSSC" if fssc else "FSSCS-RM" if fast else
                                "CA-SCL" if scl else "SCS")
                               + (" sweep PC(1024,512)+CRC16 L=%d" % L if scl else
                                  " sweep PC(1024,512)+CRC16 D=%d L=%d" % (D, L))
                               + (" Eb/N0 1.0-3.0 dB" if points == list(POINTS) else
                                  " Eb/N0 %s dB" % ",".join("%g" % p for p in points)),
                   "N": N, "K": K, "crc_bits": CRC, "D": D, "L": L,
                   "ebn0_db": points, "frames_per_point": B, "global_batch": B * len(points),
                   "launches_per_step": len(points), "parallelism": "single GPU",
                   "launch_shape": launch_shape},
        "latency": {"request_ms_p50": float(np.percentile(req_ms, 50)),
                    "request_ms_p99": float(np.percentile(req_ms, 99)),
                    "request": "%d closed-loop requests of 1-256 frames at %.1f dB, one in "
                               "flight, host clock from submission to completion"
                               % (args.latency_requests, lat_eb),
                    "batch_launch_ms_p50": float(np.percentile(all_ms, 50)),
                    "batch_launch_ms_p99": float(np.percentile(all_ms, 99))},
        "per_point": {str(k): v for k, v in per_point.items()},
        "k_bit_mbps": value * K / kp,
        "paper_context": paper_context(args.decoder),
        "end_to_end_from_host": e2e,
        "wall_s": wall, "input_generation_s": gen_s,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def paper_context(decoder: str):
    """The paper's per-thread CPU throughput for the same decoder, with its setup."""
    if decoder not in PAPER_TP_MBPS:
        return None
    name, tp = PAPER_TP_MBPS[decoder]
    return {"decoder": name, "mbps_per_thread": {str(e): v for e, v in zip(POINTS, tp)},
            "hardware": "AMD Ryzen 5 1600 at 3.2 GHz, 6 threads, average per thread",
            "workload": "PC(1024,512), 5G information set, CRC-24C, L=8, D=8192",
            "note": "the paper's figures on its own machine and code; context, not vs_baseline"}


def mixed_batch(torch, dev, B, seed, pcs, codes, stream, Lp=8, crc=16):
    """Frames of the mixed workload generated on the device, laid out grouped by (code, D):
    returns (frames descriptors, LLRs, reference payloads, groups, grouped order, payload
    bits per frame)."""
    from paper_1809_03606_amd import binding, channel

    cidx, Dv, eb = channel.mixed_draw(seed, B)
    dsel = {8: 0, 32: 1, 64: 2}
    gkey = cidx.astype(np.int64) * 3 + np.vectorize(dsel.get)(Dv)
    grouped = np.argsort(gkey, kind="stable")  # frames grouped by (code, D)
    Nf = np.array([codes[c][0] for c in cidx], np.int64)
    kpf = np.array([codes[c][1] - crc for c in cidx], np.int64)
    llr_off = np.zeros(B, np.int64)
    out_off = np.zeros(B, np.int64)
    llr_off[grouped] = np.concatenate([[0], np.cumsum(Nf[grouped])[:-1]])
    out_off[grouped] = np.concatenate([[0], np.cumsum(kpf[grouped])[:-1]])
    tot_llr, tot_out = int(Nf.sum()), int(kpf.sum())
    llr = torch.empty(tot_llr, dtype=torch.float32, device=dev)
    pay_ref = torch.empty(tot_out, dtype=torch.uint8, device=dev)
    groups = []  # (code, D, first grouped position, count)
    t0 = time.time()
    with torch.cuda.stream(stream):
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        bounds = np.nonzero(np.diff(gkey[grouped]))[0] + 1
        for a, b in zip(np.concatenate([[0], bounds]), np.concatenate([bounds, [B]])):
            f0 = grouped[a]
            c, d = int(cidx[f0]), int(Dv[f0])
            n, k = codes[c]
            lo, lo_o = int(llr_off[f0]), int(out_off[f0])
            cnt = int(b - a)
            pay = channel.device_payload(torch, gen, cnt, k - crc, dev)
            cw = torch.empty((cnt, n), dtype=torch.uint8, device=dev)
            pcs[c].encode_device(pay, cw, stream)
            ebs = torch.from_numpy(eb[grouped[a:b]]).to(dev)
            llr[lo:lo + cnt * n] = channel.device_llr_per_frame(torch, gen, cw, ebs, k / n).reshape(-1)
            pay_ref[lo_o:lo_o + cnt * (k - crc)] = pay.reshape(-1)
            groups.append((c, d, lo, lo_o, cnt))
    stream.synchronize()
    log("mixed inputs ready: %d frames in %d (code, D) groups, %.1f s" % (B, len(groups), time.time() - t0))
    frames = np.zeros(B, binding.FRAME_DTYPE)
    frames["code"], frames["D"], frames["L"] = cidx, Dv, Lp
    frames["llr_off"], frames["out_off"] = llr_off, out_off
    return frames, llr, pay_ref, groups, grouped, kpf


def run_mixed(args):
    """Mixed batch: frames drawn uniformly over N in {128..2048}, rate in {1/4..5/6} (25
    codes, CRC-16), D in {8, 32, 64}, L = 8, Eb/N0 ~ U[1.5, 3.5] dB, decoded (a) in one
    persistent launch replayed from a captured graph and (b) as one launch per (code, D)."""
    import torch

    from paper_1809_03606_amd import binding, channel

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    B, Lp, crc, seed = args.mixed_frames, 8, 16, 4
    codes = channel.mixed_codes()
    pcs = [binding.PolarCode(n, k, crc, 2.0) for (n, k) in codes]
    stream = torch.cuda.Stream(device=dev)
    frames, llr, pay_ref, groups, grouped, kpf = mixed_batch(torch, dev, B, seed, pcs, codes,
                                                             stream, Lp, crc)
    tot_out = int(kpf.sum())
    ctx = binding.ScsContext(0)
    ctx_plain = binding.ScsContext(0)  # one launch per configuration, library launch shapes
    pay_m = torch.empty(tot_out, dtype=torch.uint8, device=dev)
    st_m = torch.empty(B, dtype=torch.uint8, device=dev)
    pay_p = torch.empty(tot_out, dtype=torch.uint8, device=dev)
    st_p = torch.empty(B, dtype=torch.uint8, device=dev)
    handles = [p.handle for p in pcs]
    launch_shape = {"waves_per_block": 4, "source": "library default"}
    if args.wpb:
        ctx.configure(args.wpb)
        launch_shape = {"waves_per_block": args.wpb, "source": "flags"}
    elif args.tune != "off":
        from paper_1809_03606_amd import tune

        entry = None if args.tune == "force" else tune.apply_mixed(ctx, pcs, frames)
        source = "cache"
        if entry is None:
            t0 = time.time()
            entry = tune.tune_mixed(ctx, pcs, frames, llr, pay_m, st_m, stream)
            source = "tuned in %.1f s on %d frames" % (time.time() - t0, entry["frames"])
        launch_shape = {"waves_per_block": entry["waves_per_block"], "source": source,
                        "candidates_ms": entry["candidates_ms"]}
    log("mixed launch shape: %s" % launch_shape)
    binding.scs_mixed_prepare(ctx.handle, handles, frames, stream)
    stream.synchronize()

    def plain():
        pos = 0
        for (c, d, lo, lo_o, cnt) in groups:
            n, k = codes[c]
            binding.scs_decode_batch(ctx_plain.handle, pcs[c].handle, d, Lp, binding.SCS_LLR_F32,
                                     llr[lo:].data_ptr(), cnt, pay_p[lo_o:].data_ptr(),
                                     st_p[pos:].data_ptr(), None, stream)
            pos += cnt

    # graph of the prepared persistent launch
    g = torch.cuda.CUDAGraph()
    binding.scs_mixed_launch(ctx.handle, binding.SCS_LLR_F32, llr, pay_m, st_m, None, stream)
    stream.synchronize()
    with torch.cuda.graph(g, stream=stream):
        binding.scs_mixed_launch(ctx.handle, binding.SCS_LLR_F32, llr, pay_m, st_m, None,
                                 torch.cuda.current_stream())
    plain()
    stream.synchronize()
    same = bool(torch.equal(pay_m, pay_p)) and bool(torch.equal(st_m[torch.from_numpy(grouped).to(dev)], st_p))
    # frame errors: compare per frame via segment sums over the payload bytes
    bad = (pay_m != pay_ref).to(torch.int64)
    seg = torch.from_numpy(np.repeat(np.arange(B)[grouped], kpf[grouped])).to(dev)
    err_frames = torch.zeros(B, dtype=torch.int64, device=dev).index_add_(0, seg, bad)
    fer = float((err_frames > 0).float().mean().item())
    log("mixed: outputs equal to the per-configuration launches: %s, FER %.3e" % (same, fer))

    def timed(fn, reps):
        ev = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            ev.append((a, b))
        stream.synchronize()
        return [a.elapsed_time(b) for a, b in ev]

    with torch.cuda.stream(stream):
        timed(g.replay, args.warmup)
        ms_m = timed(g.replay, args.steps)
    timed(plain, args.warmup)
    ms_p = timed(plain, args.steps)
    bits = B * float(kpf.mean())
    v_m = bits / (np.mean(ms_m) * 1e-3) / 1e6
    v_p = bits / (np.mean(ms_p) * 1e-3) / 1e6
    line = {
        "metric": "info Mbit/s decoded, mixed batch (N 128-2048, rate 1/4-5/6, D 8/32/64) in one persistent launch",
        "value": v_m, "unit": "Mbit/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": float(np.mean(ms_m)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded BPSK/AWGN frames generated on the device",
        "config": {"workload": "mixed batch: 25 codes (CRC-16) x D in {8,32,64}, L=8, Eb/N0 U[1.5,3.5]",
                   "frames": B, "groups": len(groups), "parallelism": "single GPU",
                   "launch_shape": launch_shape},
        "frames_per_s": B / (np.mean(ms_m) * 1e-3),
        "plain_one_launch_per_config": {"value": v_p, "unit": "Mbit/s", "launches": len(groups),
                                        "ms_per_step": float(np.mean(ms_p))},
        "mixed_over_plain": v_m / v_p,
        "outputs_equal": same, "fer": fer,
    }
    print(json.dumps(line))


def wilson(k, n, z=1.959964):
    """95% Wilson score interval of a binomial proportion."""
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return (float(c - h), float(c + h))


def run_fixed(args):
    """Fixed point at 2 dB: the same 10^6 noisy frames decoded with binary32 LLRs and with
    int8 LLRs q = clamp(rint(T y)) (int8 tree, int16 path metric); FER of both with 95%
    intervals, the quantiser scale T chosen by a sweep on the first 200,000 frames, and the
    throughput of both decoders."""
    import torch

    from paper_1809_03606_amd import binding, channel

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    B, eb, kp = args.frames, 2.0, K - CRC
    code = binding.PolarCode(N, K, CRC, 2.0)
    ctx = binding.ScsContext(0)
    stream = torch.cuda.Stream(device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(SEED * 1000 + 2)
    pay = channel.device_payload(torch, gen, B, kp, dev)
    y = torch.empty((B, N), dtype=torch.float64, device=dev)  # channel output, for quantising
    llr = torch.empty((B, N), dtype=torch.float32, device=dev)
    s2 = channel.sigma2(eb, K / N)
    chunk = 1 << 17
    for lo in range(0, B, chunk):
        hi = min(B, lo + chunk)
        cw = torch.empty((hi - lo, N), dtype=torch.uint8, device=dev)
        code.encode_device(pay[lo:hi], cw)
        nz = channel.device_noise(torch, gen, hi - lo, N, dev)
        llr[lo:hi] = channel.device_llr_from_noise(torch, cw, nz, eb, K / N, "f32")
        y[lo:hi] = (1.0 - 2.0 * cw.to(torch.float64)) + np.sqrt(s2) * nz
        del cw, nz
    torch.cuda.synchronize()
    out = torch.empty((B, kp), dtype=torch.uint8, device=dev)
    st = torch.empty((B,), dtype=torch.uint8, device=dev)

    from paper_1809_03606_amd import tune

    def decode(x, n):
        dt = binding.SCS_LLR_F32 if x.dtype == torch.float32 else binding.SCS_LLR_I8
        # each precision at its tuned workgroup size (the library default when none is stored)
        ctx.configure(0)
        tune.apply(ctx, code, D, L, "f32" if dt == binding.SCS_LLR_F32 else "i8")
        # x was just written on the default stream: the decoder's stream waits for it
        stream.wait_stream(torch.cuda.current_stream())
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        binding.scs_decode_batch(ctx.handle, code.handle, D, L, dt, x, n, out, st, None, stream)
        b.record(stream)
        stream.synchronize()
        errs = int((out[:n] != pay[:n]).any(dim=1).sum().item())
        return errs, a.elapsed_time(b)

    # quantiser scale: 200k frames per candidate
    ns = min(B, 200_000)
    sweep = {}
    for T in (2.0, 4.0, 8.0, 16.0):
        q = torch.clamp(torch.round(T * y[:ns]), -127, 127).to(torch.int8)
        sweep[T] = decode(q, ns)[0] / ns
        log("fixed: T=%g FER %.4f on %d frames" % (T, sweep[T], ns))
    T = min(sweep, key=lambda t: (sweep[t], t))
    q = torch.empty((B, N), dtype=torch.int8, device=dev)
    for lo in range(0, B, chunk):
        hi = min(B, lo + chunk)
        q[lo:hi] = torch.clamp(torch.round(T * y[lo:hi]), -127, 127).to(torch.int8)
    decode(llr, B)
    decode(q, B)  # warm-up
    e32, ms32 = decode(llr, B)
    e8, ms8 = decode(q, B)
    line = {
        "metric": "FER of int8/int16 fixed-point SCS vs binary32 at 2 dB, and throughput",
        "value": B * kp / (ms8 * 1e-3) / 1e6, "unit": "Mbit/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": ms8, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i8",
        "data": "synthetic: seeded BPSK/AWGN frames generated on the device",
        "config": {"workload": "fixed point PC(1024,512)+CRC16 D=32 L=8 Eb/N0 2.0 dB",
                   "frames": B, "quantiser_scale": T, "scale_sweep_fer": sweep},
        "fer_i8": e8 / B, "fer_i8_ci95": wilson(e8, B),
        "fer_f32": e32 / B, "fer_f32_ci95": wilson(e32, B),
        "f32_payload_mbps": B * kp / (ms32 * 1e-3) / 1e6,
    }
    print(json.dumps(line))


DEPTHS = (8, 16, 32, 64, 128, 256)


def run_depth(args):
    """Stack depth and L: FER and throughput of SCS and FSSCS-RM on the same 10^6 noisy
    frames of PC(1024,512)+CRC-16 at each Eb/N0 point, for D in {8, 16, 32, 64, 128, 256}
    and L in {2, 4, 8}, with CA-SCL (L in {1, 2, 4, 8}) on the same frames; every
    configuration at the autotuner's stored workgroup size where there is one."""
    import torch

    from paper_1809_03606_amd import binding, channel, tune

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    B, kp = args.frames, K - CRC
    code = binding.PolarCode(N, K, CRC, 2.0)
    ctx = binding.ScsContext(0)

    def shape(dec, d, lp):
        """The autotuner's stored workgroup size for this configuration, else the default."""
        ctx.configure(0)
        e = tune.apply(ctx, code, d, lp, "f32", decoder=dec)
        return e["waves_per_block"] if e else 0

    stream = torch.cuda.Stream(device=dev)
    out = torch.empty((B, kp), dtype=torch.uint8, device=dev)
    st = torch.empty((B,), dtype=torch.uint8, device=dev)
    rows = []
    for pi, eb in enumerate([float(x) for x in args.points.split(",")]):
        gen = torch.Generator(device=dev)
        gen.manual_seed(SEED * 1000 + 7 + pi)
        pay = channel.device_payload(torch, gen, B, kp, dev)
        llr = torch.empty((B, N), dtype=torch.float32, device=dev)
        chunk = 1 << 17
        for lo in range(0, B, chunk):
            hi = min(B, lo + chunk)
            cw = torch.empty((hi - lo, N), dtype=torch.uint8, device=dev)
            code.encode_device(pay[lo:hi], cw)
            llr[lo:hi] = channel.device_llr(torch, gen, cw, eb, K / N, "f32")
            del cw
        torch.cuda.synchronize()
        for dec in ("scs", "fsscs"):
            fn = binding.fsscs_decode_batch if dec == "fsscs" else binding.scs_decode_batch
            for d in DEPTHS:
                for Lp in (2, 4, 8):
                    wpb = shape(dec, d, Lp)
                    fn(ctx.handle, code.handle, d, Lp, binding.SCS_LLR_F32, llr, B, out, st,
                       None, stream)  # warm-up
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    fn(ctx.handle, code.handle, d, Lp, binding.SCS_LLR_F32, llr, B, out, st,
                       None, stream)
                    b.record(stream)
                    stream.synchronize()
                    ms = a.elapsed_time(b)
                    errs = int((out != pay).any(dim=1).sum().item())
                    rows.append({"decoder": dec, "ebn0_db": eb, "D": d, "L": Lp, "fer": errs / B,
                                 "fer_ci95": wilson(errs, B), "launch_ms": ms,
                                 "payload_mbps": B * kp / (ms * 1e-3) / 1e6,
                                 "waves_per_block": wpb or "default"})
                    log("depth: %s Eb/N0 %.1f D=%d L=%d FER %.5f %.0f Mbit/s" % (
                        dec, eb, d, Lp, errs / B, rows[-1]["payload_mbps"]))
        for Lp in (1, 2, 4, 8):
            wpb = shape("scl", 0, Lp)
            binding.scl_decode_batch(ctx.handle, code.handle, Lp, binding.SCS_LLR_F32, llr, B, out,
                                     st, None, stream)  # warm-up
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            binding.scl_decode_batch(ctx.handle, code.handle, Lp, binding.SCS_LLR_F32, llr, B, out,
                                     st, None, stream)
            b.record(stream)
            stream.synchronize()
            ms = a.elapsed_time(b)
            errs = int((out != pay).any(dim=1).sum().item())
            rows.append({"decoder": "scl", "ebn0_db": eb, "D": None, "L": Lp, "fer": errs / B,
                         "fer_ci95": wilson(errs, B), "launch_ms": ms,
                         "payload_mbps": B * kp / (ms * 1e-3) / 1e6,
                         "waves_per_block": wpb or "default"})
            log("depth: scl Eb/N0 %.1f L=%d FER %.5f %.0f Mbit/s" % (
                eb, Lp, errs / B, rows[-1]["payload_mbps"]))
        del llr, pay
    ref = [r for r in rows if r["decoder"] == "scs" and r["D"] == D and r["L"] == L]
    line = {
        "metric": "FER and info Mbit/s vs stack depth D and L, SCS and FSSCS-RM",
        "value": ref[0]["payload_mbps"] if ref else None, "unit": "Mbit/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded BPSK/AWGN frames generated on the device",
        "config": {"workload": "depth study PC(1024,512)+CRC16, D in {8,16,32,64,128,256}, "
                               "L in {2,4,8}; CA-SCL L in {1,2,4,8}",
                   "frames": B},
        "rows": rows,
    }
    print(json.dumps(line))


# Device-memory budget of the serving run's admission: a request's footprint counts its
# LLRs, its outputs and, for every frame, a decoder state as if the frame were resident
# (stack rows of D slots, L counters, alpha tree; serve.request_footprint), about 12 KB per
# frame of the mixed distribution; 16 GiB (of the MI355X's 288) lets the four slots' full
# batches of 16,384 frames be in flight together.
SERVE_BUDGET = 16 << 30


def serve_pool(seed, n_req, codes, pcs, on_device=True):
    """A pool of requests of the mixed distribution (code, D, Eb/N0 per request), 1..256
    frames each, LLRs generated on the device with the library's encoder; they stay there
    (device-resident requests) or are copied to host memory."""
    import torch

    from paper_1809_03606_amd import channel
    from paper_1809_03606_amd.serve import Request

    rng = np.random.default_rng(seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    pool = []
    for rid in range(n_req):
        c = int(rng.integers(len(codes)))
        n, k = codes[c]
        m = int(rng.integers(1, 257))
        pay = channel.device_payload(torch, gen, m, k - 16, "cuda")
        cw = torch.empty((m, n), dtype=torch.uint8, device="cuda")
        pcs[c].encode_device(pay, cw)
        ebs = torch.full((m,), float(rng.uniform(1.5, 3.5)), dtype=torch.float64, device="cuda")
        llr = channel.device_llr_per_frame(torch, gen, cw, ebs, k / n)
        pool.append(Request(rid=rid, code=c, D=int(rng.choice([8, 32, 64])), L=8,
                            llr=llr if on_device else llr.cpu().numpy()))
    torch.cuda.synchronize()
    return pool


def run_serve(args):
    """Poisson arrivals of requests (1..256 frames of one code / D from the mixed
    distribution, LLRs resident on the device) at args.serve_load x the sustained frame
    rate of the mixed batch's persistent launch (measured here on an i.i.d. batch of the same
    distribution), admitted by device-memory budget into 4 slots that share the GPU (a
    quarter of the CUs each); reports request latency percentiles and sustained payload
    bit/s."""
    import copy
    import gc

    import torch

    from paper_1809_03606_amd import binding, channel, tune
    from paper_1809_03606_amd.serve import GpuBackend, Server

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    codes = channel.mixed_codes()
    pcs = [binding.PolarCode(n, k, 16, 2.0) for (n, k) in codes]
    shapes = [(n, k - 16) for (n, k) in codes]
    # the mixed batch's sustained rate: one persistent launch over an i.i.d. batch
    stream = torch.cuda.Stream(device=dev)
    Bm = args.serve_rate_frames
    frames, llr, _, _, _, kpf = mixed_batch(torch, dev, Bm, 44, pcs, codes, stream)
    ctx = binding.ScsContext(0)
    if tune.apply_mixed(ctx, pcs, frames) is None:
        ctx.configure(4)
    pay = torch.empty(int(kpf.sum()), dtype=torch.uint8, device=dev)
    st = torch.empty(Bm, dtype=torch.uint8, device=dev)
    binding.scs_mixed_prepare(ctx.handle, [p.handle for p in pcs], frames, stream)
    ms = []
    for r in range(4):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        binding.scs_mixed_launch(ctx.handle, binding.SCS_LLR_F32, llr, pay, st, None, stream)
        b.record(stream)
        stream.synchronize()
        if r:
            ms.append(a.elapsed_time(b))
    c4_fps = Bm / (np.mean(ms) * 1e-3)
    del llr, pay, st
    ctx.close()
    log("serve: mixed-batch sustained rate %.0f frames/s (%d frames, %.1f ms per launch)"
        % (c4_fps, Bm, np.mean(ms)))
    pool = serve_pool(5, args.serve_pool, codes, pcs, on_device=True)
    pool_frames = sum(r.frames for r in pool)
    log("serve: pool of %d device-resident requests (%d frames) ready" % (len(pool), pool_frames))
    be = GpuBackend(pcs, n_slots=4, max_frames=16384, host_inputs=False)
    # saturated capacity of the server: the whole pool submitted at once, six times
    srv = Server(be, shapes, budget_bytes=SERVE_BUDGET, max_batch_frames=16384, keep_completed=False)
    t0 = time.perf_counter()
    for rep_ in range(6):
        for r in pool:
            srv.submit(copy.copy(r))
    srv.drain()
    cap_fps = 6 * pool_frames / (time.perf_counter() - t0)
    log("serve: saturated server capacity %.0f frames/s" % cap_fps)
    # Poisson arrivals at the offered load for the run time
    rng = np.random.default_rng(6)
    mean_frames = pool_frames / len(pool)
    offered_fps = args.serve_load * c4_fps
    rate = offered_fps / mean_frames  # requests per second
    arrivals, t, k = [], 0.0, 0
    while t < args.serve_seconds:
        t += float(rng.exponential(1.0 / rate))
        r = copy.copy(pool[int(rng.integers(len(pool)))])
        r.rid = k
        arrivals.append((t, r))
        k += 1
    srv = Server(be, shapes, budget_bytes=SERVE_BUDGET, max_batch_frames=16384, keep_completed=False)
    log("serve: replaying %d requests over %.0f s (%.0f frames/s offered)"
        % (len(arrivals), args.serve_seconds, offered_fps))
    # The million pre-generated requests would make every full collection of Python's cyclic
    # garbage collector walk them all (pauses of a large fraction of a second, which queue
    # up requests); the server makes no reference cycles, so the collector is parked for
    # the run and the objects that exist now are frozen out of its view.
    gc.collect()
    gc.freeze()
    gc.disable()
    try:
        rep = srv.run(arrivals, progress=lambda msg: log("serve: " + msg))
    finally:
        gc.enable()
        gc.unfreeze()
    line = {
        "metric": "p50/p99 request latency and sustained info Mbit/s, continuous-batching server",
        "value": rep["payload_mbps"], "unit": "Mbit/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": rep["span_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded BPSK/AWGN requests of the mixed distribution, LLRs on the device",
        "config": {"workload": "serving: Poisson requests of 1-256 frames, mixed codes/D, "
                               "4 slots sharing the GPU, 16 GiB budget, device-resident LLRs",
                   "offered_load": args.serve_load,
                   "mixed_batch_frames_per_s": c4_fps,
                   "offered_frames_per_s": offered_fps,
                   "server_capacity_frames_per_s": cap_fps,
                   "requests": len(arrivals), "seconds": args.serve_seconds},
        "latency_ms": {"p50": rep["latency_ms_p50"], "p99": rep["latency_ms_p99"],
                       "mean": rep["latency_ms_mean"]},
        "sustained_frames_per_s": rep["frames"] / rep["span_s"],
        "batches": rep["batches"], "max_concurrent_batches": be.max_concurrent,
        "host_submit_ms_per_batch": rep["host_submit_ms_per_batch"],
        "budget_bytes": rep["budget_bytes"], "peak_budget_bytes": rep["peak_budget_bytes"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
