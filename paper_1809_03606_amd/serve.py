"""Continuous-batching decode server over the C-ABI.

Requests (one code, one D and L, 1..256 frames each) arrive over time.  The server keeps a
FIFO of waiting requests and several device slots (one HIP stream and one decoder context
each).  Whenever a slot is free it admits waiting requests, oldest first, while their
device footprint fits the free part of the memory budget, and enqueues one mixed-batch
decode (``scs_decode_mixed``) of all their frames; the results are copied back once the
batch is done.  Batches of different slots run concurrently on the GPU.  A request's LLRs are either in host memory
(packed into the slot's pinned staging buffer and copied to the device with the batch) or
already on the device (a CUDA tensor, for example written there by a demodulator): then the
batch's descriptors point at them where they are and nothing is copied in.  A request that arrives while others are decoding joins the next
free slot: slots and budget are released as batches finish.

Footprint of a request (bytes of device memory its frames hold while in flight): LLRs
(4 N per frame), payload and status bytes, and the decoder's per-frame LDS state.  A
request larger than the whole budget is rejected at submission.

The backend interface (``submit`` / ``done`` / ``collect`` / ``free_slots``) is what the
scheduler talks to, so the scheduling logic can be exercised with any object that
implements it.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import binding


def frame_state_bytes(N: int, D: int) -> int:
    """On-chip decoder state of one frame (stack rows, L counters, alpha tree, spare)."""
    W = N // 32 if N >= 32 else 1
    return 4 * (D * W + (N + 3) // 4 + N + 64)


def request_footprint(N: int, kp: int, D: int, frames: int) -> int:
    return frames * (4 * N + kp + 1 + frame_state_bytes(N, D))


@dataclasses.dataclass
class Request:
    rid: int
    code: int            # index into the server's code list
    D: int
    L: int
    llr: object          # float32 [frames][N]: numpy array, or CUDA tensor on the device
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    payload: np.ndarray | None = None  # uint8 [frames][kp]
    status: np.ndarray | None = None   # uint8 [frames]
    footprint: int = 0

    @property
    def frames(self) -> int:
        return int(self.llr.shape[0])


class AdmissionError(ValueError):
    pass


class GpuBackend:
    """Device slots: a stream, a decoder context, output buffers and (host_inputs) pinned
    staging buffers for requests whose LLRs are in host memory.  Requests with device LLRs
    must have them written (and the writing stream synchronised) before submission."""

    def __init__(self, codes, n_slots: int = 4, max_frames: int = 4096, device: int = 0,
                 host_inputs: bool = True, share_gpu: bool = True):
        """share_gpu: each slot's launches take 1 / n_slots of the CUs, so that the slots'
        batches run side by side instead of one batch's last frames holding up the next.
        Side by side needs a hardware queue per slot stream: HIP shares its queues
        (GPU_MAX_HW_QUEUES, 4 by default) among all streams of the process, and launches in
        one queue run one after another, so the process should allow n_slots + 2 or more."""
        import torch

        self.torch = torch
        self.codes = codes  # list of binding.PolarCode
        self.Ns = np.array([c.N for c in codes], np.int64)
        self.kps = np.array([c.payload_bits for c in codes], np.int64)
        self.handles = [c.handle for c in codes]
        self.dev = torch.device("cuda", device)
        maxN = max(c.N for c in codes)
        maxkp = max(c.payload_bits for c in codes)
        self.max_frames = max_frames
        self.max_concurrent = 0  # most batches seen in flight at once
        self.slots = []
        stage = max_frames * maxN if host_inputs else 0
        cus = torch.cuda.get_device_properties(self.dev).multi_processor_count
        share = max(1, cus // n_slots) if share_gpu and n_slots > 1 else 0
        for _ in range(n_slots):
            s = {
                "stream": torch.cuda.Stream(device=self.dev),
                "ctx": binding.ScsContext(device),
                "h_llr": torch.empty(stage, dtype=torch.float32, pin_memory=True),
                "d_llr": torch.empty(stage, dtype=torch.float32, device=self.dev),
                "d_pay": torch.empty(max_frames * maxkp, dtype=torch.uint8, device=self.dev),
                "d_st": torch.empty(max_frames, dtype=torch.uint8, device=self.dev),
                "h_pay": torch.empty(max_frames * maxkp, dtype=torch.uint8, pin_memory=True),
                "h_st": torch.empty(max_frames, dtype=torch.uint8, pin_memory=True),
                "event": None, "batch": None, "busy": False,
            }
            if share:
                s["ctx"].set_grid_cus(share)
            # size the context's plan buffers once, so that no submission has to grow them
            big = max(range(len(codes)), key=lambda c: codes[c].N)
            plan = np.zeros(max_frames, binding.FRAME_DTYPE)
            plan["code"], plan["D"], plan["L"] = big, 1, 1
            binding.scs_mixed_prepare(s["ctx"].handle, [c.handle for c in codes], plan, s["stream"])
            s["stream"].synchronize()
            self.slots.append(s)

    def free_slots(self):
        return [i for i, s in enumerate(self.slots) if not s["busy"]]

    def submit(self, slot: int, reqs):
        torch = self.torch
        s = self.slots[slot]
        nr = len(reqs)
        m = np.fromiter((r.frames for r in reqs), np.int64, nr)
        n = int(m.sum())
        if n > self.max_frames:
            raise AdmissionError("batch of %d frames exceeds the slot size %d" % (n, self.max_frames))
        code = np.fromiter((r.code for r in reqs), np.int64, nr)
        Nr, kpr = self.Ns[code], self.kps[code]
        first = np.cumsum(m) - m                          # first frame of each request
        j = np.arange(n, dtype=np.int64) - np.repeat(first, m)  # frame within its request
        frames = np.zeros(n, binding.FRAME_DTYPE)
        frames["code"] = np.repeat(code, m)
        frames["D"] = np.repeat(np.fromiter((r.D for r in reqs), np.int64, nr), m)
        frames["L"] = np.repeat(np.fromiter((r.L for r in reqs), np.int64, nr), m)
        out0 = np.cumsum(m * kpr) - m * kpr
        frames["out_off"] = np.repeat(out0, m) + j * np.repeat(kpr, m)
        lo_o = int((m * kpr).sum())
        on_device = [getattr(r.llr, "is_cuda", False) for r in reqs]
        st = s["stream"]
        if all(on_device):
            # descriptors point at the requests' own device LLRs, relative to the lowest
            ptrs = np.fromiter((r.llr.data_ptr() for r in reqs), np.int64, nr)
            base = int(ptrs.min())
            if ((ptrs - base) % 4).any():
                raise AdmissionError("device LLRs must be 4-byte aligned float32")
            frames["llr_off"] = np.repeat((ptrs - base) // 4, m) + j * np.repeat(Nr, m)
            llr_arg = base
        elif not any(on_device):
            if s["h_llr"].numel() == 0:
                raise AdmissionError("this backend takes device LLRs only (host_inputs=False)")
            hl = s["h_llr"].numpy()
            l0 = np.cumsum(m * Nr) - m * Nr
            for r, a in zip(reqs, l0):
                hl[a:a + r.llr.size] = r.llr.reshape(-1)
            lo = int((m * Nr).sum())
            frames["llr_off"] = np.repeat(l0, m) + j * np.repeat(Nr, m)
            with torch.cuda.stream(st):
                s["d_llr"][:lo].copy_(s["h_llr"][:lo], non_blocking=True)
            llr_arg = s["d_llr"]
        else:
            raise AdmissionError("a batch holds requests with host and with device LLRs")
        spans = list(zip(first.tolist(), out0.tolist(), m.tolist(), kpr.tolist()))
        with torch.cuda.stream(st):
            binding.scs_decode_mixed(s["ctx"].handle, self.handles, frames, binding.SCS_LLR_F32,
                                     llr_arg, s["d_pay"], s["d_st"], None, st)
            ev = torch.cuda.Event()
            ev.record(st)
        # The results are copied back in collect(), once the batch is done: an asynchronous
        # device-to-host copy enqueued here was measured to hold back the other slots'
        # launches until this batch had finished, serialising the slots.
        s.update(event=ev, batch=(reqs, spans, lo_o, n), busy=True)
        self.max_concurrent = max(self.max_concurrent, sum(x["busy"] for x in self.slots))

    def done(self, slot: int) -> bool:
        s = self.slots[slot]
        return s["busy"] and s["event"].query()

    def collect(self, slot: int):
        s = self.slots[slot]
        reqs, spans, lo_o, n = s["batch"]
        with self.torch.cuda.stream(s["stream"]):  # the batch is done: these return at once
            s["h_pay"][:lo_o].copy_(s["d_pay"][:lo_o])
            s["h_st"][:n].copy_(s["d_st"][:n])
        hp, hs = s["h_pay"].numpy(), s["h_st"].numpy()
        for r, (f, lo_o, m, kp) in zip(reqs, spans):
            r.payload = hp[lo_o:lo_o + m * kp].reshape(m, kp).copy()
            r.status = hs[f:f + m].copy()
        s.update(event=None, batch=None, busy=False)
        return reqs


class Server:
    """FIFO admission under a device-memory budget, continuous batching over the slots."""

    def __init__(self, backend, code_shapes, budget_bytes: int = 512 << 20,
                 max_batch_frames: int = 4096, clock=time.perf_counter,
                 keep_completed: bool = True, on_complete=None):
        """keep_completed: finished requests are appended to `completed` (a long-running
        server passes False and takes them through `on_complete(request)` instead, so that
        it holds nothing per finished request beyond its latency)."""
        self.backend = backend
        self.shapes = code_shapes  # list of (N, kp)
        self.budget = int(budget_bytes)
        self.max_batch_frames = int(max_batch_frames)
        self.clock = clock
        self.keep_completed = keep_completed
        self.on_complete = on_complete
        self.waiting = collections.deque()
        self.in_use = 0
        self.peak_in_use = 0
        self.completed = []
        self.batches = 0
        # running totals of the finished requests, for report()
        self.latencies = []  # seconds, arrival to completion
        self.done_frames = 0
        self.done_bits = 0
        self.t_first = float("inf")
        self.t_last = float("-inf")
        self.submit_s = 0.0  # host time spent handing batches to the backend

    def footprint(self, r: Request) -> int:
        N, kp = self.shapes[r.code]
        return request_footprint(N, kp, r.D, r.frames)

    def submit(self, r: Request, now: float | None = None):
        r.footprint = self.footprint(r)
        if r.footprint > self.budget or r.frames > self.max_batch_frames:
            raise AdmissionError("request %d needs %d bytes / %d frames, budget %d bytes / %d frames"
                                 % (r.rid, r.footprint, r.frames, self.budget, self.max_batch_frames))
        r.t_arrival = self.clock() if now is None else now
        self.waiting.append(r)

    def cancel(self, rid: int) -> bool:
        """Drop a request that is still waiting; a request already on the device finishes."""
        for r in list(self.waiting):
            if r.rid == rid:
                self.waiting.remove(r)
                return True
        return False

    def step(self) -> int:
        """Retire finished batches, then admit waiting requests into free slots.  Returns the
        number of requests completed by this call."""
        now = self.clock()
        finished = 0
        for slot in range(len(self.backend.slots)):
            if self.backend.done(slot):
                for r in self.backend.collect(slot):
                    r.t_done = now
                    self.in_use -= r.footprint
                    self.latencies.append(now - r.t_arrival)
                    self.done_frames += r.frames
                    self.done_bits += r.frames * self.shapes[r.code][1]
                    self.t_first = min(self.t_first, r.t_arrival)
                    self.t_last = max(self.t_last, now)
                    if self.keep_completed:
                        self.completed.append(r)
                    if self.on_complete is not None:
                        self.on_complete(r)
                    finished += 1
        for slot in self.backend.free_slots():
            if not self.waiting:
                break
            batch, frames, need = [], 0, 0
            while self.waiting:
                r = self.waiting[0]
                if self.in_use + need + r.footprint > self.budget:
                    break
                if frames + r.frames > self.max_batch_frames:
                    break
                batch.append(self.waiting.popleft())
                frames += r.frames
                need += r.footprint
            if not batch:
                break
            for r in batch:
                r.t_admit = now
            self.in_use += need
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            t_sub = time.perf_counter()
            self.backend.submit(slot, batch)
            self.submit_s += time.perf_counter() - t_sub
            self.batches += 1
        return finished

    def busy(self) -> bool:
        return bool(self.waiting) or any(s["busy"] for s in self.backend.slots)

    def drain(self, timeout_s: float = 120.0):
        t0 = self.clock()
        while self.busy():
            if self.clock() - t0 > timeout_s:
                raise TimeoutError("server did not drain in %.0f s" % timeout_s)
            if self.step() == 0:
                time.sleep(0.0002)

    def run(self, arrivals, poll_s: float = 0.0002, progress=None, every_s: float = 10.0):
        """arrivals: list of (offset_seconds, Request), ascending offsets.  Replays them in
        real time against the backend and drains the server; `progress(text)` is called
        about every `every_s` seconds."""
        t0 = self.clock()
        k = 0
        next_report = every_s
        while k < len(arrivals) or self.busy():
            now = self.clock() - t0
            while k < len(arrivals) and arrivals[k][0] <= now:
                self.submit(arrivals[k][1], now=t0 + arrivals[k][0])
                k += 1
            if progress is not None and now >= next_report:
                progress("%.0f s: %d arrived, %d completed, %d waiting, %d batches"
                         % (now, k, len(self.latencies), len(self.waiting), self.batches))
                next_report += every_s
            if self.step() == 0:
                time.sleep(poll_s)
        return self.report()

    def report(self):
        lat = np.asarray(self.latencies)
        if lat.size == 0:
            return {"requests": 0}
        span = self.t_last - self.t_first
        return {"requests": int(lat.size), "frames": self.done_frames, "batches": self.batches,
                "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
                "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
                "latency_ms_mean": float(lat.mean() * 1e3),
                "payload_mbps": self.done_bits / max(span, 1e-9) / 1e6,
                "span_s": span, "peak_budget_bytes": self.peak_in_use,
                "budget_bytes": self.budget,
                "host_submit_ms_per_batch": 1e3 * self.submit_s / max(self.batches, 1)}
