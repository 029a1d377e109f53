"""The continuous-batching server on the GPU: requests of mixed codes arriving while
others decode are admitted as slots and budget free up, batches overlap on the device, and
every request's result is the same as decoding it alone (and as the oracle)."""
import sys

import numpy as np
import pytest

import oracle
from cases import THREADS
from paper_1809_03606_amd import channel

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_gpu_server_results_alone_equal_results_in_the_mix(cuda):
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.serve import GpuBackend, Request, Server

    rng = np.random.default_rng(5)
    allc = channel.mixed_codes()
    pick = [0, 7, 12, 16, 23]  # N 128 .. 2048, several rates
    codes = [allc[c] for c in pick]
    pcs = [binding.PolarCode(N, K, 16, 2.0) for N, K in codes]
    infos = [oracle.construct(N, K, 2.0) for N, K in codes]
    reqs, t = [], 0.0
    arrivals = []
    for rid in range(160):
        c = int(rng.integers(len(codes)))
        N, K = codes[c]
        m = int(rng.integers(1, 65))
        pay = channel.payload_bits(5, rid, 0, m, K - 16)
        llr = channel.bpsk_awgn_llr(oracle.encode_batch(infos[c], 16, pay),
                                    channel.noise(5, 50_000 + rid, 0, m, N), float(rng.uniform(1.5, 3.5)), K / N)
        r = Request(rid=rid, code=c, D=int(rng.choice([8, 32, 64])), L=8, llr=llr)
        reqs.append(r)
        t += float(rng.exponential(0.0004))
        arrivals.append((t, r))
    be = GpuBackend(pcs, n_slots=4, max_frames=1024)
    shapes = [(N, K - 16) for N, K in codes]
    srv = Server(be, shapes, budget_bytes=48 << 20, max_batch_frames=1024)
    _say("gpu: serving %d requests" % len(reqs))
    rep = srv.run(arrivals)
    assert rep["requests"] == len(reqs)
    assert be.max_concurrent >= 2, "batches never overlapped"
    assert srv.peak_in_use <= srv.budget and srv.in_use == 0
    ctx = binding.ScsContext(0)
    for r in reqs:
        x = cuda.from_numpy(r.llr).cuda()
        kp = shapes[r.code][1]
        p = cuda.zeros((r.frames, kp), dtype=cuda.uint8, device="cuda")
        s = cuda.zeros((r.frames,), dtype=cuda.uint8, device="cuda")
        ctx.decode(pcs[r.code], r.D, r.L, x, p, s)
        cuda.cuda.synchronize()
        assert (p.cpu().numpy() == r.payload).all() and (s.cpu().numpy() == r.status).all(), r.rid
    for r in reqs[::16]:
        rp, rs, _ = oracle.scs_decode_batch(oracle.F32, infos[r.code], 16, r.D, r.L, r.llr, threads=THREADS)
        assert (rp == r.payload).all() and (rs == r.status).all(), r.rid
    _say("served: %s" % rep)


def test_gpu_server_device_resident_requests(cuda):
    """Requests whose LLRs are already on the device (no staging copy): the batch's
    descriptors point at each request's own tensor; every result equals the request decoded
    alone and the oracle."""
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.serve import GpuBackend, Request, Server

    rng = np.random.default_rng(8)
    allc = channel.mixed_codes()
    pick = [2, 8, 13, 19, 24]
    codes = [allc[c] for c in pick]
    pcs = [binding.PolarCode(N, K, 16, 2.0) for N, K in codes]
    infos = [oracle.construct(N, K, 2.0) for N, K in codes]
    arrivals, t, host = [], 0.0, {}
    for rid in range(200):
        c = int(rng.integers(len(codes)))
        N, K = codes[c]
        m = int(rng.integers(1, 97))
        pay = channel.payload_bits(8, rid, 0, m, K - 16)
        llr = channel.bpsk_awgn_llr(oracle.encode_batch(infos[c], 16, pay),
                                    channel.noise(8, 70_000 + rid, 0, m, N),
                                    float(rng.uniform(1.5, 3.5)), K / N)
        host[rid] = llr
        r = Request(rid=rid, code=c, D=int(rng.choice([8, 32, 64])), L=8,
                    llr=cuda.from_numpy(llr).cuda())
        t += float(rng.exponential(0.0003))
        arrivals.append((t, r))
    cuda.cuda.synchronize()
    be = GpuBackend(pcs, n_slots=4, max_frames=2048, host_inputs=False)
    shapes = [(N, K - 16) for N, K in codes]
    srv = Server(be, shapes, budget_bytes=64 << 20, max_batch_frames=2048)
    _say("gpu: serving %d device-resident requests" % len(arrivals))
    rep = srv.run(arrivals)
    assert rep["requests"] == len(arrivals) and be.max_concurrent >= 2
    ctx = binding.ScsContext(0)
    for _, r in arrivals:
        kp = shapes[r.code][1]
        p = cuda.zeros((r.frames, kp), dtype=cuda.uint8, device="cuda")
        s = cuda.zeros((r.frames,), dtype=cuda.uint8, device="cuda")
        ctx.decode(pcs[r.code], r.D, r.L, r.llr, p, s)
        cuda.cuda.synchronize()
        assert (p.cpu().numpy() == r.payload).all() and (s.cpu().numpy() == r.status).all(), r.rid
    for _, r in arrivals[::20]:
        rp, rs, _ = oracle.scs_decode_batch(oracle.F32, infos[r.code], 16, r.D, r.L, host[r.rid],
                                            threads=THREADS)
        assert (rp == r.payload).all() and (rs == r.status).all(), r.rid
