"""Scheduler logic of the decode server, on the CPU with an oracle backend."""
import numpy as np
import pytest

import oracle
from fake_backend import OracleBackend
from paper_1809_03606_amd import channel
from paper_1809_03606_amd.serve import AdmissionError, Request, Server, request_footprint

CODES = [(64, 40), (128, 64), (256, 128)]
CRC = 16


def make_requests(n, seed, max_frames=8):
    rng = np.random.default_rng(seed)
    infos = [oracle.construct(N, K, 2.0) for N, K in CODES]
    reqs = []
    for rid in range(n):
        c = int(rng.integers(len(CODES)))
        N, K = CODES[c]
        m = int(rng.integers(1, max_frames + 1))
        pay = channel.payload_bits(seed, rid, 0, m, K - CRC)
        llr = channel.bpsk_awgn_llr(oracle.encode_batch(infos[c], CRC, pay),
                                    channel.noise(seed, 10_000 + rid, 0, m, N), 2.0, K / N)
        reqs.append(Request(rid=rid, code=c, D=int(rng.choice([4, 16])), L=8, llr=llr))
    return infos, reqs


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4
        return self.t


def test_every_request_completes_with_its_own_result():
    infos, reqs = make_requests(40, seed=3)
    shapes = [(N, K - CRC) for N, K in CODES]
    be = OracleBackend(infos, CRC, n_slots=3)
    srv = Server(be, shapes, budget_bytes=10 ** 9, max_batch_frames=32, clock=FakeClock())
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert len(srv.completed) == 40 and be.max_concurrent >= 2
    for r in reqs:
        alone = oracle.scs_decode_batch(oracle.F32, infos[r.code], CRC, r.D, r.L, r.llr)
        assert (r.payload == alone[0]).all() and (r.status == alone[1]).all()
        assert r.t_done >= r.t_admit >= r.t_arrival


def test_budget_is_respected_and_fifo_kept():
    infos, reqs = make_requests(30, seed=4)
    shapes = [(N, K - CRC) for N, K in CODES]
    biggest = max(request_footprint(CODES[r.code][0], CODES[r.code][1] - CRC, r.D, r.frames) for r in reqs)
    budget = 2 * biggest
    be = OracleBackend(infos, CRC, n_slots=4)
    srv = Server(be, shapes, budget_bytes=budget, max_batch_frames=64, clock=FakeClock())
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert srv.peak_in_use <= budget
    assert srv.in_use == 0
    admits = [r.t_admit for r in sorted(reqs, key=lambda r: r.rid)]
    assert admits == sorted(admits)  # admission in arrival order


def test_over_budget_request_is_rejected_and_cancel_works():
    infos, reqs = make_requests(3, seed=5)
    shapes = [(N, K - CRC) for N, K in CODES]
    srv = Server(OracleBackend(infos, CRC), shapes, budget_bytes=1000, clock=FakeClock())
    with pytest.raises(AdmissionError):
        srv.submit(reqs[0])
    srv2 = Server(OracleBackend(infos, CRC, n_slots=1), shapes, budget_bytes=10 ** 9, clock=FakeClock())
    for r in reqs:
        srv2.submit(r)
    assert srv2.cancel(reqs[2].rid) and not srv2.cancel(999)
    srv2.drain()
    assert sorted(r.rid for r in srv2.completed) == [reqs[0].rid, reqs[1].rid]


def test_long_running_server_keeps_totals_not_requests():
    """keep_completed=False: finished requests go to the callback only; the report comes from
    running totals and equals the one a keeping server gives on the same requests."""
    infos, reqs = make_requests(25, seed=6)
    shapes = [(N, K - CRC) for N, K in CODES]
    got = []
    reps = []
    for keep in (True, False):
        be = OracleBackend(infos, CRC, n_slots=2)
        srv = Server(be, shapes, budget_bytes=10 ** 9, max_batch_frames=16, clock=FakeClock(),
                     keep_completed=keep, on_complete=None if keep else got.append)
        for r in reqs:
            srv.submit(r)
        srv.drain()
        assert len(srv.completed) == (25 if keep else 0)
        reps.append(srv.report())
    assert sorted(r.rid for r in got) == list(range(25))
    a, b = reps
    assert a["requests"] == b["requests"] == 25 and a["frames"] == b["frames"] == sum(r.frames for r in reqs)
    assert b["payload_mbps"] > 0 and b["latency_ms_p99"] >= b["latency_ms_p50"] > 0


def test_progress_counts_completions_without_keeping_them():
    """The progress line of run() counts finished requests from the running totals, so a
    long-running server (keep_completed=False) reports them too."""
    infos, reqs = make_requests(12, seed=8)
    shapes = [(N, K - CRC) for N, K in CODES]
    be = OracleBackend(infos, CRC, n_slots=2)
    srv = Server(be, shapes, budget_bytes=10 ** 9, max_batch_frames=16, clock=FakeClock(),
                 keep_completed=False, on_complete=lambda r: None)
    msgs = []
    srv.run([(0.0, r) for r in reqs], poll_s=0.0, progress=msgs.append, every_s=2e-4)
    done = [int(m.split(" arrived, ")[1].split(" completed")[0]) for m in msgs]
    assert done and max(done) > 0 and srv.report()["requests"] == 12
