"""Mixed batches (frames of 25 codes, N 128..2048, rates 1/4..5/6, D in {8, 32, 64},
CRC-16, Eb/N0 uniform in [1.5, 3.5]) in one persistent launch: every frame equals the
oracle and equals its own one-launch-per-configuration result; a captured graph of the
prepared launch replays to the same bytes."""
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


def build_mixed(B, seed, L=8, crc=16):
    """Frames of the mixed workload encoded by the oracle; returns the per-frame
    descriptors, one flat LLR array, per-frame reference payloads and oracle results."""
    from paper_1809_03606_amd.binding import FRAME_DTYPE

    codes = channel.mixed_codes()
    cidx, D, eb = channel.mixed_draw(seed, B)
    infos = [oracle.construct(N, K, 2.0) for (N, K) in codes]
    frames = np.zeros(B, FRAME_DTYPE)
    llr_parts, off, out_off = [], 0, 0
    want = {}
    per = [None] * B
    for c in range(len(codes)):
        idx = np.nonzero(cidx == c)[0]
        if idx.size == 0:
            continue
        N, K = codes[c]
        pay = channel.payload_bits(seed, 1000 + c, 0, idx.size, K - crc)
        nz = channel.noise(seed, 2000 + c, 0, idx.size, N)
        cw = oracle.encode_batch(infos[c], crc, pay)
        for j, f in enumerate(idx):
            per[f] = (c, pay[j], channel.bpsk_awgn_llr(cw[j:j + 1], nz[j:j + 1], eb[f], K / N)[0])
    llr = []
    for f in range(B):
        c, pay, l = per[f]
        N, K = codes[c]
        frames[f] = (c, D[f], L, 0, off, out_off)
        llr.append(l)
        off += N
        out_off += K - crc
    flat = np.concatenate(llr).astype(np.float32)
    # the oracle, frame by frame
    ref_pay, ref_st, ref_stats = [], np.zeros(B, np.uint8), []
    for c in range(len(codes)):
        idx = np.nonzero(frames["code"] == c)[0]
        for d in np.unique(frames["D"][idx]):
            sel = idx[frames["D"][idx] == d]
            x = np.stack([per[f][2] for f in sel])
            p, s, st = oracle.scs_decode_batch(oracle.F32, infos[c], crc, int(d), L, x, threads=THREADS)
            for j, f in enumerate(sel):
                want[f] = (p[j], s[j], st[j])
    return codes, frames, flat, per, want, out_off


def _gpu_mixed(cuda, codes_h, frames, flat, total_out, stats=True, ctx=None):
    from paper_1809_03606_amd import binding

    dev = "cuda"
    x = cuda.from_numpy(flat).to(dev)
    pay = cuda.full((max(total_out, 1),), 0xEE, dtype=cuda.uint8, device=dev)
    st = cuda.full((len(frames),), 0xEE, dtype=cuda.uint8, device=dev)
    sts = cuda.zeros((len(frames), 8), dtype=cuda.int32, device=dev) if stats else None
    own = ctx is None
    if own:
        ctx = binding.ScsContext(0)
    binding.scs_decode_mixed(ctx.handle, codes_h, frames, binding.SCS_LLR_F32, x, pay, st, sts)
    cuda.cuda.synchronize()
    return pay.cpu().numpy(), st.cpu().numpy(), (sts.cpu().numpy().view(np.uint32) if stats else None)


def test_gpu_mixed_batch_matches_oracle_and_uniform_launches(cuda):
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import PolarCode

    B = 1500
    codes, frames, flat, per, want, total_out = build_mixed(B, seed=4)
    pcs = [PolarCode(N, K, 16, 2.0) for (N, K) in codes]
    _say("gpu: mixed batch of %d frames" % B)
    pay, st, stats = _gpu_mixed(cuda, [p.handle for p in pcs], frames, flat, total_out)
    fields = binding.STATS_FIELDS
    for f in range(B):
        c = frames["code"][f]
        kp = codes[c][1] - 16
        o = frames["out_off"][f]
        rp, rs, rstat = want[f]
        assert (pay[o:o + kp] == rp).all() and st[f] == rs, "frame %d (code %d)" % (f, c)
        for name in ("iterations", "switches", "completions", "evictions", "drops", "prunes"):
            assert stats[f, fields.index(name)] == rstat[name], (f, name)
    # the same frames, one launch per (code, D)
    ctx = binding.ScsContext(0)
    for c in range(len(codes)):
        idx = np.nonzero(frames["code"] == c)[0]
        for d in np.unique(frames["D"][idx]):
            sel = idx[frames["D"][idx] == d]
            x = cuda.from_numpy(np.stack([per[f][2] for f in sel])).cuda()
            kp = codes[c][1] - 16
            p = cuda.zeros((sel.size, kp), dtype=cuda.uint8, device="cuda")
            s = cuda.zeros((sel.size,), dtype=cuda.uint8, device="cuda")
            ctx.decode(pcs[c], int(d), 8, x, p, s)
            cuda.cuda.synchronize()
            p, s = p.cpu().numpy(), s.cpu().numpy()
            for j, f in enumerate(sel):
                o = frames["out_off"][f]
                assert (pay[o:o + kp] == p[j]).all() and st[f] == s[j]


def test_gpu_mixed_graph_replay(cuda):
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import PolarCode

    B = 400
    codes, frames, flat, per, want, total_out = build_mixed(B, seed=44)
    pcs = [PolarCode(N, K, 16, 2.0) for (N, K) in codes]
    handles = [p.handle for p in pcs]
    ctx = binding.ScsContext(0)
    x = cuda.from_numpy(flat).cuda()
    pay = cuda.zeros((total_out,), dtype=cuda.uint8, device="cuda")
    st = cuda.zeros((B,), dtype=cuda.uint8, device="cuda")
    stream = cuda.cuda.Stream()
    binding.scs_mixed_prepare(ctx.handle, handles, frames, stream)
    stream.synchronize()
    _say("gpu: mixed eager launch")
    binding.scs_mixed_launch(ctx.handle, binding.SCS_LLR_F32, x, pay, st, None, stream)
    stream.synchronize()
    eager_pay, eager_st = pay.cpu().numpy().copy(), st.cpu().numpy().copy()
    for f in range(B):
        c = frames["code"][f]
        kp = codes[c][1] - 16
        o = frames["out_off"][f]
        assert (eager_pay[o:o + kp] == want[f][0]).all() and eager_st[f] == want[f][1]
    g = cuda.cuda.CUDAGraph()
    with cuda.cuda.graph(g, stream=stream):
        binding.scs_mixed_launch(ctx.handle, binding.SCS_LLR_F32, x, pay, st, None,
                                 cuda.cuda.current_stream())
    for rep in range(3):
        pay.fill_(0xEE)
        st.fill_(0xEE)
        cuda.cuda.synchronize()
        _say("gpu: graph replay %d" % rep)
        g.replay()
        cuda.cuda.synchronize()
        assert (pay.cpu().numpy() == eager_pay).all() and (st.cpu().numpy() == eager_st).all()
        # eager work of the program between replays
        ctx.decode(pcs[0], 8, 8, cuda.zeros((3, codes[0][0]), device="cuda"),
                   cuda.zeros((3, codes[0][1] - 16), dtype=cuda.uint8, device="cuda"),
                   cuda.zeros((3,), dtype=cuda.uint8, device="cuda"))
        cuda.cuda.synchronize()


def test_gpu_mixed_rejects_bad_descriptors(cuda):
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import FRAME_DTYPE, PolarCode

    pc = PolarCode(128, 64, 16)
    ctx = binding.ScsContext(0)
    x = cuda.zeros((256,), device="cuda")
    pay = cuda.zeros((128,), dtype=cuda.uint8, device="cuda")
    st = cuda.zeros((2,), dtype=cuda.uint8, device="cuda")
    good = np.zeros(2, FRAME_DTYPE)
    good[1]["llr_off"] = 128
    good["D"], good["L"] = 8, 8
    for field, val in [("code", 1), ("code", -1), ("D", 0), ("D", 65), ("L", 0), ("L", 256),
                       ("_pad", 1), ("llr_off", -1), ("out_off", -5)]:
        bad = good.copy()
        bad[1][field] = val
        with pytest.raises(binding.PolarError) as e:
            binding.scs_decode_mixed(ctx.handle, [pc.handle], bad, binding.SCS_LLR_F32, x, pay, st)
        assert e.value.code == binding.POLAR_EINVAL, field
    binding.scs_decode_mixed(ctx.handle, [pc.handle], good, binding.SCS_LLR_F32, x, pay, st)
    cuda.cuda.synchronize()
    assert binding.scs_ctx_last_error(ctx.handle) == 0


@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_gpu_mixed_every_workgroup_size_matches_oracle(cuda, wpb):
    """Every launch shape the mixed-plan tuner can choose gives the oracle's bits."""
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import PolarCode

    B = 500
    codes, frames, flat, per, want, total_out = build_mixed(B, seed=50 + wpb)
    pcs = [PolarCode(N, K, 16, 2.0) for (N, K) in codes]
    ctx = binding.ScsContext(0, wpb)
    _say("gpu: mixed batch at %d wavefronts per workgroup" % wpb)
    pay, st, stats = _gpu_mixed(cuda, [p.handle for p in pcs], frames, flat, total_out, ctx=ctx)
    for f in range(B):
        c = frames["code"][f]
        kp = codes[c][1] - 16
        o = frames["out_off"][f]
        assert (pay[o:o + kp] == want[f][0]).all() and st[f] == want[f][1], (wpb, f)


@pytest.mark.parametrize("grid_cus", [1, 37, 0])
def test_gpu_mixed_grid_share_matches_oracle(cuda, grid_cus):
    """A persistent launch confined to a part of the CUs (scs_ctx_set_grid_cus, as the
    serving slots use it) gives the oracle's bits; out-of-range settings are refused."""
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import PolarCode, PolarError

    B = 400
    codes, frames, flat, per, want, total_out = build_mixed(B, seed=70 + grid_cus)
    pcs = [PolarCode(N, K, 16, 2.0) for (N, K) in codes]
    ctx = binding.ScsContext(0)
    cus = cuda.cuda.get_device_properties(0).multi_processor_count
    for bad in (-1, cus + 1):
        with pytest.raises(PolarError):
            ctx.set_grid_cus(bad)
    ctx.set_grid_cus(grid_cus)
    _say("gpu: mixed batch on %d CUs' worth of workgroups" % grid_cus)
    pay, st, stats = _gpu_mixed(cuda, [p.handle for p in pcs], frames, flat, total_out, ctx=ctx)
    for f in range(B):
        c = frames["code"][f]
        kp = codes[c][1] - 16
        o = frames["out_off"][f]
        assert (pay[o:o + kp] == want[f][0]).all() and st[f] == want[f][1], (grid_cus, f)


def test_gpu_mixed_plan_tuner(cuda, tmp_path):
    """tune_mixed times the persistent launch at every workgroup size on the caller's plan,
    checks the bytes agree, stores the fastest under the plan's key and applies it."""
    from paper_1809_03606_amd import binding, tune
    from paper_1809_03606_amd.binding import PolarCode

    B = 2000
    codes, frames, flat, per, want, total_out = build_mixed(B, seed=57)
    pcs = [PolarCode(N, K, 16, 2.0) for (N, K) in codes]
    ctx = binding.ScsContext(0)
    x = cuda.from_numpy(flat).cuda()
    pay = cuda.zeros((total_out,), dtype=cuda.uint8, device="cuda")
    st = cuda.zeros((B,), dtype=cuda.uint8, device="cuda")
    stream = cuda.cuda.Stream()
    path = str(tmp_path / "tune.json")
    _say("gpu: mixed plan tuner on %d frames" % B)
    entry = tune.tune_mixed(ctx, pcs, frames, x, pay, st, stream, path=path)
    assert set(entry["candidates_ms"]) == {"1", "2", "4"}
    assert entry["waves_per_block"] in (1, 2, 4)
    got = tune.apply_mixed(binding.ScsContext(0), pcs, frames, path=path)
    assert got["waves_per_block"] == entry["waves_per_block"]
    # the context is left with the whole plan prepared at the chosen size
    binding.scs_mixed_launch(ctx.handle, binding.SCS_LLR_F32, x, pay, st, None, stream)
    stream.synchronize()
    p, s = pay.cpu().numpy(), st.cpu().numpy()
    for f in range(B):
        c = frames["code"][f]
        kp = codes[c][1] - 16
        o = frames["out_off"][f]
        assert (p[o:o + kp] == want[f][0]).all() and s[f] == want[f][1], f


def test_gpu_mixed_one_context_two_streams(cuda):
    """Two different plans decoded on one context from two streams with no host
    synchronisation in between: the context orders its own calls, both results are exact."""
    from paper_1809_03606_amd import binding
    from paper_1809_03606_amd.binding import PolarCode

    runs = []
    for seed, B in ((71, 700), (72, 300)):
        codes, frames, flat, per, want, total_out = build_mixed(B, seed=seed)
        runs.append((codes, frames, cuda.from_numpy(flat).cuda(), want, total_out))
    pcs = [PolarCode(N, K, 16, 2.0) for (N, K) in runs[0][0]]
    ctx = binding.ScsContext(0)
    streams = [cuda.cuda.Stream(), cuda.cuda.Stream()]
    outs = [(cuda.full((r[4],), 0xEE, dtype=cuda.uint8, device="cuda"),
             cuda.full((len(r[1]),), 0xEE, dtype=cuda.uint8, device="cuda")) for r in runs]
    cuda.cuda.synchronize()
    _say("gpu: two mixed plans on one context, two streams")
    for (codes, frames, x, want, total_out), s, (pay, st) in zip(runs, streams, outs):
        binding.scs_decode_mixed(ctx.handle, [p.handle for p in pcs], frames,
                                 binding.SCS_LLR_F32, x, pay, st, None, s)
    cuda.cuda.synchronize()
    for (codes, frames, x, want, total_out), (pay, st) in zip(runs, outs):
        p, s_ = pay.cpu().numpy(), st.cpu().numpy()
        for f in range(len(frames)):
            kp = codes[frames["code"][f]][1] - 16
            o = frames["out_off"][f]
            assert (p[o:o + kp] == want[f][0]).all() and s_[f] == want[f][1], f
    assert binding.scs_ctx_last_error(ctx.handle) == 0
