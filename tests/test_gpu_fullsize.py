"""Full-size batches in the launch configuration the benchmark times (10^6 frames of
PC(1024,512)+CRC-16, D=32, L=8, one launch; for each of the three decoders), checked on a
sample of frames against the oracle.  The batch is generated on the device; for the sampled frames the payload and the
noise are copied back, encoded with the oracle's encoder and passed through the channel on
the host, and those host LLRs (which must equal the device LLRs bit for bit) are what the
oracle decodes."""
import sys

import numpy as np
import pytest

import oracle
from cases import THREADS
from paper_1809_03606_amd import channel

pytestmark = pytest.mark.gpu

N, K, CRC, D, L = 1024, 512, 16, 32, 8
FRAMES = 1_000_000
SAMPLE = 240


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _full(cuda, ebn0, dtype, seed, decoder="scs", list_size=L):
    from paper_1809_03606_amd import binding

    torch = cuda
    code = binding.PolarCode(N, K, CRC, 2.0)
    info = oracle.construct(N, K, 2.0)
    assert (code.info_mask == info).all()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    kp = K - CRC
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(FRAMES, SAMPLE, replace=False))
    pay = channel.device_payload(torch, gen, FRAMES, kp, "cuda")
    llr = torch.empty((FRAMES, N), dtype=torch.float32 if dtype == "f32" else torch.int8, device="cuda")
    s_noise = np.zeros((SAMPLE, N))
    chunk = 1 << 17
    for lo in range(0, FRAMES, chunk):
        hi = min(FRAMES, lo + chunk)
        cw = torch.empty((hi - lo, N), dtype=torch.uint8, device="cuda")
        code.encode_device(pay[lo:hi], cw)
        nz = channel.device_noise(torch, gen, hi - lo, N, "cuda")
        llr[lo:hi] = channel.device_llr_from_noise(torch, cw, nz, ebn0, K / N, dtype)
        sel = sample[(sample >= lo) & (sample < hi)]
        if sel.size:
            s_noise[np.searchsorted(sample, sel)] = nz[torch.from_numpy(sel - lo).cuda()].cpu().numpy()
        del cw, nz
    out = torch.empty((FRAMES, kp), dtype=torch.uint8, device="cuda")
    st = torch.empty((FRAMES,), dtype=torch.uint8, device="cuda")
    ctx = binding.ScsContext(0)
    # the workgroup size the benchmark applies: the tuner's stored choice, else the library's
    from paper_1809_03606_amd import tune

    entry = tune.apply(ctx, code, D, list_size, dtype, decoder=decoder)
    _say("gpu: full-size %s %s batch at %.1f dB (list %d), %s wavefronts per workgroup"
         % (decoder, dtype, ebn0, list_size, entry["waves_per_block"] if entry else "default"))
    if decoder == "scl":
        ctx.decode_list(code, list_size, llr, out, st)
    else:
        ctx.decode(code, D, L, llr, out, st, fast=decoder == "fsscs")
    torch.cuda.synchronize()
    idx = torch.from_numpy(sample).cuda()
    g_pay, g_st = out[idx].cpu().numpy(), st[idx].cpu().numpy()
    d_llr = llr[idx].cpu().numpy()
    # host reconstruction of the sampled inputs, independent of the library
    s_pay = pay[idx].cpu().numpy()
    cw_h = oracle.encode_batch(info, CRC, s_pay)
    if dtype == "f32":
        h_llr = channel.bpsk_awgn_llr(cw_h, s_noise, ebn0, K / N)
        mode = oracle.F32
    else:
        h_llr = channel.bpsk_awgn_i8(cw_h, s_noise, ebn0, K / N)
        mode = oracle.FIX
    assert np.array_equal(h_llr.view(np.uint8), d_llr.view(np.uint8))
    if decoder == "scl":
        rp, rs, _ = oracle.scl_decode_batch(mode, info, CRC, list_size, h_llr, threads=THREADS)
    elif decoder == "fsscs":
        rp, rs, _ = oracle.fsscs_decode_batch(mode, info, CRC, D, L, h_llr, threads=THREADS)
    else:
        rp, rs, _ = oracle.scs_decode_batch(mode, info, CRC, D, L, h_llr, threads=THREADS)
    assert np.array_equal(rp, g_pay) and np.array_equal(rs, g_st)
    fer = float((out != pay).any(dim=1).float().mean().item())
    _say("full-size %s %s %.1f dB: FER %.4f" % (decoder, dtype, ebn0, fer))
    return fer


@pytest.mark.parametrize("ebn0", [1.0, 2.0])
def test_gpu_full_size_float32_sampled_against_oracle(cuda, ebn0):
    _full(cuda, ebn0, "f32", seed=20 + int(ebn0 * 10))


def test_gpu_full_size_fixed_point_sampled_against_oracle(cuda):
    _full(cuda, 2.0, "i8", seed=30)


@pytest.mark.parametrize("decoder", ["fsscs", "scl"])
def test_gpu_full_size_other_decoders_sampled_against_oracle(cuda, decoder):
    _full(cuda, 2.0, "f32", seed=40, decoder=decoder)


@pytest.mark.parametrize("list_size", [1, 4])
def test_gpu_full_size_packed_list_decoder_sampled_against_oracle(cuda, list_size):
    # 8 / L frames share a wavefront; the sample falls anywhere in the packed batch
    _full(cuda, 2.0, "f32", seed=50 + list_size, decoder="scl", list_size=list_size)


def test_gpu_mixed_full_batch_sampled_against_oracle(cuda):
    """The mixed workload at its full size (2 x 10^6 frames over 25 codes x D in {8, 32, 64},
    L = 8, Eb/N0 uniform in [1.5, 3.5]) in one persistent launch, at the workgroup size the
    benchmark uses (the tuner's cached choice for this plan, else the library's); a sample
    of frames is rebuilt on the host with the oracle's encoder and decoded by the oracle."""
    from paper_1809_03606_amd import binding, tune

    torch = cuda
    B, Lm, crc, seed = 2_000_000, 8, 16, 4
    codes = channel.mixed_codes()
    pcs = [binding.PolarCode(n, k, crc, 2.0) for (n, k) in codes]
    cidx, Dv, eb = channel.mixed_draw(seed, B)
    Nf = np.array([codes[c][0] for c in cidx], np.int64)
    kpf = np.array([codes[c][1] - crc for c in cidx], np.int64)
    # the LLRs and payloads are laid out grouped by code (descriptors stay in draw order)
    grouped = np.argsort(cidx, kind="stable")
    llr_off = np.zeros(B, np.int64)
    out_off = np.zeros(B, np.int64)
    llr_off[grouped] = np.concatenate([[0], np.cumsum(Nf[grouped])[:-1]])
    out_off[grouped] = np.concatenate([[0], np.cumsum(kpf[grouped])[:-1]])
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(B, SAMPLE, replace=False))
    llr = torch.empty(int(Nf.sum()), dtype=torch.float32, device="cuda")
    s_pay, s_noise = {}, {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    for c in range(len(codes)):  # frames of one code at a time
        idx = np.nonzero(cidx == c)[0]
        n, k = codes[c]
        for lo in range(0, idx.size, 1 << 16):
            part = idx[lo:lo + (1 << 16)]
            pay = channel.device_payload(torch, gen, part.size, k - crc, "cuda")
            cw = torch.empty((part.size, n), dtype=torch.uint8, device="cuda")
            pcs[c].encode_device(pay, cw)
            nz = channel.device_noise(torch, gen, part.size, n, "cuda")
            x = channel.device_llr_from_noise_per_frame(torch, cw, nz, eb[part], k / n)
            base = int(llr_off[part[0]])  # frames of one code are contiguous, in order
            llr[base:base + part.size * n] = x.reshape(-1)
            hit = np.nonzero(np.isin(part, sample))[0]
            for j in hit:
                s_pay[int(part[j])] = pay[j].cpu().numpy()
                s_noise[int(part[j])] = nz[j].cpu().numpy()
            del pay, cw, nz, x
    frames = np.zeros(B, binding.FRAME_DTYPE)
    frames["code"], frames["D"], frames["L"] = cidx, Dv, Lm
    frames["llr_off"], frames["out_off"] = llr_off, out_off
    ctx = binding.ScsContext(0)
    tune.apply_mixed(ctx, pcs, frames)
    out = torch.full((int(kpf.sum()),), 0xEE, dtype=torch.uint8, device="cuda")
    st = torch.full((B,), 0xEE, dtype=torch.uint8, device="cuda")
    _say("gpu: full-size mixed batch, %d frames in one persistent launch" % B)
    binding.scs_decode_mixed(ctx.handle, [p.handle for p in pcs], frames, binding.SCS_LLR_F32,
                             llr, out, st)
    torch.cuda.synchronize()
    assert binding.scs_ctx_last_error(ctx.handle) == 0
    g_st = st.cpu().numpy()
    assert set(np.unique(g_st)) <= {1, 2, 6}
    # the sample, rebuilt on the host and decoded by the oracle per (code, D)
    infos = {}
    for c, d in sorted({(int(cidx[f]), int(Dv[f])) for f in sample}):
        sel = [int(f) for f in sample if cidx[f] == c and Dv[f] == d]
        n, k = codes[c]
        info = infos.setdefault(c, oracle.construct(n, k, 2.0))
        cw_h = oracle.encode_batch(info, crc, np.stack([s_pay[f] for f in sel]))
        h_llr = channel.bpsk_awgn_llr_per_frame(cw_h, np.stack([s_noise[f] for f in sel]),
                                                eb[sel], k / n)
        d_llr = np.stack([llr[int(llr_off[f]):int(llr_off[f]) + n].cpu().numpy() for f in sel])
        assert np.array_equal(h_llr.view(np.uint8), d_llr.view(np.uint8))
        rp, rs, _ = oracle.scs_decode_batch(oracle.F32, info, crc, d, Lm, h_llr, threads=THREADS)
        for j, f in enumerate(sel):
            o = int(out_off[f])
            got = out[o:o + k - crc].cpu().numpy()
            assert np.array_equal(got, rp[j]) and g_st[f] == rs[j], (f, c, d)
