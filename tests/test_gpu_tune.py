"""GPU: the launch-shape autotuner and the waves-per-workgroup knob.  Every launch shape
must give the oracle's bits; the tuner must store a choice among its candidates and
``apply`` must configure a context with it."""
import numpy as np
import pytest

from cases import assert_parity, gpu_decode, make_frames, oracle_decode

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_every_launch_shape_matches_oracle(cuda, wpb):
    from paper_1809_03606_amd.binding import PolarCode

    N, K, crc, D, L = 512, 256, 16, 32, 8
    info, pay, llr = make_frames(N, K, crc, 1.5, 53, seed=97)
    ref = oracle_decode(info, crc, D, L, llr)
    print("gpu: launch shape wpb=%d" % wpb, flush=True)
    got = gpu_decode(cuda, PolarCode(N, K, crc, 2.0), D, L, llr, wpb=wpb)
    assert_parity(got, ref, "wpb=%d" % wpb)


def test_tuner_stores_and_applies(cuda, tmp_path):
    from paper_1809_03606_amd import binding, tune

    code = binding.PolarCode(256, 128, 16)
    path = str(tmp_path / "tune.json")
    print("gpu: tuner on PC(256,128)", flush=True)
    entry = tune.tune(code, 16, 8, "f32", frames=4096, reps=1, path=path)
    assert entry["waves_per_block"] in tune.CANDIDATES
    assert len(entry["candidates_ms"]) == len(tune.CANDIDATES)
    ctx = binding.ScsContext(0)
    got = tune.apply(ctx, code, 16, 8, "f32", path=path)
    assert got["waves_per_block"] == entry["waves_per_block"]
    assert tune.apply(ctx, binding.PolarCode(128, 64, 0), 16, 8, "f32", path=path) is None
    # the configured context still decodes to the oracle's bits
    info, pay, llr = make_frames(256, 128, 16, 2.0, 40, seed=5)
    ref = oracle_decode(info, 16, 16, 8, llr)
    torch = cuda
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(llr).to(dev)
    out = torch.empty((40, code.payload_bits), dtype=torch.uint8, device=dev)
    st = torch.empty((40,), dtype=torch.uint8, device=dev)
    ctx.decode(code, 16, 8, x, out, st)
    torch.cuda.synchronize()
    ctx.close()
    assert np.array_equal(out.cpu().numpy(), ref[0]) and np.array_equal(st.cpu().numpy(), ref[1])


def test_tuner_command_line_in_a_fresh_process(cuda, tmp_path):
    """The tuner as its own process: its first library call comes right after PyTorch's
    device set-up (which shares the HIP runtime with the library)."""
    import json
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = str(tmp_path / "tuned.json")
    print("gpu: tuner command line", flush=True)
    r = subprocess.run([sys.executable, "-m", "paper_1809_03606_amd.tune", "--N", "128", "--K",
                        "64", "--D", "8", "--frames", "2048", "--out", out],
                       cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    entry = json.loads(r.stdout.strip().splitlines()[-1])
    assert entry["waves_per_block"] in __import__("paper_1809_03606_amd.tune",
                                                 fromlist=["x"]).CANDIDATES
    assert json.load(open(out))


def test_tuner_list_decoder(cuda, tmp_path):
    """The list decoder's workgroup size through the tuner: a stored choice among its
    candidates, applied to a context that still decodes to the oracle's bits."""
    import oracle
    from paper_1809_03606_amd import binding, tune

    code = binding.PolarCode(256, 128, 16)
    path = str(tmp_path / "tune.json")
    print("gpu: tuner, list decoder L=4 on PC(256,128)", flush=True)
    entry = tune.tune(code, 0, 4, "f32", frames=2048, reps=1, path=path, decoder="scl")
    assert entry["waves_per_block"] in tune.candidates("scl")
    assert entry["frames"] == 2048 * 2  # two frames per wavefront at L = 4
    ctx = binding.ScsContext(0)
    assert tune.apply(ctx, code, 32, 4, "f32", path=path, decoder="scl") is not None
    info, pay, llr = make_frames(256, 128, 16, 2.0, 41, seed=6)
    rp, rs, _ = oracle.scl_decode_batch(oracle.F32, info, 16, 4, llr, threads=4)
    torch = cuda
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(llr).to(dev)
    out = torch.empty((41, code.payload_bits), dtype=torch.uint8, device=dev)
    st = torch.empty((41,), dtype=torch.uint8, device=dev)
    ctx.decode_list(code, 4, x, out, st)
    torch.cuda.synchronize()
    ctx.close()
    assert np.array_equal(out.cpu().numpy(), rp) and np.array_equal(st.cpu().numpy(), rs)
