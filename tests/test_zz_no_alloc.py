"""The entry point that allocates nothing (mdn_denoise_noalloc) against mdn_denoise, through the C ABI:
the same kernels over a static device scratch instead of a caller workspace, so the outputs are
equal bit for bit. Two calls in a row, the second on a smaller image (the scratch keeps the first
call's contents), in float16 and float32 storage; a request above the scratch's size is refused."""

import numpy as np
import pytest

import synth
from mdn_testlib import gpu_bank, trained_bank_multiscale

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f16", "f32"])
def test_noalloc_equals_denoise_on_two_calls(storage):
    import torch
    import paper_1802_06130_amd as M
    f16 = storage == "f16"
    print(f"noalloc vs denoise, {storage} storage", flush=True)
    bank = trained_bank_multiscale(levels=3)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16 if f16 else torch.float32)
    code = M.F16 if f16 else M.F32
    dt = np.float16 if f16 else np.float32
    for i, (H, W) in enumerate([(1080, 1920), (301, 257)]):
        z = torch.from_numpy(synth.noisy_pair(6100 + i, H, W, 3, 25, dtype=dt)[0]).cuda()
        a = M.denoise(z, gb, storage=code)
        out = torch.empty_like(z)
        b = M.denoise_noalloc(z, gb, storage=code, out=out)
        torch.cuda.synchronize()
        print(f"  call {i + 1}: {H}x{W}", flush=True)
        assert b.data_ptr() == out.data_ptr()
        assert torch.equal(a, b), f"call {i + 1} ({H}x{W}) differs from mdn_denoise"


def test_noalloc_refuses_images_above_the_scratch():
    import torch
    import paper_1802_06130_amd as M
    bank = trained_bank_multiscale(levels=3)
    gb = gpu_bank(bank, 3)
    assert M.denoise_workspace_size(4032, 3024, 3, 3, M.F32) <= M.NOALLOC_SCRATCH_BYTES
    z = torch.empty((3, 8192, 8192), dtype=torch.float32, device="cuda")
    with pytest.raises(M.MdnError) as e:
        M.denoise_noalloc(z, gb, storage=M.F32)
    assert e.value.status == M.MDN_ENOMEM


@pytest.mark.parametrize("storage", ["f16", "f32"])
def test_noalloc_under_graph_capture(storage):
    """The callers it is for: the cascade captured into a HIP graph (it allocates nothing, so the
    capture holds only kernel launches) and replayed three times, with eager calls of the same entry
    point between the replays; every replay and every eager call equals mdn_denoise bit for bit."""
    import torch
    import paper_1802_06130_amd as M
    f16 = storage == "f16"
    print(f"noalloc under graph capture, {storage} storage", flush=True)
    bank = trained_bank_multiscale(levels=3)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16 if f16 else torch.float32)
    code = M.F16 if f16 else M.F32
    dt = np.float16 if f16 else np.float32
    z = torch.from_numpy(synth.noisy_pair(6200, 333, 517, 3, 25, dtype=dt)[0]).cuda()
    z2 = torch.from_numpy(synth.noisy_pair(6201, 200, 150, 3, 25, dtype=dt)[0]).cuda()
    want = M.denoise(z, gb, storage=code)
    want2 = M.denoise(z2, gb, storage=code)
    out = torch.empty_like(z)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        M.denoise_noalloc(z, gb, storage=code, out=out)      # first use of the scratch, outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        M.denoise_noalloc(z, gb, storage=code, out=out)
    out2 = torch.empty_like(z2)
    for r in range(3):
        out.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), f"replay {r + 1} differs from mdn_denoise"
        M.denoise_noalloc(z2, gb, storage=code, out=out2)     # eager, smaller, on the same scratch
        torch.cuda.synchronize()
        assert torch.equal(out2, want2), f"eager call after replay {r + 1} differs from mdn_denoise"
    del graph
