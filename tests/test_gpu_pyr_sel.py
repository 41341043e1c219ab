"""The cascade's shared launch of a pyramid step and its level's selection pass, against the
separate calls: mdn_denoise runs the selection pass of every RGB level whose filtering reads a
selector map inside the launch of that level's pyramid step. The same cascade assembled from the
separate entry points (mdn_pyramid_build, mdn_select_filters, then mdn_apply_level on the map)
must give the same output bit for bit, for float16 (column walk) and float32 (LDS bank)
coefficients, both storages and ragged sizes down to one pixel."""

import numpy as np
import pytest

import synth
from mdn_testlib import gpu_bank, trained_bank_multiscale

pytestmark = pytest.mark.gpu

SIZES = [(1, 1), (3, 5), (57, 59), (130, 97), (481, 321), (768, 1024)]
# (float16 coefficients, storage, input dtype)
CASES = [(True, "F16", np.float16), (True, "F16", np.float32), (True, "F32", np.float32), (False, "F32", np.float32)]


@pytest.fixture(scope="module")
def bank():
    return trained_bank_multiscale(levels=3)


@pytest.mark.parametrize("coeff16, storage_name, in_dtype", CASES)
@pytest.mark.parametrize("H, W", SIZES)
def test_denoise_equals_separate_calls(bank, H, W, coeff16, storage_name, in_dtype):
    import torch
    import paper_1802_06130_amd as M
    print(f"shared launch vs separate calls {H}x{W} coeff16={coeff16} storage={storage_name} "
          f"input={np.dtype(in_dtype).name}", flush=True)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16 if coeff16 else torch.float32)
    storage = getattr(M, storage_name)
    sdt = torch.float16 if storage == M.F16 else torch.float32
    z = torch.from_numpy(synth.noisy_pair(3100 + H + W, H, W, 3, 25, dtype=in_dtype)[0]).cuda()
    want = M.denoise(z, gb, storage=storage)
    L = len(gb.levels)
    pyr = [z] + M.pyramid_build(z, L, storage=sdt)
    coarse, cc = pyr[L], M.RGB
    for lev in reversed(range(L)):
        lv = gb.levels[lev]
        s = M.select_filters(pyr[lev], lv)
        last = lev == 0
        coarse = M.apply_level(pyr[lev], lv, u_coarse=coarse, coarse_color=cc, s=s,
                               out_color=M.RGB if last else None, out_dtype=z.dtype if last else sdt)
        cc = M.YCC
    torch.cuda.synchronize()
    assert torch.equal(coarse, want)
