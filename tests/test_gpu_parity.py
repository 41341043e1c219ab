"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: pyramid levels bit-exact (float64 arithmetic rounded once); bucket maps equal except
at pixels whose oracle features lie within 1e-6 of a bucket boundary, such flips capped per level;
every output pixel within 1e-4 max-abs (float32 storage) or 2e-3 (float16 storage) of the oracle
cascade run on the GPU's own maps at the same storage rounding, with the max-abs and |dPSNR|
against the pure float64 oracle reported beside it.
"""

import numpy as np
import pytest

import oracle as O
import synth
from mdn_testlib import (TOL_F16, TOL_F32, cascade_parity, gpu_bank, gpu_level, index_parity,
                         trained_bank_multiscale, trained_bank_single)

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(a, dtype=None):
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


SIZES = [(1, 1), (3, 5), (7, 7), (17, 33), (64, 64), (130, 97)]


@pytest.mark.parametrize("H,W", SIZES + [(768, 1024)])
@pytest.mark.parametrize("C", [1, 3])
def test_pyramid_bit_exact_f32(H, W, C):
    import paper_1802_06130_amd as M
    print(f"pyramid f32 C={C} {H}x{W}", flush=True)
    z, _ = synth.noisy_pair(10 + H + W, H, W, C, 25)
    got = M.pyramid_build(_dev(z), 3)
    want = O.build_pyramid(z, 4, storage=np.float32)
    for lev in range(3):
        g = got[lev].cpu().numpy()
        w = want[lev + 1].astype(np.float32)
        assert g.shape == w.shape
        assert np.array_equal(g, w), f"level {lev + 1}: {np.sum(g != w)} of {g.size} differ"


@pytest.mark.parametrize("H,W", [(5, 3), (64, 80), (301, 257)])
def test_pyramid_bit_exact_f16(H, W):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"pyramid f16 {H}x{W}", flush=True)
    z, _ = synth.noisy_pair(20 + H, H, W, 3, 25, dtype=np.float16)
    got = M.pyramid_build(_dev(z), 3, storage=torch.float16)
    want = O.build_pyramid(z, 4, storage=np.float16)
    for lev in range(3):
        g = got[lev].cpu().numpy()
        w = want[lev + 1].astype(np.float16)
        assert np.array_equal(g, w), f"level {lev + 1}: {np.sum(g != w)} of {g.size} differ"


@pytest.mark.parametrize("H,W", SIZES + [(256, 256)])
def test_select_parity_grey(H, W):
    import paper_1802_06130_amd as M
    print(f"select grey {H}x{W}", flush=True)
    lb = trained_bank_single().levels[0]
    z, _ = synth.noisy_pair(30 + H, H, W, 1, 25)
    s = M.select_filters(_dev(z), gpu_level(lb, 1))
    _, n_mis, n_near = index_parity(s.cpu().numpy(), z, lb)
    print(f"  mismatches={n_mis} near-boundary={n_near}")


@pytest.mark.parametrize("H,W", SIZES + [(768, 1024)])
def test_select_parity_rgb(H, W):
    import paper_1802_06130_amd as M
    print(f"select rgb {H}x{W}", flush=True)
    lb = trained_bank_multiscale().levels[0]
    z, _ = synth.noisy_pair(40 + W, H, W, 3, 25)
    s = M.select_filters(_dev(z), gpu_level(lb, 3))
    _, n_mis, n_near = index_parity(s.cpu().numpy(), z, lb)
    print(f"  mismatches={n_mis} near-boundary={n_near}")


def test_select_constant_and_ramp():
    import paper_1802_06130_amd as M
    lb = trained_bank_multiscale().levels[0]
    z = np.full((3, 40, 70), 0.3, np.float32)
    s = M.select_filters(_dev(z), gpu_level(lb, 3)).cpu().numpy()
    assert np.all(s == (12 * 3 + 0) * 3 + 0)
    yy, xx = np.mgrid[0:40, 0:70]
    ramp = np.stack([0.2 + 0.004 * xx + 0.002 * yy] * 3).astype(np.float32)
    s = M.select_filters(_dev(ramp), gpu_level(lb, 3)).cpu().numpy()
    index_parity(s, ramp, lb)


@pytest.mark.parametrize("H,W", SIZES + [(256, 256)])
def test_single_scale_grey(H, W):
    """Eq. (1) on a grey image (5 x 5 filters, 16 x 3 x 3 buckets)."""
    print(f"single-scale grey {H}x{W}", flush=True)
    bank = trained_bank_single()
    z, u = synth.noisy_pair(1001, H, W, 1, 25)
    cascade_parity(z, bank, gpu_bank(bank, 1), np.float32, TOL_F32, u=u)


@pytest.mark.parametrize("H,W", [(7, 9), (130, 97), (256, 256)])
def test_single_scale_rgb(H, W):
    """Eq. (1) on a colour image: colour structure tensor, YCbCr filtering, RGB output."""
    print(f"single-scale rgb {H}x{W}", flush=True)
    bank = trained_bank_single(channels=3)
    z, u = synth.noisy_pair(1003, H, W, 3, 25)
    r = cascade_parity(z, bank, gpu_bank(bank, 3), np.float32, TOL_F32, u=u)
    if H * W > 10000:
        assert O.psnr(r["out"], u) > O.psnr(z, u) + 3


@pytest.mark.parametrize("H,W", SIZES + [(768, 1024)])
def test_denoise_three_level_rgb(H, W):
    print(f"denoise 3-level rgb {H}x{W}", flush=True)
    bank = trained_bank_multiscale(levels=2)
    z, u = synth.noisy_pair(2001, H, W, 3, 25)
    r = cascade_parity(z, bank, gpu_bank(bank, 3), np.float32, TOL_F32, u=u)
    if H * W > 10000:
        assert O.psnr(r["out"], u) > O.psnr(z, u) + 5


@pytest.mark.parametrize("H,W", [(9, 13), (200, 328), (600, 808)])
def test_denoise_four_level_rgb(H, W):
    print(f"denoise 4-level rgb {H}x{W}", flush=True)
    bank = trained_bank_multiscale(levels=3)
    z, u = synth.noisy_pair(3001 + H, H, W, 3, 25)
    cascade_parity(z, bank, gpu_bank(bank, 3), np.float32, TOL_F32, u=u)


def test_apply_level_precomputed_selector_matches_fused():
    import paper_1802_06130_amd as M
    bank = trained_bank_multiscale(levels=2)
    gb = gpu_bank(bank, 3)
    z, _ = synth.noisy_pair(77, 96, 130, 3, 25)
    zt = _dev(z)
    coarse = M.pyramid_build(zt, 1)[0]
    s = M.select_filters(zt, gb.levels[0])
    a = M.apply_level(zt, gb.levels[0], u_coarse=coarse, coarse_color=M.RGB)
    b = M.apply_level(zt, gb.levels[0], u_coarse=coarse, coarse_color=M.RGB, s=s)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_empty_images_are_noops():
    import paper_1802_06130_amd as M
    torch = _torch()
    bank = trained_bank_multiscale(levels=2)
    gb = gpu_bank(bank, 3)
    for shape in [(3, 0, 5), (3, 4, 0), (3, 0, 0)]:
        z = torch.zeros(shape, device="cuda")
        out = M.denoise(z, gb)
        assert out.shape == shape


def test_run_twice_bitwise_identical():
    import paper_1802_06130_amd as M
    bank = trained_bank_multiscale(levels=2)
    gb = gpu_bank(bank, 3)
    z, _ = synth.noisy_pair(5, 333, 271, 3, 25)
    zt = _dev(z)
    a = M.denoise(zt, gb).cpu().numpy()
    b = M.denoise(zt, gb).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("H,W", [(5, 9), (130, 97), (600, 808)])
@pytest.mark.parametrize("coeff16", [False, True])
def test_denoise_four_level_fp16_storage(H, W, coeff16):
    """FP16 pyramid/outputs (FP32 accumulation): indices equal the oracle's in FP16-storage mode
    except near boundaries; every pixel within 2e-3 of it on the GPU's maps; PSNR within 0.01 dB of
    the pure FP64 oracle."""
    torch = _torch()
    print(f"denoise 4-level fp16 {H}x{W} coeff16={coeff16}", flush=True)
    bank = trained_bank_multiscale(levels=3)
    z, u = synth.noisy_pair(4001 + H, H, W, 3, 25, dtype=np.float16)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16 if coeff16 else torch.float32)
    cascade_parity(z, bank, gb, np.float16, TOL_F16, u=u, dpsnr_tol=0.01 if H * W > 10000 else None)


@pytest.mark.parametrize("H,W", [(1, 1), (2, 3), (57, 59), (113, 175), (200, 116), (57, 1)])
def test_walk_kernel_fp16_bank_sizes(H, W):
    """The float16-bank kernel (column walk, strips of 58 columns x 56 rows) across strip edges."""
    torch = _torch()
    print(f"walk fp16 {H}x{W}", flush=True)
    bank = trained_bank_multiscale(levels=2)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16)
    for in_dt in (np.float16, np.float32):
        z, u = synth.noisy_pair(5001 + H + W, H, W, 3, 25, dtype=in_dt)
        print(f"  input {np.dtype(in_dt).name}", flush=True)
        cascade_parity(z, bank, gb, in_dt, TOL_F16)
