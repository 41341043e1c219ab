"""Filtering with the bank staged in LDS one channel at a time (colour multiscale levels whose bank
fits, such as float32 7x7/7x7 banks of up to 219 buckets), against the oracle's Eq. (9) on the same
selector map.

The map is given (random buckets, so every bucket row is exercised), so the comparison is of the
filtering alone: float32 outputs within 1e-4 of the oracle's, float16 outputs within 2e-3; a
selector outside the bank gives NaN. The cascade tests of test_gpu_parity.py run this kernel through
mdn_denoise for float32 banks.
"""

import numpy as np
import pytest

import oracle as O
import synth
from mdn_testlib import TOL_F16, TOL_F32, gpu_level, max_abs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def _level(q, rf, rg, seed, coeff_dtype=np.float32):
    q_theta, q_s, q_c = q
    K = q_theta * q_s * q_c
    D = (2 * rf + 1) ** 2 + (2 * rg + 1) ** 2
    co = np.random.default_rng(seed).normal(0.0, 0.06, (K, 3, D))
    co = co.astype(coeff_dtype).astype(np.float64)
    t_s = np.linspace(0.01, 0.05, q_s - 1)
    t_c = np.linspace(0.2, 0.6, q_c - 1)
    return O.LevelBank(q_theta, t_s, t_c, rg, rf, co)


@pytest.mark.parametrize("q,rf,rg", [((24, 3, 3), 3, 3), ((8, 3, 3), 2, 3), ((16, 2, 2), 2, 2),
                                     ((8, 6, 6), 1, 1), ((10, 3, 3), 1, 2)])
@pytest.mark.parametrize("H,W", [(1, 1), (7, 9), (33, 65), (200, 328)])
@pytest.mark.parametrize("storage,coarse_rgb", [(np.float32, False), (np.float16, False), (np.float32, True)])
def test_lds_bank_filter_matches_oracle(q, rf, rg, H, W, storage, coarse_rgb):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"lds apply q={q} rf={rf} rg={rg} {H}x{W} {np.dtype(storage).name} coarse {'rgb' if coarse_rgb else 'ycc'}",
          flush=True)
    lb = _level(q, rf, rg, seed=H + W + rf)
    K = lb.K
    z, _ = synth.noisy_pair(40 + W, H, W, 3, 25, dtype=storage)
    uc_rgb = synth.noisy_pair(50 + W, (H + 1) // 2, (W + 1) // 2, 3, 10)[0].astype(np.float64)
    uc = (uc_rgb if coarse_rgb else O.rgb_to_ycc(uc_rgb)).astype(storage)
    mdt = np.uint16 if K > 256 else np.uint8
    s = np.random.default_rng(W).integers(0, K, (H, W)).astype(mdt)
    lv = gpu_level(lb, 3)
    st = _dev(s)
    out = M.apply_level(_dev(z), lv, u_coarse=_dev(uc), coarse_color=M.RGB if coarse_rgb else M.YCC, s=st,
                        out_dtype=torch.float32 if storage == np.float32 else torch.float16)
    ucf = O.to_filter_space(uc.astype(np.float64)) if coarse_rgb else uc.astype(np.float64)
    ref = O.apply_level(O.to_filter_space(z.astype(np.float64)), s.astype(np.int64), lb, u_coarse=ucf)
    err = max_abs(_host(out), ref)
    print(f"  max-abs {err:.3g}")
    assert err <= (TOL_F32 if storage == np.float32 else TOL_F16)


@pytest.mark.parametrize("q,rf,rg", [((8, 3, 3), 2, 3), ((16, 2, 2), 2, 2), ((8, 6, 6), 1, 1)])
@pytest.mark.parametrize("H,W", [(7, 9), (200, 328)])
def test_lds_bank_float16_coefficients(q, rf, rg, H, W):
    """Float16 banks of other radii than 7x7/7x7 take the same kernel (their rows are copied to LDS
    as float32, pairs of taps at a time): exact conversion, so the float32 bar holds."""
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"lds apply f16 coefficients q={q} rf={rf} rg={rg} {H}x{W}", flush=True)
    lb = _level(q, rf, rg, seed=7 + H, coeff_dtype=np.float16)
    K = lb.K
    z, _ = synth.noisy_pair(60 + W, H, W, 3, 25)
    uc = O.rgb_to_ycc(synth.noisy_pair(61 + W, (H + 1) // 2, (W + 1) // 2, 3, 10)[0].astype(np.float64))
    uc = uc.astype(np.float32)
    s = np.random.default_rng(H).integers(0, K, (H, W)).astype(np.uint16 if K > 256 else np.uint8)
    out = M.apply_level(_dev(z), gpu_level(lb, 3, coeff_dtype=torch.float16), u_coarse=_dev(uc), s=_dev(s))
    ref = O.apply_level(O.to_filter_space(z.astype(np.float64)), s.astype(np.int64), lb, u_coarse=uc.astype(np.float64))
    err = max_abs(_host(out), ref)
    print(f"  max-abs {err:.3g}")
    assert err <= TOL_F32


def test_lds_bank_selector_outside_the_bank_is_nan():
    import paper_1802_06130_amd as M
    torch = _torch()
    lb = _level((24, 3, 3), 3, 3, seed=1)
    z, _ = synth.noisy_pair(3, 40, 70, 3, 25)
    uc = O.rgb_to_ycc(synth.noisy_pair(4, 20, 35, 3, 10)[0].astype(np.float64)).astype(np.float32)
    s = np.random.default_rng(2).integers(0, lb.K, (40, 70)).astype(np.uint8)
    s[5, 7] = 250
    out = _host(M.apply_level(_dev(z), gpu_level(lb, 3), u_coarse=_dev(uc), s=_dev(s)))
    assert np.isnan(out[:, 5, 7]).all()
    out[:, 5, 7] = 0.0
    assert np.isfinite(out).all()
    del torch


def test_lds_bank_cascade_level_by_level_equals_denoise():
    """mdn_denoise with a float32 bank (selection pass, then the LDS-bank filtering at every level)
    equals the same kernels called level by level through mdn_apply_level, bit for bit."""
    import paper_1802_06130_amd as M
    from mdn_testlib import gpu_bank, trained_bank_multiscale
    torch = _torch()
    bank = trained_bank_multiscale(levels=3)
    gb = gpu_bank(bank, 3)
    z, _ = synth.noisy_pair(2007, 181, 263, 3, 25)
    zt = _dev(z)
    out = _host(M.denoise(zt, gb))
    pyr = [zt] + M.pyramid_build(zt, 3)
    u, color = pyr[3], M.RGB
    for lev in range(2, -1, -1):
        s = M.select_filters(pyr[lev], gb.levels[lev])
        u = M.apply_level(pyr[lev], gb.levels[lev], u_coarse=u, coarse_color=color, s=s,
                          out_color=M.RGB if lev == 0 else M.YCC)
        color = M.YCC
    assert np.array_equal(out, _host(u))
    del torch
