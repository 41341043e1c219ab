"""Phase-aware buckets (the other reading of the non-integer i/2 of Eq. (9)):
the parity of the pixel on the coarser grid joins the bucket index, s' = 4 s + 2 (y mod 2) + (x mod 2),
on the GPU through the C ABI, against the oracle.

Bars as everywhere: maps equal the oracle's except within 1e-6 of a bucket boundary (the phase
itself is exact); float32 cascades within 1e-4; the normal equations' counts exact; a bank trained
with phases gives outputs close to the oracle's phase-aware bank.
"""

import numpy as np
import pytest

import oracle as O
import synth
from mdn_testlib import TOL_F32, cascade_parity, gpu_bank, gpu_level, index_parity

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def _bank(L=2, q=(24, 3, 3), r=3, seed=8):
    zs = [synth.noisy_pair(700 + i, 128, 128, 3, 25)[0].astype(np.float64) for i in range(2)]
    levels = []
    for lev in range(L):
        f = [O.level_features(O.build_pyramid(z, lev + 1)[lev]) for z in zs]
        t_s = O.thresholds_from_features(np.concatenate([x[0] for x in f]), q[1])
        t_c = O.thresholds_from_features(np.concatenate([x[1] for x in f]), q[2])
        K = q[0] * q[1] * q[2] * 4
        co = synth.random_bank_coeffs(seed + lev, K, 3, (2 * r + 1) ** 2, (2 * r + 1) ** 2)
        levels.append(O.LevelBank(q[0], t_s, t_c, r, r, co, phases=4))
    return O.Bank(levels)


@pytest.mark.parametrize("q", [(24, 3, 3), (8, 2, 2)])
@pytest.mark.parametrize("H,W", [(1, 1), (2, 3), (17, 33), (301, 257)])
@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_select_phase_aware(q, H, W, dtype):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"select phases q={q} {H}x{W} {np.dtype(dtype).name}", flush=True)
    lb = _bank(1, q).levels[0]
    z, _ = synth.noisy_pair(710 + W, H, W, 3, 25, dtype=dtype)
    s = M.select_filters(_dev(z), gpu_level(lb, 3))
    K = q[0] * q[1] * q[2] * 4
    assert s.dtype == (torch.uint16 if K > 256 else torch.uint8)
    sn = s.cpu().numpy().astype(np.int64)
    yy, xx = np.mgrid[0:H, 0:W]
    assert np.array_equal(sn % 4, 2 * (yy % 2) + (xx % 2))
    _, n_mis, n_near = index_parity(sn, z.astype(np.float64), lb)
    print(f"  mismatches={n_mis} near-boundary={n_near}")


def test_denoise_phase_aware_f32():
    import paper_1802_06130_amd as M
    torch = _torch()
    print("denoise phase-aware 3-level", flush=True)
    bank = _bank(2)
    z, u = synth.noisy_pair(2020, 200, 248, 3, 25)
    gb = gpu_bank(bank, 3)
    cascade_parity(z, bank, gb, np.float32, TOL_F32, u=u)


def test_train_phase_aware_end_to_end():
    import paper_1802_06130_amd as M
    print("train phase-aware multiscale", flush=True)
    pairs = [synth.noisy_pair(720 + i, 96, 96, 3, 25) for i in range(3)]
    p64 = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    thr = [([0.03, 0.06], [0.25, 0.5]), ([0.02, 0.04], [0.25, 0.5])]
    bank_o, stats_o, fb_o = O.train_multiscale(p64, 2, 8, 3, 3, 3, 3, 1e-3, thresholds=thr, storage=np.float32,
                                               phases=4)
    bank_g, grams, fb_g = M.train_multiscale([(_dev(z), _dev(u)) for z, u in pairs], 2, 8, 3, 3, 3, 3, 1e-3,
                                             thresholds=thr, phases=4)
    assert grams[0].n.numel() == 8 * 9 * 4
    assert np.array_equal(grams[1].n.cpu().numpy(), stats_o[1].n)
    z, u = synth.noisy_pair(2021, 120, 160, 3, 25)
    lvls = [O.LevelBank(8, np.array(t[0]), np.array(t[1]), 3, 3, lg.coeffs.double().cpu().numpy(), phases=4)
            for t, lg in zip(thr, bank_g.levels)]
    out_g = O.denoise(z, O.Bank(lvls), storage=np.float32)
    out_o = O.denoise(z, bank_o, storage=np.float32)
    err = float(np.max(np.abs(out_g - out_o)))
    print(f"  fallbacks GPU {fb_g} oracle {[3 * int(f.sum()) for f in fb_o]}; output max-abs {err:.3g}; "
          f"PSNR {O.psnr(z, u):.2f} -> {O.psnr(out_g, u):.2f} dB")
    assert err < 1e-3
