"""Padding is never read, nor workspace bytes before they are written, nor anything written outside
an output: inputs whose row and plane padding hold NaN, outputs inside NaN-filled buffers and
workspaces filled with NaN bytes give finite results, bit for bit those of dense inputs and zeroed
workspaces, and leave the output padding as it was. Covers the cascade (float16 column walk,
float32 LDS-bank kernel, single-scale tiled kernel), the pyramid, the selector, the batched form and
the normal equations, through the C ABI."""

import numpy as np
import pytest

import synth
from mdn_testlib import gpu_bank, gpu_level, trained_bank_multiscale, trained_bank_single

pytestmark = pytest.mark.gpu

PAD_X, PAD_Y = 13, 5


def _torch():
    import torch
    return torch


def _padded(t, pad_x=PAD_X, pad_y=PAD_Y):
    """A view of t inside a NaN-filled buffer with extra columns per row and extra rows per plane."""
    torch = _torch()
    C, H, W = t.shape
    buf = torch.full((C, H + pad_y, W + pad_x), float("nan"), dtype=t.dtype, device=t.device)
    buf[:, :H, :W] = t
    return buf, buf[:, :H, :W]


def _nan_outside(buf, H, W):
    pad = torch_mask(buf, H, W)
    return bool(_torch().isnan(buf[pad]).all())


def torch_mask(buf, H, W):
    torch = _torch()
    m = torch.ones(buf.shape, dtype=torch.bool, device=buf.device)
    m[:, :H, :W] = False
    return m


@pytest.mark.parametrize("case", ["f16_walk", "f32_lds", "grey_single"])
def test_cascade_ignores_padding_and_workspace_contents(case):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"padding: cascade {case}", flush=True)
    H, W = 181, 243
    if case == "grey_single":
        bank = trained_bank_single()
        gb = gpu_bank(bank, 1)
        z = torch.from_numpy(synth.noisy_pair(61, H, W, 1, 25)[0]).cuda()
        code, levels = M.F32, 1
    else:
        f16 = case == "f16_walk"
        bank = trained_bank_multiscale(levels=3)
        gb = gpu_bank(bank, 3, coeff_dtype=torch.float16 if f16 else torch.float32)
        dt = np.float16 if f16 else np.float32
        z = torch.from_numpy(synth.noisy_pair(62, H, W, 3, 25, dtype=dt)[0]).cuda()
        code, levels = (M.F16 if f16 else M.F32), 3
    C = z.shape[0]
    need = M.denoise_workspace_size(W, H, C, levels, code)
    ws0 = torch.zeros(max(need, 1), dtype=torch.uint8, device="cuda")
    ref = M.denoise(z, gb, storage=code, ws=ws0)
    _, zp = _padded(z)
    obuf, op = _padded(torch.empty_like(z))
    wsn = torch.full((max(need, 1),), 0xFF, dtype=torch.uint8, device="cuda")     # NaN in float16 and float32
    M.denoise(zp, gb, storage=code, ws=wsn, out=op)
    torch.cuda.synchronize()
    assert torch.isfinite(op).all()
    assert torch.equal(op, ref)
    assert _nan_outside(obuf, H, W), "a write landed in the output's padding"


def test_pyramid_and_selector_ignore_padding():
    import paper_1802_06130_amd as M
    torch = _torch()
    print("padding: pyramid and selector", flush=True)
    z = torch.from_numpy(synth.noisy_pair(63, 130, 97, 3, 25, dtype=np.float16)[0]).cuda()
    _, zp = _padded(z)
    outs, views = [], []
    h, w = 130, 97
    for _ in range(3):
        h, w = (h + 1) // 2, (w + 1) // 2
        b, v = _padded(torch.empty((3, h, w), dtype=torch.float16, device="cuda"))
        outs.append(b)
        views.append(v)
    M.pyramid_build(zp, 3, storage=torch.float16, out=views)
    ref = M.pyramid_build(z, 3, storage=torch.float16)
    torch.cuda.synchronize()
    for b, v, r in zip(outs, views, ref):
        assert torch.equal(v, r)
        assert _nan_outside(b, v.shape[1], v.shape[2])
    lv = gpu_bank(trained_bank_multiscale(levels=3), 3).levels[0]
    smap = torch.full((130, 97 + 11), 0xAB, dtype=torch.uint8, device="cuda")
    M.select_filters(zp, lv, out=smap[:, :97])
    torch.cuda.synchronize()
    assert torch.equal(smap[:, :97], M.select_filters(z, lv))
    assert bool((smap[:, 97:] == 0xAB).all())


def test_batched_form_ignores_padding():
    import paper_1802_06130_amd as M
    torch = _torch()
    print("padding: batched form", flush=True)
    gb = gpu_bank(trained_bank_multiscale(levels=3), 3, coeff_dtype=torch.float16)
    zs = [torch.from_numpy(synth.noisy_pair(64 + i, h, w, 3, 25, dtype=np.float16)[0]).cuda()
          for i, (h, w) in enumerate([(200, 150), (61, 97), (33, 40)])]
    plan = M.Plan(gb, M.F16, max_images=4)
    ref = [t.clone() for t in plan.denoise_batch(zs, use_graph=False)]
    zp = [_padded(t)[1] for t in zs]
    obufs = [_padded(torch.empty_like(t)) for t in zs]
    plan.denoise_batch(zp, [v for _, v in obufs], use_graph=True)
    torch.cuda.synchronize()
    for (b, v), r in zip(obufs, ref):
        assert torch.equal(v, r)
        assert _nan_outside(b, v.shape[1], v.shape[2])
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_normal_equations_ignore_padding(precision):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"padding: normal equations precision={precision}", flush=True)
    lb = trained_bank_multiscale(levels=2).levels[0]
    sel = gpu_level(lb, 3)
    z, u = (torch.from_numpy(a).cuda() for a in synth.noisy_pair(65, 96, 130, 3, 25))
    zc = M.pyramid_build(z, 1)[0]
    grams = []
    for zz, uu, cc in ((z, u, zc), (_padded(z)[1], _padded(u)[1], _padded(zc)[1])):
        g = M.Gram(sel.K, 3, 3, 3)
        M.train_accumulate(g, zz, uu, sel, u_coarse=cc, coarse_color=M.RGB, precision=precision)
        grams.append(g)
    torch.cuda.synchronize()
    assert torch.equal(grams[0].n, grams[1].n)
    assert torch.equal(grams[0].G, grams[1].G) and torch.equal(grams[0].b, grams[1].b)
    assert torch.isfinite(grams[1].G).all()
