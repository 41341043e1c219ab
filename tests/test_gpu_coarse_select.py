"""Selection on the coarser output (selector = SELECT_COARSE): the structure tensor of the coarser
level's output u^{l+1}, upsampled onto the level's grid (linear interpolation on the pyramid's
alignment) and taken back to RGB, instead of the noisy z^l; the alternative that Eq. (9) leaves
open. GPU through the C ABI against the oracle.

Bars as for the other selectors: bucket maps equal to the oracle's (run on the same coarser output)
except at pixels whose features lie within 1e-6 of a bucket boundary; features to 1e-13 (strength)
and 1e-9 (coherence); float32 cascades within 1e-4 of the oracle run on the GPU's index maps, float16
storage within 2e-3 of its float16-storage mode. The GPU converts YCbCr to RGB before interpolating
and the oracle after (both float64 and linear), so their selector images differ by rounding only.
"""

import numpy as np
import pytest

import oracle as O
import synth
from mdn_testlib import (FLIP_CAP, TOL_F16, TOL_F32, check_gram, gpu_bank, gpu_level, index_parity, max_abs,
                         trained_bank_multiscale)

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def _coarse_output(seed, H, W, dtype=np.float32, ycc=True):
    """A coarser output as the cascade holds it (ceil(H/2) x ceil(W/2); YCbCr, or RGB at the
    coarsest level), stored in dtype: a lightly noisy seeded scene."""
    rgb = synth.noisy_pair(seed, (H + 1) // 2, (W + 1) // 2, 3, 5)[0].astype(np.float64)
    return (O.rgb_to_ycc(rgb) if ycc else rgb).astype(dtype)


def _filter_space(uc, ycc):
    uc = np.asarray(uc, np.float64)
    return uc if ycc else O.to_filter_space(uc)


def _coarse_level(q_theta, q_s, q_c, seed=3):
    f = []
    for i in range(3):
        uc = _coarse_output(seed + i, 96, 96)
        f.append(O.level_features(np.zeros((3, 96, 96)), "coarse", uc.astype(np.float64)))
    t_s = O.thresholds_from_features(np.concatenate([x[0] for x in f]), q_s)
    t_c = O.thresholds_from_features(np.concatenate([x[1] for x in f]), q_c)
    K = q_theta * q_s * q_c
    return O.LevelBank(q_theta, t_s, t_c, 3, 3, np.zeros((K, 3, 98)), "coarse")


@pytest.mark.parametrize("q", [(24, 3, 3), (10, 4, 2)])
@pytest.mark.parametrize("H,W", [(1, 1), (7, 7), (17, 33), (130, 97), (768, 1024)])
@pytest.mark.parametrize("dtype,ycc", [(np.float32, True), (np.float16, True), (np.float32, False)])
def test_select_parity_coarse(q, H, W, dtype, ycc):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"select coarse q={q} {H}x{W} {np.dtype(dtype).name} {'ycc' if ycc else 'rgb'}", flush=True)
    lb = _coarse_level(*q)
    uc = _coarse_output(70 + W, H, W, dtype, ycc)
    z = torch.empty((3, H, W), device="cuda")          # gives the size only
    s = M.select_filters(z, gpu_level(lb, 3), u_coarse=_dev(uc), coarse_color=M.YCC if ycc else M.RGB)
    s = s.cpu().numpy()
    _, n_mis, n_near = index_parity(s, np.zeros((3, H, W)), lb, u_coarse=_filter_space(uc, ycc))
    print(f"  mismatches={n_mis} near-boundary={n_near}")


def test_coarse_features_match_oracle():
    import paper_1802_06130_amd as M
    torch = _torch()
    for ycc, (H, W) in [(True, (70, 90)), (False, (69, 91))]:
        uc = _coarse_output(8, H, W, np.float32, ycc)
        st, co = M.level_features(torch.empty((3, H, W), device="cuda"), M.SELECT_COARSE, _dev(uc),
                                  M.YCC if ycc else M.RGB)
        sel = O.selector_image(np.zeros((3, H, W)), "coarse", _filter_space(uc, ycc))
        _, s_o, c_o = O.eigen_features(*O.structure_tensor(sel))
        assert np.max(np.abs(st.cpu().numpy() - s_o)) < 1e-13
        assert np.max(np.abs(co.cpu().numpy() - c_o)) < 1e-9


def test_coarse_selector_reads_the_coarser_output_only():
    """Two different noisy inputs with the same coarser output select the same buckets inline
    (and the same as the selector-only call), while the noisy-input selector does not."""
    import paper_1802_06130_amd as M
    torch = _torch()
    H, W = 96, 130
    bank = trained_bank_multiscale(levels=1, selector="coarse")
    lv = gpu_level(bank.levels[0], 3)
    uc = _dev(_coarse_output(11, H, W))
    maps = []
    for seed in (1, 2):
        z = _dev(synth.noisy_pair(seed, H, W, 3, 25)[0])
        s_out = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        M.apply_level(z, lv, u_coarse=uc, s_out=s_out)
        maps.append(s_out.cpu().numpy())
    assert np.array_equal(maps[0], maps[1])
    s_sel = M.select_filters(torch.empty((3, H, W), device="cuda"), lv, u_coarse=uc).cpu().numpy()
    assert np.array_equal(maps[0], s_sel)


def _gpu_levels(img, gb, storage_t, coeff16):
    """The cascade level by level through mdn_apply_level (inline selection on the coarser output),
    returning the output, the maps and the coarser outputs each level selected on."""
    import paper_1802_06130_amd as M
    torch = _torch()
    L = len(gb.levels)
    zt = _dev(img)
    pyr = [zt] + M.pyramid_build(zt, L, storage=storage_t)
    u, color = pyr[L], M.RGB
    maps, coarse = [None] * L, [None] * L
    for lev in range(L - 1, -1, -1):
        H, W = pyr[lev].shape[1:]
        coarse[lev] = (_host(u), color == M.YCC)
        s_out = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        out_color = M.RGB if lev == 0 else M.YCC
        out_dtype = zt.dtype if lev == 0 else storage_t
        u = M.apply_level(pyr[lev], gb.levels[lev], u_coarse=u, coarse_color=color, s_out=s_out,
                          out_color=out_color, out_dtype=out_dtype)
        maps[lev] = s_out.cpu().numpy()
        color = M.YCC
    return u, maps, coarse, pyr


def _oracle_on_maps(img, bank, maps, storage):
    """The oracle cascade with the GPU's index maps."""
    return O.denoise(img, bank, storage=storage, maps=maps)


def _check_maps(maps, coarse, pyr_host, bank):
    for lev, (uc, ycc) in enumerate(coarse):
        _, n_mis, n_near = index_parity(maps[lev], pyr_host[lev], bank.levels[lev], u_coarse=_filter_space(uc, ycc))
        print(f"  level {lev}: mismatches={n_mis} near-boundary={n_near}")
        assert n_mis <= max(1, FLIP_CAP * maps[lev].size)


@pytest.mark.parametrize("H,W", [(9, 13), (200, 328)])
def test_denoise_coarse_bank_f32(H, W):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"denoise coarse-selector 3-level f32 {H}x{W}", flush=True)
    bank = trained_bank_multiscale(levels=2, selector="coarse")
    gb = gpu_bank(bank, 3)
    z, u = synth.noisy_pair(2005, H, W, 3, 25)
    out = _host(M.denoise(_dev(z), gb, storage=M.F32))
    out_l, maps, coarse, pyr = _gpu_levels(z, gb, torch.float32, False)
    assert np.array_equal(out, _host(out_l))                  # the same kernels, level by level
    _check_maps(maps, coarse, [_host(p) for p in pyr], bank)
    err = max_abs(out, _oracle_on_maps(z.astype(np.float64), bank, maps, np.float32))
    print(f"  max-abs vs oracle on the GPU's maps {err:.3g}")
    assert err <= TOL_F32
    ref = O.denoise(z, bank, storage=np.float32)
    print(f"  max-abs vs pure oracle {max_abs(out, ref):.3g}")
    if H * W > 10000:
        assert O.psnr(out, u) > O.psnr(z, u) + 5


def test_denoise_coarse_bank_f16_column_walk():
    """float16 storage and coefficients: the coarse selection fills the map the filtering walk reads."""
    import paper_1802_06130_amd as M
    torch = _torch()
    print("denoise coarse-selector 4-level f16", flush=True)
    bank = trained_bank_multiscale(levels=3, selector="coarse")
    z, u = synth.noisy_pair(4011, 250, 330, 3, 25, dtype=np.float16)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16)
    out = _host(M.denoise(_dev(z), gb, storage=M.F16))
    out_l, maps, coarse, pyr = _gpu_levels(z, gb, torch.float16, True)
    assert np.array_equal(out, _host(out_l))
    _check_maps(maps, coarse, [_host(p) for p in pyr], bank)
    err = max_abs(out, _oracle_on_maps(z.astype(np.float64), bank, maps, np.float16))
    print(f"  max-abs vs fp16-mode oracle on the GPU's maps {err:.3g}")
    assert err <= TOL_F16
    assert O.psnr(out, u) > O.psnr(z, u) + 5
    with pytest.raises(M.MdnError) as e:
        M.Plan(gb, M.F16, max_images=4)
    assert e.value.status == M.MDN_ENOTSUP


@pytest.mark.parametrize("precision,tol", [(0, 2e-5), (1, 2e-4)])
def test_gram_coarse_selector(precision, tol):
    """Normal equations of a coarse-selector level: given the same coarser output, the buckets are the
    oracle's (counts exact) and G, b, yy lie within the accumulation bound of the training tests."""
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"gram coarse selector precision={precision}", flush=True)
    lb = _coarse_level(24, 3, 3)
    K = lb.K
    st = O.GramStats.zeros(K, 3, 98)
    g = M.Gram(K, 3, 3, 3)
    sel = gpu_level(lb, 3)
    for i, (H, W) in enumerate([(80, 80), (61, 90)]):
        z, u = synth.noisy_pair(300 + i, H, W, 3, 25)
        uc = _coarse_output(310 + i, H, W)
        s_o = O.select(z.astype(np.float64), lb.q_theta, lb.t_s, lb.t_c, selector="coarse",
                       u_coarse=uc.astype(np.float64))
        s_g = M.select_filters(_dev(z), sel, u_coarse=_dev(uc)).cpu().numpy()
        index_parity(s_g, z, lb, u_coarse=uc.astype(np.float64))
        assert np.array_equal(s_g, s_o)           # no pixel of these inputs lies at a boundary
        O.accumulate_level(st, s_o, O.to_filter_space(z.astype(np.float64)), O.to_filter_space(u.astype(np.float64)),
                           3, 3, uc.astype(np.float64))
        M.train_accumulate(g, _dev(z), _dev(u), sel, u_coarse=_dev(uc), coarse_color=M.YCC, precision=precision)
    worst = check_gram(g, st, tol)
    print(f"  worst ratio {worst:.3g}")
    del torch


def test_train_coarse_end_to_end():
    """Training with the coarse selector end to end. The coarsest trained level selects on z^L, the
    same input on both sides: its thresholds agree to rounding and its filters to the float32 normal
    equations. Finer levels select on the trained cascade's own outputs, which differ by those
    normal equations, so a pixel near a boundary may change bucket there (either bucket is correct):
    the oracle is trained again with the GPU's thresholds and the two banks must denoise a held-out
    image to the same PSNR (0.02 dB)."""
    import paper_1802_06130_amd as M
    print("train multiscale, coarse selector", flush=True)
    pairs = [synth.noisy_pair(90 + i, 96, 96, 3, 25) for i in range(3)]
    p64 = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    bank_g, _, _ = M.train_multiscale([(_dev(z), _dev(u)) for z, u in pairs], 2, 8, 3, 3, 3, 3, 1e-3,
                                      selector=M.SELECT_COARSE)
    bank_o, _, _ = O.train_multiscale(p64, 2, 8, 3, 3, 3, 3, 1e-3, storage=np.float32, selector="coarse")
    top_o, top_g = bank_o.levels[-1], bank_g.levels[-1]
    assert np.max(np.abs(top_o.t_s - top_g.t_s)) < 1e-12 and np.max(np.abs(top_o.t_c - top_g.t_c)) < 1e-9
    for lo, lg in zip(bank_o.levels, bank_g.levels):
        print(f"  thresholds: strength {np.max(np.abs(lo.t_s - lg.t_s)):.3g} coherence {np.max(np.abs(lo.t_c - lg.t_c)):.3g}")
        assert np.allclose(lo.t_s, lg.t_s, rtol=1e-3) and np.allclose(lo.t_c, lg.t_c, rtol=1e-3)
        assert lg.selector == M.SELECT_COARSE
    thr = [(lg.t_s, lg.t_c) for lg in bank_g.levels]
    bank_o, _, _ = O.train_multiscale(p64, 2, 8, 3, 3, 3, 3, 1e-3, thresholds=thr, storage=np.float32,
                                      selector="coarse")
    z, u = synth.noisy_pair(2006, 120, 160, 3, 25)
    lvls = [O.LevelBank(8, lg.t_s, lg.t_c, 3, 3, lg.coeffs.double().cpu().numpy(), "coarse") for lg in bank_g.levels]
    # the coarsest trained level alone: same buckets on both sides
    pyr = O.build_pyramid(z, 3, np.float32)
    zc = O.to_filter_space(pyr[2])
    s1 = O.select(pyr[1], 8, *thr[1], selector="coarse", u_coarse=zc)
    top = [O.apply_level(O.to_filter_space(pyr[1]), s1, b.levels[1], zc) for b in (O.Bank(lvls), bank_o)]
    err_top = max_abs(top[0], top[1])
    out_g = O.denoise(z, O.Bank(lvls), storage=np.float32)
    out_o = O.denoise(z, bank_o, storage=np.float32)
    d_psnr = O.psnr(out_g, u) - O.psnr(out_o, u)
    print(f"  coarsest level max-abs {err_top:.3g}; full cascade max-abs {max_abs(out_g, out_o):.3g}, "
          f"PSNR {O.psnr(z, u):.2f} -> {O.psnr(out_g, u):.3f} (GPU-trained) / {O.psnr(out_o, u):.3f} dB")
    assert err_top < 1e-3
    assert abs(d_psnr) < 0.02
