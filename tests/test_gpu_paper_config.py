"""The paper's experimental configuration (Section 5) on the GPU, through the
C ABI, against the oracle: 16 x 16 x 16 = 4096 buckets (uint16 selector maps), 7x7 denoise and 5x5
upscale filters, pyramid depth from the noise level.

Bars as everywhere: bucket maps equal the oracle's except at pixels within 1e-6 of a bucket
boundary; cascades within 1e-4 (float32) or 2e-3 (float16) of the oracle run on the GPU's maps,
every pixel; the normal equations' sample counts exact and G within 2e-5 sqrt(G_pp G_qq). The
batched form runs such banks on the tiled kernel in table mode and equals the per-image form bit
for bit.
"""

import numpy as np
import pytest

import oracle as O
import synth
from mdn_testlib import TOL_F16, TOL_F32, cascade_parity, gpu_bank, gpu_level, index_parity

pytestmark = pytest.mark.gpu

Q = (16, 16, 16)
K = 16 * 16 * 16


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def _thresholds(zs, q=16):
    f = [O.level_features(z.astype(np.float64)) for z in zs]
    return (O.thresholds_from_features(np.concatenate([x[0] for x in f]), q),
            O.thresholds_from_features(np.concatenate([x[1] for x in f]), q))


def _bank(L, rf, rg, seed=5):
    """Random (normalised) filters for inference plumbing; thresholds per level from the features of
    seeded scenes at that level (equal-population quantiles)."""
    zs = [synth.noisy_pair(300 + i, 160, 160, 3, 25)[0].astype(np.float64) for i in range(3)]
    levels = []
    for lev in range(L):
        t_s, t_c = _thresholds([O.build_pyramid(z, lev + 1)[lev] for z in zs])
        co = synth.random_bank_coeffs(seed + lev, K, 3, (2 * rf + 1) ** 2, (2 * rg + 1) ** 2)
        levels.append(O.LevelBank(16, t_s, t_c, rg, rf, co))
    return O.Bank(levels)


@pytest.mark.parametrize("H,W", [(1, 1), (17, 33), (130, 97), (768, 1024)])
@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_select_4096_buckets_uint16_map(H, W, dtype):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"select 4096 buckets {H}x{W} {np.dtype(dtype).name}", flush=True)
    lb = _bank(1, 2, 3).levels[0]
    z, _ = synth.noisy_pair(400 + W, H, W, 3, 25, dtype=dtype)
    s = M.select_filters(_dev(z), gpu_level(lb, 3))
    assert s.dtype == torch.uint16
    sn = s.cpu().numpy()
    _, n_mis, n_near = index_parity(sn, z.astype(np.float64), lb)
    print(f"  mismatches={n_mis} near-boundary={n_near} buckets used={len(np.unique(sn))}")
    if H * W > 100000:
        assert len(np.unique(sn)) > 2000 and int(sn.max()) > 255


def test_denoise_paper_configuration_f32():
    """sigma = 25: five-level pyramid (four trained levels), 7x7 denoise / 5x5 upscale filters."""
    L, rf, rg, q = O.paper_setup(25)
    assert (L, rf, rg, q) == (4, 2, 3, Q)
    bank = _bank(L, rf, rg)
    z, u = synth.noisy_pair(2010, 300, 412, 3, 25)
    gb = gpu_bank(bank, 3)
    cascade_parity(z, bank, gb, np.float32, TOL_F32, u=u)


@pytest.mark.parametrize("sigma", [5, 25])
def test_denoise_paper_configuration_f16(sigma):
    """Float16 pyramid, outputs and coefficients (float32 accumulation) at the paper's configuration
    for sigma: indices equal the oracle's in float16-storage mode except near boundaries, every pixel
    within 2e-3 of it on the GPU's maps, PSNR within 0.01 dB of the pure FP64 oracle."""
    torch = _torch()
    L, rf, rg, q = O.paper_setup(sigma)
    print(f"paper configuration f16 sigma={sigma}: {L + 1} levels, f {2 * rf + 1}x{2 * rf + 1}, "
          f"g {2 * rg + 1}x{2 * rg + 1}", flush=True)
    bank = _bank(L, rf, rg, seed=7)
    z, u = synth.noisy_pair(2030 + sigma, 300, 412, 3, sigma, dtype=np.float16)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16)
    cascade_parity(z, bank, gb, np.float16, TOL_F16, u=u, dpsnr_tol=0.01)


def test_apply_with_precomputed_uint16_map_equals_inline():
    import paper_1802_06130_amd as M
    torch = _torch()
    lb = _bank(1, 2, 3).levels[0]
    z, _ = synth.noisy_pair(2011, 120, 150, 3, 25)
    zc = M.pyramid_build(_dev(z), 1)[0]
    lv = gpu_level(lb, 3)
    s_out = torch.empty((120, 150), dtype=torch.uint16, device="cuda")
    a = M.apply_level(_dev(z), lv, u_coarse=zc, coarse_color=M.RGB, s_out=s_out)
    b = M.apply_level(_dev(z), lv, u_coarse=zc, coarse_color=M.RGB, s=M.select_filters(_dev(z), lv))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(s_out, M.select_filters(_dev(z), lv))
    with pytest.raises(M.MdnError):
        M.apply_level(_dev(z), lv, u_coarse=zc, coarse_color=M.RGB, s=torch.zeros((120, 150), dtype=torch.uint8,
                                                                                  device="cuda"))


def test_normal_equations_4096_buckets():
    import paper_1802_06130_amd as M
    print("gram 4096 buckets, 7x7 + 5x5", flush=True)
    pairs = [synth.noisy_pair(500 + i, 96, 112, 3, 25) for i in range(2)]
    t_s, t_c = _thresholds([z for z, _ in pairs])
    lb = O.LevelBank(16, t_s, t_c, 3, 2, np.zeros((K, 3, 74)))
    sel = gpu_level(lb, 3)
    g = M.Gram(K, 3, 3, 2)
    st = O.GramStats.zeros(K, 3, 74)
    for z, u in pairs:
        z64, u64 = z.astype(np.float64), u.astype(np.float64)
        zc = M.pyramid_build(_dev(z), 1)[0]
        M.train_accumulate(g, _dev(z), _dev(u), sel, u_coarse=zc, coarse_color=M.RGB)
        s = M.select_filters(_dev(z), sel).cpu().numpy().astype(np.int64)
        index_parity(s, z64, lb)
        pz = O.build_pyramid(z64, 2, storage=np.float32)
        O.accumulate_level(st, s, O.to_filter_space(z64), O.to_filter_space(u64), 3, 2, O.to_filter_space(pz[1]))
    assert np.array_equal(g.n.cpu().numpy(), st.n)
    Gg = g.G.cpu().numpy().reshape(st.G.shape)
    diag = np.sqrt(np.maximum(np.einsum("kcii->kci", st.G), 0.0))
    bound = 2e-5 * diag[:, :, :, None] * diag[:, :, None, :] + 1e-12
    worst = float((np.abs(Gg - st.G) / bound).max())
    print(f"  buckets hit {int((st.n > 0).sum())}, worst |dG| / bound = {worst:.3g}")
    assert worst <= 1.0


def test_train_paper_configuration_end_to_end():
    """sigma = 5: three-level pyramid, 5x5 denoise / 3x3 upscale filters, 4096 buckets (most fall back
    to the pooled solution with this little data), trained on both sides."""
    import paper_1802_06130_amd as M
    L, rf, rg, (qt, qs, qc) = O.paper_setup(5)
    assert (L, rf, rg) == (2, 1, 2)
    pairs = [synth.noisy_pair(600 + i, 96, 96, 3, 5) for i in range(3)]
    p64 = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    bank_o, _, fb_o = O.train_multiscale(p64, L, qt, qs, qc, rf, rg, 1e-3, storage=np.float32)
    bank_g, _, fb_g = M.train_multiscale([(_dev(z), _dev(u)) for z, u in pairs], L, qt, qs, qc, rf, rg, 1e-3)
    for lo, lg in zip(bank_o.levels, bank_g.levels):
        assert np.max(np.abs(lo.t_s - lg.t_s)) < 1e-12 and np.max(np.abs(lo.t_c - lg.t_c)) < 1e-9
    z, u = synth.noisy_pair(2012, 120, 160, 3, 5)
    lvls = [O.LevelBank(qt, lg.t_s, lg.t_c, rg, rf, lg.coeffs.double().cpu().numpy()) for lg in bank_g.levels]
    out_g = O.denoise(z, O.Bank(lvls), storage=np.float32)
    out_o = O.denoise(z, bank_o, storage=np.float32)
    err = float(np.max(np.abs(out_g - out_o)))
    print(f"  fallback systems GPU {fb_g} oracle {[3 * int(f.sum()) for f in fb_o]}; output max-abs {err:.3g}; "
          f"PSNR {O.psnr(z, u):.2f} -> {O.psnr(out_g, u):.2f} dB")
    assert err < 1e-3


@pytest.mark.parametrize("sigma,storage", [(25, "f16"), (5, "f16"), (25, "f32")])
def test_batched_form_equals_plain_on_the_paper_configuration(sigma, storage):
    """The batched form (one tiled launch per level over every image's 64 x 16 tiles, hipGraph
    replay) on 4096-bucket banks with the sigma's footprints and depth equals mdn_denoise bit for
    bit, on ragged images whose sizes cut tiles, strips and pyramid levels unevenly."""
    import paper_1802_06130_amd as M
    torch = _torch()
    L, rf, rg, _ = O.paper_setup(sigma)
    f16 = storage == "f16"
    print(f"batched paper configuration sigma={sigma} {storage}", flush=True)
    gb = gpu_bank(_bank(L, rf, rg, seed=11), 3, coeff_dtype=torch.float16 if f16 else torch.float32)
    code = M.F16 if f16 else M.F32
    dt = np.float16 if f16 else np.float32
    sizes = [(300, 412), (61, 97), (17, 129), (128, 40), (1, 1)]
    zs = [_dev(synth.noisy_pair(2100 + i, h, w, 3, sigma, dtype=dt)[0]) for i, (h, w) in enumerate(sizes)]
    plan = M.Plan(gb, code, max_images=8)
    rows = plan.autotune(zs)
    outs = None
    for _ in range(2):                 # capture, then replay
        outs = plan.denoise_batch(zs, outs, use_graph=True)
    torch.cuda.synchronize()
    for zt, ob, (h, w) in zip(zs, outs, sizes):
        op = M.denoise(zt, gb, storage=code)
        torch.cuda.synchronize()
        assert torch.equal(ob, op), f"{h}x{w}: batched differs from per-image"
    kt = plan.kernel_times(zs, reps=1)
    print(f"  rows {rows}; kernel us per level {kt}", flush=True)
    plan.close()


def test_batched_form_equals_plain_on_a_phase_aware_bank():
    import paper_1802_06130_amd as M
    torch = _torch()
    print("batched phase-aware bank", flush=True)
    zs0 = [synth.noisy_pair(300 + i, 160, 160, 3, 25)[0].astype(np.float64) for i in range(3)]
    levels = []
    for lev in range(3):
        t_s, t_c = _thresholds([O.build_pyramid(z, lev + 1)[lev] for z in zs0], 3)
        co = synth.random_bank_coeffs(60 + lev, 24 * 3 * 3 * 4, 3, 49, 49)
        levels.append(O.LevelBank(24, t_s, t_c, 3, 3, co, phases=4))
    gb = gpu_bank(O.Bank(levels), 3, coeff_dtype=torch.float16)
    zs = [_dev(synth.noisy_pair(2200 + i, h, w, 3, 25, dtype=np.float16)[0])
          for i, (h, w) in enumerate([(250, 330), (61, 97), (33, 40)])]
    plan = M.Plan(gb, M.F16, max_images=4)
    outs = plan.denoise_batch(zs, use_graph=True)
    torch.cuda.synchronize()
    for zt, ob in zip(zs, outs):
        assert torch.equal(ob, M.denoise(zt, gb, storage=M.F16))
    plan.close()


def test_plan_refusals():
    """Single-scale banks and float32 banks that fit in LDS one channel at a time stay per-image."""
    import paper_1802_06130_amd as M
    torch = _torch()
    from mdn_testlib import trained_bank_multiscale, trained_bank_single
    for bank, dt in ((trained_bank_single(channels=3), torch.float32), (trained_bank_multiscale(levels=2), torch.float32)):
        with pytest.raises(M.MdnError) as e:
            M.Plan(gpu_bank(bank, 3, coeff_dtype=dt), M.F32, max_images=2)
        assert e.value.status == M.MDN_ENOTSUP
