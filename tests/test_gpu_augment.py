"""Training-set augmentation (Section 5) on the GPU, through the C ABI, against the oracle.

- mdn_dihedral moves every element of every plane bit for bit as the oracle's symmetry does,
  for both dtypes, ragged sizes and all eight symmetries;
- the normal equations of an augmented training set match the oracle's, accumulated over the
  GPU's own selector maps (each map checked first: mismatches only near bucket boundaries);
- a multiscale bank trained with augmentation gives outputs close to the oracle's augmented bank.
"""

import numpy as np
import pytest

import oracle as O
import synth
from mdn_testlib import index_parity

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("shape", [(1, 37, 53), (3, 70, 33), (3, 64, 96), (3, 1, 40)])
@pytest.mark.parametrize("dtype", [np.float16, np.float32])
def test_dihedral_matches_oracle_bitwise(shape, dtype):
    import paper_1802_06130_amd as M
    print(f"dihedral {shape} {np.dtype(dtype).name}", flush=True)
    x = np.random.default_rng(3).random(shape).astype(dtype)
    xd = _dev(x)
    for t in range(8):
        got = M.dihedral(xd, t).cpu().numpy()
        ref = O.dihedral(x, t)
        assert got.shape == ref.shape
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), f"transform {t}"


def test_augmented_normal_equations_match_oracle():
    import paper_1802_06130_amd as M
    print("augmented gram (rgb multiscale)", flush=True)
    pairs = [synth.noisy_pair(60 + i, 48, 40, 3, 25) for i in range(2)]
    q_theta, t_s, t_c = 24, [0.03, 0.06], [0.25, 0.5]
    K = q_theta * 9
    lb = O.LevelBank(q_theta, np.array(t_s), np.array(t_c), 3, 3, np.zeros((K, 3, 98)))
    sel = M.Level(q_theta, t_s, t_c, 3, 3, _torch().zeros((K, 3, 98), device="cuda"), 3)
    g = M.Gram(K, 3, 3, 3)
    st = O.GramStats.zeros(K, 3, 98)
    aug = M.augment_pairs([(_dev(z), _dev(u)) for z, u in pairs])
    assert len(aug) == 16
    for zt, ut in aug:
        zc = M.pyramid_build(zt, 1)[0]
        M.train_accumulate(g, zt, ut, sel, u_coarse=zc, coarse_color=M.RGB)
        z64, u64 = zt.cpu().numpy().astype(np.float64), ut.cpu().numpy().astype(np.float64)
        s = M.select_filters(zt, sel).cpu().numpy()
        index_parity(s, z64, lb)
        pz = O.build_pyramid(z64, 2, storage=np.float32)
        O.accumulate_level(st, s.astype(np.int64), O.to_filter_space(z64), O.to_filter_space(u64), 3, 3,
                           O.to_filter_space(pz[1]))
    Gg = g.G.cpu().numpy().reshape(st.G.shape)
    assert np.array_equal(g.n.cpu().numpy(), st.n)
    diag = np.sqrt(np.maximum(np.einsum("kcii->kci", st.G), 0.0))
    bound = 2e-5 * diag[:, :, :, None] * diag[:, :, None, :] + 1e-12
    worst = float((np.abs(Gg - st.G) / bound).max())
    print(f"  samples {int(st.n.sum())}, worst |dG| / (2e-5 sqrt(GppGqq)) = {worst:.3g}")
    assert worst <= 1.0


def test_train_multiscale_augmented_end_to_end():
    import paper_1802_06130_amd as M
    print("train multiscale with augmentation", flush=True)
    pairs = [synth.noisy_pair(70 + i, 64, 64, 3, 25) for i in range(2)]
    p64 = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    thr = [([0.03, 0.06], [0.25, 0.5]), ([0.02, 0.04], [0.25, 0.5])]
    bank_o, _, _ = O.train_multiscale(p64, 2, 8, 3, 3, 3, 3, 1e-3, thresholds=thr, storage=np.float32, augment=True)
    bank_g, grams, _ = M.train_multiscale([(_dev(z), _dev(u)) for z, u in pairs], 2, 8, 3, 3, 3, 3, 1e-3,
                                          thresholds=thr, augment=True)
    assert int(grams[0].n.sum()) == 8 * 2 * 64 * 64
    z, u = synth.noisy_pair(2002, 120, 160, 3, 25)
    lvls = [O.LevelBank(8, np.array(t[0]), np.array(t[1]), 3, 3, lv.coeffs.double().cpu().numpy())
            for t, lv in zip(thr, bank_g.levels)]
    out_g = O.denoise(z, O.Bank(lvls), storage=np.float32)
    out_o = O.denoise(z, bank_o, storage=np.float32)
    err = float(np.max(np.abs(out_g - out_o)))
    print(f"  output max-abs (GPU-trained vs oracle-trained, oracle cascade) {err:.3g}; "
          f"PSNR {O.psnr(z, u):.2f} -> {O.psnr(out_g, u):.2f} dB")
    assert err < 1e-3
