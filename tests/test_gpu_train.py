"""GPU training path against the FP64 oracle (Eq. (7)-(8)), through the C ABI.

- normal equations: sample counts exact; G, b, yy entrywise within the FP32 (or BF16 hi/lo)
  accumulation bound |dG_pq| <= tol * sqrt(G_pp G_qq) (Cauchy-Schwarz bound on sum |x_p x_q|);
- solve: the GPU float64 Cholesky on the oracle's own normal equations reproduces the oracle's
  coefficients (1e-9) and fallback set;
- planted filters are recovered from noise-free pairs;
- end to end, filters trained on the GPU give outputs close to the oracle-trained filters'.
"""

import numpy as np
import pytest

import oracle as O
import synth
from mdn_testlib import check_gram as _check_gram

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _pairs(n, size, C, sigma=25.0, seed0=1):
    return [synth.noisy_pair(seed0 + i, size, size, C, sigma) for i in range(n)]


def _oracle_single_stats(pairs, q_theta, t_s, t_c, radius):
    K = q_theta * (len(t_s) + 1) * (len(t_c) + 1)
    C = pairs[0][0].shape[0]
    st = O.GramStats.zeros(K, C, (2 * radius + 1) ** 2)
    for z, u in pairs:
        s = O.select(z.astype(np.float64), q_theta, t_s, t_c)
        O.accumulate_level(st, s, O.to_filter_space(z), O.to_filter_space(u), radius)
    return st


@pytest.mark.parametrize("precision,tol", [(0, 2e-5), (1, 2e-4)])
def test_gram_single_scale_grey(precision, tol):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"gram grey precision={precision}", flush=True)
    pairs = _pairs(4, 96, 1)
    feats = [O.level_features(z.astype(np.float64)) for z, _ in pairs]
    t_s = O.thresholds_from_features(np.concatenate([f[0] for f in feats]), 3)
    t_c = O.thresholds_from_features(np.concatenate([f[1] for f in feats]), 3)
    st = _oracle_single_stats(pairs, 16, t_s, t_c, 2)
    g = M.Gram(144, 1, 2)
    sel = M.Level(16, t_s, t_c, 2, None, torch.zeros((144, 1, 25), device="cuda"), 1)
    for z, u in pairs:
        M.train_accumulate(g, _dev(z), _dev(u), sel, precision=precision)
    worst = _check_gram(g, st, tol)
    print(f"  worst |dG| / (tol sqrt(GppGqq)) = {worst:.3g}")


@pytest.mark.parametrize("precision,tol", [(0, 2e-5), (1, 2e-4)])
def test_gram_multiscale_rgb(precision, tol):
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"gram rgb multiscale precision={precision}", flush=True)
    pairs = _pairs(2, 80, 3)
    q_theta, t_s, t_c = 24, [0.03, 0.06], [0.25, 0.5]
    K = q_theta * 9
    st = O.GramStats.zeros(K, 3, 98)
    g = M.Gram(K, 3, 3, 3)
    sel = M.Level(q_theta, t_s, t_c, 3, 3, torch.zeros((K, 3, 98), device="cuda"), 3)
    for z, u in pairs:
        z64, u64 = z.astype(np.float64), u.astype(np.float64)
        pz = O.build_pyramid(z64, 2, storage=np.float32)
        pu = O.build_pyramid(u64, 2, storage=np.float32)
        s = O.select(z64, q_theta, t_s, t_c)
        O.accumulate_level(st, s, O.to_filter_space(z64), O.to_filter_space(u64), 3, 3, O.to_filter_space(pz[1]))
        zc = M.pyramid_build(_dev(z), 1)[0]
        M.train_accumulate(g, _dev(z), _dev(u), sel, u_coarse=zc, coarse_color=M.RGB, precision=precision)
        del pu
    worst = _check_gram(g, st, tol)
    print(f"  worst ratio {worst:.3g}")


def _gap_thresholds(f, q):
    """q - 1 thresholds near the feature's quantiles, each the midpoint of the widest gap between
    neighbouring sorted values in a small window, so that no pixel sits within rounding of one."""
    v = np.sort(np.asarray(f, dtype=np.float64).ravel())
    t = []
    for j in range(1, q):
        i = int(j * len(v) / q)
        lo, hi = max(0, i - 8), min(len(v) - 1, i + 8)
        k = lo + int(np.argmax(np.diff(v[lo:hi + 1])))
        t.append(0.5 * (v[k] + v[k + 1]))
    return t


@pytest.mark.parametrize("q_theta,q,phases,H,W,n", [(64, 16, 1, 96, 96, 3), (64, 16, 4, 96, 96, 3),
                                                     (16, 16, 1, 512, 768, 1), (2, 1, 1, 256, 320, 2)])
def test_gram_with_many_buckets(q_theta, q, phases, H, W, n):
    """The bucket grouping at its limits: 16384 buckets and 65536 with phases (the largest K, 16-bit
    keys, running positions in global memory), 4096 buckets over 393216 pixels (slices of 512 pixels,
    768 scan blocks, positions in LDS), and 2 buckets (one-bit keys; runs of about 80000 samples, so
    each bucket's partial sums span many work items): the normal equations match bucket by bucket."""
    import paper_1802_06130_amd as M
    torch = _torch()
    K = q_theta * q * q * phases
    print(f"gram grey K={K} {H}x{W} x{n}", flush=True)
    pairs = _pairs(n, H, 1, seed0=40) if H == W else [synth.noisy_pair(40 + i, H, W, 1, 25.0) for i in range(n)]
    feats = [O.level_features(z.astype(np.float64)) for z, _ in pairs]
    t_s = _gap_thresholds(np.concatenate([f[0].ravel() for f in feats]), q)
    t_c = _gap_thresholds(np.concatenate([f[1].ravel() for f in feats]), q)
    st = O.GramStats.zeros(K, 1, 9)
    for z, u in pairs:
        s = O.select(z.astype(np.float64), q_theta, t_s, t_c, phases=phases)
        O.accumulate_level(st, s, O.to_filter_space(z), O.to_filter_space(u), 1)
    assert np.count_nonzero(st.n) > min(1000, K - 1)
    g = M.Gram(K, 1, 1)
    sel = M.Level(q_theta, t_s, t_c, 1, None, torch.zeros((K, 1, 9), device="cuda"), 1, phases=phases)
    for z, u in pairs:
        M.train_accumulate(g, _dev(z), _dev(u), sel, precision=0)
    worst = _check_gram(g, st, 2e-5)
    print(f"  worst ratio {worst:.3g}")


@pytest.mark.parametrize("precision,tol", [(0, 2e-5), (1, 2e-4)])
@pytest.mark.parametrize("H,W", [(1, 1), (2, 3), (7, 1), (17, 33), (66, 130)])
def test_gram_multiscale_rgb_small_and_ragged(H, W, precision, tol):
    """Single pixels, slivers and sizes with ragged 64-sample chunks: one work item or a few, slices
    of the grouping shorter than a wave, margins wider than the image."""
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"gram rgb multiscale {H}x{W} precision={precision}", flush=True)
    pairs = [synth.noisy_pair(90 + i, H, W, 3, 25.0) for i in range(3)]
    q_theta, t_s, t_c = 24, [0.03, 0.06], [0.25, 0.5]
    K = q_theta * 9
    st = O.GramStats.zeros(K, 3, 98)
    g = M.Gram(K, 3, 3, 3)
    sel = M.Level(q_theta, t_s, t_c, 3, 3, torch.zeros((K, 3, 98), device="cuda"), 3)
    for z, u in pairs:
        z64, u64 = z.astype(np.float64), u.astype(np.float64)
        pz = O.build_pyramid(z64, 2, storage=np.float32)
        s = O.select(z64, q_theta, t_s, t_c)
        O.accumulate_level(st, s, O.to_filter_space(z64), O.to_filter_space(u64), 3, 3, O.to_filter_space(pz[1]))
        zc = M.pyramid_build(_dev(z), 1)[0]
        M.train_accumulate(g, _dev(z), _dev(u), sel, u_coarse=zc, coarse_color=M.RGB, precision=precision)
    assert int(st.n.sum()) == 3 * H * W
    worst = _check_gram(g, st, tol)
    print(f"  worst ratio {worst:.3g}")


@pytest.mark.parametrize("precision,tol", [(0, 2e-5), (1, 2e-4)])
def test_gram_cross_channel_147(precision, tol):
    """Cross-channel layout (x = the three channels' 7x7 patches, D = 147, three right-hand sides)
    against the oracle's cross-channel normal equations; then the solved filters' output-space error
    against the oracle's solution, relative to the target energy."""
    import paper_1802_06130_amd as M
    torch = _torch()
    print(f"gram cross-channel precision={precision}", flush=True)
    pairs = _pairs(3, 72, 3)
    q_theta, t_s, t_c = 8, [0.03, 0.06], [0.25, 0.5]
    K, C, D = q_theta * 9, 3, 147
    st = O.CrossGramStats.zeros(K, C, D)
    g = M.Gram(K, 3, 3, None, layout=M.X_CROSS_CHANNEL)
    sel = M.Level(q_theta, t_s, t_c, 3, None, torch.zeros((K, 3, 49), device="cuda"), 3)
    for z, u in pairs:
        z64, u64 = z.astype(np.float64), u.astype(np.float64)
        s = O.select(z64, q_theta, t_s, t_c)
        O.accumulate_level_cross(st, s, O.to_filter_space(z64), O.to_filter_space(u64), 3)
        M.train_accumulate(g, _dev(z), _dev(u), sel, precision=precision)
    G = g.G.cpu().numpy().reshape(K, D, D)
    b = g.b.cpu().numpy().reshape(K, C, D)
    assert np.array_equal(g.n.cpu().numpy(), st.n), "sample counts differ"
    diag = np.sqrt(np.maximum(np.einsum("kii->ki", st.G), 0.0))
    ratio = np.abs(G - st.G) / (tol * diag[:, :, None] * diag[:, None, :] + 1e-12)
    assert ratio.max() <= 1.0, f"G outside bound (worst ratio {ratio.max():.3g})"
    yd = np.sqrt(np.maximum(st.yy, 0.0))
    assert np.all(np.abs(b - st.b) <= tol * diag[:, None, :] * yd[:, :, None] + 1e-12)
    lam = 1e-3
    h_ref, fb = O.solve_level_cross(st, lam)
    co, nfb = M.train_solve(g, lam)
    assert nfb == int(fb.sum())
    dh = co.double().cpu().numpy() - h_ref
    err = sum(dh[k, c] @ st.G[k] @ dh[k, c] for k in range(K) for c in range(C))
    rel = float(np.sqrt(err / st.yy.sum()))
    print(f"  worst G ratio {ratio.max():.3g}; output-space rms error / target rms {rel:.3g}")
    assert rel <= (1e-4 if precision == 0 else 1e-3)


def test_solve_on_oracle_normal_equations():
    import paper_1802_06130_amd as M
    torch = _torch()
    pairs = _pairs(4, 96, 1)
    t_s, t_c = [0.04, 0.08], [0.2, 0.45]
    st = _oracle_single_stats(pairs, 16, t_s, t_c, 2)
    want, fb = O.solve_level(st, 1e-3)
    g = M.Gram(144, 1, 2)
    g.G.copy_(torch.from_numpy(st.G.reshape(-1)))
    g.b.copy_(torch.from_numpy(st.b.reshape(-1)))
    g.n.copy_(torch.from_numpy(st.n))
    g.yy.copy_(torch.from_numpy(st.yy.reshape(-1)))
    co, nfb = M.train_solve(g, 1e-3)
    got = co.double().cpu().numpy()
    assert nfb == int(fb.sum())
    # float32 output of a float64 solve: compare to float32 rounding of the oracle
    assert np.max(np.abs(got - want.astype(np.float32))) <= 4 * np.finfo(np.float32).eps * max(1.0, np.abs(want).max())


def test_solve_cross_channel_three_rhs():
    import paper_1802_06130_amd as M
    torch = _torch()
    rng = np.random.default_rng(3)
    K, D = 4, 147
    g = M.Gram(K, 3, 3, None, layout=M.X_CROSS_CHANNEL)
    assert (g.D, g.nrhs, g.systems) == (147, 3, K)
    Gs, bs, hs = [], [], []
    for k in range(K):
        X = rng.normal(0, 1, (600, D))
        Y = rng.normal(0, 1, (600, 3))
        Gs.append(X.T @ X)
        bs.append((X.T @ Y).T)
        hs.append(np.linalg.solve(X.T @ X / 600 + 1e-3 * np.eye(D), (X.T @ Y / 600)))
    g.G.copy_(torch.from_numpy(np.stack(Gs).reshape(-1)))
    g.b.copy_(torch.from_numpy(np.stack(bs).reshape(-1)))
    g.n.fill_(600)
    co, nfb = M.train_solve(g, 1e-3)
    got = co.double().cpu().numpy()        # [K][3][147]
    want = np.stack([h.T for h in hs])
    assert nfb == 0
    assert np.max(np.abs(got - want)) < 1e-5


@pytest.mark.parametrize("precision,tol", [(0, 2e-4), (1, 2e-3)])
def test_planted_recovery_single_scale(precision, tol):
    """Noise-free targets made by planted per-bucket filters are recovered at lambda = 0."""
    import paper_1802_06130_amd as M
    torch = _torch()
    rng = np.random.default_rng(9)
    q_theta, t_s, t_c = 4, [0.3], [0.3]
    K, D = 16, 25
    planted = rng.normal(0, 0.3, (K, 1, D))
    zs = [rng.uniform(0, 1, (1, 96, 96)).astype(np.float32) for _ in range(6)]
    pairs = []
    for z in zs:
        s = O.select(z.astype(np.float64), q_theta, t_s, t_c)
        u = O.apply_level(z.astype(np.float64), s, O.LevelBank(q_theta, np.array(t_s), np.array(t_c), 2, None, planted))
        pairs.append((_dev(z), _dev(u.astype(np.float32))))
    bank, g, nfb = M.train_single(pairs, q_theta, 2, 2, 2, 0.0, thresholds=(t_s, t_c), precision=precision)
    assert nfb == 0
    got = bank.levels[0].coeffs.double().cpu().numpy()
    err = np.max(np.abs(got - planted))
    print(f"  planted recovery max coefficient error {err:.3g}")
    assert err < tol


def test_train_single_end_to_end_close_to_oracle():
    import paper_1802_06130_amd as M
    print("train single end-to-end", flush=True)
    pairs = _pairs(8, 128, 1)
    bank_o, _, fb_o = O.train_single([(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs], 16, 3, 3, 2, 1e-3)
    lb = bank_o.levels[0]
    bank_g, _, nfb = M.train_single([(_dev(z), _dev(u)) for z, u in pairs], 16, 3, 3, 2, 1e-3,
                                    thresholds=(lb.t_s, lb.t_c))
    assert nfb == int(fb_o.sum())
    cg = bank_g.levels[0].coeffs.double().cpu().numpy()
    # output-space error on a held-out image, both filter sets applied by the oracle on the same selection
    z, u = synth.noisy_pair(1001, 256, 256, 1, 25)
    s = O.select(z.astype(np.float64), 16, lb.t_s, lb.t_c)
    out_o = O.apply_level(z.astype(np.float64), s, lb)
    out_g = O.apply_level(z.astype(np.float64), s, O.LevelBank(16, lb.t_s, lb.t_c, 2, None, cg))
    err = float(np.max(np.abs(out_o - out_g)))
    coef = float(np.max(np.abs(cg - lb.coeffs)))
    print(f"  coefficient max-abs {coef:.3g}, output max-abs {err:.3g}")
    assert err < 1e-4


def test_train_multiscale_end_to_end():
    import paper_1802_06130_amd as M
    print("train multiscale end-to-end", flush=True)
    pairs = _pairs(4, 96, 3)
    p64 = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    thr = [([0.03, 0.06], [0.25, 0.5]), ([0.02, 0.04], [0.25, 0.5])]
    bank_o, _, fbs_o = O.train_multiscale(p64, 2, 8, 3, 3, 3, 3, 1e-3, thresholds=thr, storage=np.float32)
    bank_g, _, fbs = M.train_multiscale([(_dev(z), _dev(u)) for z, u in pairs], 2, 8, 3, 3, 3, 3, 1e-3,
                                        thresholds=thr)
    assert fbs == [3 * int(f.sum()) for f in fbs_o]      # fallback systems = buckets x channels
    z, u = synth.noisy_pair(2001, 200, 240, 3, 25)
    lvls = [O.LevelBank(8, np.array(t[0]), np.array(t[1]), 3, 3, lv.coeffs.double().cpu().numpy())
            for t, lv in zip(thr, bank_g.levels)]
    out_g = O.denoise(z, O.Bank(lvls), storage=np.float32)
    out_o = O.denoise(z, bank_o, storage=np.float32)
    err = float(np.max(np.abs(out_g - out_o)))
    print(f"  output max-abs (GPU-trained vs oracle-trained, oracle cascade) {err:.3g}; "
          f"PSNR {O.psnr(z, u):.2f} -> {O.psnr(out_g, u):.2f} dB")
    assert err < 1e-3


def test_thresholds_match_oracle_quantiles():
    import paper_1802_06130_amd as M
    pairs = _pairs(3, 64, 3)
    zs = [z for z, _ in pairs]
    t_s, t_c = M.level_thresholds([_dev(z) for z in zs], 3, 3)
    feats = [O.level_features(z.astype(np.float64)) for z in zs]
    ws = O.thresholds_from_features(np.concatenate([f[0] for f in feats]), 3)
    wc = O.thresholds_from_features(np.concatenate([f[1] for f in feats]), 3)
    assert np.max(np.abs(t_s - ws)) < 1e-12 and np.max(np.abs(t_c - wc)) < 1e-12


def test_features_match_oracle():
    import paper_1802_06130_amd as M
    z, _ = synth.noisy_pair(8, 70, 90, 3, 25)
    st, co = M.level_features(_dev(z))
    a, b, c = O.structure_tensor(z.astype(np.float64))
    _, s_o, c_o = O.eigen_features(a, b, c)
    assert np.max(np.abs(st.cpu().numpy() - s_o)) < 1e-13
    assert np.max(np.abs(co.cpu().numpy() - c_o)) < 1e-9
