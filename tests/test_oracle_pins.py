"""Pins of the FP64 oracle against closed forms, invariants, published constants and
brute force, so that a plausible slip in the oracle (a dropped term, a wrong sign or
index, a transposed operand) fails here. CPU only."""

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


# ------------------------------------------------------------------ colour (footnote of Section 3)

def test_ycc_matches_published_bt601_matrix():
    rows = _golden_rows("bt601_full_range.txt")
    M = np.array([[float(v) for v in r.split()] for r in rows[:3]])
    off = np.array([float(v) for v in rows[3].split()[1:]])
    rgb = np.random.default_rng(0).uniform(0, 1, (3, 5, 7))
    want = np.einsum("ij,jhw->ihw", M, rgb) + off[:, None, None]
    assert np.max(np.abs(O.rgb_to_ycc(rgb) - want)) < 2e-6


def test_ycc_grey_and_round_trip():
    v = np.linspace(0, 1, 11)
    grey = np.stack([v, v, v])[:, None, :]
    ycc = O.rgb_to_ycc(grey)
    assert np.max(np.abs(ycc[0] - v)) < 1e-15
    assert np.max(np.abs(ycc[1:] - 0.5)) < 1e-15
    rgb = np.random.default_rng(1).uniform(0, 1, (3, 6, 4))
    assert np.max(np.abs(O.ycc_to_rgb(O.rgb_to_ycc(rgb)) - rgb)) < 1e-14


# ------------------------------------------------------------------ pyramid (Section 4)

def test_down2_weights_closed_form():
    rows = _golden_rows("down2_bicubic_weights.txt")
    num = np.array([float(v) for v in rows[0].split()])
    assert np.array_equal(O.down2_weights() * 1024.0, num)
    assert O.down2_weights().sum() == 1.0
    gain = float(rows[1])
    assert abs((O.down2_weights() ** 2).sum() - gain) < 1e-15


def test_down2_constant_sizes_and_ramp():
    for H, W in [(1, 1), (3, 5), (8, 8), (33, 17)]:
        x = np.full((2, H, W), 0.37)
        y = O.down2(x)
        assert y.shape == (2, (H + 1) // 2, (W + 1) // 2)
        assert np.max(np.abs(y - 0.37)) < 1e-15
    # a linear ramp is reproduced exactly at the output sample positions 2m + 1/2
    H, W = 40, 48
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    alpha, beta, c0 = 0.013, -0.007, 0.4
    x = (c0 + alpha * xx + beta * yy)[None]
    y = O.down2(x)[0]
    m_y, m_x = np.mgrid[0:H // 2, 0:W // 2].astype(float)
    want = c0 + alpha * (2 * m_x + 0.5) + beta * (2 * m_y + 0.5)
    inner = (slice(2, H // 2 - 2), slice(2, W // 2 - 2))
    assert np.max(np.abs(y[inner] - want[inner])) < 1e-14


def test_down2_halves_noise():
    """The paper: downsampling by two roughly halves the noise level (Section 4)."""
    n = np.random.default_rng(5).standard_normal((1, 1024, 1024))
    g = O.down2(n)[0][8:-8, 8:-8].std()
    assert abs(g - 0.40442) < 0.004


def test_down2_brute_force():
    x = np.random.default_rng(3).uniform(0, 1, (1, 7, 9))
    w = [-12, -36, 116, 444, 444, 116, -36, -12]
    H, W = 7, 9
    out = np.zeros((4, 5))
    for m in range(4):
        for n in range(5):
            acc = 0.0
            for i, ty in enumerate(range(-3, 5)):
                for j, tx in enumerate(range(-3, 5)):
                    yy = min(max(2 * m + ty, 0), H - 1)
                    xx = min(max(2 * n + tx, 0), W - 1)
                    acc += w[i] * w[j] * x[0, yy, xx]
            out[m, n] = acc / 1024.0 / 1024.0
    assert np.max(np.abs(O.down2(x)[0] - out)) < 1e-14


# ------------------------------------------------------------------ selection (Section 3, Eq. (3)-(6))

def _ramp(H, W, alpha, beta, C=3, c0=0.3):
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    return np.stack([c0 + alpha * xx + beta * yy] * C)


@pytest.mark.parametrize("alpha,beta", [(0.01, 0.0), (0.0, 0.02), (0.011, 0.004), (-0.006, 0.013), (0.009, -0.009)])
def test_ramp_orientation_strength_coherence(alpha, beta):
    H, W, C = 20, 24, 3
    z = _ramp(H, W, alpha, beta, C)
    gx, gy = O.gradients(z)
    inner = (slice(1, H - 1), slice(1, W - 1))
    assert np.max(np.abs(gx[:, 1:-1, 1:-1] - alpha)) < 1e-15
    assert np.max(np.abs(gy[:, 1:-1, 1:-1] - beta)) < 1e-15
    a, b, c = O.structure_tensor(z)
    theta, strength, coh = O.eigen_features(a, b, c)
    core = (slice(3, H - 3), slice(3, W - 3))
    want_theta = np.mod(np.arctan2(beta, alpha) + np.pi / 2, np.pi)
    d = np.abs(theta[core] - want_theta)
    d = np.minimum(d, np.pi - d)
    assert np.max(d) < 1e-7
    assert np.max(np.abs(strength[core] - np.sqrt(C * (alpha ** 2 + beta ** 2)))) < 1e-15
    assert np.min(coh[core]) > 1 - 1e-6
    del inner


def test_orientation_is_edge_direction():
    """A vertical edge (intensity varies along x) has orientation pi/2 (the edge runs along y)."""
    z = np.zeros((3, 16, 16))
    z[:, :, 8:] = 1.0
    a, b, c = O.structure_tensor(z)
    theta, strength, coh = O.eigen_features(a, b, c)
    assert abs(theta[8, 8] - np.pi / 2) < 1e-12 and coh[8, 8] > 0.999
    zt = np.transpose(z, (0, 2, 1)).copy()   # horizontal edge
    a, b, c = O.structure_tensor(zt)
    theta, _, _ = O.eigen_features(a, b, c)
    assert min(theta[8, 8], np.pi - theta[8, 8]) < 1e-12


def test_features_against_eigh_and_mpmath():
    import mpmath as mp
    mp.mp.dps = 50
    rng = np.random.default_rng(7)
    a = rng.uniform(0, 1, 200) ** 3
    c = rng.uniform(0, 1, 200) ** 3
    b = rng.uniform(-1, 1, 200) * np.sqrt(a * c)
    theta, strength, coh = O.eigen_features(a, b, c)
    for i in range(200):
        T = np.array([[a[i], b[i]], [b[i], c[i]]])
        w, V = np.linalg.eigh(T)       # ascending eigenvalues
        minor = V[:, 0]
        ang = np.mod(np.arctan2(minor[1], minor[0]), np.pi)
        d = abs(ang - theta[i])
        assert min(d, np.pi - d) < 1e-7
        am, bm, cm = mp.mpf(a[i]), mp.mpf(b[i]), mp.mpf(c[i])
        tr = am + cm
        mu = mp.sqrt((am - cm) ** 2 + 4 * bm * bm)
        l1, l2 = (tr + mu) / 2, max((tr - mu) / 2, mp.mpf(0))
        assert abs(float(mp.sqrt(l1)) - strength[i]) < 1e-14
        cm_ = (mp.sqrt(l1) - mp.sqrt(l2)) / (mp.sqrt(l1) + mp.sqrt(l2))
        assert abs(float(cm_) - coh[i]) < 1e-7 * max(1.0, float(mp.sqrt(l1 / max(l2, mp.mpf(1e-300)))) * 1e-8)


def _structure_tensor_exact(z_frac, H, W, C, r=2):
    """Eq. (5)-(6) literally, in exact rational arithmetic: sum_j w_j G_j G_j^T with the
    2 x C colour Jacobian G_j, box weights 1/25, all indices clamped."""
    def cl(v, n):
        return min(max(v, 0), n - 1)

    def jac(y, x):
        G = [[None] * C, [None] * C]
        for ch in range(C):
            G[0][ch] = (z_frac[ch][y][cl(x + 1, W)] - z_frac[ch][y][cl(x - 1, W)]) / 2
            G[1][ch] = (z_frac[ch][cl(y + 1, H)][x] - z_frac[ch][cl(y - 1, H)][x]) / 2
        return G

    n = (2 * r + 1) ** 2
    T = {}
    for y in range(H):
        for x in range(W):
            acc = [[Fraction(0)] * 2 for _ in range(2)]
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    G = jac(cl(y + dy, H), cl(x + dx, W))
                    for p in range(2):
                        for q in range(2):
                            acc[p][q] += sum(G[p][ch] * G[q][ch] for ch in range(C)) / n
            T[y, x] = acc
    return T


@pytest.mark.parametrize("H,W,C", [(1, 1, 3), (3, 5, 3), (7, 6, 1), (9, 7, 3)])
def test_structure_tensor_exact_rational(H, W, C):
    rng = np.random.default_rng(H * 100 + W)
    k = rng.integers(0, 256, (C, H, W))
    z = k / 255.0
    zf = [[[Fraction(int(k[ch, y, x]), 255) for x in range(W)] for y in range(H)] for ch in range(C)]
    T = _structure_tensor_exact(zf, H, W, C)
    a, b, c = O.structure_tensor(z)
    for (y, x), t in T.items():
        scale = float(t[0][0] + t[1][1]) + 1e-300
        assert abs(float(t[0][0]) - a[y, x]) <= 1e-14 * scale
        assert abs(float(t[0][1]) - b[y, x]) <= 1e-14 * scale
        assert abs(float(t[1][0]) - b[y, x]) <= 1e-14 * scale
        assert abs(float(t[1][1]) - c[y, x]) <= 1e-14 * scale


def test_constant_image_flat_bucket():
    for q_theta in (16, 24):
        z = np.full((3, 12, 10), 0.42)
        s = O.select(z, q_theta, [0.01, 0.02], [0.3, 0.6])
        assert np.all(s == ((q_theta // 2) * 3 + 0) * 3 + 0)


def test_quantize_layout_and_ties():
    theta = np.array([0.0, np.pi / 24 * 1.5, np.pi - 1e-12, np.pi / 2])
    st = np.array([0.1, 0.2, 0.3, 0.2])
    co = np.array([0.5, 0.6, 0.0, 0.99])
    s = O.quantize(theta, st, co, 24, [0.2, 0.3], [0.6, 0.9])
    # bins: theta -> 0, 1, 23, 12; strength: 0, 1 (tie goes up), 2, 1; coherence: 0, 1 (tie), 0, 2
    want = [(0 * 3 + 0) * 3 + 0, (1 * 3 + 1) * 3 + 1, (23 * 3 + 2) * 3 + 0, (12 * 3 + 1) * 3 + 2]
    assert list(s) == want


def _rot90_fixture(seed):
    z, _ = synth.noisy_pair(seed, 48, 48, 3, 25)
    return z.astype(np.float64)


def test_rot90_shifts_orientation_by_half_the_bins():
    z = _rot90_fixture(11)
    q = 24
    t_s, t_c = [0.02, 0.05], [0.2, 0.5]
    s, m = O.select(z, q, t_s, t_c, return_margin=True)
    zr = np.rot90(z, 1, axes=(1, 2)).copy()
    sr, mr = O.select(zr, q, t_s, t_c, return_margin=True)
    s_back = np.rot90(sr, -1)
    ok = (m > 1e-9) & (np.rot90(mr, -1) > 1e-9)
    qs_qc = 9
    assert ok.sum() > 1500
    assert np.all((s_back % qs_qc)[ok] == (s % qs_qc)[ok])
    assert np.all(((s_back // qs_qc) % q)[ok] == ((s // qs_qc + q // 2) % q)[ok])


def test_flip_mirrors_orientation():
    z = _rot90_fixture(12)
    q = 24
    t_s, t_c = [0.02, 0.05], [0.2, 0.5]
    s, m = O.select(z, q, t_s, t_c, return_margin=True)
    sf, mf = O.select(z[:, :, ::-1].copy(), q, t_s, t_c, return_margin=True)
    sf = sf[:, ::-1]
    ok = (m > 1e-9) & (mf[:, ::-1] > 1e-9)
    assert ok.sum() > 1500
    assert np.all((sf % 9)[ok] == (s % 9)[ok])
    assert np.all(((sf // 9))[ok] == (q - 1 - s // 9)[ok])


def test_margin_detects_boundary():
    a = np.array([1.0, 1.0, 1.0])
    c = np.array([0.5, 1.0, 0.2])
    b = np.array([0.0, 0.0, 0.3])
    th, st, co = O.eigen_features(a, b, c)
    m = O.select_margins(a, b, c, th, st, co, 24, [st[2]], [])
    assert m[0] < 1e-12          # a > c, b = 0: theta = pi/2 exactly on a boundary (bin 12 edge)
    assert m[1] == 0.0           # isotropic
    assert m[2] == 0.0           # strength equal to the threshold


# ------------------------------------------------------------------ filtering (Eq. (1), (9)-(10))

def _bank_level(K_theta, t_s, t_c, rg, rf, coeffs):
    return O.LevelBank(K_theta, np.asarray(t_s, float), np.asarray(t_c, float), rg, rf, coeffs)


def test_delta_filter_is_identity_single_scale():
    z, _ = synth.noisy_pair(3, 19, 23, 3, 25)
    K = 24 * 9
    co = np.zeros((K, 3, 49))
    co[:, :, 24] = 1.0
    lb = _bank_level(24, [0.02, 0.05], [0.2, 0.5], 3, None, co)
    out = O.denoise(z, O.Bank([lb]))
    assert np.max(np.abs(out - z)) < 1e-14


def test_delta_filters_multiscale():
    z, _ = synth.noisy_pair(4, 37, 29, 3, 25)
    K = 24 * 9
    g_only = np.zeros((K, 3, 98))
    g_only[:, :, 49 + 24] = 1.0
    levels = [_bank_level(24, [0.02, 0.05], [0.2, 0.5], 3, 3, g_only) for _ in range(3)]
    out = O.denoise(z, O.Bank(levels))
    assert np.max(np.abs(out - z)) < 1e-14
    # f = delta, g = 0: nearest-neighbour upsampling of the coarser output
    f_only = np.zeros((K, 3, 98))
    f_only[:, :, 24] = 1.0
    lb = _bank_level(24, [0.02, 0.05], [0.2, 0.5], 3, 3, f_only)
    zf = O.to_filter_space(z)
    coarse = O.down2(zf)
    s = O.select(z.astype(float), 24, lb.t_s, lb.t_c)
    out = O.apply_level(zf, s, lb, u_coarse=coarse)
    H, W = z.shape[1:]
    want = coarse[:, np.arange(H)[:, None] // 2, np.arange(W)[None, :] // 2]
    assert np.max(np.abs(out - want)) < 1e-15


def test_apply_brute_force():
    rng = np.random.default_rng(21)
    C, H, W = 2, 5, 7
    z = rng.uniform(0, 1, (C, H, W))
    uc = rng.uniform(0, 1, (C, 3, 4))
    K = 4
    rf, rg = 1, 2
    co = rng.normal(0, 1, (K, C, 9 + 25))
    s = rng.integers(0, K, (H, W))
    lb = _bank_level(1, [], [], rg, rf, co)
    got = O.apply_level(z, s, lb, u_coarse=uc)

    def cl(v, n):
        return min(max(v, 0), n - 1)
    for ch in range(C):
        for y in range(H):
            for x in range(W):
                acc = 0.0
                t = 0
                for dy in range(-rf, rf + 1):
                    for dx in range(-rf, rf + 1):
                        acc += co[s[y, x], ch, t] * uc[ch, cl(y // 2 + dy, 3), cl(x // 2 + dx, 4)]
                        t += 1
                for dy in range(-rg, rg + 1):
                    for dx in range(-rg, rg + 1):
                        acc += co[s[y, x], ch, t] * z[ch, cl(y + dy, H), cl(x + dx, W)]
                        t += 1
                assert abs(acc - got[ch, y, x]) < 1e-13


def test_apply_is_linear_for_fixed_selection():
    rng = np.random.default_rng(22)
    z1, z2 = rng.uniform(0, 1, (2, 3, 9, 11))
    u1, u2 = rng.uniform(0, 1, (2, 3, 5, 6))
    co = rng.normal(0, 1, (216, 3, 98))
    s = rng.integers(0, 216, (9, 11))
    lb = _bank_level(24, [0.1, 0.2], [0.3, 0.6], 3, 3, co)
    al, be = 0.7, -1.3
    lhs = O.apply_level(al * z1 + be * z2, s, lb, al * u1 + be * u2)
    rhs = al * O.apply_level(z1, s, lb, u1) + be * O.apply_level(z2, s, lb, u2)
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_constant_fixed_point_dc_normalised():
    co = synth.random_bank_coeffs(5, 216, 3, 49, 49)      # each filter's taps sum to 1
    levels = [_bank_level(24, [0.02, 0.05], [0.2, 0.5], 3, 3, co) for _ in range(3)]
    z = np.full((3, 30, 26), 0.61)
    out = O.denoise(z, O.Bank(levels))
    assert np.max(np.abs(out - 0.61)) < 1e-13


# ------------------------------------------------------------------ training (Eq. (7)-(8))

def test_ridge_one_dimensional_closed_form():
    rng = np.random.default_rng(31)
    x = rng.normal(0, 1, 200)
    y = 0.7 * x + rng.normal(0, 0.1, 200)
    st = O.GramStats.zeros(1, 1, 1)
    st.G[0, 0, 0, 0] = x @ x
    st.b[0, 0, 0] = x @ y
    st.n[0] = 200
    for lam in (0.0, 1e-3, 0.5):
        h, _ = O.solve_level(st, lam, n_min=1)
        assert abs(h[0, 0, 0] - (x @ y) / (x @ x + 200 * lam)) < 1e-14


def test_planted_single_scale_recovery_matches_lstsq():
    rng = np.random.default_rng(41)
    q_theta, r = 4, 2
    K = q_theta * 2 * 2
    D = 25
    planted = rng.normal(0, 0.3, (K, 1, D))
    zs = [rng.uniform(0, 1, (1, 48, 48)) for _ in range(6)]
    st, co = (np.concatenate(v) for v in zip(*[O.level_features(z) for z in zs]))
    t_s, t_c = [float(np.median(st))], [float(np.median(co))]
    pairs = []
    for z in zs:
        s = O.select(z, q_theta, t_s, t_c)
        u = O.apply_level(z, s, _bank_level(q_theta, t_s, t_c, r, None, planted))
        pairs.append((z, u))
    bank, stats, fb = O.train_single(pairs, q_theta, 2, 2, r, 0.0, t_s=t_s, t_c=t_c, n_min=D)
    assert not fb.any()
    assert np.max(np.abs(bank.levels[0].coeffs - planted)) < 1e-10
    # the same per-bucket fit by a library least-squares solve on the stacked samples
    k = int(np.argmax(stats.n))
    Xs, ys = [], []
    for z, u in pairs:
        s = O.select(z, q_theta, t_s, t_c).ravel()
        X = O.patch_matrix(z[0], r)
        Xs.append(X[s == k])
        ys.append(u[0].ravel()[s == k])
    X = np.concatenate(Xs)
    y = np.concatenate(ys)
    h_ls = np.linalg.lstsq(X, y, rcond=None)[0]
    assert np.max(np.abs(h_ls - bank.levels[0].coeffs[k, 0])) < 1e-10
    # residual identity sum (y - x.h)^2 = yy - 2 b.h + h.G.h
    h = bank.levels[0].coeffs[k, 0]
    res = np.sum((y - X @ h) ** 2)
    ident = stats.yy[k, 0] - 2 * stats.b[k, 0] @ h + h @ stats.G[k, 0] @ h
    assert abs(res - ident) < 1e-9


def test_planted_cross_channel_recovery_147_taps():
    """Three-channel 7x7 patches (D = 147), three right-hand sides: planted filters are recovered at
    lambda = 0, and one bucket's solution equals a library least-squares fit of its samples."""
    rng = np.random.default_rng(45)
    q_theta, r = 2, 3
    K, C, D = q_theta * 2 * 2, 3, 147
    planted = rng.normal(0, 0.2, (K, C, D))
    zs = [rng.uniform(0, 1, (3, 60, 60)) for _ in range(5)]
    st, co = (np.concatenate(v) for v in zip(*[O.level_features(z) for z in zs]))
    t_s, t_c = [float(np.median(st))], [float(np.median(co))]
    stats = O.CrossGramStats.zeros(K, C, D)
    samples = []
    for z in zs:
        s = O.select(z, q_theta, t_s, t_c)
        u = O.apply_level_cross(z, s, planted, r)
        O.accumulate_level_cross(stats, s, z, u, r)
        samples.append((s.ravel(), z, u))
    h, fb = O.solve_level_cross(stats, 0.0)
    assert not fb.any()
    assert np.max(np.abs(h - planted)) < 1e-9
    k = int(np.argmax(stats.n))
    X = np.concatenate([np.concatenate([O.patch_matrix(z[c], r) for c in range(C)], axis=1)[s == k]
                        for s, z, _ in samples])
    for ch in range(C):
        y = np.concatenate([u[ch].ravel()[s == k] for s, _, u in samples])
        assert np.max(np.abs(np.linalg.lstsq(X, y, rcond=None)[0] - h[k, ch])) < 1e-9
    # the per-channel layout is the special case of block-diagonal cross filters
    diag = np.zeros((K, C, D))
    for ch in range(C):
        diag[:, ch, ch * 49:(ch + 1) * 49] = planted[:, ch, ch * 49:(ch + 1) * 49]
    s0 = samples[0][0].reshape(60, 60)
    want = np.stack([O.apply_level(zs[0][ch:ch + 1], s0, _bank_level(q_theta, t_s, t_c, r, None,
                                                                     diag[:, ch:ch + 1, ch * 49:(ch + 1) * 49]))[0]
                     for ch in range(C)])
    assert np.max(np.abs(O.apply_level_cross(zs[0], s0, diag, r) - want)) < 1e-12


def test_pooled_fallback_is_sum_of_bucket_statistics():
    rng = np.random.default_rng(43)
    K, C, D = 5, 1, 3
    st = O.GramStats.zeros(K, C, D)
    for k in range(K):
        X = rng.normal(0, 1, (10 + 5 * k, D))
        y = rng.normal(0, 1, 10 + 5 * k)
        st.G[k, 0] = X.T @ X
        st.b[k, 0] = X.T @ y
        st.n[k] = len(y)
    st.n[0] = 2
    h, fb = O.solve_level(st, 1e-3, n_min=D)
    assert fb.tolist() == [True, False, False, False, False]
    Gp, bp, n = st.G[:, 0].sum(0), st.b[:, 0].sum(0), st.n.sum()
    assert np.max(np.abs(h[0, 0] - np.linalg.solve(Gp / n + 1e-3 * np.eye(D), bp / n))) < 1e-14


def test_planted_multiscale_recovery():
    """Targets generated by a planted two-level cascade are recovered level by level at lambda = 0."""
    rng = np.random.default_rng(47)
    q_theta = 2
    rf, rg = 1, 1
    K = q_theta * 2
    D = 18
    planted = [rng.normal(0, 0.3, (K, 3, D)) for _ in range(2)]
    pyrs = [O.build_pyramid(rng.uniform(0, 1, (3, 40, 44)), 3) for _ in range(5)]
    thr = []
    for lev in range(2):
        st = np.concatenate([O.level_features(p[lev])[0] for p in pyrs])
        thr.append(([float(np.median(st))], []))
    banks = [_bank_level(q_theta, thr[lev][0], thr[lev][1], rg, rf, planted[lev]) for lev in range(2)]
    # targets: the planted cascade (u^2 = z^2, then level 1, then level 0)
    targets = []
    for pz in pyrs:
        u2 = O.to_filter_space(pz[2])
        s1 = O.select(pz[1], q_theta, *thr[1])
        u1 = O.apply_level(O.to_filter_space(pz[1]), s1, banks[1], u2)
        s0 = O.select(pz[0], q_theta, *thr[0])
        u0 = O.apply_level(O.to_filter_space(pz[0]), s0, banks[0], u1)
        targets.append((u0, u1))
    # level 1 fit from (z^1, u^2 = z^2) against u1; then level 0 from (z^0, fitted level-1 output)
    st1 = O.GramStats.zeros(K, 3, D)
    for pz, (_, u1) in zip(pyrs, targets):
        s1 = O.select(pz[1], q_theta, *thr[1])
        O.accumulate_level(st1, s1, O.to_filter_space(pz[1]), u1, rg, rf, O.to_filter_space(pz[2]))
    h1, fb1 = O.solve_level(st1, 0.0)
    assert not fb1.any()
    assert np.max(np.abs(h1 - planted[1])) < 1e-9
    fitted1 = _bank_level(q_theta, thr[1][0], thr[1][1], rg, rf, h1)
    st0 = O.GramStats.zeros(K, 3, D)
    for pz, (u0, _) in zip(pyrs, targets):
        s1 = O.select(pz[1], q_theta, *thr[1])
        uh1 = O.apply_level(O.to_filter_space(pz[1]), s1, fitted1, O.to_filter_space(pz[2]))
        s0 = O.select(pz[0], q_theta, *thr[0])
        O.accumulate_level(st0, s0, O.to_filter_space(pz[0]), u0, rg, rf, uh1)
    h0, fb0 = O.solve_level(st0, 0.0)
    assert not fb0.any()
    assert np.max(np.abs(h0 - planted[0])) < 1e-9


def test_train_multiscale_runs_and_denoises():
    pairs = [synth.noisy_pair(100 + i, 64, 64, 3, 25) for i in range(4)]
    pairs = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    bank, _, _ = O.train_multiscale(pairs, 2, 8, 2, 2, 2, 2, 1e-3)
    z, u = synth.noisy_pair(500, 64, 64, 3, 25)
    out = O.denoise(z, bank)
    assert O.psnr(out, u) > O.psnr(z, u) + 2.0


def test_noise_model_statistics():
    u = np.full((1, 256, 256), 0.5, dtype=np.float32)
    z = synth.add_noise(u, 25.0, 9)
    k = np.rint(z.astype(np.float64) * 255)
    assert np.max(np.abs(k / 255 - z)) < 1e-7
    assert abs((z.astype(np.float64) - 0.5).std() * 255 - 25.0) < 0.5


def test_thresholds_equal_population():
    v = np.random.default_rng(3).uniform(0, 1, 30000)
    t = O.thresholds_from_features(v, 3)
    counts = [(v < t[0]).sum(), ((v >= t[0]) & (v < t[1])).sum(), (v >= t[1]).sum()]
    assert max(counts) - min(counts) <= 2


# ----------------------------------------------------------------------------- augmentation (Section 5)

def test_dihedral_transforms_form_the_group_of_the_square():
    rng = np.random.default_rng(11)
    x = rng.random((2, 5, 7))                         # generic: no symmetry of its own
    imgs = [O.dihedral(x, t) for t in range(8)]
    # eight distinct images, each a rearrangement of the same pixels
    for i in range(8):
        assert np.array_equal(np.sort(imgs[i].ravel()), np.sort(x.ravel()))
        for j in range(i):
            assert imgs[i].shape != imgs[j].shape or not np.array_equal(imgs[i], imgs[j])
    # closed under composition, each row of the composition table a permutation (a group)
    def index_of(y):
        hits = [t for t in range(8) if imgs[t].shape == y.shape and np.array_equal(imgs[t], y)]
        assert len(hits) == 1
        return hits[0]
    table = np.array([[index_of(O.dihedral(imgs[a], b)) for b in range(8)] for a in range(8)])
    for row in table:
        assert sorted(row) == list(range(8))
    # quarter turns against numpy's rotation (an independent definition): order 4; mirrors: order 2
    assert np.array_equal(imgs[5], np.rot90(x, -1, axes=(1, 2)))
    assert np.array_equal(imgs[6], np.rot90(x, 1, axes=(1, 2)))
    y = x
    for _ in range(4):
        y = O.dihedral(y, 5)
    assert np.array_equal(y, x)
    for t in (1, 2, 4):
        assert np.array_equal(O.dihedral(O.dihedral(x, t), t), x)


def test_augmented_training_depends_only_on_the_orbit():
    """Training on the eight symmetries of a pair equals training on those of any symmetric copy of
    it: the same eight images in another order, so only the FP64 summation order differs. A set of
    transforms that is not the whole group (a missing or repeated symmetry) breaks this."""
    pairs = [synth.noisy_pair(40 + i, 24, 24, 3, 25) for i in range(2)]
    pairs = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    ref, _, _ = O.train_single(pairs, 8, 2, 2, 1, 1e-3, augment=True)
    for t in (1, 5, 6):
        moved = [(O.dihedral(z, t), O.dihedral(u, t)) for z, u in pairs]
        got, _, _ = O.train_single(moved, 8, 2, 2, 1, 1e-3, augment=True)
        assert np.max(np.abs(got.levels[0].coeffs - ref.levels[0].coeffs)) < 1e-9
        plain_ref, _, _ = O.train_single(pairs, 8, 2, 2, 1, 1e-3)
        plain_got, _, _ = O.train_single(moved, 8, 2, 2, 1, 1e-3)
        assert np.max(np.abs(plain_got.levels[0].coeffs - plain_ref.levels[0].coeffs)) > 1e-3
    # multiscale: each symmetric copy has its own pyramid and cascade
    pairs = [synth.noisy_pair(50, 32, 32, 3, 25)]
    pairs = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    ref, _, _ = O.train_multiscale(pairs, 2, 8, 2, 2, 1, 1, 1e-3, augment=True)
    moved = [(O.dihedral(z, 6), O.dihedral(u, 6)) for z, u in pairs]
    got, _, _ = O.train_multiscale(moved, 2, 8, 2, 2, 1, 1, 1e-3, augment=True)
    for a, b in zip(ref.levels, got.levels):
        assert np.max(np.abs(a.coeffs - b.coeffs)) < 1e-9


# ----------------------------------------------------------------------------- luma-only selector (Section 3, Fig. 2)

def test_luma_of_grey_is_the_grey_value():
    """The published luma weights sum to one: a grey pixel (v, v, v) has luma v."""
    v = np.random.default_rng(5).random((1, 9, 11))
    y = O.luma(np.concatenate([v, v, v]))
    assert y.shape == (1, 9, 11)
    assert np.max(np.abs(y - v)) <= 2 * np.finfo(float).eps
    assert abs(O.KR + O.KG + O.KB - 1.0) <= np.finfo(float).eps


@pytest.mark.parametrize("slopes", [((0.01, 0.0), (0.0, 0.02), (0.004, 0.004)),
                                    ((-0.006, 0.013), (0.011, 0.004), (0.0, -0.01))])
def test_luma_selector_on_colour_ramps(slopes):
    """Channels with different ramps: the luma is the ramp with the luma-weighted slope, whose
    orientation and strength the luma selector reports (coherence 1), while the colour tensor
    sums the three channels' tensors."""
    H, W = 20, 24
    z = np.concatenate([_ramp(H, W, a, b, 1) for a, b in slopes])
    K = np.array([O.KR, O.KG, O.KB])
    al = float(K @ [s[0] for s in slopes])
    be = float(K @ [s[1] for s in slopes])
    core = (slice(3, H - 3), slice(3, W - 3))
    a, b, c = O.structure_tensor(O.selector_image(z, "luma"))
    theta, strength, coh = O.eigen_features(a, b, c)
    want = np.mod(np.arctan2(be, al) + np.pi / 2, np.pi)
    d = np.abs(theta[core] - want)
    assert np.max(np.minimum(d, np.pi - d)) < 1e-7
    assert np.max(np.abs(strength[core] - np.hypot(al, be))) < 1e-14
    assert np.min(coh[core]) > 1 - 1e-6
    a2, b2, c2 = O.structure_tensor(z)
    assert np.max(np.abs(a2[core] - sum(s[0] ** 2 for s in slopes))) < 1e-15
    assert np.max(np.abs(b2[core] - sum(s[0] * s[1] for s in slopes))) < 1e-15


def test_luma_misses_an_equal_luma_colour_edge():
    """Section 3 / Fig. 2: an edge between two colours of (nearly) equal luma is invisible to the
    luma structure tensor and strong in the colour one."""
    c1 = np.array([0.9, 0.3, 0.5])
    y1 = O.KR * c1[0] + O.KG * c1[1] + O.KB * c1[2]
    c2 = np.array([0.2, 0.6, 0.0])
    c2[2] = (y1 - O.KR * c2[0] - O.KG * c2[1]) / O.KB
    z = np.empty((3, 16, 16))
    z[:, :, :8] = c1[:, None, None]
    z[:, :, 8:] = c2[:, None, None]
    t_s, t_c = [0.01, 0.05], [0.3, 0.6]
    _, s_rgb, _ = O.eigen_features(*O.structure_tensor(z))
    _, s_luma, _ = O.eigen_features(*O.structure_tensor(O.selector_image(z, "luma")))
    assert s_rgb[8, 8] > 0.1 and np.max(s_luma) < 1e-12
    q = O.select(z, 8, t_s, t_c, selector="luma") // 3 % 3   # strength bin
    assert np.all(q == 0)
    assert O.select(z, 8, t_s, t_c)[8, 8] // 3 % 3 == 2


# ----------------------------------------------------------------------------- the paper's configuration (Section 5)

def test_down2_noise_gain_closed_form_and_measured():
    w = O.down2_weights()
    assert abs(O.down2_noise_gain() - float(np.sum(w * w))) == 0.0
    assert abs(O.down2_noise_gain() - 424064 / 1024 ** 2) < 1e-15      # 2 (12^2 + 36^2 + 116^2 + 444^2) / 1024^2
    rng = np.random.default_rng(21)
    x = rng.standard_normal((1, 1024, 1024))
    y = O.down2(x)[:, 8:-8, 8:-8]
    assert abs(float(np.std(y)) - O.down2_noise_gain()) < 5e-3


def test_pyramid_noise_gain_against_white_noise():
    """The cascade's noise deviation per level: level 1 is the white-noise gain exactly; deeper
    levels match the deviation measured on a pyramid of white noise (within sampling error)."""
    assert abs(O.pyramid_noise_gain(1) - O.down2_noise_gain()) < 1e-15
    rng = np.random.default_rng(22)
    pyr = O.build_pyramid(rng.standard_normal((1, 1024, 1024)), 5)
    for lev in range(1, 5):
        m = 8
        measured = float(np.std(pyr[lev][:, m:-m, m:-m]))
        assert abs(measured / O.pyramid_noise_gain(lev) - 1) < 0.03, (lev, measured, O.pyramid_noise_gain(lev))
    assert O.pyramid_noise_gain(2) > O.down2_noise_gain() ** 2      # correlated after the first level


@pytest.mark.parametrize("sigma,want", [(5, (2, 1, 2)), (15, (3, 2, 3)), (25, (4, 2, 3)), (50, (5, 2, 3))])
def test_paper_setup_levels_and_footprints(sigma, want):
    L, rf, rg, q = O.paper_setup(sigma)
    assert (L, rf, rg) == want and q == (16, 16, 16)
    assert sigma * O.pyramid_noise_gain(L) < 2.0 <= sigma * O.pyramid_noise_gain(L - 1)


# ----------------------------------------------------------------------------- phase-aware buckets (Eq. (9), "i/2")

def test_phase_index_layout():
    s = np.arange(12).reshape(3, 4)
    sp = O.add_phase(s, 4)
    assert sp[0, 0] == 0 and sp[0, 1] == 4 * 1 + 1 and sp[1, 0] == 4 * 4 + 2 and sp[1, 1] == 4 * 5 + 3
    assert np.array_equal(sp // 4, s) and np.array_equal(O.add_phase(s, 1), s)


def test_phase_copies_of_a_blind_bank_change_nothing():
    """Four identical phase rows per bucket give exactly the phase-blind cascade."""
    pairs = [synth.noisy_pair(70 + i, 48, 48, 3, 25) for i in range(2)]
    pairs = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    bank, _, _ = O.train_multiscale(pairs, 2, 8, 2, 2, 2, 2, 1e-3)
    rep = O.Bank([O.LevelBank(lb.q_theta, lb.t_s, lb.t_c, lb.radius_g, lb.radius_f,
                              np.repeat(lb.coeffs, 4, axis=0), phases=4) for lb in bank.levels])
    z, _ = synth.noisy_pair(77, 50, 62, 3, 25)
    assert np.array_equal(O.denoise(z, rep), O.denoise(z, bank))


def test_phase_aware_upscale_reproduces_a_ramp():
    """Each fine pixel i sits at (i - 1/2)/2 on the coarse grid (down2 is centred at 2m + 1/2):
    m - 1/4 for even i and m + 1/4 for odd i. Bilinear upscale filters per phase, 3/4 of the
    nearest coarse sample and 1/4 of the next one on the pixel's side, therefore reproduce a
    linear ramp exactly; one phase-blind filter cannot serve both parities."""
    H, W = 24, 28
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    a, bx, by = 0.3, 0.011, -0.007
    fine = a + bx * xx + by * yy
    cy, cx = np.mgrid[0:H // 2, 0:W // 2].astype(float)
    coarse = (a + bx * (2 * cx + 0.5) + by * (2 * cy + 0.5))[None]
    r = 1
    taps = O.tap_offsets(r)
    K, q_theta = 2, 2                       # one orientation bin pair, one strength and coherence bin
    coeffs = np.zeros((4 * K, 1, len(taps) + len(taps)))
    for p in range(4):
        wy = {-1: 0.25, 0: 0.75, 1: 0.0} if p // 2 == 0 else {-1: 0.0, 0: 0.75, 1: 0.25}
        wx = {-1: 0.25, 0: 0.75, 1: 0.0} if p % 2 == 0 else {-1: 0.0, 0: 0.75, 1: 0.25}
        for t, (dy, dx) in enumerate(taps):
            coeffs[[4 * k + p for k in range(K)], 0, t] = wy[dy] * wx[dx]
    lb = O.LevelBank(q_theta, np.array([]), np.array([]), r, r, coeffs, phases=4)
    s = O.add_phase(np.zeros((H, W), np.int64), 4)
    out = O.apply_level(fine[None] * 0, s, lb, u_coarse=coarse)
    core = (slice(2, H - 2), slice(2, W - 2))
    assert np.max(np.abs(out[0][core] - fine[core])) < 1e-14
    blind = O.LevelBank(q_theta, np.array([]), np.array([]), r, r, coeffs[0::4], phases=1)
    out_b = O.apply_level(fine[None] * 0, np.zeros((H, W), np.int64), blind, u_coarse=coarse)
    assert np.max(np.abs(out_b[0][core] - fine[core])) > 1e-3


def test_planted_phase_aware_recovery():
    """Noise-free targets made by phase-dependent planted filters are recovered exactly with
    phases = 4 (lambda = 0) and not by the phase-blind fit."""
    rng = np.random.default_rng(42)
    q_theta, r = 2, 1
    K = q_theta * 2 * 2 * 4
    planted = rng.normal(0, 0.3, (K, 1, 9))
    zs = [rng.uniform(0, 1, (1, 40, 40)) for _ in range(4)]
    t_s, t_c = [1e9], [1e9]                 # every pixel in strength and coherence bin 0
    pairs = []
    for z in zs:
        s = O.select(z, q_theta, t_s, t_c, phases=4)
        lb = O.LevelBank(q_theta, np.array(t_s), np.array(t_c), r, None, planted, phases=4)
        pairs.append((z, O.apply_level(z, s, lb)))
    bank, _, fb = O.train_single(pairs, q_theta, 2, 2, r, 0.0, t_s=t_s, t_c=t_c, n_min=9, phases=4)
    idx = [4 * b + p for b in (0, 4) for p in range(4)]      # buckets (q_theta bin 0 or 1, 0, 0) x phases
    assert not fb[idx].any()
    assert np.max(np.abs(bank.levels[0].coeffs[idx] - planted[idx])) < 1e-10
    blind, _, _ = O.train_single(pairs, q_theta, 2, 2, r, 0.0, t_s=t_s, t_c=t_c, n_min=9)
    for b in (0, 4):
        assert np.max(np.abs(blind.levels[0].coeffs[b] - planted[4 * b])) > 1e-3


# ----------------------------------------------------------------------------- selection on the coarser output

def test_upsample2_impulse_closed_form():
    """A coarse impulse spreads as the outer product of the linear-interpolation weights
    (1/4, 3/4, 3/4, 1/4) over fine pixels 2m-1 .. 2m+2; at the first sample the clamp folds the
    missing 1/4 onto pixel 0 (weights 1, 3/4, 1/4)."""
    w = np.array([0.25, 0.75, 0.75, 0.25])
    x = np.zeros((1, 6, 7))
    x[0, 2, 3] = 1.0
    u = O.upsample2(x, 12, 14)
    want = np.zeros((12, 14))
    want[3:7, 5:9] = np.outer(w, w)
    assert np.array_equal(u[0], want)
    x = np.zeros((1, 6, 7))
    x[0, 0, 0] = 1.0
    u = O.upsample2(x, 11, 13)                 # odd sizes: ceil(11/2) = 6, ceil(13/2) = 7
    e = np.array([1.0, 0.75, 0.25])
    want = np.zeros((11, 13))
    want[:3, :3] = np.outer(e, e)
    assert np.array_equal(u[0], want)


def test_upsample2_constants_sums_and_ramps():
    """Constants stay constant; on even sizes every coarse sample hands out total weight 4 (the sum
    is preserved up to the factor 4); a ramp sampled at the coarse centres 2m + 1/2 (which is what
    down2 makes of a fine ramp) comes back as the fine ramp away from the edges."""
    for H, W in [(1, 1), (2, 3), (9, 8), (33, 17)]:
        x = np.full((2, (H + 1) // 2, (W + 1) // 2), 0.61)
        assert np.max(np.abs(O.upsample2(x, H, W) - 0.61)) < 1e-15
    x = np.random.default_rng(8).random((3, 5, 6))
    assert abs(O.upsample2(x, 10, 12).sum() - 4 * x.sum()) < 1e-12
    H, W = 40, 48
    alpha, beta, c0 = 0.013, -0.007, 0.4
    m_y, m_x = np.mgrid[0:H // 2, 0:W // 2].astype(float)
    coarse = (c0 + alpha * (2 * m_x + 0.5) + beta * (2 * m_y + 0.5))[None]
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    fine = c0 + alpha * xx + beta * yy
    inner = (slice(1, H - 1), slice(1, W - 1))
    assert np.max(np.abs(O.upsample2(coarse, H, W)[0][inner] - fine[inner])) < 1e-15
    ramp = fine[None]
    back = O.upsample2(O.down2(ramp), H, W)[0]
    core = (slice(5, H - 5), slice(5, W - 5))
    assert np.max(np.abs(back[core] - fine[core])) < 1e-14


@pytest.mark.parametrize("k", [(1.0, 0.5, -2.0), (0.3, 1.2, 0.7)])
def test_coarse_selector_follows_the_coarser_output(k):
    """The coarse selector reads u^{l+1} (held in YCbCr), upsamples it and takes it back to RGB:
    with RGB channels that are parallel ramps k_c (alpha, beta) the features at the fine level are
    those of the fine ramp, coherence 1 and strength |k| |(alpha, beta)|, whatever the noisy level
    holds. Features taken on the YCbCr channels themselves would weigh the channels differently."""
    H, W = 24, 28
    alpha, beta = 0.011, -0.006
    m_y, m_x = np.mgrid[0:H // 2, 0:W // 2].astype(float)
    base = alpha * (2 * m_x + 0.5) + beta * (2 * m_y + 0.5)
    coarse_rgb = np.stack([0.5 + kc * base for kc in k])
    u_coarse = O.to_filter_space(coarse_rgb)
    z = np.random.default_rng(3).random((3, H, W))
    core = (slice(4, H - 4), slice(4, W - 4))
    a, b, c = O.structure_tensor(O.selector_image(z, "coarse", u_coarse))
    theta, strength, coh = O.eigen_features(a, b, c)
    want = np.mod(np.arctan2(beta, alpha) + np.pi / 2, np.pi)
    d = np.abs(theta[core] - want)
    assert np.max(np.minimum(d, np.pi - d)) < 1e-7
    assert np.max(np.abs(strength[core] - np.linalg.norm(k) * np.hypot(alpha, beta))) < 1e-13
    assert np.min(coh[core]) > 1 - 1e-6
    _, s_ycc, _ = O.eigen_features(*O.structure_tensor(O.upsample2(u_coarse, H, W)))
    assert np.max(np.abs(s_ycc[core] - strength[core])) > 1e-4
    t_s, t_c = [0.5 * float(np.median(strength))], [0.5]
    s1 = O.select(z, 8, t_s, t_c, selector="coarse", u_coarse=u_coarse)
    s2 = O.select(np.zeros_like(z), 8, t_s, t_c, selector="coarse", u_coarse=u_coarse)
    assert np.array_equal(s1, s2)
    with pytest.raises(ValueError):
        O.select(z, 8, t_s, t_c, selector="coarse")


def test_planted_recovery_with_coarse_selection():
    """A level whose buckets come from the upsampled coarser output: targets made by planted
    per-bucket filters (bucket chosen on the coarser input u^{l+1}) are recovered at lambda = 0."""
    rng = np.random.default_rng(48)
    q_theta, rf, rg = 2, 1, 1
    K, D = q_theta * 2, 18
    planted = rng.normal(0, 0.3, (K, 3, D))
    pyrs = [O.build_pyramid(rng.uniform(0, 1, (3, 40, 44)), 2) for _ in range(5)]
    st = np.concatenate([O.level_features(p[0], "coarse", O.to_filter_space(p[1]))[0] for p in pyrs])
    t_s, t_c = [float(np.median(st))], []
    lb = O.LevelBank(q_theta, np.array(t_s), np.array(t_c), rg, rf, planted, selector="coarse")
    stats = O.GramStats.zeros(K, 3, D)
    for pz in pyrs:
        uc = O.to_filter_space(pz[1])
        s = O.select(pz[0], q_theta, t_s, t_c, selector="coarse", u_coarse=uc)
        assert 0 < np.mean(s % 2) < 1                    # both strength bins occur
        target = O.apply_level(O.to_filter_space(pz[0]), s, lb, uc)
        O.accumulate_level(stats, s, O.to_filter_space(pz[0]), target, rg, rf, uc)
    h, fb = O.solve_level(stats, 0.0)
    assert not fb.any()
    assert np.max(np.abs(h - planted)) < 1e-9
    # the cascade selects level 0 on its own coarser output
    bank = O.Bank([lb, O.LevelBank(q_theta, np.array(t_s), np.array(t_c), rg, rf, planted)])
    img = pyrs[0][0]
    _, maps = O.denoise(img, bank, return_index_maps=True)
    pyr = O.build_pyramid(img, 3)
    u1 = O.apply_level(O.to_filter_space(pyr[1]), maps[1], bank.levels[1], O.to_filter_space(pyr[2]))
    assert np.array_equal(maps[0], O.select(img, q_theta, t_s, t_c, selector="coarse", u_coarse=u1))
    assert not np.array_equal(maps[0], O.select(img, q_theta, t_s, t_c))


# ----------------------------------------------------------------------------- training loop (Section 4)

def _planted_level(rng, q_theta, t_s, t_c, rg, rf, K, D):
    return _bank_level(q_theta, t_s, t_c, rg, rf, rng.normal(0, 0.3, (K, 3, D)))


def test_train_multiscale_recovers_a_planted_level():
    """One trained level through train_multiscale itself: clean images made by a planted level
    (upscale block on the coarser level z^1 = u^1-hat, denoise block on z^0) are recovered at
    lambda = 0, whatever the loop does around accumulate and solve."""
    rng = np.random.default_rng(61)
    q_theta, rf, rg = 4, 1, 1
    t_s, t_c = [0.375], []                              # about the median strength of this white noise
    K, D = q_theta * 2, 18
    planted = _planted_level(rng, q_theta, t_s, t_c, rg, rf, K, D)
    pairs = []
    for _ in range(6):
        z = rng.uniform(0, 1, (3, 44, 50))
        pz = O.build_pyramid(z, 2)
        s0 = O.select(pz[0], q_theta, t_s, t_c)
        u_ycc = O.apply_level(O.to_filter_space(pz[0]), s0, planted, O.to_filter_space(pz[1]))
        pairs.append((z, O.ycc_to_rgb(u_ycc)))
    bank, stats, fb = O.train_multiscale(pairs, 1, q_theta, 2, 1, rf, rg, 0.0, thresholds=[(t_s, t_c)])
    assert not fb[0].any()
    assert stats[0].n.min() > 20 * D
    assert np.max(np.abs(bank.levels[0].coeffs - planted.coeffs)) < 1e-9


def test_train_multiscale_feeds_each_level_the_fitted_coarser_output():
    """Two trained levels: level 1 is fitted on (z^1, u^2-hat = z^2) against u^1, and level 0 on
    (z^0, the fitted level 1's own output) against u^0; each level's thresholds are the
    equal-population quantiles of that level's features. Feeding z^1 in place of the fitted output,
    or the other level's thresholds, fails below."""
    pairs = [synth.noisy_pair(300 + i, 40, 48, 3, 25) for i in range(3)]
    pairs = [(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs]
    q_theta, q_s, q_c, rf, rg = 4, 2, 2, 1, 1
    bank, stats, _ = O.train_multiscale(pairs, 2, q_theta, q_s, q_c, rf, rg, 1e-3)
    pz = [O.build_pyramid(z, 3) for z, _ in pairs]
    pu = [O.build_pyramid(u, 3) for _, u in pairs]
    # thresholds of level l: the medians (q = 2) of level l's strength and coherence
    for lev in range(2):
        feats = [O.level_features(p[lev]) for p in pz]
        st = np.concatenate([f[0] for f in feats])
        co = np.concatenate([f[1] for f in feats])
        assert np.allclose(bank.levels[lev].t_s, [np.median(st)], rtol=0, atol=1e-15)
        assert np.allclose(bank.levels[lev].t_c, [np.median(co)], rtol=0, atol=1e-15)
    assert abs(bank.levels[0].t_s[0] - bank.levels[1].t_s[0]) > 1e-3
    K, D = q_theta * q_s * q_c, 18
    want1 = O.GramStats.zeros(K, 3, D)
    want0 = O.GramStats.zeros(K, 3, D)
    wrong0 = O.GramStats.zeros(K, 3, D)
    for p, q in zip(pz, pu):
        lb1, lb0 = bank.levels[1], bank.levels[0]
        s1 = O.select(p[1], q_theta, lb1.t_s, lb1.t_c)
        O.accumulate_level(want1, s1, O.to_filter_space(p[1]), O.to_filter_space(q[1]), rg, rf,
                           O.to_filter_space(p[2]))
        uh1 = O.apply_level(O.to_filter_space(p[1]), s1, lb1, O.to_filter_space(p[2]))
        s0 = O.select(p[0], q_theta, lb0.t_s, lb0.t_c)
        O.accumulate_level(want0, s0, O.to_filter_space(p[0]), O.to_filter_space(q[0]), rg, rf, uh1)
        O.accumulate_level(wrong0, s0, O.to_filter_space(p[0]), O.to_filter_space(q[0]), rg, rf,
                           O.to_filter_space(p[1]))
    for got, want in ((stats[1], want1), (stats[0], want0)):
        assert np.array_equal(got.n, want.n)
        scale = np.max(np.abs(want.G))
        assert np.max(np.abs(got.G - want.G)) <= 1e-12 * scale
        assert np.max(np.abs(got.b - want.b)) <= 1e-12 * scale
    assert np.max(np.abs(wrong0.G - want0.G)) > 1e-3 * np.max(np.abs(want0.G))


# ----------------------------------------------------------------------------- margins (near-boundary pixels)

def _tensor_from_eigen(theta, lam1, lam2):
    """[[a, b], [b, c]] with minor eigenvector (cos theta, sin theta) of eigenvalue lam2 and major
    eigenvector (-sin theta, cos theta) of eigenvalue lam1."""
    s, c = np.sin(theta), np.cos(theta)
    return lam1 * s * s + lam2 * c * c, (lam2 - lam1) * s * c, lam1 * c * c + lam2 * s * s


def test_select_margins_against_mpmath_distances():
    """Each margin recomputed in 50-digit arithmetic from its definition: the distance of sqrt(lam1)
    and of the coherence from the nearest threshold, and the distance of the unit-trace point
    ((a - c), 2b) / tr from the nearest boundary line, taken as a cross product with the line's
    direction (cos 2 theta_b, sin 2 theta_b), theta_b = b pi / Q (no angle of the tensor needed)."""
    import mpmath as mp
    mp.mp.dps = 50
    rng = np.random.default_rng(71)
    n = 300
    a = rng.uniform(0, 1, n) ** 3
    c = rng.uniform(0, 1, n) ** 3
    b = rng.uniform(-1, 1, n) * np.sqrt(a * c)
    q_theta, t_s, t_c = 24, [0.2, 0.5], [0.1, 0.4, 0.7]
    th, st, co = O.eigen_features(a, b, c)
    m = O.select_margins(a, b, c, th, st, co, q_theta, t_s, t_c)
    for i in range(n):
        am, bm, cm = mp.mpf(a[i]), mp.mpf(b[i]), mp.mpf(c[i])
        tr = am + cm
        mu = mp.sqrt((am - cm) ** 2 + 4 * bm * bm)
        s1 = mp.sqrt((tr + mu) / 2)
        s2 = mp.sqrt(max((tr - mu) / 2, mp.mpf(0)))
        coh = (s1 - s2) / (s1 + s2)
        ms = min(abs(s1 - t) for t in t_s)
        mc = min(abs(coh - t) for t in t_c)
        mo = min(abs((am - cm) * mp.sin(2 * k * mp.pi / q_theta) - 2 * bm * mp.cos(2 * k * mp.pi / q_theta)) / tr
                 for k in range(q_theta))
        want = float(min(ms, mc, mo))
        assert abs(m[i] - want) <= 1e-12 * max(1.0, want) + 1e-14, (i, m[i], want)


def test_select_margins_planted_distances():
    """Features planted at a known distance from one boundary: strength t + 3e-7, coherence
    t + 5e-7, and an orientation Delta past a bin edge, whose margin is the anisotropy
    (lam1 - lam2) / (lam1 + lam2) times |sin 2 Delta| (the doubled angle of the tensor)."""
    q_theta = 16
    mid = (5 + 0.5) * np.pi / q_theta                 # middle of orientation bin 5
    # strength: sqrt(lam1) planted 3e-7 above the threshold, coherence far from its thresholds
    a, b, c = _tensor_from_eigen(mid, 0.09, 0.01)
    th, st, co = O.eigen_features(np.array([a]), np.array([b]), np.array([c]))
    m = O.select_margins(np.array([a]), np.array([b]), np.array([c]), th, st, co, q_theta,
                         [st[0] - 3e-7], [co[0] + 0.2])
    assert abs(m[0] - 3e-7) < 1e-15
    m = O.select_margins(np.array([a]), np.array([b]), np.array([c]), th, st, co, q_theta,
                         [st[0] + 0.2], [co[0] - 5e-7])
    assert abs(m[0] - 5e-7) < 1e-15
    # orientation: Delta past the edge of bin 7 (theta_b = 7 pi / 16)
    for delta in (1e-3, -2e-4, 4e-2):
        lam1, lam2 = 0.3, 0.05
        a, b, c = _tensor_from_eigen(7 * np.pi / q_theta + delta, lam1, lam2)
        th, st, co = O.eigen_features(np.array([a]), np.array([b]), np.array([c]))
        assert abs(th[0] - (7 * np.pi / q_theta + delta)) < 1e-12
        m = O.select_margins(np.array([a]), np.array([b]), np.array([c]), th, st, co, q_theta, [10.0], [10.0])
        want = (lam1 - lam2) / (lam1 + lam2) * abs(np.sin(2 * delta))
        assert abs(m[0] - want) < 1e-10 * want, (delta, m[0], want)
    # the margin is a distance: a threshold just inside it never changes the bucket
    a, b, c = _tensor_from_eigen(mid, 0.09, 0.01)
    A, B, Cc = np.array([a]), np.array([b]), np.array([c])
    th, st, co = O.eigen_features(A, B, Cc)
    for t in (st[0] - 1e-6, st[0] + 1e-6):
        m = O.select_margins(A, B, Cc, th, st, co, q_theta, [t], [])
        s_lo = O.quantize(th, st - 0.99 * m, co, q_theta, [t], [])
        s_hi = O.quantize(th, st + 0.99 * m, co, q_theta, [t], [])
        assert s_lo[0] == s_hi[0] == O.quantize(th, st, co, q_theta, [t], [])[0]


# ----------------------------------------------------------------------------- PSNR (quality measure, Section 5)

def test_psnr_closed_form_and_clip():
    ref = np.full((3, 8, 8), 0.5)
    assert abs(O.psnr(ref + 0.1, ref) - 20.0) < 1e-12          # MSE 1e-2 at peak 1
    assert abs(O.psnr(ref - 0.01, ref) - 40.0) < 1e-12
    est = ref.copy()
    est[0] += 0.1                                               # one channel of three: MSE 1e-2 / 3
    assert abs(O.psnr(est, ref) - 10 * np.log10(300.0)) < 1e-12
    one = np.ones((1, 4, 4))
    assert O.psnr(one + 0.7, one) == float("inf")             # clipped to the peak: no error
    assert abs(O.psnr(-0.5 * one, 0.2 * one) - 20 * np.log10(1 / 0.2)) < 1e-12


# ----------------------------------------------------------------------------- cascade at given index maps

def test_denoise_at_given_maps():
    """The cascade run at given per-level index maps: its own maps change nothing; a different
    bucket at one level-0 pixel changes that pixel only, to Eq. (9) with that bucket's filters; a
    different bucket at one level-1 pixel changes level 0 only inside that pixel's cone (coarse taps
    at floor(i/2) + j, |j| <= radius_f)."""
    bank = O.Bank([_bank_level(8, [0.03], [0.5], 1, 1, np.random.default_rng(5 + lev).normal(0, 0.2, (32, 3, 18)))
                   for lev in range(2)])
    z, _ = synth.noisy_pair(91, 30, 34, 3, 25)
    z = z.astype(np.float64)
    out, maps = O.denoise(z, bank, return_index_maps=True)
    assert np.array_equal(O.denoise(z, bank, maps=maps), out)
    assert np.array_equal(O.denoise(z, bank, maps=[None, maps[1]]), out)
    y, x = 13, 21
    m0 = [maps[0].copy(), maps[1]]
    m0[0][y, x] = (maps[0][y, x] + 5) % 32
    alt = O.denoise(z, bank, maps=m0)
    diff = np.any(alt != out, axis=0)
    assert diff[y, x] and diff.sum() == 1
    pyr = O.build_pyramid(z, 3)
    u2 = O.to_filter_space(pyr[2])
    u1 = O.apply_level(O.to_filter_space(pyr[1]), maps[1], bank.levels[1], u2)
    z0 = O.to_filter_space(pyr[0])
    h = bank.levels[0].coeffs[m0[0][y, x]]
    pix = np.zeros(3)
    for ch in range(3):
        for t, (dy, dx) in enumerate(O.tap_offsets(1)):
            pix[ch] += h[ch, t] * u1[ch, min(max(y // 2 + dy, 0), 14), min(max(x // 2 + dx, 0), 16)]
        for t, (dy, dx) in enumerate(O.tap_offsets(1)):
            pix[ch] += h[ch, 9 + t] * z0[ch, min(max(y + dy, 0), 29), min(max(x + dx, 0), 33)]
    assert np.max(np.abs(O.ycc_to_rgb(pix[:, None, None])[:, 0, 0] - alt[:, y, x])) < 1e-12
    yc, xc = 6, 9
    m1 = [maps[0], maps[1].copy()]
    m1[1][yc, xc] = (maps[1][yc, xc] + 3) % 32
    alt = O.denoise(z, bank, maps=m1)
    diff = np.argwhere(np.any(alt != out, axis=0))
    assert len(diff) > 0
    assert np.all(np.abs(diff[:, 0] // 2 - yc) <= 1) and np.all(np.abs(diff[:, 1] // 2 - xc) <= 1)
    with pytest.raises(ValueError):
        O.denoise(z, bank, maps=[maps[0]])
    with pytest.raises(ValueError):
        O.denoise(z, bank, maps=[maps[0][:-1], maps[1]])
