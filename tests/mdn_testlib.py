"""Shared helpers for the tests: oracle-trained banks, GPU bank upload, index-map checks and the
cascade parity protocol (every output pixel compared with the oracle run on the GPU's own maps)."""

from __future__ import annotations

import functools

import numpy as np

import oracle as O
import synth

NEAR = 1e-6          # features this close to a bucket boundary may take either bucket
TOL_F32 = 1e-4       # max-abs on [0, 1] images, float32 storage
TOL_F16 = 2e-3       # max-abs, float16 storage
FLIP_CAP = 1e-3      # near-boundary index flips allowed per level, as a fraction of its pixels


@functools.lru_cache(maxsize=None)
def trained_bank_multiscale(levels: int = 2, n_pairs: int = 8, size: int = 128, q_theta: int = 24,
                            q_s: int = 3, q_c: int = 3, radius: int = 3, lam: float = 1e-3, sigma: float = 25.0,
                            selector: str = "rgb"):
    """Oracle-trained multiscale bank (float64) on seeded synthetic RGB pairs."""
    pairs = []
    for i in range(n_pairs):
        z, u = synth.noisy_pair(1 + i, size, size, 3, sigma)
        pairs.append((z.astype(np.float64), u.astype(np.float64)))
    bank, _, _ = O.train_multiscale(pairs, levels, q_theta, q_s, q_c, radius, radius, lam, selector=selector)
    return bank


@functools.lru_cache(maxsize=None)
def trained_bank_single(n_pairs: int = 8, size: int = 128, q_theta: int = 16, q_s: int = 3, q_c: int = 3,
                        radius: int = 2, lam: float = 1e-3, sigma: float = 25.0, channels: int = 1):
    """Oracle-trained single-scale bank (grey by default), Eq. (1)."""
    pairs = []
    for i in range(n_pairs):
        z, u = synth.noisy_pair(1 + i, size, size, channels, sigma)
        pairs.append((z.astype(np.float64), u.astype(np.float64)))
    bank, _, _ = O.train_single(pairs, q_theta, q_s, q_c, radius, lam)
    return bank


def gpu_level(lb: O.LevelBank, channels: int, coeff_dtype=None, device="cuda"):
    import torch
    import paper_1802_06130_amd as M
    dt = coeff_dtype or torch.float32
    co = torch.tensor(np.ascontiguousarray(lb.coeffs), dtype=torch.float64).to(dt).to(device)
    sel = {"rgb": M.SELECT_RGB, "luma": M.SELECT_LUMA, "coarse": M.SELECT_COARSE}[lb.selector]
    return M.Level(lb.q_theta, lb.t_s, lb.t_c, lb.radius_g, lb.radius_f, co, channels, sel, lb.phases)


def gpu_bank(bank: O.Bank, channels: int, coeff_dtype=None, device="cuda"):
    import paper_1802_06130_amd as M
    return M.Bank([gpu_level(lb, channels, coeff_dtype, device) for lb in bank.levels])


def index_parity(s_gpu: np.ndarray, z_level: np.ndarray, lb: O.LevelBank, u_coarse=None):
    """Compare a GPU bucket map with the oracle's; every mismatch must be near a boundary.
    u_coarse: the coarser output (filter colour space, float64) for coarse-selector levels.

    Returns (mismatch mask, number of mismatches, number of near-boundary pixels).
    """
    s_ref, margin = O.select(np.asarray(z_level, np.float64), lb.q_theta, lb.t_s, lb.t_c, return_margin=True,
                             selector=lb.selector, phases=lb.phases, u_coarse=u_coarse)
    mism = s_gpu.astype(np.int64) != s_ref
    near = margin < NEAR
    bad = mism & ~near
    assert not bad.any(), f"{int(bad.sum())} index mismatches away from bucket boundaries (first at {np.argwhere(bad)[0]})"
    return mism, int(mism.sum()), int(near.sum())


def max_abs(a, b, mask=None):
    d = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))
    if mask is not None:
        d = d[..., ~mask]
    return float(d.max()) if d.size else 0.0


def gpu_cascade(img, gb, storage=np.float32):
    """The GPU cascade of one (C, H, W) image run level by level through mdn_apply_level, with each
    level's selector map captured (s_out) as its filtering pass used it. The storage of the pyramid
    and of the coarser outputs, and the colour and dtype of every output, are those of mdn_denoise.
    Returns (output tensor, [map of level 0 .. L-1] as int64 arrays)."""
    import torch
    import paper_1802_06130_amd as M
    img = np.ascontiguousarray(img)
    zt = torch.from_numpy(img).cuda()
    C = img.shape[0]
    L = len(gb.levels)
    rgb = M.GRAY if C == 1 else M.RGB
    maps = [None] * L
    if gb.levels[0].radius_f < 0:
        s_out = torch.empty(img.shape[1:], dtype=M.selector_dtype(gb.levels[0]), device="cuda")
        out = M.apply_level(zt, gb.levels[0], s_out=s_out, out_color=rgb)
        maps[0] = s_out.cpu().numpy().astype(np.int64)
        return out, maps
    st = torch.float32 if storage == np.float32 else torch.float16
    pyr = [zt] + M.pyramid_build(zt, L, storage=st)
    u, color = pyr[L], rgb
    for lev in range(L - 1, -1, -1):
        s_out = torch.empty(pyr[lev].shape[1:], dtype=M.selector_dtype(gb.levels[lev]), device="cuda")
        u = M.apply_level(pyr[lev], gb.levels[lev], u_coarse=u, coarse_color=color, s_out=s_out,
                          out_color=rgb if lev == 0 else (M.GRAY if C == 1 else M.YCC),
                          out_dtype=zt.dtype if lev == 0 else st)
        maps[lev] = s_out.cpu().numpy().astype(np.int64)
        color = M.GRAY if C == 1 else M.YCC
    return u, maps


def cascade_parity(img, bank, gb, storage=np.float32, tol=TOL_F32, u=None, dpsnr_tol=None, out=None):
    """The parity protocol of a whole cascade (Section 4; Eq. (1) for a single-scale bank).

    1. The GPU output of mdn_denoise (``out`` if the caller already has it) equals the level-by-level
       run that captures each level's map, bit for bit.
    2. Every level's map equals the oracle's selection on the same (bit-identical) pyramid level
       except at pixels whose oracle features lie within 1e-6 of a bucket boundary, and such flips
       stay below FLIP_CAP of the level's pixels.
    3. Every output pixel is within ``tol`` of the oracle cascade run on those maps, at the same
       storage rounding (float64 arithmetic); no pixel is left out.
    4. Reported beside it: flips per level and the max-abs against the pure float64 oracle (its own
       selection, no storage rounding); with the clean image ``u``, |dPSNR| against that oracle,
       bounded by ``dpsnr_tol`` when given.
    Returns a dict of these figures."""
    import torch
    import paper_1802_06130_amd as M
    img = np.ascontiguousarray(img)
    code = M.F32 if storage == np.float32 else M.F16
    if out is None:
        out = M.denoise(torch.from_numpy(img).cuda(), gb, storage=code)
    out_l, maps = gpu_cascade(img, gb, storage)
    torch.cuda.synchronize()
    got = out.float().cpu().numpy().astype(np.float64)
    assert np.array_equal(got, out_l.float().cpu().numpy().astype(np.float64)), \
        "mdn_denoise differs from the same kernels run level by level"
    L = len(bank.levels)
    if bank.levels[0].radius_f is None:
        pyr = [O.round_storage(np.asarray(img, np.float64), storage)]
    else:
        pyr = O.build_pyramid(img, L + 1, storage)
    flips = []
    for lev in range(L):
        _, n_mis, _ = index_parity(maps[lev], pyr[lev], bank.levels[lev])
        npx = maps[lev].size
        assert n_mis <= max(1, FLIP_CAP * npx), f"level {lev}: {n_mis} of {npx} pixels flipped bucket"
        flips.append(n_mis)
    ref = O.denoise(img, bank, storage=storage, maps=maps)
    err = max_abs(got, ref)
    ref64 = O.denoise(np.asarray(img, np.float64), bank)
    err64 = max_abs(got, ref64)
    res = {"max_abs": err, "flips": flips, "max_abs_fp64": err64}
    msg = f"  max-abs at the GPU's maps {err:.3g} (all pixels), flips per level {flips}, max-abs vs pure FP64 {err64:.3g}"
    if u is not None:
        res["dpsnr"] = abs(O.psnr(got, u) - O.psnr(ref64, u))
        msg += f", |dPSNR| vs FP64 {res['dpsnr']:.4f} dB"
    print(msg, flush=True)
    assert err <= tol, f"max-abs {err:.3g} > {tol:g}"
    if dpsnr_tol is not None and u is not None:
        assert res["dpsnr"] <= dpsnr_tol
    res["out"] = got
    return res


def check_gram(g, st, tol):
    """GPU normal equations against the oracle's: counts exact; G, b, yy within the accumulation
    bound |dG_pq| <= tol sqrt(G_pp G_qq) (Cauchy-Schwarz bound on sum |x_p x_q|). Returns the worst
    ratio to the bound."""
    K, C, D, _ = st.G.shape
    G = g.G.cpu().numpy().reshape(K, C, D, D)
    b = g.b.cpu().numpy().reshape(K, C, D)
    n = g.n.cpu().numpy()
    yy = g.yy.cpu().numpy().reshape(K, C)
    assert np.array_equal(n, st.n), "sample counts differ"
    diag = np.sqrt(np.maximum(np.einsum("kcii->kci", st.G), 0.0))
    bound = tol * diag[:, :, :, None] * diag[:, :, None, :] + 1e-12
    rel = np.abs(G - st.G) / bound
    assert rel.max() <= 1.0, f"G outside bound (worst ratio {rel.max():.3g})"
    yd = np.sqrt(np.maximum(st.yy, 0.0))
    assert np.all(np.abs(b - st.b) <= tol * diag * yd[:, :, None] + 1e-12)
    assert np.all(np.abs(yy - st.yy) <= tol * st.yy + 1e-12)
    return float(rel.max())
