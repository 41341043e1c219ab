"""Shared helpers for the tests: oracle-trained banks, GPU bank upload, index-map checks."""

from __future__ import annotations

import functools

import numpy as np

import oracle as O
import synth

NEAR = 1e-6          # features this close to a bucket boundary may take either bucket
TOL_F32 = 1e-4       # max-abs on [0, 1] images, float32 storage
TOL_F16 = 2e-3       # max-abs, float16 storage


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


def propagate_mask(mask_coarse: np.ndarray, shape_fine, radius_f: int) -> np.ndarray:
    """Fine pixels whose coarse taps (at floor(i/2) + j, |j| <= radius_f) touch a masked coarse pixel."""
    if not mask_coarse.any():
        return np.zeros(shape_fine, bool)
    Hc, Wc = mask_coarse.shape
    dil = np.zeros_like(mask_coarse)
    for dy in range(-radius_f, radius_f + 1):
        for dx in range(-radius_f, radius_f + 1):
            dil |= O.shift(mask_coarse.astype(np.int8), dy, dx).astype(bool)
    H, W = shape_fine
    return dil[np.arange(H)[:, None] // 2, np.arange(W)[None, :] // 2]


def max_abs(a, b, mask=None):
    d = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))
    if mask is not None:
        d = d[..., ~mask]
    return float(d.max()) if d.size else 0.0


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
