"""Seeded synthetic scenes, noise and workload mixes.

The paper evaluates on natural photographs (68 Berkeley test images, a large
private training corpus and 1 MP timing images, all in Section 5); none of them
is available here, so these generators stand in for them with piecewise-smooth
colour scenes that contain the structures the selector is built to tell apart:
flat regions, straight and curved edges, corners and oriented textures.

Recipe of ``synth_scene(seed, H, W, C)``, drawn with ``numpy.random.default_rng(seed)``:

1. background: a constant colour plus a linear ramp (at most 0.3 across the
   image) plus one or two low-frequency sinusoids of amplitude at most 0.1;
2. 6-14 rotated rectangles and 6-14 ellipses, extent U[0.05, 0.4]*min(H, W),
   painted in random order, colour U[0.1, 0.9]^C with a linear shading of at
   most 0.3 across the shape;
3. 2-4 sinusoidal gratings inside random rectangular or elliptical masks:
   period U[4, 32] px, orientation U[0, pi), phase U[0, 2 pi), amplitude
   U[0.05, 0.25] times a random colour vector;
4. clip to [0, 1] and round to the storage dtype.

Noise follows the paper's protocol (Section 5): additive white Gaussian noise
of standard deviation sigma/255, then quantised to 8 bits and clamped, drawn
from ``default_rng(seed + 10**6)``.
"""

from __future__ import annotations

import numpy as np

SIGMAS_8BIT = (15.0, 25.0, 50.0)


def _shape_mask(rng, H, W, kind, extent, center, angle):
    """Return (slice_y, slice_x, mask, u, v) for a shape inside its bounding box.

    u, v are the shape-local coordinates normalised to [-1, 1] along the two axes.
    """
    cy, cx = center
    ha, hb = extent[0] / 2.0, extent[1] / 2.0
    ca, sa = np.cos(angle), np.sin(angle)
    ey = abs(ha * sa) + abs(hb * ca)
    ex = abs(ha * ca) + abs(hb * sa)
    y0, y1 = int(max(0, np.floor(cy - ey))), int(min(H, np.ceil(cy + ey) + 1))
    x0, x1 = int(max(0, np.floor(cx - ex))), int(min(W, np.ceil(cx + ex) + 1))
    if y0 >= y1 or x0 >= x1:
        return None
    yy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
    xx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
    u = (xx * ca + yy * sa) / max(ha, 1e-9)
    v = (-xx * sa + yy * ca) / max(hb, 1e-9)
    if kind == "rect":
        mask = (np.abs(u) <= 1.0) & (np.abs(v) <= 1.0)
    else:
        mask = (u * u + v * v) <= 1.0
    return slice(y0, y1), slice(x0, x1), mask, u, v


def synth_scene(seed: int, H: int, W: int, C: int = 3, dtype=np.float32) -> np.ndarray:
    """Clean seeded scene, planar (C, H, W), values in [0, 1], in ``dtype``."""
    rng = np.random.default_rng(seed)
    img = np.empty((C, H, W), dtype=np.float64)
    yy = np.arange(H, dtype=np.float64)[:, None]
    xx = np.arange(W, dtype=np.float64)[None, :]
    # 1. background
    base = rng.uniform(0.25, 0.75, C)
    ramp_dir = rng.uniform(0.0, 2.0 * np.pi)
    ramp_amp = rng.uniform(0.0, 0.3, C)
    diag = max(np.hypot(H, W), 1.0)
    t = (np.cos(ramp_dir) * xx + np.sin(ramp_dir) * yy) / diag - 0.5
    for c in range(C):
        img[c] = base[c] + ramp_amp[c] * t
    for _ in range(int(rng.integers(1, 3))):
        period = rng.uniform(0.5, 2.0) * max(H, W)
        ang = rng.uniform(0.0, np.pi)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        amp = rng.uniform(0.0, 0.1, C)
        wave = np.sin(2.0 * np.pi * (np.cos(ang) * xx + np.sin(ang) * yy) / period + ph)
        for c in range(C):
            img[c] += amp[c] * wave
    # 2. rectangles and ellipses in painter's order
    kinds = ["rect"] * int(rng.integers(6, 15)) + ["ellipse"] * int(rng.integers(6, 15))
    order = rng.permutation(len(kinds))
    m = float(min(H, W))
    for idx in order:
        kind = kinds[idx]
        extent = rng.uniform(0.05, 0.4, 2) * m
        center = (rng.uniform(0, H), rng.uniform(0, W))
        angle = rng.uniform(0.0, np.pi)
        color = rng.uniform(0.1, 0.9, C)
        shade = rng.uniform(-0.3, 0.3, C)
        shade_dir = rng.uniform(0.0, 2.0 * np.pi)
        got = _shape_mask(rng, H, W, kind, extent, center, angle)
        if got is None:
            continue
        sy, sx, mask, u, v = got
        lin = 0.5 * (np.cos(shade_dir) * u + np.sin(shade_dir) * v)  # in [-1, 1] over the shape
        for c in range(C):
            region = img[c, sy, sx]
            region[mask] = (color[c] + shade[c] * lin)[mask]
    # 3. oriented gratings inside masks
    for _ in range(int(rng.integers(2, 5))):
        kind = "rect" if rng.uniform() < 0.5 else "ellipse"
        extent = rng.uniform(0.1, 0.5, 2) * m
        center = (rng.uniform(0, H), rng.uniform(0, W))
        angle = rng.uniform(0.0, np.pi)
        period = rng.uniform(4.0, 32.0)
        g_ang = rng.uniform(0.0, np.pi)
        g_ph = rng.uniform(0.0, 2.0 * np.pi)
        g_amp = rng.uniform(0.05, 0.25)
        cvec = rng.uniform(0.2, 1.0, C)
        got = _shape_mask(rng, H, W, kind, extent, center, angle)
        if got is None:
            continue
        sy, sx, mask, _, _ = got
        ly = np.arange(sy.start, sy.stop, dtype=np.float64)[:, None]
        lx = np.arange(sx.start, sx.stop, dtype=np.float64)[None, :]
        wave = np.sin(2.0 * np.pi * (np.cos(g_ang) * lx + np.sin(g_ang) * ly) / period + g_ph)
        for c in range(C):
            region = img[c, sy, sx]
            region[mask] += (g_amp * cvec[c] * wave)[mask]
    np.clip(img, 0.0, 1.0, out=img)
    return img.astype(dtype)


def add_noise(clean: np.ndarray, sigma_8bit: float, seed: int, dtype=None) -> np.ndarray:
    """Noisy observation z = clip(rint(255*(u + sigma/255*n))/255, 0, 1), n ~ N(0, 1) iid.

    ``rint`` rounds half to even. The noise generator is ``default_rng(seed + 10**6)``.
    """
    rng = np.random.default_rng(seed + 10**6)
    u = clean.astype(np.float64)
    n = rng.standard_normal(u.shape)
    z = np.clip(np.rint(255.0 * (u + (sigma_8bit / 255.0) * n)) / 255.0, 0.0, 1.0)
    return z.astype(dtype if dtype is not None else clean.dtype)


def noisy_pair(seed: int, H: int, W: int, C: int, sigma_8bit: float, dtype=np.float32):
    """(noisy z, clean u) for one seeded scene."""
    u = synth_scene(seed, H, W, C, dtype=dtype)
    return add_noise(u, sigma_8bit, seed, dtype=dtype), u


def ragged_sizes(seed: int, n: int, lo: int = 480, hi: int = 4032, step: int = 8,
                 max_pixels: int = 4032 * 3024):
    """n (W, H) pairs, each uniform over {lo, lo+step, ..., hi}, rejected if W*H > max_pixels."""
    rng = np.random.default_rng(seed)
    choices = np.arange(lo, hi + 1, step)
    out = []
    while len(out) < n:
        w, h = (int(v) for v in rng.choice(choices, 2))
        if w * h <= max_pixels:
            out.append((w, h))
    return out


def poisson_arrivals(rate_hz: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))


def random_bank_coeffs(seed: int, K: int, C: int, taps_f: int, taps_g: int) -> np.ndarray:
    """Stand-in filter coefficients [K][C][taps_f + taps_g], float64.

    Each filter is a positive, centre-weighted random kernel plus small signed
    jitter, scaled so that its taps sum to 1. Used only where a trained bank is
    not needed (timing runs, kernel plumbing), never as an expected value.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((K, C, taps_f + taps_g), dtype=np.float64)
    for part, n in ((0, taps_f), (1, taps_g)):
        if n == 0:
            continue
        r = int(round((np.sqrt(n) - 1) / 2))
        dy, dx = np.mgrid[-r:r + 1, -r:r + 1]
        d2 = (dy * dy + dx * dx).ravel().astype(np.float64)
        width = rng.uniform(0.6, 2.5, (K, C, 1))
        w = np.exp(-d2[None, None, :] / (2.0 * width * width))
        w += rng.normal(0.0, 0.05, w.shape)
        lo = 0 if part == 0 else taps_f
        out[:, :, lo:lo + n] = w
    out /= out.sum(axis=2, keepdims=True)
    return out
