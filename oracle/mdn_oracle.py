"""FP64 oracle of "Fast, Trainable, Multiscale Denoising" (Choi, Isidoro, Getreuer, Milanfar).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the GPU library, with which it shares no
code. Everything is float64 NumPy, written to be checked against the paper by
eye rather than to be fast.

Where the paper leaves a detail open, the reading taken here is named in the
docstring (colour matrix, gradient operator, box weighting, borders, bicubic
variant, orientation convention, thresholds, bucket layout, the meaning of
"i/2", ridge normalisation). The margin helpers report how close each pixel's
features lie to a bucket boundary, so that a second implementation may
legitimately pick the neighbouring bucket there.

Parity unpinned: agreement with the paper's Table 1 PSNR figures (its test and
training images are not available) and the authors' own threshold values and
bicubic variant.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "KR", "KB", "KG", "rgb_to_ycc", "ycc_to_rgb", "to_filter_space", "from_filter_space",
    "keys_cubic", "down2_weights", "down2", "build_pyramid",
    "shift", "coarse_shift", "gradients", "structure_tensor", "eigen_features",
    "quantize", "select", "select_margins", "tap_offsets",
    "LevelBank", "Bank", "apply_level", "denoise",
    "thresholds_from_features", "level_features", "GramStats", "patch_matrix",
    "accumulate_level", "solve_level", "train_single", "train_multiscale",
    "CrossGramStats", "accumulate_level_cross", "solve_level_cross", "apply_level_cross",
    "psnr", "round_storage", "dihedral", "augment_pairs", "luma", "selector_image", "upsample2",
    "down2_noise_gain", "pyramid_noise_gain", "paper_setup", "add_phase",
]

# --------------------------------------------------------------------------------------
# Colour conversion: footnote of Section 3 (YCbCr, ITU-R BT.601).
# Reading: full-range BT.601 built from Kr = 0.299, Kb = 0.114, chroma offset +1/2,
# no clamping; the inverse is the exact inverse matrix.
# --------------------------------------------------------------------------------------
KR = 0.299
KB = 0.114
KG = 1.0 - KR - KB


def _ycc_matrix() -> np.ndarray:
    m = np.zeros((3, 3))
    m[0] = [KR, KG, KB]                                   # Y
    m[1] = (np.array([0.0, 0.0, 1.0]) - m[0]) / (2.0 * (1.0 - KB))   # Cb = (B - Y) / 1.772
    m[2] = (np.array([1.0, 0.0, 0.0]) - m[0]) / (2.0 * (1.0 - KR))   # Cr = (R - Y) / 1.402
    return m


_YCC_OFFSET = np.array([0.0, 0.5, 0.5])


def rgb_to_ycc(rgb: np.ndarray) -> np.ndarray:
    """(3, H, W) RGB -> (3, H, W) YCbCr, float64."""
    x = np.asarray(rgb, dtype=np.float64)
    return np.einsum("ij,jhw->ihw", _ycc_matrix(), x) + _YCC_OFFSET[:, None, None]


def ycc_to_rgb(ycc: np.ndarray) -> np.ndarray:
    """Exact inverse of ``rgb_to_ycc``."""
    x = np.asarray(ycc, dtype=np.float64) - _YCC_OFFSET[:, None, None]
    return np.einsum("ij,jhw->ihw", np.linalg.inv(_ycc_matrix()), x)


def to_filter_space(img: np.ndarray) -> np.ndarray:
    """Colour images are filtered in YCbCr; grey images as they are."""
    img = np.asarray(img, dtype=np.float64)
    return rgb_to_ycc(img) if img.shape[0] == 3 else img.copy()


def from_filter_space(img: np.ndarray) -> np.ndarray:
    img = np.asarray(img, dtype=np.float64)
    return ycc_to_rgb(img) if img.shape[0] == 3 else img.copy()


def round_storage(x: np.ndarray, storage) -> np.ndarray:
    """Round to a storage type (float32/float16) and back to float64; None keeps float64."""
    if storage is None:
        return np.asarray(x, dtype=np.float64)
    return np.asarray(x).astype(storage).astype(np.float64)


# --------------------------------------------------------------------------------------
# Borders. Reading: every stencil (gradients, box, filter taps, coarse taps,
# downsampling) replicates the edge pixel: index clamp(i, 0, n-1).
# --------------------------------------------------------------------------------------

def shift(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """out[..., y, x] = x[..., clamp(y + dy), clamp(x + dx)]."""
    H, W = x.shape[-2:]
    ys = np.clip(np.arange(H) + dy, 0, H - 1)
    xs = np.clip(np.arange(W) + dx, 0, W - 1)
    return x[..., ys[:, None], xs[None, :]]


def coarse_shift(xc: np.ndarray, dy: int, dx: int, H: int, W: int) -> np.ndarray:
    """out[y, x] = xc[clamp(floor(y/2) + dy), clamp(floor(x/2) + dx)], an H x W field.

    Reading of "i/2" in Eq. (9)-(10): the coarse patch is centred on floor(i/2)
    per coordinate (the nearest coarse sample for both parities of i).
    """
    Hc, Wc = xc.shape[-2:]
    ys = np.clip(np.arange(H) // 2 + dy, 0, Hc - 1)
    xs = np.clip(np.arange(W) // 2 + dx, 0, Wc - 1)
    return xc[..., ys[:, None], xs[None, :]]


# --------------------------------------------------------------------------------------
# Pyramid: Section 4, "Multiscale filtering" (factor-two bicubic downsampling of
# the noisy and the clean images).
# Reading: Keys' cubic convolution kernel with a = -1/2, stretched by the factor
# two so that it low-passes before decimation, and centred between input samples
# 2m and 2m+1; the output of an n-sample axis has ceil(n/2) samples.
# --------------------------------------------------------------------------------------

def keys_cubic(t: float, a: float = -0.5) -> float:
    """Keys' cubic convolution kernel."""
    t = abs(t)
    if t < 1.0:
        return (a + 2.0) * t ** 3 - (a + 3.0) * t ** 2 + 1.0
    if t < 2.0:
        return a * t ** 3 - 5.0 * a * t ** 2 + 8.0 * a * t - 4.0 * a
    return 0.0


def down2_weights() -> np.ndarray:
    """Weights of input samples 2m-3 .. 2m+4 for output sample m."""
    w = np.array([keys_cubic((t - 0.5) / 2.0) for t in range(-3, 5)])
    return w / w.sum()


def _down2_axis(x: np.ndarray, axis: int) -> np.ndarray:
    w = down2_weights()
    n = x.shape[axis]
    m = (n + 1) // 2
    out = 0.0
    for k, t in enumerate(range(-3, 5)):
        idx = np.clip(2 * np.arange(m) + t, 0, n - 1)
        out = out + w[k] * np.take(x, idx, axis=axis)
    return out


def down2(x: np.ndarray) -> np.ndarray:
    """Separable factor-two bicubic downsampling of (C, H, W): rows, then columns."""
    x = np.asarray(x, dtype=np.float64)
    return _down2_axis(_down2_axis(x, axis=-1), axis=-2)


def build_pyramid(img: np.ndarray, n_levels: int, storage=None) -> List[np.ndarray]:
    """[z^0, ..., z^{n_levels-1}], z^{l+1} = down2(z^l), each rounded to ``storage``."""
    levels = [round_storage(img, storage)]
    for _ in range(n_levels - 1):
        levels.append(round_storage(down2(levels[-1]), storage))
    return levels


# --------------------------------------------------------------------------------------
# Filter selection: Section 3, "Filter selection", Eq. (3)-(6).
# --------------------------------------------------------------------------------------

def gradients(z: np.ndarray):
    """Per-channel gradients (g_x, g_y) of (C, H, W).

    Reading: central differences, g_x = (z[y, x+1] - z[y, x-1]) / 2 along columns
    and g_y = (z[y+1, x] - z[y-1, x]) / 2 along rows (rows grow downwards).
    """
    z = np.asarray(z, dtype=np.float64)
    gx = (shift(z, 0, 1) - shift(z, 0, -1)) / 2.0
    gy = (shift(z, 1, 0) - shift(z, -1, 0)) / 2.0
    return gx, gy


def structure_tensor(z: np.ndarray, box_radius: int = 2):
    """Entries (a, b, c) of the spatially filtered colour structure tensor, Eq. (6).

    T_i = sum_c sum_j w_j [[gx gx, gx gy], [gx gy, gy gy]] with the sum over the
    colour channels of z. Reading of the spatial weighting w: the mean over a
    (2r+1) x (2r+1) box (r = 2, i.e. 5 x 5), borders clamped.
    """
    gx, gy = gradients(z)
    A = (gx * gx).sum(axis=0)
    B = (gx * gy).sum(axis=0)
    Cc = (gy * gy).sum(axis=0)
    n = (2 * box_radius + 1) ** 2
    a = np.zeros_like(A)
    b = np.zeros_like(A)
    c = np.zeros_like(A)
    for dy in range(-box_radius, box_radius + 1):
        for dx in range(-box_radius, box_radius + 1):
            a += shift(A, dy, dx)
            b += shift(B, dy, dx)
            c += shift(Cc, dy, dx)
    return a / n, b / n, c / n


def eigen_features(a, b, c):
    """Orientation, strength and coherence of the 2x2 tensors [[a, b], [b, c]].

    lambda1 >= lambda2 are the eigenvalues; strength = sqrt(lambda1); coherence =
    (sqrt(l1) - sqrt(l2)) / (sqrt(l1) + sqrt(l2)) (Section 3). Orientation theta is
    the angle of the eigenvector of the smaller eigenvalue (the edge direction),
    measured from +x towards +y, in [0, pi).

    Readings for the degenerate cases: lambda2 is clamped at 0; coherence is 0
    when lambda1 = 0; when a = c and b = 0 the angle is pi/2 (atan2(0, 0) = 0,
    with -0 treated as +0).
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    tr = a + c
    mu = np.sqrt((a - c) ** 2 + 4.0 * b * b)
    lam1 = (tr + mu) / 2.0
    lam2 = np.maximum((tr - mu) / 2.0, 0.0)
    s1 = np.sqrt(np.maximum(lam1, 0.0))
    s2 = np.sqrt(lam2)
    with np.errstate(invalid="ignore", divide="ignore"):
        coh = np.where(s1 + s2 > 0.0, (s1 - s2) / (s1 + s2), 0.0)
    two_b = 2.0 * b + 0.0            # canonicalise -0 to +0
    a_m_c = (a - c) + 0.0
    major = 0.5 * np.arctan2(two_b, a_m_c)          # angle of the larger eigenvalue's vector
    theta = np.mod(major + np.pi / 2.0, np.pi)
    return theta, s1, coh


def quantize(theta, strength, coherence, q_theta: int, t_s: Sequence[float], t_c: Sequence[float]):
    """Bucket index s = (q_theta_bin * Qs + qs) * Qc + qc.

    Orientation: Qθ uniform bins over [0, pi). Strength and coherence: the number
    of thresholds the feature reaches (thresholds ascending, ties go up). The
    paper gives only the bin counts (Section 5 and the caption of Fig. 4).
    """
    q_s = len(t_s) + 1
    q_c = len(t_c) + 1
    qt = np.minimum(np.floor(theta * q_theta / np.pi).astype(np.int64), q_theta - 1)
    qs = np.zeros(np.shape(strength), dtype=np.int64)
    for t in t_s:
        qs += (strength >= t)
    qc = np.zeros(np.shape(coherence), dtype=np.int64)
    for t in t_c:
        qc += (coherence >= t)
    return (qt * q_s + qs) * q_c + qc


def select_margins(a, b, c, theta, strength, coherence, q_theta, t_s, t_c):
    """Distance of each pixel's features from the nearest bucket boundary.

    strength, coherence: min |feature - threshold|. Orientation: the distance of
    the unit-trace point ((a - c), 2b) / tr from the nearest boundary line, i.e.
    (mu / tr) * min_b |sin(2 (theta - b pi / Q))|; isotropic pixels (mu = 0, or tr
    = 0) are at distance 0 from every orientation boundary.
    """
    tr = np.asarray(a) + np.asarray(c)
    mu = np.sqrt((np.asarray(a) - np.asarray(c)) ** 2 + 4.0 * np.asarray(b) ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        aniso = np.where(tr > 0.0, mu / tr, 0.0)
    ang = np.min(np.abs(np.sin(2.0 * (theta[..., None] - np.arange(q_theta) * np.pi / q_theta))), axis=-1)
    m_theta = aniso * ang
    m_s = np.full(np.shape(strength), np.inf)
    for t in t_s:
        m_s = np.minimum(m_s, np.abs(strength - t))
    m_c = np.full(np.shape(coherence), np.inf)
    for t in t_c:
        m_c = np.minimum(m_c, np.abs(coherence - t))
    return np.minimum(np.minimum(m_theta, m_s), m_c)


def luma(rgb: np.ndarray) -> np.ndarray:
    """BT.601 luma Y = Kr R + Kg G + Kb B of an RGB (3, H, W) image, as a (1, H, W) image
    (the first row of the colour matrix of the footnote of Section 3)."""
    rgb = np.asarray(rgb, dtype=np.float64)
    return (KR * rgb[0] + KG * rgb[1] + KB * rgb[2])[None]


def _up2_axis(x: np.ndarray, axis: int, n: int) -> np.ndarray:
    """Linear interpolation by two along one axis, onto n fine samples: coarse sample m sits at
    fine coordinate 2m + 1/2, so fine 2m lies a quarter step left of it (3/4 of m, 1/4 of m-1) and
    fine 2m+1 a quarter step right (3/4 of m, 1/4 of m+1); indices clamped at the edges."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, 0)
    nc = x.shape[0]
    i = np.arange(n)
    m = i // 2
    other = np.clip(np.where(i % 2 == 0, m - 1, m + 1), 0, nc - 1)
    out = 0.75 * x[m] + 0.25 * x[other]
    return np.moveaxis(out, 0, axis)


def upsample2(x: np.ndarray, H: int, W: int) -> np.ndarray:
    """Factor-two upsampling of a (C, ceil(H/2), ceil(W/2)) level onto the (C, H, W) grid of the
    next finer level, on the pyramid's alignment (a coarse sample is centred between fine pixels
    2m and 2m+1): separable linear interpolation, rows then columns (_up2_axis)."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape[1] != (H + 1) // 2 or x.shape[2] != (W + 1) // 2:
        raise ValueError("coarse level must be ceil(H/2) x ceil(W/2)")
    return _up2_axis(_up2_axis(x, 1, H), 2, W)


def selector_image(z_sel: np.ndarray, selector: str = "rgb", u_coarse: Optional[np.ndarray] = None) -> np.ndarray:
    """The image whose structure tensor selects the filters.

    "rgb": the colour image itself, the channels summed in Eq. (6) (the paper's choice).
    "luma": its luma channel alone, the structure tensor of the earlier methods that Section 3
    compares against (Fig. 2: luma alone can miss structure that is visible in colour).
    Grey images are their own luma.
    "coarse": not the noisy level but the coarser level's denoised output u^{l+1} (in the filter
    colour space, as the cascade of Section 4 holds it), upsampled onto this level's grid
    (upsample2) and taken back to RGB; z_sel then only fixes the size. The alternative to
    selecting on the noisy z^l that Eq. (9) leaves open: the coarser output has less noise but
    half the resolution.
    """
    z_sel = np.asarray(z_sel, dtype=np.float64)
    if selector == "coarse":
        if u_coarse is None:
            raise ValueError("the coarse selector needs the coarser output")
        return from_filter_space(upsample2(u_coarse, z_sel.shape[1], z_sel.shape[2]))
    if selector == "luma" and z_sel.shape[0] == 3:
        return luma(z_sel)
    if selector not in ("rgb", "luma"):
        raise ValueError(selector)
    return z_sel


def add_phase(s: np.ndarray, phases: int) -> np.ndarray:
    """Phase-aware buckets (reading of the non-integer "i/2" of Eq. (9) for odd i): with phases = 4
    the parity of the pixel's row and column, p = 2 (y mod 2) + (x mod 2), joins the bucket index as
    s' = 4 s + p, so that each bucket has one upscale (and denoise) filter per phase of i relative to
    the coarser grid. phases = 1 leaves s as it is (one phase-blind filter per bucket)."""
    if phases == 1:
        return s
    if phases != 4:
        raise ValueError(phases)
    H, W = np.shape(s)
    p = 2 * (np.arange(H)[:, None] % 2) + (np.arange(W)[None, :] % 2)
    return 4 * np.asarray(s, dtype=np.int64) + p


def select(z_sel: np.ndarray, q_theta: int, t_s, t_c, return_margin: bool = False, selector: str = "rgb",
           phases: int = 1, u_coarse: Optional[np.ndarray] = None):
    """Filter selector s(i) from the image the structure tensor is taken on.

    Colour images: z_sel is RGB (the channels summed in Eq. (6)), or its luma with
    selector="luma"; grey: one channel. selector="coarse": the upsampled coarser output
    u_coarse instead (selector_image). phases = 4: phase-aware buckets (add_phase).
    """
    a, b, c = structure_tensor(selector_image(z_sel, selector, u_coarse))
    theta, strength, coh = eigen_features(a, b, c)
    s = add_phase(quantize(theta, strength, coh, q_theta, t_s, t_c), phases)
    if return_margin:
        return s, select_margins(a, b, c, theta, strength, coh, q_theta, t_s, t_c)
    return s


# --------------------------------------------------------------------------------------
# Filters and the cascade: Eq. (1)-(2) (single scale) and Eq. (9)-(10) (multiscale).
# --------------------------------------------------------------------------------------

def tap_offsets(radius: int):
    """Footprint F of a (2r+1)^2 filter as (dy, dx) offsets in row-major order."""
    return [(dy, dx) for dy in range(-radius, radius + 1) for dx in range(-radius, radius + 1)]


@dataclass
class LevelBank:
    """Filters of one level: coeffs[k, c] = [f taps (upscale block); g taps] (Eq. (10)).

    radius_f is None for the single-scale filter of Eq. (1) (no upscale block).
    K = q_theta * (len(t_s) + 1) * (len(t_c) + 1).
    """
    q_theta: int
    t_s: np.ndarray
    t_c: np.ndarray
    radius_g: int
    radius_f: Optional[int]
    coeffs: np.ndarray
    selector: str = "rgb"          # "rgb" (Eq. (6) over R, G, B), "luma" or "coarse" (selector_image)
    phases: int = 1                # 1, or 4 phase-aware buckets (add_phase); coeffs then has 4K rows

    @property
    def q_s(self):
        return len(self.t_s) + 1

    @property
    def q_c(self):
        return len(self.t_c) + 1

    @property
    def K(self):
        return self.q_theta * self.q_s * self.q_c * self.phases

    @property
    def taps_f(self):
        return 0 if self.radius_f is None else (2 * self.radius_f + 1) ** 2

    @property
    def taps_g(self):
        return (2 * self.radius_g + 1) ** 2


@dataclass
class Bank:
    """levels[l] holds the filters of trained level l = 0 (finest) .. L-1."""
    levels: List[LevelBank] = field(default_factory=list)


def apply_level(z_f: np.ndarray, s: np.ndarray, lb: LevelBank, u_coarse: Optional[np.ndarray] = None):
    """One filtering step, per channel of the filter colour space.

    Single scale (Eq. (1)): u_i = sum_j h^{s(i)}_j z_{i+j}.
    Multiscale (Eq. (9)): u_i = sum_j f^{s(i)}_j u^{l+1}_{i/2+j} + sum_j g^{s(i)}_j z^l_{i+j}.
    """
    z_f = np.asarray(z_f, dtype=np.float64)
    C, H, W = z_f.shape
    out = np.zeros((C, H, W))
    tf = lb.taps_f
    for ch in range(C):
        if lb.radius_f is not None:
            assert u_coarse is not None
            for t, (dy, dx) in enumerate(tap_offsets(lb.radius_f)):
                out[ch] += lb.coeffs[s, ch, t] * coarse_shift(u_coarse[ch], dy, dx, H, W)
        for t, (dy, dx) in enumerate(tap_offsets(lb.radius_g)):
            out[ch] += lb.coeffs[s, ch, tf + t] * shift(z_f[ch], dy, dx)
    return out


def _given_map(maps, lev: int, shape) -> Optional[np.ndarray]:
    """The caller's bucket map of level ``lev`` (None: select as usual)."""
    if maps is None or maps[lev] is None:
        return None
    s = np.asarray(maps[lev]).astype(np.int64)
    if s.shape != tuple(shape):
        raise ValueError(f"index map of level {lev} is {s.shape}, the level is {tuple(shape)}")
    return s


def denoise(img: np.ndarray, bank: Bank, storage=None, return_index_maps: bool = False, maps=None):
    """Coarse-to-fine cascade of Section 4: u^L = z^L, then Eq. (9) for l = L-1 .. 0.

    With a single level whose filters have no upscale block this is the plain
    single-scale filter of Eq. (1). ``storage`` (None, float32 or float16) rounds
    every stored pyramid level and every intermediate output to that type, to
    mirror a storage precision; arithmetic stays float64.

    ``maps``: optional list, one entry per trained level, of (H_l, W_l) bucket maps that
    replace the selection of that level (None entries select as usual). A pixel whose
    features lie on a bucket boundary may legitimately take either bucket; with the maps
    another implementation actually used, the cascade is then defined for every pixel.
    """
    L = len(bank.levels)
    multiscale = bank.levels[0].radius_f is not None
    img = round_storage(img, storage)
    if maps is not None and len(maps) != L:
        raise ValueError(f"maps: one entry per trained level ({L}), got {len(maps)}")
    if not multiscale:
        lb = bank.levels[0]
        s = _given_map(maps, 0, img.shape[1:])
        if s is None:
            s = select(img, lb.q_theta, lb.t_s, lb.t_c, selector=lb.selector, phases=lb.phases)
        out = from_filter_space(apply_level(to_filter_space(img), s, lb))
        out = round_storage(out, storage)
        return (out, [s]) if return_index_maps else out
    pyr = build_pyramid(img, L + 1, storage)
    u = to_filter_space(pyr[L])
    out_maps = [None] * L
    for lev in range(L - 1, -1, -1):
        lb = bank.levels[lev]
        s = _given_map(maps, lev, pyr[lev].shape[1:])
        if s is None:
            s = select(pyr[lev], lb.q_theta, lb.t_s, lb.t_c, selector=lb.selector, phases=lb.phases, u_coarse=u)
        out_maps[lev] = s
        u = apply_level(to_filter_space(pyr[lev]), s, lb, u_coarse=u)
        if lev > 0:
            u = round_storage(u, storage)
    out = round_storage(from_filter_space(u), storage)
    return (out, out_maps) if return_index_maps else out


# --------------------------------------------------------------------------------------
# Training: Eq. (7)-(8), one least-squares regression per bucket and channel,
# trained level by level from the second-coarsest level down (Section 4).
# --------------------------------------------------------------------------------------

def level_features(z_sel: np.ndarray, selector: str = "rgb", u_coarse: Optional[np.ndarray] = None):
    """(strength, coherence) of every pixel, flattened."""
    a, b, c = structure_tensor(selector_image(z_sel, selector, u_coarse))
    _, strength, coh = eigen_features(a, b, c)
    return strength.ravel(), coh.ravel()


def thresholds_from_features(values: np.ndarray, q: int) -> np.ndarray:
    """Equal-population thresholds: the k/q quantiles, k = 1 .. q-1 (linear interpolation).

    Reading: the paper gives only the number of strength and coherence bins.
    """
    if q <= 1:
        return np.zeros(0)
    return np.quantile(np.asarray(values, dtype=np.float64), np.arange(1, q) / q)


def patch_matrix(x: np.ndarray, radius: int, coarse_of_shape=None) -> np.ndarray:
    """Rows R_i x for every pixel i (row-major), columns in tap order.

    With ``coarse_of_shape=(H, W)`` the patches are taken on the coarse image at
    floor(i/2) for the H x W fine grid (the R_{i/2} of Eq. (10)).
    """
    cols = []
    for dy, dx in tap_offsets(radius):
        if coarse_of_shape is None:
            cols.append(shift(x, dy, dx).ravel())
        else:
            cols.append(coarse_shift(x, dy, dx, *coarse_of_shape).ravel())
    return np.stack(cols, axis=1)


@dataclass
class GramStats:
    """Per bucket k and channel c: G = sum x x^T, b = sum x y, yy = sum y^2; n = count."""
    G: np.ndarray   # (K, C, D, D)
    b: np.ndarray   # (K, C, D)
    n: np.ndarray   # (K,)
    yy: np.ndarray  # (K, C)

    @staticmethod
    def zeros(K: int, C: int, D: int) -> "GramStats":
        return GramStats(np.zeros((K, C, D, D)), np.zeros((K, C, D)), np.zeros(K, dtype=np.int64),
                         np.zeros((K, C)))


def accumulate_level(stats: GramStats, s: np.ndarray, z_f: np.ndarray, target_f: np.ndarray,
                     radius_g: int, radius_f: Optional[int] = None, u_coarse: Optional[np.ndarray] = None):
    """Add one training pair's samples to the normal equations of Eq. (8).

    x_i = [R_{i/2} u^{l+1}_c ; R_i z^l_c] (or R_i z_c single-scale), y_i = u^l_{i,c}, k = s(i).
    """
    C, H, W = z_f.shape
    sk = np.asarray(s).ravel()
    K = stats.G.shape[0]
    stats.n += np.bincount(sk, minlength=K)
    for ch in range(C):
        blocks = []
        if radius_f is not None:
            blocks.append(patch_matrix(u_coarse[ch], radius_f, coarse_of_shape=(H, W)))
        blocks.append(patch_matrix(z_f[ch], radius_g))
        X = np.concatenate(blocks, axis=1)
        y = np.asarray(target_f[ch], dtype=np.float64).ravel()
        for k in np.unique(sk):
            sel = sk == k
            Xk = X[sel]
            yk = y[sel]
            stats.G[k, ch] += Xk.T @ Xk
            stats.b[k, ch] += Xk.T @ yk
            stats.yy[k, ch] += yk @ yk
    return stats


def solve_level(stats: GramStats, lam: float, n_min: Optional[int] = None):
    """Per-bucket ridge solution h_k = (G_k / n_k + lam I)^{-1} b_k / n_k.

    Readings: the regression details are deferred by the paper to BLADE; the
    ridge term is taken on the mean-normalised normal equations. Buckets with
    fewer than ``n_min`` samples (default: the tap count D) take the pooled
    solution of the whole level. Returns (coeffs (K, C, D), fallback mask (K,)).
    """
    K, C, D, _ = stats.G.shape
    if n_min is None:
        n_min = D
    eye = np.eye(D)
    n_all = stats.n.sum()
    out = np.zeros((K, C, D))
    fallback = stats.n < n_min
    for ch in range(C):
        Gp = stats.G[:, ch].sum(axis=0)
        bp = stats.b[:, ch].sum(axis=0)
        pooled = np.linalg.solve(Gp / max(n_all, 1) + lam * eye, bp / max(n_all, 1)) if n_all > 0 else np.zeros(D)
        for k in range(K):
            if fallback[k]:
                out[k, ch] = pooled
            else:
                nk = stats.n[k]
                out[k, ch] = np.linalg.solve(stats.G[k, ch] / nk + lam * eye, stats.b[k, ch] / nk)
    return out, fallback


# --------------------------------------------------------------------------------------
# Cross-channel regression (a reading of a literal 147-tap feature vector: the 7x7 patches of
# all three filter-space channels concatenated, one system per bucket with one right-hand side
# per output channel). Not used by the paper's per-channel inference; kept for the training
# precision study.

@dataclass
class CrossGramStats:
    """Per bucket k: G = sum x x^T (one matrix), b[c] = sum x y_c, yy[c] = sum y_c^2; n = count."""
    G: np.ndarray   # (K, D, D), D = C * taps
    b: np.ndarray   # (K, C, D)
    n: np.ndarray   # (K,)
    yy: np.ndarray  # (K, C)

    @staticmethod
    def zeros(K: int, C: int, D: int) -> "CrossGramStats":
        return CrossGramStats(np.zeros((K, D, D)), np.zeros((K, C, D)), np.zeros(K, dtype=np.int64),
                              np.zeros((K, C)))


def _cross_patches(z_f: np.ndarray, radius: int) -> np.ndarray:
    return np.concatenate([patch_matrix(z_f[ch], radius) for ch in range(z_f.shape[0])], axis=1)


def accumulate_level_cross(stats: CrossGramStats, s: np.ndarray, z_f: np.ndarray, target_f: np.ndarray,
                           radius: int):
    """x_i = [R_i z_0; R_i z_1; ...; R_i z_{C-1}], y_i = target at i (all channels), k = s(i)."""
    C = z_f.shape[0]
    sk = np.asarray(s).ravel()
    K = stats.G.shape[0]
    stats.n += np.bincount(sk, minlength=K)
    X = _cross_patches(z_f, radius)
    Y = np.asarray(target_f, dtype=np.float64).reshape(C, -1)
    for k in np.unique(sk):
        sel = sk == k
        Xk = X[sel]
        stats.G[k] += Xk.T @ Xk
        for ch in range(C):
            yk = Y[ch, sel]
            stats.b[k, ch] += Xk.T @ yk
            stats.yy[k, ch] += yk @ yk
    return stats


def solve_level_cross(stats: CrossGramStats, lam: float, n_min: Optional[int] = None):
    """h_{k,c} = (G_k / n_k + lam I)^{-1} b_{k,c} / n_k, pooled solution for sparse buckets.

    Returns (coeffs (K, C, D), fallback mask (K,))."""
    K, C, D = stats.b.shape
    if n_min is None:
        n_min = D
    eye = np.eye(D)
    n_all = stats.n.sum()
    fallback = stats.n < n_min
    out = np.zeros((K, C, D))
    Gp, bp = stats.G.sum(axis=0), stats.b.sum(axis=0)
    for ch in range(C):
        pooled = np.linalg.solve(Gp / max(n_all, 1) + lam * eye, bp[ch] / max(n_all, 1)) if n_all > 0 else np.zeros(D)
        for k in range(K):
            if fallback[k]:
                out[k, ch] = pooled
            else:
                out[k, ch] = np.linalg.solve(stats.G[k] / stats.n[k] + lam * eye, stats.b[k, ch] / stats.n[k])
    return out, fallback


def apply_level_cross(z_f: np.ndarray, s: np.ndarray, coeffs: np.ndarray, radius: int) -> np.ndarray:
    """Output channel c at i: sum over input channels c' and taps j of h[s(i)][c][c' taps + j] z_{c'}(i+j)."""
    C, H, W = z_f.shape
    X = _cross_patches(z_f, radius)
    sk = np.asarray(s).ravel()
    out = np.empty((C, H * W))
    for ch in range(C):
        out[ch] = np.einsum("nd,nd->n", X, coeffs[sk, ch])
    return out.reshape(C, H, W)


# --------------------------------------------------------------------------------------
# Training-set augmentation: Section 5 adds the axial flips and 90-degree rotations of
# every noisy/clean pair so that the filters learn the symmetries.
# Reading: all eight symmetries of the square (the dihedral group D4), numbered by three
# bits applied in this order: bit 2 transposes (rows <-> columns), then bit 0 mirrors
# the columns (x -> W-1-x) and bit 1 mirrors the rows (y -> H-1-y).
# --------------------------------------------------------------------------------------

def dihedral(img: np.ndarray, t: int) -> np.ndarray:
    """Symmetry t (0..7) of the square applied to the last two axes of img."""
    x = np.asarray(img)
    if t & 4:
        x = np.swapaxes(x, -1, -2)
    if t & 1:
        x = x[..., :, ::-1]
    if t & 2:
        x = x[..., ::-1, :]
    return np.ascontiguousarray(x)


def augment_pairs(pairs):
    """Every pair followed by its seven other symmetries (the same symmetry on both images)."""
    return [(dihedral(z, t), dihedral(u, t)) for z, u in pairs for t in range(8)]


def train_single(pairs, q_theta: int, q_s: int, q_c: int, radius: int, lam: float,
                 t_s=None, t_c=None, n_min=None, augment: bool = False, selector: str = "rgb",
                 phases: int = 1):
    """Single-scale bank (Eq. (1), (7)-(8)) from (noisy, clean) pairs of (C, H, W) images.

    augment: train on the eight symmetries of every pair (Section 5).
    selector: structure tensor of the colour image ("rgb") or of its luma ("luma"); a single
    level has no coarser output, so "coarse" is refused."""
    if selector == "coarse":
        raise ValueError("a single-scale level has no coarser output to select on")
    if augment:
        pairs = augment_pairs(pairs)
    zs = [np.asarray(z, dtype=np.float64) for z, _ in pairs]
    if t_s is None or t_c is None:
        feats = [level_features(z, selector) for z in zs]
        st = np.concatenate([f[0] for f in feats])
        co = np.concatenate([f[1] for f in feats])
        t_s = thresholds_from_features(st, q_s) if t_s is None else np.asarray(t_s, float)
        t_c = thresholds_from_features(co, q_c) if t_c is None else np.asarray(t_c, float)
    K = q_theta * q_s * q_c * phases
    C = zs[0].shape[0]
    D = (2 * radius + 1) ** 2
    stats = GramStats.zeros(K, C, D)
    for (z, u) in pairs:
        s = select(np.asarray(z, np.float64), q_theta, t_s, t_c, selector=selector, phases=phases)
        accumulate_level(stats, s, to_filter_space(z), to_filter_space(u), radius)
    coeffs, fb = solve_level(stats, lam, n_min)
    lb = LevelBank(q_theta, np.asarray(t_s, float), np.asarray(t_c, float), radius, None, coeffs, selector, phases)
    return Bank([lb]), stats, fb


def train_multiscale(pairs, n_trained_levels: int, q_theta: int, q_s: int, q_c: int,
                     radius_f: int, radius_g: int, lam: float, thresholds=None, n_min=None,
                     storage=None, augment: bool = False, selector: str = "rgb", phases: int = 1):
    """Multiscale bank, trained from the second-coarsest level down (Section 4).

    Level l is fitted with u^{l+1} = the output of the already trained level l+1
    on the same pair (u^L = z^L); targets are the clean pyramid levels.
    ``thresholds``: optional list (per level) of (t_s, t_c); otherwise the
    equal-population quantiles of each level's training features.
    ``augment``: train on the eight symmetries of every pair (Section 5); each
    symmetric copy is a pair of its own, with its own pyramid and cascade.
    ``selector``: structure tensor of the colour levels ("rgb"), of their luma ("luma"), or of
    the upsampled coarser output of the pair's own training cascade ("coarse", selector_image).
    ``phases``: 1, or 4 for phase-aware buckets (add_phase).
    """
    if augment:
        pairs = augment_pairs(pairs)
    L = n_trained_levels
    pz = [build_pyramid(z, L + 1, storage) for z, _ in pairs]
    pu = [build_pyramid(u, L + 1, storage) for _, u in pairs]
    C = pz[0][0].shape[0]
    levels: List[Optional[LevelBank]] = [None] * L
    stats_all = [None] * L
    fallbacks = [None] * L
    uhat = [to_filter_space(p[L]) for p in pz]
    for lev in range(L - 1, -1, -1):
        if thresholds is not None:
            t_s, t_c = (np.asarray(t, float) for t in thresholds[lev])
        else:
            feats = [level_features(p[lev], selector, uhat[i]) for i, p in enumerate(pz)]
            t_s = thresholds_from_features(np.concatenate([f[0] for f in feats]), q_s)
            t_c = thresholds_from_features(np.concatenate([f[1] for f in feats]), q_c)
        K = q_theta * q_s * q_c * phases
        D = (2 * radius_f + 1) ** 2 + (2 * radius_g + 1) ** 2
        stats = GramStats.zeros(K, C, D)
        smaps = []
        for i in range(len(pairs)):
            s = select(pz[i][lev], q_theta, t_s, t_c, selector=selector, phases=phases, u_coarse=uhat[i])
            smaps.append(s)
            accumulate_level(stats, s, to_filter_space(pz[i][lev]), to_filter_space(pu[i][lev]),
                             radius_g, radius_f, uhat[i])
        coeffs, fb = solve_level(stats, lam, n_min)
        lb = LevelBank(q_theta, t_s, t_c, radius_g, radius_f, coeffs, selector, phases)
        levels[lev] = lb
        stats_all[lev] = stats
        fallbacks[lev] = fb
        uhat = [round_storage(apply_level(to_filter_space(pz[i][lev]), smaps[i], lb, uhat[i]), storage)
                for i in range(len(pairs))]
    return Bank(levels), stats_all, fallbacks


# --------------------------------------------------------------------------------------
# The paper's experimental configuration (Section 5): 16 orientation x 16 strength x 16
# coherence buckets at every level; 5x5 filters at the finer level and 3x3 at the coarser one
# for sigma < 10, 7x7 and 5x5 otherwise; as many levels as make the coarsest level's noise
# standard deviation fall below 2 (in 8-bit units).
# Readings: "finer level" is the level's own input (the g taps, Eq. (10)) and "coarser level"
# the upsampled coarser output (the f taps); the noise of level l is the standard deviation of
# the pyramid of white noise of standard deviation sigma at level l. Through the first down2 the
# white noise keeps only 0.4044 of its deviation (R12); the output is no longer white, so the
# deviation of later levels follows from the whole cascade, not from that factor alone.
# --------------------------------------------------------------------------------------

def down2_noise_gain() -> float:
    """Standard deviation of down2 applied to unit white noise: the 2-D filter's root sum of
    squared weights, i.e. the 1-D sum of squared weights (about 0.4044, R12)."""
    w = down2_weights()
    return float(np.sum(w * w))


def pyramid_noise_gain(level: int) -> float:
    """Standard deviation at pyramid level `level` of unit white noise at level 0 (away from the
    borders): the root sum of squares of the cascade's weights on the level-0 samples, per axis,
    squared for the separable 2-D cascade."""
    n = 64 * 2 ** level
    rows = np.eye(n)
    for _ in range(level):
        rows = _down2_axis(rows, 0)          # row j: weights of output sample j on the inputs
    r = rows[rows.shape[0] // 2]
    return float(np.sum(r * r))


def paper_setup(sigma_8bit: float):
    """(trained levels L, radius_f, radius_g, (q_theta, q_s, q_c)) for noise sigma (8-bit units);
    the pyramid has L + 1 levels and the noise of its coarsest one is below 2."""
    L = 1
    while sigma_8bit * pyramid_noise_gain(L) >= 2.0:
        L += 1
    rf, rg = (1, 2) if sigma_8bit < 10 else (2, 3)
    return L, rf, rg, (16, 16, 16)


def psnr(est: np.ndarray, ref: np.ndarray) -> float:
    """PSNR in dB with peak 1 over all channels, of clip(est, 0, 1) against ref."""
    e = np.clip(np.asarray(est, np.float64), 0.0, 1.0) - np.asarray(ref, np.float64)
    mse = float(np.mean(e * e))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(1.0 / mse)
