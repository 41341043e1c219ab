"""ctypes binding of libmdn (include/mdn.h): argument marshalling only.

Every step of the denoiser runs in the HIP library; this module turns torch tensors
(device memory and the current stream) into the C descriptors and raises on a
non-OK status. It fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes as ct
import os
import re
from typing import List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# MDN_LIB names another build of the same library (the sanitizer variants of build.py)
LIB_PATH = os.environ.get("MDN_LIB") or os.path.join(_PKG, "libmdn.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "mdn.h")

MDN_OK, MDN_EINVAL, MDN_ENOMEM, MDN_EDEVICE, MDN_ENOTSUP, MDN_ETIMEOUT, MDN_ECANCELED = range(7)
F32, F16 = 0, 1
GRAY, RGB, YCC = 0, 1, 2
SELECT_RGB, SELECT_LUMA, SELECT_COARSE = 0, 1, 2       # mdn_selector
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOTSUP", 5: "ETIMEOUT", 6: "ECANCELED"}


class MdnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mdn {_STATUS.get(status, status)}: {msg}")
        self.status = status


class MdnImage(ct.Structure):
    _fields_ = [("data", ct.c_void_p), ("width", ct.c_int32), ("height", ct.c_int32),
                ("channels", ct.c_int32), ("dtype", ct.c_int32), ("color", ct.c_int32),
                ("reserved", ct.c_int32), ("row_pitch", ct.c_int64), ("plane_pitch", ct.c_int64)]


class MdnLevel(ct.Structure):
    _fields_ = [("q_theta", ct.c_int32), ("q_s", ct.c_int32), ("q_c", ct.c_int32),
                ("radius_f", ct.c_int32), ("radius_g", ct.c_int32), ("channels", ct.c_int32),
                ("coeff_dtype", ct.c_int32), ("selector", ct.c_int32), ("phases", ct.c_int32),
                ("reserved", ct.c_int32),
                ("t_s", ct.POINTER(ct.c_double)), ("t_c", ct.POINTER(ct.c_double)),
                ("coeffs", ct.c_void_p)]


class MdnBank(ct.Structure):
    _fields_ = [("levels", ct.c_int32), ("reserved", ct.c_int32), ("level", ct.POINTER(MdnLevel))]


_lib = None


def lib() -> ct.CDLL:
    """Load libmdn.so (built in-tree). Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmdn.so not built at {LIB_PATH}; run python -m paper_1802_06130_amd.build")
        L = ct.CDLL(LIB_PATH)
        vp, i32, i64 = ct.c_void_p, ct.c_int32, ct.c_int64
        P = ct.POINTER
        sig = {
            "mdn_pyramid_build": [P(MdnImage), i32, P(MdnImage), vp],
            "mdn_dihedral": [P(MdnImage), i32, P(MdnImage), vp],
            "mdn_select_filters": [P(MdnImage), P(MdnLevel), vp, i64, vp],
            "mdn_select_filters_coarse": [P(MdnImage), i32, i32, P(MdnLevel), vp, i64, vp],
            "mdn_apply_level": [P(MdnImage), P(MdnImage), vp, i64, P(MdnLevel), P(MdnImage), vp, vp],
            "mdn_denoise_workspace_size": [i32, i32, i32, i32, i32, P(ct.c_size_t)],
            "mdn_denoise": [P(MdnImage), P(MdnBank), i32, vp, ct.c_size_t, P(MdnImage), vp],
            "mdn_denoise_noalloc": [P(MdnImage), P(MdnBank), i32, P(MdnImage), vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ct.c_int
        L.mdn_last_error.restype = ct.c_char_p
        L.mdn_version.restype = ct.c_char_p
        _lib = L
    return _lib


def header_functions() -> List[str]:
    """Names of the functions declared in include/mdn.h."""
    with open(HEADER_PATH) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(mdn_[a-z_0-9]+)\s*\(", text, re.M)))


def _check(status: int):
    if status != MDN_OK:
        raise MdnError(status, lib().mdn_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float16:
        return F16
    raise TypeError(f"unsupported image dtype {t.dtype}")


def image(t, color: Optional[int] = None) -> MdnImage:
    """Descriptor of a (C, H, W) CUDA tensor with unit stride along W."""
    if t.dim() != 3:
        raise ValueError("images are (C, H, W)")
    C, H, W = t.shape
    if W > 1 and t.stride(2) != 1:
        raise ValueError("images need unit stride along W")
    if color is None:
        color = GRAY if C == 1 else RGB
    return MdnImage(ct.c_void_p(t.data_ptr()), W, H, C, _dtype_code(t), color, 0, t.stride(1), t.stride(0))


class Level:
    """One trained level: thresholds on the host, coefficients on the device."""

    def __init__(self, q_theta: int, t_s: Sequence[float], t_c: Sequence[float], radius_g: int,
                 radius_f: Optional[int], coeffs, channels: int, selector: int = 0, phases: int = 1):
        self.q_theta = int(q_theta)
        self.selector = int(selector)          # SELECT_RGB, SELECT_LUMA or SELECT_COARSE
        self.phases = int(phases)              # 1, or 4 phase-aware buckets
        self.t_s = np.ascontiguousarray(np.asarray(t_s, dtype=np.float64))
        self.t_c = np.ascontiguousarray(np.asarray(t_c, dtype=np.float64))
        self.radius_g = int(radius_g)
        self.radius_f = -1 if radius_f is None else int(radius_f)
        self.coeffs = coeffs.contiguous()          # device tensor [K][C][D]
        self.channels = int(channels)
        self._ts_arr = (ct.c_double * max(1, len(self.t_s)))(*self.t_s.tolist())
        self._tc_arr = (ct.c_double * max(1, len(self.t_c)))(*self.t_c.tolist())

    @property
    def K(self):
        return self.q_theta * (len(self.t_s) + 1) * (len(self.t_c) + 1) * self.phases

    def desc(self) -> MdnLevel:
        return MdnLevel(self.q_theta, len(self.t_s) + 1, len(self.t_c) + 1, self.radius_f, self.radius_g,
                        self.channels, _dtype_code(self.coeffs), self.selector, self.phases, 0,
                        ct.cast(self._ts_arr, ct.POINTER(ct.c_double)),
                        ct.cast(self._tc_arr, ct.POINTER(ct.c_double)),
                        ct.c_void_p(self.coeffs.data_ptr()))


class Bank:
    def __init__(self, levels: List[Level]):
        self.levels = list(levels)

    def desc(self) -> MdnBank:
        self._arr = (MdnLevel * len(self.levels))(*[lv.desc() for lv in self.levels])
        return MdnBank(len(self.levels), 0, ct.cast(self._arr, ct.POINTER(MdnLevel)))


def pyramid_build(level0, n_out: int, storage=None, out=None):
    """Levels 1..n_out of the factor-two bicubic pyramid of ``level0`` (C, H, W)."""
    torch = _torch()
    C, H, W = level0.shape
    dt = level0.dtype if storage is None else storage
    if out is None:
        out = []
        h, w = H, W
        for _ in range(n_out):
            h, w = (h + 1) // 2, (w + 1) // 2
            out.append(torch.empty((C, h, w), dtype=dt, device=level0.device))
    color = GRAY if C == 1 else RGB
    descs = (MdnImage * max(1, n_out))(*[image(o, color) for o in out])
    _check(lib().mdn_pyramid_build(ct.byref(image(level0, color)), n_out, descs, _stream_ptr()))
    return out


def dihedral(img, transform: int, out=None):
    """Symmetry ``transform`` (0..7) of the square applied to every plane of ``img`` (C, H, W):
    bit 2 transposes (first), bit 0 mirrors the columns, bit 1 the rows (Section 5)."""
    torch = _torch()
    C, H, W = img.shape
    if out is None:
        shape = (C, W, H) if transform & 4 else (C, H, W)
        out = torch.empty(shape, dtype=img.dtype, device=img.device)
    color = GRAY if C == 1 else RGB
    _check(lib().mdn_dihedral(ct.byref(image(img, color)), int(transform), ct.byref(image(out, color)), _stream_ptr()))
    return out


def augment_pairs(pairs):
    """Every (noisy, clean) pair followed by its seven other symmetries, made on the GPU."""
    return [(dihedral(z, t), dihedral(u, t)) for z, u in pairs for t in range(8)]


def selector_dtype(level: Level):
    """Element type of a level's selector maps: uint8 for K <= 256 buckets, uint16 above."""
    torch = _torch()
    return torch.uint16 if level.K > 256 else torch.uint8


def _check_map(t, level: Level, name: str):
    if t is not None and t.dtype != selector_dtype(level):
        raise MdnError(MDN_EINVAL, f"{name}: selector maps of a {level.K}-bucket level are {selector_dtype(level)}")


def select_filters(z, level: Level, out=None, u_coarse=None, coarse_color=None):
    """(H, W) bucket map of the RGB/grey image z (uint8, or uint16 when K > 256). A level with
    selector=SELECT_COARSE selects on the coarser output u_coarse instead (YCbCr unless coarse_color
    says otherwise); z then only gives the size."""
    torch = _torch()
    C, H, W = z.shape
    if out is None:
        out = torch.empty((H, W), dtype=selector_dtype(level), device=z.device)
    _check_map(out, level, "out")
    lv = level.desc()
    pitch = out.stride(0) if H > 0 else W
    if level.selector == SELECT_COARSE and u_coarse is not None:
        uc = image(u_coarse, coarse_color if coarse_color is not None else (GRAY if C == 1 else YCC))
        _check(lib().mdn_select_filters_coarse(ct.byref(uc), W, H, ct.byref(lv), ct.c_void_p(out.data_ptr()),
                                               pitch, _stream_ptr()))
        return out
    _check(lib().mdn_select_filters(ct.byref(image(z)), ct.byref(lv), ct.c_void_p(out.data_ptr()), pitch,
                                    _stream_ptr()))
    return out


def apply_level(z, level: Level, u_coarse=None, s=None, out=None, out_color=None, coarse_color=None,
                out_dtype=None, s_out=None):
    """One filtering step; returns u_out (C, H, W) in YCbCr unless out_color says otherwise.
    ``s_out`` ((H, W) map, uint8 or uint16 as for select_filters) receives the selector used when
    selecting inline."""
    torch = _torch()
    C, H, W = z.shape
    if out_color is None:
        out_color = GRAY if C == 1 else YCC
    if out is None:
        out = torch.empty((C, H, W), dtype=out_dtype or z.dtype, device=z.device)
    uc = None
    if u_coarse is not None:
        uc = image(u_coarse, coarse_color if coarse_color is not None else (GRAY if C == 1 else YCC))
    lv = level.desc()
    if s is None and s_out is None and u_coarse is not None and level.coeffs.dtype == torch.float16 and C == 3:
        s_out = torch.empty((H, W), dtype=selector_dtype(level), device=z.device)   # the float16 path's map
    _check_map(s, level, "s")
    _check_map(s_out, level, "s_out")
    sp = s.stride(0) if s is not None else (s_out.stride(0) if s_out is not None else 0)
    _check(lib().mdn_apply_level(ct.byref(image(z)), ct.byref(uc) if uc is not None else None,
                                 ct.c_void_p(s.data_ptr()) if s is not None else None, sp, ct.byref(lv),
                                 ct.byref(image(out, out_color)),
                                 ct.c_void_p(s_out.data_ptr()) if s_out is not None else None, _stream_ptr()))
    return out


def denoise_workspace_size(width: int, height: int, channels: int, levels: int, storage: int = F32) -> int:
    n = ct.c_size_t(0)
    _check(lib().mdn_denoise_workspace_size(width, height, channels, levels, storage, ct.byref(n)))
    return n.value


def denoise(img, bank: Bank, storage: int = F32, ws=None, out=None):
    """Whole cascade of one (C, H, W) image; returns the denoised image in the input's colour."""
    torch = _torch()
    C, H, W = img.shape
    if out is None:
        out = torch.empty_like(img)
    need = denoise_workspace_size(W, H, C, len(bank.levels), storage)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=img.device)
    b = bank.desc()
    _check(lib().mdn_denoise(ct.byref(image(img)), ct.byref(b), storage, ct.c_void_p(ws.data_ptr()),
                             ws.numel(), ct.byref(image(out)), _stream_ptr()))
    return out


NOALLOC_SCRATCH_BYTES = 128 << 20     # MDN_NOALLOC_SCRATCH_BYTES of include/mdn.h


def denoise_noalloc(img, bank: Bank, storage: int = F32, out=None):
    """mdn_denoise_noalloc: the cascade with the library's static device scratch as workspace (the
    library allocates nothing; ``out`` is allocated here unless given). Calls that overlap on one
    device race on that scratch."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(img)
    b = bank.desc()
    _check(lib().mdn_denoise_noalloc(ct.byref(image(img)), ct.byref(b), storage, ct.byref(image(out)), _stream_ptr()))
    return out


# ----------------------------------------------------------------------------- training

X_PER_CHANNEL, X_CROSS_CHANNEL = 0, 1
GRAM_F32, GRAM_BF16X3 = 0, 1


class MdnGram(ct.Structure):
    _fields_ = [("K", ct.c_int32), ("channels", ct.c_int32), ("layout", ct.c_int32), ("radius_f", ct.c_int32),
                ("radius_g", ct.c_int32), ("reserved", ct.c_int32), ("G", ct.c_void_p), ("b", ct.c_void_p),
                ("n", ct.c_void_p), ("yy", ct.c_void_p)]


def _train_sigs(L):
    vp, i32, i64 = ct.c_void_p, ct.c_int32, ct.c_int64
    P = ct.POINTER
    sig = {
        "mdn_gram_dims": [P(MdnGram), P(i32), P(i32), P(i32)],
        "mdn_gram_zero": [P(MdnGram), vp],
        "mdn_train_workspace_size": [P(MdnGram), i32, i32, P(ct.c_size_t)],
        "mdn_train_accumulate": [P(MdnGram), P(MdnImage), P(MdnImage), P(MdnImage), P(MdnLevel), i32, vp,
                                 ct.c_size_t, vp],
        "mdn_train_solve_workspace_size": [P(MdnGram), P(ct.c_size_t)],
        "mdn_train_solve": [P(MdnGram), ct.c_double, i64, vp, i32, vp, vp, ct.c_size_t, vp],
        "mdn_level_features": [P(MdnImage), i32, vp, vp, vp],
        "mdn_level_features_coarse": [P(MdnImage), i32, i32, vp, vp, vp],
        "mdn_quantiles_workspace_size": [i64, P(ct.c_size_t)],
        "mdn_quantiles": [vp, i64, i32, P(ct.c_double), vp, ct.c_size_t, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ct.c_int


class Gram:
    """Normal equations of one level (device float64 accumulators)."""

    def __init__(self, K: int, channels: int, radius_g: int, radius_f: Optional[int] = None,
                 layout: int = X_PER_CHANNEL, device="cuda"):
        torch = _torch()
        _train_sigs(lib())
        self.cfg = (int(K), int(channels), int(layout), -1 if radius_f is None else int(radius_f), int(radius_g))
        d = MdnGram(*self.cfg, 0, None, None, None, None)
        D, nrhs, nsys = ct.c_int32(), ct.c_int32(), ct.c_int32()
        _check(lib().mdn_gram_dims(ct.byref(d), ct.byref(D), ct.byref(nrhs), ct.byref(nsys)))
        self.D, self.nrhs, self.systems = D.value, nrhs.value, nsys.value
        self.G = torch.zeros(self.systems * self.D * self.D, dtype=torch.float64, device=device)
        self.b = torch.zeros(self.systems * self.nrhs * self.D, dtype=torch.float64, device=device)
        self.n = torch.zeros(K, dtype=torch.int64, device=device)
        self.yy = torch.zeros(self.systems * self.nrhs, dtype=torch.float64, device=device)

    def desc(self) -> MdnGram:
        return MdnGram(*self.cfg, 0, ct.c_void_p(self.G.data_ptr()), ct.c_void_p(self.b.data_ptr()),
                       ct.c_void_p(self.n.data_ptr()), ct.c_void_p(self.yy.data_ptr()))

    def zero(self):
        _check(lib().mdn_gram_zero(ct.byref(self.desc()), _stream_ptr()))


def _ws(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def train_accumulate(gram: Gram, z, target, level: Level, u_coarse=None, precision: int = GRAM_F32,
                     coarse_color=None, ws=None):
    C, H, W = z.shape
    _train_sigs(lib())
    need = ct.c_size_t()
    _check(lib().mdn_train_workspace_size(ct.byref(gram.desc()), W, H, ct.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = _ws(need.value, z.device)
    uc = None
    if u_coarse is not None:
        uc = image(u_coarse, GRAY if C == 1 else (coarse_color if coarse_color is not None else YCC))
    lv = level.desc()
    _check(lib().mdn_train_accumulate(ct.byref(gram.desc()), ct.byref(image(z)),
                                      ct.byref(uc) if uc is not None else None, ct.byref(image(target)),
                                      ct.byref(lv), precision, ct.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream_ptr()))
    return ws


def train_solve(gram: Gram, lam: float, min_count: Optional[int] = None, coeff_dtype=None):
    """Solve every system; returns (coeffs [K][C][D] device tensor, number of fallback systems)."""
    torch = _torch()
    dev = gram.G.device
    dt = coeff_dtype or torch.float32
    K, C = gram.cfg[0], gram.cfg[1]
    out = torch.empty((K, C, gram.D), dtype=dt, device=dev)
    nfb = torch.zeros(1, dtype=torch.int32, device=dev)
    need = ct.c_size_t()
    _check(lib().mdn_train_solve_workspace_size(ct.byref(gram.desc()), ct.byref(need)))
    ws = _ws(need.value, dev)
    mc = gram.D if min_count is None else int(min_count)
    _check(lib().mdn_train_solve(ct.byref(gram.desc()), float(lam), mc, ct.c_void_p(out.data_ptr()),
                                 _dtype_code(out), ct.c_void_p(nfb.data_ptr()), ct.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream_ptr()))
    return out, int(nfb.item())


def level_features(z, selector: int = 0, u_coarse=None, coarse_color=None):
    """(strength, coherence) float64 device tensors [H][W] of the RGB/grey image z (structure tensor
    of the colour image, of its luma with selector=SELECT_LUMA, or of the upsampled coarser output
    u_coarse with selector=SELECT_COARSE, YCbCr unless coarse_color says otherwise)."""
    torch = _torch()
    _train_sigs(lib())
    C, H, W = z.shape
    st = torch.empty((H, W), dtype=torch.float64, device=z.device)
    co = torch.empty((H, W), dtype=torch.float64, device=z.device)
    if selector == SELECT_COARSE:
        if u_coarse is None:
            raise MdnError(MDN_EINVAL, "the coarse selector needs u_coarse")
        uc = image(u_coarse, coarse_color if coarse_color is not None else (GRAY if C == 1 else YCC))
        _check(lib().mdn_level_features_coarse(ct.byref(uc), W, H, ct.c_void_p(st.data_ptr()),
                                               ct.c_void_p(co.data_ptr()), _stream_ptr()))
        return st, co
    _check(lib().mdn_level_features(ct.byref(image(z)), int(selector), ct.c_void_p(st.data_ptr()),
                                    ct.c_void_p(co.data_ptr()), _stream_ptr()))
    return st, co


def quantiles(values, q: int) -> np.ndarray:
    """k/q quantiles (k = 1..q-1) of a float64 device tensor, computed by the library."""
    _train_sigs(lib())
    v = values.contiguous().view(-1)
    n = v.numel()
    need = ct.c_size_t()
    _check(lib().mdn_quantiles_workspace_size(n, ct.byref(need)))
    ws = _ws(need.value, v.device)
    out = (ct.c_double * (q - 1))()
    _check(lib().mdn_quantiles(ct.c_void_p(v.data_ptr()), n, q, out, ct.c_void_p(ws.data_ptr()), ws.numel(),
                               _stream_ptr()))
    return np.array(list(out))


def level_thresholds(zs, q_s: int, q_c: int, selector: int = 0, u_coarse=None, coarse_color=None):
    """Equal-population strength / coherence thresholds over the given level images (for the
    coarse selector, over the upsampled coarser outputs u_coarse[i] of the same levels)."""
    torch = _torch()
    ucs = u_coarse if u_coarse is not None else [None] * len(zs)
    feats = [level_features(z, selector, uc, coarse_color) for z, uc in zip(zs, ucs)]
    st = torch.cat([f[0].view(-1) for f in feats])
    co = torch.cat([f[1].view(-1) for f in feats])
    t_s = quantiles(st, q_s) if q_s > 1 else np.zeros(0)
    t_c = quantiles(co, q_c) if q_c > 1 else np.zeros(0)
    return t_s, t_c


def train_single(pairs, q_theta: int, q_s: int, q_c: int, radius: int, lam: float, thresholds=None,
                 precision: int = GRAM_F32, coeff_dtype=None, min_count=None, augment: bool = False,
                 selector: int = 0, phases: int = 1):
    """Single-scale bank (Eq. (1), (7)-(8)) from (noisy, clean) (C, H, W) device tensors;
    augment: train on the eight symmetries of every pair (Section 5); selector: SELECT_RGB or
    SELECT_LUMA."""
    torch = _torch()
    if augment:
        pairs = augment_pairs(pairs)
    C = pairs[0][0].shape[0]
    if thresholds is None:
        t_s, t_c = level_thresholds([z for z, _ in pairs], q_s, q_c, selector)
    else:
        t_s, t_c = thresholds
    K = q_theta * (len(t_s) + 1) * (len(t_c) + 1) * phases
    dummy = torch.zeros((K, C, (2 * radius + 1) ** 2), dtype=torch.float32, device=pairs[0][0].device)
    sel = Level(q_theta, t_s, t_c, radius, None, dummy, C, selector, phases)
    g = Gram(K, C, radius, None, device=pairs[0][0].device)
    ws = None
    for z, u in pairs:
        ws = train_accumulate(g, z, u, sel, precision=precision, ws=ws)
    co, nfb = train_solve(g, lam, min_count, coeff_dtype)
    return Bank([Level(q_theta, t_s, t_c, radius, None, co, C, selector, phases)]), g, nfb


def train_multiscale(pairs, n_trained_levels: int, q_theta: int, q_s: int, q_c: int, radius_f: int,
                     radius_g: int, lam: float, thresholds=None, precision: int = GRAM_F32, coeff_dtype=None,
                     min_count=None, storage=None, augment: bool = False, selector: int = 0, phases: int = 1):
    """Multiscale bank trained from the second-coarsest level down (Section 4); pairs are
    (noisy, clean) (C, H, W) device tensors. Returns (Bank, grams, fallback counts).
    augment: train on the eight symmetries of every pair (Section 5), each its own pair;
    selector: SELECT_RGB (colour structure tensor), SELECT_LUMA or SELECT_COARSE (the upsampled
    coarser output of the pair's own training cascade); phases: 1 or 4 (phase-aware buckets)."""
    torch = _torch()
    if augment:
        pairs = augment_pairs(pairs)
    L = n_trained_levels
    C = pairs[0][0].shape[0]
    dev = pairs[0][0].device
    pz = [[z] + pyramid_build(z, L, storage=storage) for z, _ in pairs]
    pu = [[u] + pyramid_build(u, L, storage=storage) for _, u in pairs]
    levels: List[Optional[Level]] = [None] * L
    grams, fbs = [None] * L, [None] * L
    uhat = [p[L] for p in pz]
    coarse_color = GRAY if C == 1 else RGB
    D = (2 * radius_f + 1) ** 2 + (2 * radius_g + 1) ** 2
    ws = None
    for lev in range(L - 1, -1, -1):
        if thresholds is not None:
            t_s, t_c = thresholds[lev]
        else:
            t_s, t_c = level_thresholds([p[lev] for p in pz], q_s, q_c, selector, uhat, coarse_color)
        K = q_theta * (len(t_s) + 1) * (len(t_c) + 1) * phases
        sel = Level(q_theta, t_s, t_c, radius_g, radius_f, torch.zeros((K, C, D), dtype=torch.float32, device=dev), C,
                    selector, phases)
        g = Gram(K, C, radius_g, radius_f, device=dev)
        for i in range(len(pairs)):
            ws = train_accumulate(g, pz[i][lev], pu[i][lev], sel, u_coarse=uhat[i], precision=precision,
                                  coarse_color=coarse_color, ws=ws)
        co, nfb = train_solve(g, lam, min_count, coeff_dtype)
        lvl = Level(q_theta, t_s, t_c, radius_g, radius_f, co, C, selector, phases)
        levels[lev], grams[lev], fbs[lev] = lvl, g, nfb
        uhat = [apply_level(pz[i][lev], lvl, u_coarse=uhat[i], coarse_color=coarse_color,
                            out_dtype=pz[i][lev].dtype) for i in range(len(pairs))]
        coarse_color = GRAY if C == 1 else YCC
    return Bank(levels), grams, fbs


# ----------------------------------------------------------------------------- batched form

def _plan_sigs(L):
    vp, i32 = ct.c_void_p, ct.c_int32
    P = ct.POINTER
    sig = {
        "mdn_plan_create": [P(MdnBank), i32, i32, P(vp)],
        "mdn_plan_create_banks": [P(MdnBank), i32, i32, i32, P(vp)],
        "mdn_plan_destroy": [vp],
        "mdn_plan_autotune": [vp, P(MdnImage), P(MdnImage), P(i32), i32, P(i32), vp],
        "mdn_denoise_batch": [vp, P(MdnImage), P(MdnImage), P(i32), i32, i32, vp],
        "mdn_plan_kernel_times": [vp, P(MdnImage), P(MdnImage), P(i32), i32, i32, P(ct.c_float), vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ct.c_int


class Plan:
    """Batched denoiser: one persistent launch per kernel, level and bank over a list of images.
    ``bank`` is one Bank or a list of them; the batch calls then take ``banks``, one index per
    image (None: bank 0 throughout)."""

    def __init__(self, bank, storage: int = F16, max_images: int = 256):
        _plan_sigs(lib())
        banks = list(bank) if isinstance(bank, (list, tuple)) else [bank]
        self.banks = banks                     # keeps the coefficient tensors alive
        self.levels = max(len(b.levels) for b in banks)
        h = ct.c_void_p()
        if len(banks) == 1:
            _check(lib().mdn_plan_create(ct.byref(banks[0].desc()), storage, max_images, ct.byref(h)))
        else:
            self._descs_b = [b.desc() for b in banks]
            arr = (MdnBank * len(banks))(*self._descs_b)
            _check(lib().mdn_plan_create_banks(arr, len(banks), storage, max_images, ct.byref(h)))
        self.handle = h

    def _descs(self, ins, outs, banks):
        n = len(ins)
        a = (MdnImage * n)(*[image(t, RGB) for t in ins])
        b = (MdnImage * n)(*[image(t, RGB) for t in outs])
        k = None if banks is None else (ct.c_int32 * n)(*[int(x) for x in banks])
        return n, a, b, k

    def autotune(self, ins, outs=None, banks=None):
        outs = outs if outs is not None else [_torch().empty_like(t) for t in ins]
        n, a, b, k = self._descs(ins, outs, banks)
        rows = (ct.c_int32 * (3 * self.levels))()
        _check(lib().mdn_plan_autotune(self.handle, a, b, k, n, rows, _stream_ptr()))
        return [tuple(rows[3 * l:3 * l + 3]) for l in range(self.levels)]

    def kernel_times(self, ins, outs=None, reps: int = 3, banks=None):
        """Mean device microseconds per launch of the batch's kernels: a list over levels of
        (pyramid, selection, filtering), from HIP events on the plan's stream (synchronises). Where a
        level's selection runs in its pyramid step's launch, that launch is the pyramid entry and
        the selection entry is 0."""
        outs = outs if outs is not None else [_torch().empty_like(t) for t in ins]
        n, a, b, k = self._descs(ins, outs, banks)
        us = (ct.c_float * (3 * self.levels))()
        _check(lib().mdn_plan_kernel_times(self.handle, a, b, k, n, int(reps), us, _stream_ptr()))
        return [tuple(float(x) for x in us[3 * l:3 * l + 3]) for l in range(self.levels)]

    def denoise_batch(self, ins, outs=None, use_graph: bool = True, banks=None):
        outs = outs if outs is not None else [_torch().empty_like(t) for t in ins]
        n, a, b, k = self._descs(ins, outs, banks)
        self._keep = (a, b, k)
        _check(lib().mdn_denoise_batch(self.handle, a, b, k, n, 1 if use_graph else 0, _stream_ptr()))
        return outs

    def close(self):
        if getattr(self, "handle", None):
            lib().mdn_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- serving loop

EXEC_HIP, EXEC_FAKE = 0, 1
FAKE_FAIL_UPLOAD, FAKE_FAIL_LAUNCH, FAKE_FAIL_TICK, FAKE_FAIL_DOWNLOAD, FAKE_STALL = range(5)


class MdnServerConfig(ct.Structure):
    _fields_ = [("banks", ct.POINTER(MdnBank)), ("n_banks", ct.c_int32), ("storage", ct.c_int32),
                ("max_slots", ct.c_int32), ("stages_per_tick", ct.c_int32),
                ("max_ticks_in_flight", ct.c_int32), ("executor", ct.c_int32), ("reserved", ct.c_int32 * 2),
                ("hbm_budget", ct.c_uint64), ("staging_bytes", ct.c_uint64), ("queue_timeout", ct.c_double),
                ("fake_h2d_gbps", ct.c_double), ("fake_d2h_gbps", ct.c_double),
                ("fake_gpx_per_s", ct.c_double), ("fake_launch_us", ct.c_double)]


class MdnRequest(ct.Structure):
    _fields_ = [("host_in", ct.c_void_p), ("host_out", ct.c_void_p), ("width", ct.c_int32),
                ("height", ct.c_int32), ("dtype", ct.c_int32), ("bank", ct.c_int32), ("tag", ct.c_uint64)]


class MdnCompletion(ct.Structure):
    _fields_ = [("id", ct.c_uint64), ("tag", ct.c_uint64), ("status", ct.c_int32), ("slot", ct.c_int32),
                ("tick_first", ct.c_int32), ("tick_last", ct.c_int32), ("t_arrival", ct.c_double),
                ("t_admit", ct.c_double), ("t_device_done", ct.c_double), ("t_host_done", ct.c_double),
                ("host_out", ct.c_void_p)]


class MdnServerCounters(ct.Structure):
    _fields_ = [(n, ct.c_uint64) for n in ("submitted", "admitted", "completed", "failed", "rejected", "ticks",
                                          "launches", "tick_items", "arena_bytes", "arena_used", "arena_peak")] + \
               [("queued", ct.c_int32), ("active", ct.c_int32)]


def _server_sigs(L):
    vp, i32, u64, dbl = ct.c_void_p, ct.c_int32, ct.c_uint64, ct.c_double
    P = ct.POINTER
    sig = {
        "mdn_server_create": [P(MdnServerConfig), P(vp)],
        "mdn_server_destroy": [vp],
        "mdn_server_submit": [vp, P(MdnRequest), P(u64)],
        "mdn_server_cancel": [vp, u64],
        "mdn_server_poll": [vp, dbl, P(MdnCompletion), i32, P(i32)],
        "mdn_server_replay": [vp, P(MdnRequest), P(dbl), i32, P(MdnCompletion)],
        "mdn_server_stats": [vp, P(MdnServerCounters)],
        "mdn_server_now": [vp, P(dbl)],
        "mdn_server_footprint": [vp, P(MdnRequest), P(u64)],
        "mdn_server_fake_advance": [vp, dbl],
        "mdn_server_fake_inject": [vp, i32, u64, dbl],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ct.c_int


def _completion(c: MdnCompletion) -> dict:
    return {k: getattr(c, k) for k, _ in MdnCompletion._fields_}


class Server:
    """Serving loop over several banks (one per noise level): admission by device footprint,
    continuous batching of cascade stages, copies on their own streams. Host images are
    (3, H, W) contiguous CPU tensors (pinned for asynchronous copies)."""

    def __init__(self, banks: List[Bank], storage: int = F16, max_slots: int = 16, stages_per_tick: int = 1,
                 max_ticks_in_flight: int = 2, hbm_budget: int = 4 << 30, staging_bytes: int = 0,
                 queue_timeout: float = 0.0, executor: int = EXEC_HIP, fake_model=(25.0, 25.0, 20.0, 5.0)):
        _server_sigs(lib())
        self.banks = list(banks)               # keeps the coefficient tensors alive
        descs = [b.desc() for b in self.banks]
        self._bank_arr = (MdnBank * len(descs))(*descs)
        cfg = MdnServerConfig()
        cfg.banks = ct.cast(self._bank_arr, ct.POINTER(MdnBank))
        cfg.n_banks = len(descs)
        cfg.storage = storage
        cfg.max_slots = max_slots
        cfg.stages_per_tick = stages_per_tick
        cfg.max_ticks_in_flight = max_ticks_in_flight
        cfg.executor = executor
        cfg.hbm_budget = hbm_budget
        cfg.staging_bytes = staging_bytes
        cfg.queue_timeout = queue_timeout
        cfg.fake_h2d_gbps, cfg.fake_d2h_gbps, cfg.fake_gpx_per_s, cfg.fake_launch_us = fake_model
        h = ct.c_void_p()
        _check(lib().mdn_server_create(ct.byref(cfg), ct.byref(h)))
        self.handle = h
        self._held = {}

    @staticmethod
    def request(host_in, bank: int, host_out=None, tag: int = 0) -> MdnRequest:
        if host_in.dim() != 3 or host_in.shape[0] != 3 or not host_in.is_contiguous():
            raise ValueError("host images are contiguous (3, H, W)")
        if host_out is not None and (host_out.shape != host_in.shape or host_out.dtype != host_in.dtype
                                     or not host_out.is_contiguous()):
            raise ValueError("host_out must match host_in")
        _, H, W = host_in.shape
        return MdnRequest(host_in.data_ptr(), host_out.data_ptr() if host_out is not None else None,
                          W, H, _dtype_code(host_in), bank, tag)

    def submit(self, host_in, bank: int, host_out=None, tag: int = 0) -> int:
        rid = ct.c_uint64()
        _check(lib().mdn_server_submit(self.handle, ct.byref(self.request(host_in, bank, host_out, tag)),
                                       ct.byref(rid)))
        self._held[rid.value] = (host_in, host_out)
        return rid.value

    def submit_request(self, req: MdnRequest) -> int:
        """Submit a prepared descriptor (the caller keeps its host buffers alive)."""
        rid = ct.c_uint64()
        _check(lib().mdn_server_submit(self.handle, ct.byref(req), ct.byref(rid)))
        return rid.value

    def footprint(self, req: MdnRequest) -> int:
        b = ct.c_uint64()
        _check(lib().mdn_server_footprint(self.handle, ct.byref(req), ct.byref(b)))
        return b.value

    def cancel(self, rid: int):
        _check(lib().mdn_server_cancel(self.handle, rid))

    def poll(self, max_wait: float = 0.0, max_out: int = 256) -> List[dict]:
        out = (MdnCompletion * max_out)()
        n = ct.c_int32()
        _check(lib().mdn_server_poll(self.handle, max_wait, out, max_out, ct.byref(n)))
        res = [_completion(out[i]) for i in range(n.value)]
        for c in res:
            self._held.pop(c["id"], None)
        return res

    def wait_all(self, max_wait: float = 1e9) -> List[dict]:
        done = []
        while True:
            got = self.poll(max_wait)
            done += got
            st = self.stats()
            if not got and st["queued"] == 0 and st["active"] == 0:
                return done

    def replay(self, requests: Sequence[MdnRequest], arrivals: Sequence[float]) -> List[dict]:
        n = len(requests)
        reqs = (MdnRequest * n)(*requests)
        arr = (ct.c_double * n)(*[float(a) for a in arrivals])
        out = (MdnCompletion * n)()
        _check(lib().mdn_server_replay(self.handle, reqs, arr, n, out))
        return [_completion(out[i]) for i in range(n)]

    def stats(self) -> dict:
        c = MdnServerCounters()
        _check(lib().mdn_server_stats(self.handle, ct.byref(c)))
        return {k: getattr(c, k) for k, _ in MdnServerCounters._fields_}

    def now(self) -> float:
        t = ct.c_double()
        _check(lib().mdn_server_now(self.handle, ct.byref(t)))
        return t.value

    def fake_advance(self, t: float):
        _check(lib().mdn_server_fake_advance(self.handle, t))

    def fake_inject(self, what: int, tag: int, value: float = 0.0):
        _check(lib().mdn_server_fake_inject(self.handle, what, tag, value))

    def close(self):
        if getattr(self, "handle", None):
            lib().mdn_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
