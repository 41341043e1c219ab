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
LIB_PATH = os.path.join(_PKG, "libmdn.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "mdn.h")

MDN_OK, MDN_EINVAL, MDN_ENOMEM, MDN_EDEVICE, MDN_ENOTSUP = range(5)
F32, F16 = 0, 1
GRAY, RGB, YCC = 0, 1, 2
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOTSUP"}


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
                ("coeff_dtype", ct.c_int32), ("reserved", ct.c_int32),
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
            "mdn_select_filters": [P(MdnImage), P(MdnLevel), vp, i64, vp],
            "mdn_apply_level": [P(MdnImage), P(MdnImage), vp, i64, P(MdnLevel), P(MdnImage), vp],
            "mdn_denoise_workspace_size": [i32, i32, i32, i32, i32, P(ct.c_size_t)],
            "mdn_denoise": [P(MdnImage), P(MdnBank), i32, vp, ct.c_size_t, P(MdnImage), vp],
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
                 radius_f: Optional[int], coeffs, channels: int):
        self.q_theta = int(q_theta)
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
        return self.q_theta * (len(self.t_s) + 1) * (len(self.t_c) + 1)

    def desc(self) -> MdnLevel:
        return MdnLevel(self.q_theta, len(self.t_s) + 1, len(self.t_c) + 1, self.radius_f, self.radius_g,
                        self.channels, _dtype_code(self.coeffs), 0,
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


def select_filters(z, level: Level, out=None):
    """uint8 (H, W) bucket map of the RGB/grey image z."""
    torch = _torch()
    C, H, W = z.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=z.device)
    lv = level.desc()
    _check(lib().mdn_select_filters(ct.byref(image(z)), ct.byref(lv), ct.c_void_p(out.data_ptr()),
                                    out.stride(0) if H > 0 else W, _stream_ptr()))
    return out


def apply_level(z, level: Level, u_coarse=None, s=None, out=None, out_color=None, coarse_color=None,
                out_dtype=None):
    """One filtering step; returns u_out (C, H, W) in YCbCr unless out_color says otherwise."""
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
    _check(lib().mdn_apply_level(ct.byref(image(z)), ct.byref(uc) if uc is not None else None,
                                 ct.c_void_p(s.data_ptr()) if s is not None else None,
                                 s.stride(0) if s is not None else 0, ct.byref(lv),
                                 ct.byref(image(out, out_color)), _stream_ptr()))
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
