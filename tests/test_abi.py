"""CPU-side checks of the C ABI: the library loads, exports every declared entry point, and
rejects bad arguments before touching the device."""

import ctypes as ct
import os
import subprocess

import numpy as np
import pytest

import paper_1802_06130_amd as M
from paper_1802_06130_amd import _lib as B


def test_library_exports_every_declared_symbol():
    L = M.lib()
    names = M.header_functions()
    assert "mdn_denoise" in names and "mdn_apply_level" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/mdn.h but not exported"


def test_exported_symbols_via_nm():
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for n in M.header_functions():
        assert n in exported


def test_version_string():
    assert b"gfx950" in M.lib().mdn_version()


def test_workspace_size_host_only():
    n = M.denoise_workspace_size(1024, 768, 3, 2, M.F32)
    # z^1, u^1 (512 x 384) and z^2 (256 x 192), pitches rounded up to 64 elements, + the uint8
    # selector maps of levels 0 and 1
    want = 3 * 4 * (512 * 384 * 2 + 256 * 192) + 1024 * 768 + 512 * 384
    assert n == want
    assert M.denoise_workspace_size(0, 0, 3, 3, M.F16) == 0
    with pytest.raises(M.MdnError):
        M.denoise_workspace_size(10, 10, 2, 2, M.F32)
    with pytest.raises(M.MdnError):
        M.denoise_workspace_size(10, 10, 3, 0, M.F32)


def _img(data=None, w=8, h=8, c=3, dtype=M.F32, color=M.RGB, reserved=0):
    return B.MdnImage(data, w, h, c, dtype, color, reserved, w, w * h)


def _level(**kw):
    ts = (ct.c_double * 2)(0.1, 0.2)
    tc = (ct.c_double * 2)(0.3, 0.6)
    d = dict(q_theta=24, q_s=3, q_c=3, radius_f=3, radius_g=3, channels=3, coeff_dtype=M.F32, selector=0, phases=1,
             t_s=ct.cast(ts, ct.POINTER(ct.c_double)), t_c=ct.cast(tc, ct.POINTER(ct.c_double)), coeffs=0x1000)
    d.update(kw)
    lv = B.MdnLevel(**d)
    lv._keep = (ts, tc)
    return lv


@pytest.mark.parametrize("img,lvl,msg", [
    (_img(data=None), _level(), "null data"),
    (_img(data=0x1000, c=2), _level(), "channels"),
    (_img(data=0x1000, color=M.GRAY), _level(), "colour"),
    (_img(data=0x1000, dtype=7), _level(), "dtype"),
    (_img(data=0x1000, reserved=1), _level(), "reserved"),
    (_img(data=0x1000), _level(q_theta=23), "q_theta"),
    (_img(data=0x1000), _level(q_theta=64, q_s=17, q_c=3), "q_s"),
    (_img(data=0x1000), _level(radius_g=4), "radius_g"),
    (_img(data=0x1000), _level(channels=1), "channels"),
    (_img(data=0x1000), _level(coeffs=None), "coeffs"),
    (_img(data=0x1000), _level(selector=3), "selector"),
    (_img(data=0x1000), _level(selector=2), "mdn_select_filters_coarse"),
    (_img(data=0x1000), _level(selector=2, radius_f=-1), "single-scale"),
    (_img(data=0x1000), _level(phases=2), "phases"),
    (B.MdnImage(0x1000, 8, 8, 3, M.F32, M.RGB, 0, 8, 1 << 28), _level(), "2 GiB"),
])
def test_select_rejects_bad_arguments(img, lvl, msg):
    st = M.lib().mdn_select_filters(ct.byref(img), ct.byref(lvl), ct.c_void_p(0x2000), 8, None)
    assert st in (B.MDN_EINVAL, B.MDN_ENOTSUP)
    assert msg in M.lib().mdn_last_error().decode()


def test_thresholds_must_ascend():
    ts = (ct.c_double * 2)(0.2, 0.1)
    lv = _level(t_s=ct.cast(ts, ct.POINTER(ct.c_double)))
    st = M.lib().mdn_select_filters(ct.byref(_img(data=0x1000)), ct.byref(lv), ct.c_void_p(0x2000), 8, None)
    assert st == B.MDN_EINVAL and b"ascending" in M.lib().mdn_last_error()


def test_pyramid_rejects_wrong_level_size():
    lv0 = _img(data=0x1000, w=9, h=7)
    outs = (B.MdnImage * 2)(_img(data=0x2000, w=5, h=4), _img(data=0x3000, w=2, h=2))
    st = M.lib().mdn_pyramid_build(ct.byref(lv0), 2, outs, None)
    assert st == B.MDN_EINVAL and b"out[1]" in M.lib().mdn_last_error()


def test_apply_requires_coarse_for_multiscale():
    z = _img(data=0x1000)
    out = _img(data=0x2000, color=M.YCC)
    st = M.lib().mdn_apply_level(ct.byref(z), None, None, 0, ct.byref(_level()), ct.byref(out), None, None)
    assert st == B.MDN_EINVAL and b"u_coarse" in M.lib().mdn_last_error()


def test_denoise_workspace_too_small():
    z = _img(data=0x1000, w=64, h=64)
    out = _img(data=0x2000, w=64, h=64)
    lv = (B.MdnLevel * 2)(_level(), _level())
    bank = B.MdnBank(2, 0, ct.cast(lv, ct.POINTER(B.MdnLevel)))
    st = M.lib().mdn_denoise(ct.byref(z), ct.byref(bank), M.F32, ct.c_void_p(0x4000), 16, ct.byref(out), None)
    assert st == B.MDN_ENOMEM


def test_noalloc_refuses_an_image_above_its_scratch_before_touching_the_device():
    """The entry point that allocates nothing checks the cascade's workspace against its static scratch
    (MDN_NOALLOC_SCRATCH_BYTES) first: a 16384 x 8192 float32 image needs more and is refused."""
    w, h = 16384, 8192
    z = B.MdnImage(0x1000, w, h, 3, M.F32, M.RGB, 0, w, w * h)
    out = B.MdnImage(0x2000, w, h, 3, M.F32, M.RGB, 0, w, w * h)
    lv = (B.MdnLevel * 3)(_level(), _level(), _level())
    bank = B.MdnBank(3, 0, ct.cast(lv, ct.POINTER(B.MdnLevel)))
    assert M.denoise_workspace_size(w, h, 3, 3, M.F32) > M.NOALLOC_SCRATCH_BYTES
    st = M.lib().mdn_denoise_noalloc(ct.byref(z), ct.byref(bank), M.F32, ct.byref(out), None)
    assert st == B.MDN_ENOMEM and b"static scratch" in M.lib().mdn_last_error()
    assert M.denoise_workspace_size(4032, 3024, 3, 4, M.F32) <= M.NOALLOC_SCRATCH_BYTES


def test_noalloc_scratch_size_matches_the_header():
    import re
    with open(B.HEADER_PATH) as fh:
        m = re.search(r"#define MDN_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", fh.read())
    assert m and int(m.group(1)) << int(m.group(2)) == M.NOALLOC_SCRATCH_BYTES


def test_library_missing_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        B.lib()


@pytest.mark.parametrize("t,out_wh,alias,msg", [
    (8, (8, 6), False, "transform"),
    (-1, (8, 6), False, "transform"),
    (4, (8, 6), False, "must be 6 x 8"),
    (1, (6, 8), False, "must be 8 x 6"),
    (0, (8, 6), True, "alias"),
])
def test_dihedral_rejects_bad_arguments(t, out_wh, alias, msg):
    src = B.MdnImage(0x1000, 8, 6, 3, M.F32, M.RGB, 0, 8, 48)
    w, h = out_wh
    dst = B.MdnImage(0x1000 if alias else 0x9000, w, h, 3, M.F32, M.RGB, 0, w, w * h)
    st = M.lib().mdn_dihedral(ct.byref(src), t, ct.byref(dst), None)
    assert st == B.MDN_EINVAL
    assert msg in M.lib().mdn_last_error().decode()


def test_coarse_selector_argument_checks():
    """The coarse selector's own calls: the level must select on the coarser output, which must be
    ceil(width/2) x ceil(height/2); the noisy-input calls send such levels to them."""
    lib = M.lib()
    B._train_sigs(lib)
    uc = _img(data=0x3000, w=4, h=4, color=M.YCC)
    smap = ct.c_void_p(0x2000)
    st = lib.mdn_select_filters_coarse(ct.byref(uc), 8, 8, ct.byref(_level()), smap, 8, None)
    assert st == B.MDN_EINVAL and b"does not select on the coarser output" in lib.mdn_last_error()
    st = lib.mdn_select_filters_coarse(ct.byref(uc), 10, 8, ct.byref(_level(selector=2)), smap, 10, None)
    assert st == B.MDN_EINVAL and b"ceil(width/2)" in lib.mdn_last_error()
    st = lib.mdn_select_filters_coarse(ct.byref(uc), 7, 8, ct.byref(_level(selector=2)), smap, 6, None)
    assert st == B.MDN_EINVAL and b"s_pitch" in lib.mdn_last_error()
    st = lib.mdn_select_filters_coarse(ct.byref(uc), 0, 0, ct.byref(_level(selector=2)), smap, 0, None)
    assert st == B.MDN_EINVAL                                  # 0 x 0 needs a 0 x 0 coarser output
    st = lib.mdn_level_features(ct.byref(_img(data=0x1000)), 2, ct.c_void_p(0x5000), ct.c_void_p(0x6000), None)
    assert st == B.MDN_EINVAL and b"mdn_level_features_coarse" in lib.mdn_last_error()
    st = lib.mdn_level_features_coarse(ct.byref(uc), 7, 7, None, None, None)
    assert st == B.MDN_EINVAL and b"null output" in lib.mdn_last_error()
    z = _img(data=0x1000)
    tgt = _img(data=0x7000)
    g = B.MdnGram(K=216, channels=3, layout=0, radius_f=-1, radius_g=3, reserved=0, G=0x8000, b=0x9000, n=0xa000,
                  yy=0xb000)
    st = lib.mdn_train_accumulate(ct.byref(g), ct.byref(z), None, ct.byref(tgt), ct.byref(_level(selector=2)), 0,
                                  ct.c_void_p(0xc000), 1 << 30, None)
    assert st == B.MDN_EINVAL and b"coarser output" in lib.mdn_last_error()
