"""The paper's experimental configuration (Section 5) against the 4-level 7x7/7x7, 24x3x3-bucket
configuration the rest of this repository measures: quality and throughput on one GPU.

Paper configuration at noise sigma: 16x16x16 buckets, 7x7 denoise / 5x5 upscale filters (5x5 / 3x3
below sigma 10), as many levels as bring the coarsest level's noise below 2 (oracle.paper_setup).
Both banks are trained on the GPU from 64 seeded 256x256 pairs with the eight symmetries (Section 5),
ridge 1e-3, float32 coefficients; PSNR over 8 held-out seeded 512x512 images. Throughput: mdn_denoise
of one seeded 4032x3024 RGB frame, HIP events, median of 5, twice: float32 storage and coefficients,
and float16 storage and coefficients (the column walk for the 216-bucket bank; the tiled kernel
with coefficients read through L2 for the 4096-bucket bank). Synthetic scenes stand in for the
paper's corpus and test set.

Run with an MI355X visible:  python tests/paper_config_study.py  (prints one JSON object)

With --frame SIGMA it only times the cascade of the paper configuration at that noise level on one
seeded 4032x3024 float16 frame: seeded stand-in coefficients (float16), thresholds at the
equal-population quantiles of a 1024x1024 crop of the frame, 3 untimed and 5 timed calls. This is
the command the kernel trace and counters of that configuration are taken on.
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
import synth  # noqa: E402


def _time_denoise(M, torch, bank, frame, storage=None):
    storage = M.F32 if storage is None else storage
    out = torch.empty_like(frame)
    M.denoise(frame, bank, storage=storage, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for a, b in ev:
        a.record()
        M.denoise(frame, bank, storage=storage, out=out)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def frame_only(sigma):
    import time
    import torch
    import paper_1802_06130_amd as M
    dev = torch.device("cuda:0")
    L, rf, rg, (qt, qs, qc) = O.paper_setup(sigma)
    frame = torch.from_numpy(synth.noisy_pair(7, 3024, 4032, 3, sigma)[0]).to(dev).half()
    t_s, t_c = M.level_thresholds([frame[:, :1024, :1024].float().contiguous()], qs, qc)
    K = qt * qs * qc
    levels = []
    for lev in range(L):
        co = synth.random_bank_coeffs(40 + lev, K, 3, (2 * rf + 1) ** 2, (2 * rg + 1) ** 2)
        levels.append(M.Level(qt, t_s, t_c, rg, rf, torch.from_numpy(co).to(dev).half(), 3))
    bank = M.Bank(levels)
    out = torch.empty_like(frame)
    ws = torch.empty(M.denoise_workspace_size(4032, 3024, 3, L, M.F16), dtype=torch.uint8, device=dev)
    for _ in range(3):
        M.denoise(frame, bank, storage=M.F16, ws=ws, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        M.denoise(frame, bank, storage=M.F16, ws=ws, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 5 * 1e3
    print(json.dumps({"sigma": sigma, "levels": L + 1, "buckets": K, "radius_f": rf, "radius_g": rg,
                      "frame_ms_f16": round(ms, 3), "MP_s_f16": round(3024 * 4032 / ms * 1e-3, 1)}))


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--frame":
        frame_only(float(sys.argv[2]))
        return
    import torch
    import paper_1802_06130_amd as M
    dev = torch.device("cuda:0")
    frame = torch.from_numpy(synth.noisy_pair(7, 3024, 4032, 3, 25)[0]).to(dev)
    res = {}
    for sigma in (5.0, 25.0, 50.0):
        pairs = [synth.noisy_pair(8200 + i, 256, 256, 3, sigma) for i in range(64)]
        dp = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
        tests = [synth.noisy_pair(9200 + i, 512, 512, 3, sigma) for i in range(8)]
        row = {"noisy_psnr_db": round(float(np.mean([O.psnr(z, u) for z, u in tests])), 4)}
        L, rf, rg, (qt, qs, qc) = O.paper_setup(sigma)
        for name, cfg in (("paper", (L, qt, qs, qc, rf, rg)), ("repo_4level_216", (3, 24, 3, 3, 3, 3))):
            l_, qt_, qs_, qc_, rf_, rg_ = cfg
            bank, _, fbs = M.train_multiscale(dp, l_, qt_, qs_, qc_, rf_, rg_, 1e-3, augment=True)
            ps = [O.psnr(M.denoise(torch.from_numpy(z).to(dev), bank).cpu().numpy().astype(np.float64), u)
                  for z, u in tests]
            ms = _time_denoise(M, torch, bank, frame)
            b16 = M.Bank([M.Level(lv.q_theta, lv.t_s, lv.t_c, lv.radius_g, lv.radius_f, lv.coeffs.half(), 3)
                          for lv in bank.levels])
            ms16 = _time_denoise(M, torch, b16, frame.half(), M.F16)
            row[name] = {"levels": l_ + 1, "buckets": qt_ * qs_ * qc_, "radius_f": rf_, "radius_g": rg_,
                         "psnr_db": round(float(np.mean(ps)), 4), "fallback_systems": [int(f) for f in fbs],
                         "frame_ms_f32": round(ms, 3), "MP_s_f32": round(3024 * 4032 / ms * 1e-3, 1),
                         "frame_ms_f16": round(ms16, 3), "MP_s_f16": round(3024 * 4032 / ms16 * 1e-3, 1)}
            del bank, b16
            torch.cuda.empty_cache()
        res[f"sigma_{int(sigma)}"] = row
    print(json.dumps(res))


if __name__ == "__main__":
    main()
