"""Selector study (Section 3 and Fig. 2: the structure tensor taken jointly over the colour channels,
Eq. (6), against the luma-only analysis of earlier methods; and, for the image the tensor is taken
on, the noisy level z^l against the upsampled coarser output u^{l+1}, the alternative Eq. (9)
leaves open): quality of banks that differ only in the selector, and the cost of each selection pass.

Quality: 3-level RGB banks (7x7/7x7, 24x3x3 buckets, ridge 1e-3, equal-population thresholds of
their own features) trained on the GPU from 16 seeded 256x256 pairs at sigma 15, 25 and 50/255;
PSNR of 8 held-out seeded 512x512 images denoised with each bank (float32 path). The synthetic
scenes stand in for the paper's corpus and test set, so the numbers are context.

Cost: the selection pass (mdn_select_filters, or mdn_select_filters_coarse from the 2016x1512
float16 YCbCr coarser output) on a 4032x3024 float16 RGB frame with each selector, and the whole
float16 cascade (mdn_denoise, float16 coefficients) with the sigma-25 banks; HIP events, median of 20.

Run with an MI355X visible:  python tests/selector_study.py  (prints one JSON object)
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
import synth  # noqa: E402


def main():
    import torch
    import paper_1802_06130_amd as M
    dev = torch.device("cuda:0")
    res = {"quality": {}, "select_us": {}, "denoise_ms": {}}
    sels = (("rgb", M.SELECT_RGB), ("luma", M.SELECT_LUMA), ("coarse", M.SELECT_COARSE))
    banks25 = {}
    for sigma in (15.0, 25.0, 50.0):
        pairs = [synth.noisy_pair(8100 + i, 256, 256, 3, sigma) for i in range(16)]
        dp = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
        tests = [synth.noisy_pair(9100 + i, 512, 512, 3, sigma) for i in range(8)]
        row = {"noisy_psnr_db": round(float(np.mean([O.psnr(z, u) for z, u in tests])), 4)}
        for name, sel in sels:
            bank, _, _ = M.train_multiscale(dp, 3, 24, 3, 3, 3, 3, 1e-3, selector=sel)
            if sigma == 25.0:
                banks25[name] = bank
            ps = [O.psnr(M.denoise(torch.from_numpy(z).to(dev), bank).cpu().numpy().astype(np.float64), u)
                  for z, u in tests]
            row[name] = round(float(np.mean(ps)), 4)
        res["quality"][f"sigma_{int(sigma)}"] = row
    z, _ = synth.noisy_pair(7, 3024, 4032, 3, 25, dtype=np.float16)
    zt = torch.from_numpy(z).to(dev)
    uc = M.pyramid_build(zt, 1)[0]                      # stands in for the coarser output (as RGB)
    s = torch.empty((3024, 4032), dtype=torch.uint8, device=dev)

    def timed(fn, n=20):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    for name, sel in sels:
        lv = M.Level(24, [0.02, 0.05], [0.25, 0.5], 3, 3, torch.zeros((216, 3, 98), device=dev), 3, sel)
        res["select_us"][name] = round(timed(lambda: M.select_filters(zt, lv, out=s, u_coarse=uc, coarse_color=M.RGB))
                                       * 1e3, 1)
        b16 = M.Bank([M.Level(l.q_theta, l.t_s, l.t_c, l.radius_g, l.radius_f, l.coeffs.half(), 3, l.selector)
                      for l in banks25[name].levels])
        ws = torch.empty(M.denoise_workspace_size(4032, 3024, 3, 3, M.F16), dtype=torch.uint8, device=dev)
        out = torch.empty_like(zt)
        res["denoise_ms"][name] = round(timed(lambda: M.denoise(zt, b16, storage=M.F16, ws=ws, out=out)), 3)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
