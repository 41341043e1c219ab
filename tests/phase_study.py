"""Phase-aware buckets (the other reading of the non-integer i/2 of Eq. (9): one filter pair per
bucket and parity of the pixel on the coarser grid) against phase-blind buckets: quality and
float32 throughput.

4-level RGB banks, 7x7/7x7 filters, 24x3x3 buckets (x4 phases), ridge 1e-3, trained on the GPU from
64 seeded 256x256 pairs with the eight symmetries, sigma 25/255; PSNR over 8 held-out seeded 512x512
images; throughput of mdn_denoise on one seeded 4032x3024 frame, float32 storage and filters, HIP
events, median of 5. Synthetic scenes stand in for the paper's corpus and test set.

Run with an MI355X visible:  python tests/phase_study.py  (prints one JSON object)
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
    pairs = [synth.noisy_pair(8300 + i, 256, 256, 3, 25) for i in range(64)]
    dp = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
    tests = [synth.noisy_pair(9300 + i, 512, 512, 3, 25) for i in range(8)]
    frame = torch.from_numpy(synth.noisy_pair(7, 3024, 4032, 3, 25)[0]).to(dev)
    res = {"noisy_psnr_db": round(float(np.mean([O.psnr(z, u) for z, u in tests])), 4)}
    for phases in (1, 4):
        bank, _, fbs = M.train_multiscale(dp, 3, 24, 3, 3, 3, 3, 1e-3, augment=True, phases=phases)
        ps = [O.psnr(M.denoise(torch.from_numpy(z).to(dev), bank).cpu().numpy().astype(np.float64), u)
              for z, u in tests]
        out = torch.empty_like(frame)
        M.denoise(frame, bank, out=out)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for a, b in ev:
            a.record()
            M.denoise(frame, bank, out=out)
            b.record()
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        res[f"phases_{phases}"] = {"buckets": 216 * phases, "psnr_db": round(float(np.mean(ps)), 4),
                                   "fallback_systems": [int(f) for f in fbs], "frame_ms_f32": round(ms, 3),
                                   "MP_s_f32": round(3024 * 4032 / ms * 1e-3, 1)}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
