"""Augmentation study (Section 5: training pairs extended by their axial flips and 90-degree
rotations): quality of banks trained with and without the eight symmetries, and the cost of the
symmetry kernel.

Quality: 3-level RGB banks (7x7/7x7, 24x3x3 buckets, ridge 1e-3) trained on the GPU from N seeded
256x256 pairs at sigma 25/255, with and without augmentation, for N = 4 and 16; PSNR of 8 held-out
seeded 512x512 images denoised with each bank (float32 path). The synthetic scenes stand in for the
paper's training corpus and test set, so the numbers are context, not a reproduction.

Cost: mdn_dihedral on a 4032x3024 float16 RGB frame, all eight symmetries, HIP events; bytes moved
= read + write of the frame.

Run with an MI355X visible:  python tests/augment_study.py  (prints one JSON object)
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
    tests = [synth.noisy_pair(9000 + i, 512, 512, 3, 25) for i in range(8)]
    res = {"quality": {}, "dihedral": {}}
    for n in (4, 16):
        pairs = [synth.noisy_pair(8000 + i, 256, 256, 3, 25) for i in range(n)]
        dp = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
        row = {}
        for aug in (False, True):
            bank, grams, fbs = M.train_multiscale(dp, 3, 24, 3, 3, 3, 3, 1e-3, augment=aug)
            ps = []
            for z, u in tests:
                out = M.denoise(torch.from_numpy(z).to(dev), bank).cpu().numpy().astype(np.float64)
                ps.append(O.psnr(out, u))
            row["augmented" if aug else "plain"] = {"psnr_db": round(float(np.mean(ps)), 4),
                                                    "fallback_systems": [int(f) for f in fbs]}
        row["noisy_psnr_db"] = round(float(np.mean([O.psnr(z, u) for z, u in tests])), 4)
        res["quality"][f"{n}_pairs"] = row
    z, _ = synth.noisy_pair(7, 3024, 4032, 3, 25, dtype=np.float16)
    zt = torch.from_numpy(z).to(dev)
    outs = [M.dihedral(zt, t) for t in range(8)]
    torch.cuda.synchronize()
    for t in range(8):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
        for a, b in ev:
            a.record()
            M.dihedral(zt, t, out=outs[t])
            b.record()
        torch.cuda.synchronize()
        us = float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e3
        res["dihedral"][str(t)] = {"us": round(us, 1), "GB_s": round(2 * zt.numel() * 2 / us * 1e-3, 1)}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
