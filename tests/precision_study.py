"""Training precision study: Gram accumulation in FP32 MFMA and in BF16 hi/lo MFMA (three
products) against the FP64 oracle, at the paper's per-channel layout (D = 98 per channel, 3-level
pyramid, two trained levels) and at the literal cross-channel D = 147 layout (single scale).

Inputs: 8 seeded 512x512 RGB pairs, sigma drawn per pair from {15, 25, 50}/255 with rng(3);
thresholds are the oracle's equal-population quantiles, given to both sides so that only the
arithmetic differs. Reports, per level and precision: the worst Gram entry error relative to
sqrt(G_pp G_qq), the coefficient error, the output-space error sqrt(sum dh^T G dh / sum y^2)
and, end to end, the PSNR of a held-out 512x512 image denoised with each bank.

Run with an MI355X visible:  python tests/precision_study.py  (prints one JSON object)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
import synth  # noqa: E402

N_PAIRS, SIZE, LEVELS = 8, 512, 2
Q_THETA, Q_S, Q_C, R = 24, 3, 3, 3
LAM = 1e-3


def _pairs():
    rng = np.random.default_rng(3)
    sig = rng.choice([15.0, 25.0, 50.0], N_PAIRS)
    return [synth.noisy_pair(1 + i, SIZE, SIZE, 3, float(s)) for i, s in enumerate(sig)], sig


def _gram_err(G, Gref):
    d = np.sqrt(np.maximum(np.einsum("...ii->...i", Gref), 0.0))
    return float(np.max(np.abs(G - Gref) / (d[..., :, None] * d[..., None, :] + 1e-300)))


def _out_err(h, href, G, yy):
    dh = h - href
    e = np.einsum("kcd,kcde,kce->", dh, G, dh) if G.ndim == 4 else np.einsum("kcd,kde,kce->", dh, G, dh)
    return float(np.sqrt(max(e, 0.0) / yy.sum()))


def _say(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def main():
    import torch
    import paper_1802_06130_amd as M
    t0 = time.time()
    pairs, sig = _pairs()
    pz = [O.build_pyramid(z.astype(np.float64), LEVELS + 1, storage=np.float32) for z, _ in pairs]
    thr = []
    for lev in range(LEVELS):
        feats = [O.level_features(p[lev]) for p in pz]
        thr.append((O.thresholds_from_features(np.concatenate([f[0] for f in feats]), Q_S),
                    O.thresholds_from_features(np.concatenate([f[1] for f in feats]), Q_C)))
    ob, ostats, ofb = O.train_multiscale([(z.astype(np.float64), u.astype(np.float64)) for z, u in pairs],
                                         LEVELS, Q_THETA, Q_S, Q_C, R, R, LAM, thresholds=thr, storage=np.float32)
    t_oracle = time.time() - t0
    _say(f"oracle multiscale training done in {t_oracle:.0f}s")
    zt, ut = synth.noisy_pair(3001, SIZE, SIZE, 3, 25.0)
    ref_out = O.denoise(zt.astype(np.float64), ob, storage=np.float32)
    report = {"pairs": N_PAIRS, "size": SIZE, "sigmas": sig.tolist(), "levels_trained": LEVELS, "lambda": LAM,
              "oracle_seconds": round(t_oracle, 1),
              "psnr_noisy_db": round(O.psnr(zt.astype(np.float64), ut), 3),
              "psnr_oracle_bank_db": round(O.psnr(ref_out, ut), 4), "per_channel_D98": {}, "cross_D147": {}}
    dev = torch.device("cuda:0")
    tp = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
    for name, prec in (("fp32_mfma", M.GRAM_F32), ("bf16x3_mfma", M.GRAM_BF16X3)):
        bank, grams, fbs = M.train_multiscale(tp, LEVELS, Q_THETA, Q_S, Q_C, R, R, LAM, thresholds=thr,
                                              precision=prec)
        torch.cuda.synchronize()
        lv = {}
        for lev in range(LEVELS):
            K, C, D = Q_THETA * Q_S * Q_C, 3, 98
            G = grams[lev].G.cpu().numpy().reshape(K, C, D, D)
            h = bank.levels[lev].coeffs.double().cpu().numpy()
            href = ob.levels[lev].coeffs
            lv[f"level{lev}"] = {
                "gram_worst_rel": _gram_err(G, ostats[lev].G),
                "coeff_max_abs": float(np.max(np.abs(h - href))),
                "output_space_rel": _out_err(h, href, ostats[lev].G, ostats[lev].yy),
                "fallback_systems": int(fbs[lev])}
        out = M.denoise(torch.from_numpy(zt).to(dev), bank, storage=M.F32).cpu().numpy().astype(np.float64)
        lv["psnr_db"] = round(O.psnr(out, ut), 4)
        lv["dpsnr_vs_oracle_bank_db"] = round(lv["psnr_db"] - report["psnr_oracle_bank_db"], 4)
        report["per_channel_D98"][name] = lv
        _say(f"per-channel {name}: {lv}")
    # cross-channel, single scale at level 0
    K, C, D = Q_THETA * Q_S * Q_C, 3, 147
    cst = O.CrossGramStats.zeros(K, C, D)
    t_s, t_c = thr[0]
    for z, u in pairs:
        z64, u64 = z.astype(np.float64), u.astype(np.float64)
        O.accumulate_level_cross(cst, O.select(z64, Q_THETA, t_s, t_c), O.to_filter_space(z64),
                                 O.to_filter_space(u64), R)
    href, cfb = O.solve_level_cross(cst, LAM)
    _say("oracle cross-channel statistics done")
    sel = M.Level(Q_THETA, t_s, t_c, R, None, torch.zeros((K, 3, 49), device=dev), 3)
    for name, prec in (("fp32_mfma", M.GRAM_F32), ("bf16x3_mfma", M.GRAM_BF16X3)):
        g = M.Gram(K, 3, R, None, layout=M.X_CROSS_CHANNEL, device=dev)
        for z, u in tp:
            M.train_accumulate(g, z, u, sel, precision=prec)
        co, nfb = M.train_solve(g, LAM)
        h = co.double().cpu().numpy()
        report["cross_D147"][name] = {
            "gram_worst_rel": _gram_err(g.G.cpu().numpy().reshape(K, D, D), cst.G),
            "coeff_max_abs": float(np.max(np.abs(h - href))),
            "output_space_rel": _out_err(h, href, cst.G, cst.yy),
            "fallback_systems": int(nfb), "oracle_fallback_systems": int(cfb.sum())}
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
