"""Parity at the full frame size (4032 x 3024, 4-level RGB, 7x7/7x7 filters, 216 buckets, float16
storage and float16 filters), in the launch configuration the benchmark times (batched plan,
autotuned strip heights, graph replay) and in the plain per-image form.

The oracle cannot run a whole frame in seconds, so the check has two parts:
* locality, a property that holds at any size: the output at a pixel depends only on a window
  around it (about 80 level-0 pixels across all four levels), so on crops whose origin is a
  multiple of 16 (pyramid levels stay aligned) the full-frame output equals the crop's own output
  bit for bit away from the crop's cut edges; crops at the four corners keep the frame's own
  edges, where clamping happens, so the borders are covered;
* the crops themselves against the oracle in its float16-storage mode, run on the GPU's own maps:
  bucket indices equal except near a boundary (flips capped), every pixel within 2e-3.
"""

import numpy as np
import pytest

import synth
from mdn_testlib import TOL_F16, cascade_parity, gpu_bank, trained_bank_multiscale

pytestmark = pytest.mark.gpu

H, W = 3024, 4032
C = 384            # crop side
M_ = 128           # margin kept from a cut edge


def _crops():
    # (y0, x0): four corners, the centre and an off-centre interior crop, origins multiple of 16
    return [(0, 0), (0, W - C), (H - C, 0), (H - C, W - C),
            ((H // 2 - C // 2) // 16 * 16, (W // 2 - C // 2) // 16 * 16), (1712, 592)]


def _valid(y0, x0):
    """Region of a crop far enough from every cut edge (frame edges are not cut)."""
    top = 0 if y0 == 0 else M_
    left = 0 if x0 == 0 else M_
    bot = C if y0 + C == H else C - M_
    right = C if x0 + C == W else C - M_
    return slice(top, bot), slice(left, right)


def test_full_frame_locality_and_oracle_parity():
    import torch
    import paper_1802_06130_amd as M
    print(f"full frame {W}x{H}", flush=True)
    bank = trained_bank_multiscale(levels=3)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16)
    z, u = synth.noisy_pair(4242, H, W, 3, 25, dtype=np.float16)
    zt = torch.from_numpy(z).cuda()

    plain = M.denoise(zt, gb, storage=M.F16)
    others = [torch.from_numpy(synth.noisy_pair(4300 + i, h, w, 3, 25, dtype=np.float16)[0]).cuda()
              for i, (h, w) in enumerate([(1080, 1920), (720, 1280)])]
    plan = M.Plan(gb, M.F16, max_images=8)
    batch_in = [others[0], zt, others[1]]
    outs = [torch.empty_like(t) for t in batch_in]
    plan.autotune(batch_in, outs)
    for _ in range(2):
        plan.denoise_batch(batch_in, outs, use_graph=True)
    torch.cuda.synchronize()
    full = plain.cpu().numpy()
    assert np.array_equal(outs[1].cpu().numpy(), full), "batched full frame differs from the plain form"
    for t, o in zip(others, (outs[0], outs[2])):
        assert np.array_equal(o.cpu().numpy(), M.denoise(t, gb, storage=M.F16).cpu().numpy())
    plan.close()

    for (y0, x0) in _crops():
        print(f"  crop at ({y0}, {x0})", flush=True)
        zc = np.ascontiguousarray(z[:, y0:y0 + C, x0:x0 + C])
        crop_gpu = M.denoise(torch.from_numpy(zc).cuda(), gb, storage=M.F16)
        sy, sx = _valid(y0, x0)
        assert np.array_equal(crop_gpu.cpu().numpy()[:, sy, sx], full[:, y0:y0 + C, x0:x0 + C][:, sy, sx]), \
            f"full-frame output at crop ({y0}, {x0}) differs from the crop's own output"
        # the crop against the oracle (float16 storage mode) on the GPU's maps, every pixel
        cascade_parity(zc, bank, gb, np.float16, TOL_F16, out=crop_gpu)
