"""Batched form (one persistent launch per kernel and level over a ragged list of images, optional
hipGraph replay): every image's output equals the plain per-image call bit for bit, alone or in
the mix, eagerly or from repeated graph replays, before and after autotuning."""

import numpy as np
import pytest

import synth
from mdn_testlib import gpu_bank, trained_bank_multiscale

pytestmark = pytest.mark.gpu

SIZES = [(1, 1), (3, 5), (57, 59), (130, 97), (481, 321), (200, 1500), (1024, 768), (64, 64)]


def _setup(dtype=np.float16):
    import torch
    bank = trained_bank_multiscale(levels=3)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16)
    zs = [torch.from_numpy(synth.noisy_pair(9000 + i, h, w, 3, 25, dtype=dtype)[0]).cuda()
          for i, (h, w) in enumerate(SIZES)]
    return gb, zs


def _plain(M, gb, zs, storage):
    return [M.denoise(z, gb, storage=storage).cpu().numpy() for z in zs]


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_per_image(use_graph):
    import torch
    import paper_1802_06130_amd as M
    gb, zs = _setup()
    want = _plain(M, gb, zs, M.F16)
    plan = M.Plan(gb, M.F16, max_images=16)
    outs = [torch.empty_like(z) for z in zs]
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        plan.denoise_batch(zs, outs, use_graph=use_graph)
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
        for i, (g, w) in enumerate(zip(got, want)):
            assert np.array_equal(g, w), f"replay {rep}, image {i} {SIZES[i]} differs"
        _ = (zs[0] * 2).sum().item()          # unrelated eager work between replays
    plan.close()


def test_batch_alone_vs_mix_and_float32_io():
    import torch
    import paper_1802_06130_amd as M
    gb, zs = _setup(np.float32)
    plan = M.Plan(gb, M.F16, max_images=16)
    mix = plan.denoise_batch(zs, use_graph=True)
    torch.cuda.synchronize()
    mix = [m.cpu().numpy() for m in mix]
    for i, z in enumerate(zs):
        alone = plan.denoise_batch([z], use_graph=False)[0].cpu().numpy()
        assert np.array_equal(alone, mix[i]), f"image {i} differs alone vs in the mix"
    plain = _plain(M, gb, zs, M.F16)
    for i in range(len(zs)):
        assert np.array_equal(plain[i], mix[i])
    plan.close()


def test_autotune_keeps_results():
    import torch
    import paper_1802_06130_amd as M
    gb, zs = _setup()
    want = _plain(M, gb, zs, M.F16)
    plan = M.Plan(gb, M.F16, max_images=16)
    rows = plan.autotune(zs)
    print("tuned rows per level (pyramid, selection, filtering):", rows)
    assert len(rows) == 3
    for d2, se, wa in rows:
        assert d2 in (8, 16, 32, 64) and se in (10, 20, 30, 60) and wa in (14, 28, 42, 56)
    got = plan.denoise_batch(zs, use_graph=True)
    torch.cuda.synchronize()
    for g, w in zip(got, want):
        assert np.array_equal(g.cpu().numpy(), w)
    plan.close()


def test_batch_rejects_bad_inputs():
    import torch
    import paper_1802_06130_amd as M
    gb, zs = _setup()
    plan = M.Plan(gb, M.F16, max_images=2)
    with pytest.raises(M.MdnError):
        plan.denoise_batch(zs[:3])                              # more than max_images
    with pytest.raises(M.MdnError):
        plan.denoise_batch([zs[2]], [torch.empty((3, 5, 5), dtype=torch.float16, device="cuda")])
    plan.close()


def test_kernel_times_runs_the_same_launches():
    """mdn_plan_kernel_times runs the batch's launches one at a time between events: positive times for
    every pyramid step and filtering launch, the selection entry 0 on every level (this single
    column-walk bank runs each level's selection in its pyramid step's launch), outputs equal to the
    batched form's bit for bit; before and after a graph replay of the same batch."""
    import torch
    import paper_1802_06130_amd as M
    gb, zs = _setup()
    plan = M.Plan(gb, M.F16, max_images=16)
    want = [o.cpu().numpy() for o in plan.denoise_batch(zs, use_graph=True)]
    outs = [torch.full_like(z, -1.0) for z in zs]
    kt = plan.kernel_times(zs, outs, reps=2)
    torch.cuda.synchronize()
    assert len(kt) == len(gb.levels) and all(lv[0] > 0.0 and lv[1] == 0.0 and lv[2] > 0.0 for lv in kt)
    for o, w in zip(outs, want):
        assert np.array_equal(o.cpu().numpy(), w)
    again = [o.cpu().numpy() for o in plan.denoise_batch(zs, use_graph=True)]
    for a, w in zip(again, want):
        assert np.array_equal(a, w)
    with pytest.raises(M.MdnError) as e:
        plan.kernel_times(zs, outs, reps=0)
    assert e.value.status == M.MDN_EINVAL
    plan.close()


def test_batch_with_many_strips_per_wave_equals_per_image():
    """A batch large enough that the level-0 filtering launch gives every wave 24 or more strips, so
    the block's waves move on to their strips together (a barrier per round): every output still
    equals the per-image call, which has a few strips per wave and no such barrier, bit for bit."""
    import torch
    import paper_1802_06130_amd as M
    H, W, n = 3024, 4032, 16
    bank = trained_bank_multiscale(levels=3)
    gb = gpu_bank(bank, 3, coeff_dtype=torch.float16)
    g = torch.Generator(device="cuda").manual_seed(1234)
    zs = [(torch.rand((3, H, W), generator=g, device="cuda") * 255).round().div(255).half() for _ in range(n)]
    # level-0 strips of the default heights: 58 columns by walk rows (28 for a 4032 x 3024 image)
    props = torch.cuda.get_device_properties(0)
    strips = n * ((W + 57) // 58) * ((H + 27) // 28)
    assert strips >= 24 * props.multi_processor_count * 8
    plan = M.Plan(gb, M.F16, max_images=n)
    outs = plan.denoise_batch(zs, use_graph=True)
    torch.cuda.synchronize()
    for i, z in enumerate(zs):
        want = M.denoise(z, gb, storage=M.F16)
        assert torch.equal(outs[i], want), f"image {i} differs"
    plan.close()


def _paper_bank(M, torch, L, rf, rg, seed):
    """4096-bucket bank of the paper's configuration (Section 5) with stand-in coefficients and the
    equal-population thresholds of seeded scenes at each level."""
    import oracle as O
    zs0 = [synth.noisy_pair(300 + i, 160, 160, 3, 25)[0].astype(np.float64) for i in range(3)]
    lvs = []
    for lev in range(L):
        f = [O.level_features(O.build_pyramid(z, lev + 1)[lev]) for z in zs0]
        t_s = O.thresholds_from_features(np.concatenate([x[0] for x in f]), 16)
        t_c = O.thresholds_from_features(np.concatenate([x[1] for x in f]), 16)
        co = synth.random_bank_coeffs(seed + lev, 4096, 3, (2 * rf + 1) ** 2, (2 * rg + 1) ** 2)
        lvs.append(M.Level(16, t_s, t_c, rg, rf, torch.from_numpy(co).to(torch.float16).cuda(), 3))
    return M.Bank(lvs)


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_with_a_bank_per_image(use_graph):
    """Every image names its bank (the per-image bank[] of the batched call): three banks of
    different depth and kernels in one plan (a 4-level column-walk bank, a 3-level 4096-bucket bank
    with 5x5 / 3x3 filters, a 5-level 4096-bucket bank with 7x7 / 5x5 filters); each output equals
    mdn_denoise with that image's bank, bit for bit, eagerly and from graph replays, after autotuning."""
    import torch
    import paper_1802_06130_amd as M
    print(f"batch with a bank per image, graph={use_graph}", flush=True)
    gb, zs = _setup()
    banks = [gb, _paper_bank(M, torch, 2, 1, 2, 90), _paper_bank(M, torch, 4, 2, 3, 95)]
    which = [i % 3 for i in range(len(zs))]
    want = [M.denoise(z, banks[b], storage=M.F16).cpu().numpy() for z, b in zip(zs, which)]
    plan = M.Plan(banks, M.F16, max_images=16)
    assert plan.levels == 4
    rows = plan.autotune(zs, banks=which)
    outs = [torch.empty_like(z) for z in zs]
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        plan.denoise_batch(zs, outs, use_graph=use_graph, banks=which)
        torch.cuda.synchronize()
        for i, (o, w) in enumerate(zip(outs, want)):
            assert np.array_equal(o.cpu().numpy(), w), f"rep {rep}: image {i} {SIZES[i]} bank {which[i]} differs"
    kt = plan.kernel_times(zs, outs, reps=1, banks=which)
    print(f"  rows {rows}; kernel us per level {kt}", flush=True)
    # the same images with the banks exchanged: a new signature, new tables and graph
    which2 = [(b + 1) % 3 for b in which]
    plan.denoise_batch(zs, outs, use_graph=use_graph, banks=which2)
    torch.cuda.synchronize()
    for i, (z, o, b) in enumerate(zip(zs, outs, which2)):
        assert np.array_equal(o.cpu().numpy(), M.denoise(z, banks[b], storage=M.F16).cpu().numpy())
    with pytest.raises(M.MdnError):
        plan.denoise_batch(zs, outs, banks=[3] * len(zs))
    plan.close()


def test_batch_float32_storage_equals_per_image():
    """Float32 pyramid storage in the batched form (each level's pyramid step and selection pass in
    one launch) with float32 images: every output equals the per-image call's bit for bit, eagerly
    and from a graph. Float16 images need float16 storage in this form."""
    import torch
    import paper_1802_06130_amd as M
    gb, zs = _setup(np.float32)
    want = _plain(M, gb, zs, M.F32)
    plan = M.Plan(gb, M.F32, max_images=16)
    for use_graph in (False, True):
        outs = plan.denoise_batch(zs, use_graph=use_graph)
        torch.cuda.synchronize()
        for i, (o, w) in enumerate(zip(outs, want)):
            assert np.array_equal(o.cpu().numpy(), w), f"image {i} {SIZES[i]} differs (graph {use_graph})"
    z16 = [z.half() for z in zs[:2]]
    with pytest.raises(M.MdnError) as e:
        plan.denoise_batch(z16)
    assert e.value.status == M.MDN_ENOTSUP
    plan.close()
