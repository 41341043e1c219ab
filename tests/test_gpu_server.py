"""Serving loop on the device: each request's result equals the plain per-image denoiser's bit for
bit, whether it ran alone or mixed with overlapping requests of other sizes and banks, for any
tick granularity, with caller buffers or slot staging buffers."""

import ctypes as ct

import numpy as np
import pytest

import synth
from mdn_testlib import gpu_bank, trained_bank_multiscale

pytestmark = pytest.mark.gpu

SIZES = [(1, 1), (3, 5), (57, 59), (130, 97), (481, 321), (200, 1500), (1024, 768), (64, 64)]


def _banks(M, torch, levels=3):
    """Three banks: the oracle-trained one and two with stand-in coefficients (same thresholds)."""
    trained = gpu_bank(trained_bank_multiscale(levels=levels), 3, coeff_dtype=torch.float16)
    banks = [trained]
    for seed in (71, 72):
        lv = []
        for l, t in enumerate(trained.levels):
            c = synth.random_bank_coeffs(seed * 10 + l, t.K, 3, 49, 49)
            lv.append(M.Level(t.q_theta, t.t_s, t.t_c, t.radius_g, t.radius_f,
                              torch.from_numpy(c).to(torch.float16).cuda(), 3))
        banks.append(M.Bank(lv))
    return banks


def _inputs(torch, dtype):
    return [torch.from_numpy(synth.noisy_pair(9100 + i, h, w, 3, 25, dtype=dtype)[0]).pin_memory()
            for i, (h, w) in enumerate(SIZES)]


def _plain(M, banks, zs, which, storage):
    return [M.denoise(z.cuda(), banks[b], storage=storage).cpu().numpy() for z, b in zip(zs, which)]


def _alone(M, srv, zs, which):
    outs = []
    for i, (z, b) in enumerate(zip(zs, which)):
        o = z.new_empty(z.shape).pin_memory()
        o.fill_(-7.0)
        srv.submit(z, b, o, tag=i)
        (c,) = srv.wait_all()
        assert c["status"] == M.MDN_OK, c
        outs.append(o.numpy().copy())
    return outs


@pytest.mark.parametrize("dtype,storage_name", [(np.float16, "F16"), (np.float32, "F32")])
def test_server_alone_vs_mix_bitwise(dtype, storage_name):
    import torch
    import paper_1802_06130_amd as M
    storage = getattr(M, storage_name)
    banks = _banks(M, torch)
    zs = _inputs(torch, dtype)
    which = [i % 3 for i in range(len(zs))]
    want = _plain(M, banks, zs, which, storage)
    srv = M.Server(banks, storage=storage, max_slots=4, hbm_budget=1 << 30)
    alone = _alone(M, srv, zs, which)
    for i, (a, w) in enumerate(zip(alone, want)):
        assert np.array_equal(a, w), f"request {i} {SIZES[i]} alone differs from the plain denoiser"
    # the mix: all requests within about a millisecond, overlapping on the device
    outs = [z.new_empty(z.shape).pin_memory() for z in zs]
    for o in outs:
        o.fill_(-7.0)
    reqs = [M.Server.request(z, b, o) for z, b, o in zip(zs, which, outs)]
    arrivals = synth.poisson_arrivals(5000.0, len(zs), 5200)
    before = srv.stats()
    done = srv.replay(reqs, arrivals)
    st = srv.stats()
    assert all(c["status"] == M.MDN_OK for c in done), done
    assert st["tick_items"] - before["tick_items"] > st["ticks"] - before["ticks"], "no tick held two requests"
    for i, (o, w) in enumerate(zip(outs, want)):
        assert np.array_equal(o.numpy(), w), f"request {i} {SIZES[i]} differs in the mix"
    assert st["arena_used"] == 0
    srv.close()


@pytest.mark.parametrize("stages_per_tick,ahead", [(3, 1), (8, 3)])
def test_server_tick_granularity_and_staging(stages_per_tick, ahead):
    import torch
    import paper_1802_06130_amd as M
    banks = _banks(M, torch)
    zs = _inputs(torch, np.float16)
    which = [(i + 1) % 3 for i in range(len(zs))]
    want = _plain(M, banks, zs, which, M.F16)
    biggest = max(z.numel() for z in zs) * 2
    srv = M.Server(banks, storage=M.F16, max_slots=3, stages_per_tick=stages_per_tick,
                   max_ticks_in_flight=ahead, hbm_budget=256 << 20, staging_bytes=biggest)
    for i, (z, b) in enumerate(zip(zs, which)):
        srv.submit(z, b, None, tag=i)
    got = {}
    while len(got) < len(zs):
        for c in srv.poll(1.0):
            assert c["status"] == M.MDN_OK, c
            z = zs[c["tag"]]
            buf = np.empty(z.shape, np.float16)
            ct.memmove(buf.ctypes.data, c["host_out"], buf.nbytes)      # valid until the slot is reused
            got[c["tag"]] = buf
    for i in range(len(zs)):
        assert np.array_equal(got[i], want[i]), f"request {i} {SIZES[i]} differs"
    srv.close()


def test_server_mixes_column_walk_and_tiled_banks():
    """A bank of the paper's own configuration (16 x 16 x 16 buckets, 7x7 denoise / 5x5 upscale
    filters, the tiled kernel with inline selection) served beside a column-walk bank: every request
    equals the plain per-image denoiser bit for bit, alone and in the mix."""
    import torch
    import paper_1802_06130_amd as M
    import oracle as O
    walk_bank = _banks(M, torch)[0]
    zs0 = [synth.noisy_pair(300 + i, 160, 160, 3, 25)[0].astype(np.float64) for i in range(3)]
    lvs = []
    for lev in range(3):
        f = [O.level_features(O.build_pyramid(z, lev + 1)[lev]) for z in zs0]
        t_s = O.thresholds_from_features(np.concatenate([x[0] for x in f]), 16)
        t_c = O.thresholds_from_features(np.concatenate([x[1] for x in f]), 16)
        co = synth.random_bank_coeffs(80 + lev, 4096, 3, 25, 49)
        lvs.append(M.Level(16, t_s, t_c, 3, 2, torch.from_numpy(co).to(torch.float16).cuda(), 3))
    tiled_bank = M.Bank(lvs)
    banks = [walk_bank, tiled_bank]
    zs = _inputs(torch, np.float16)
    which = [i % 2 for i in range(len(zs))]
    want = _plain(M, banks, zs, which, M.F16)
    srv = M.Server(banks, storage=M.F16, max_slots=4, hbm_budget=1 << 30)
    alone = _alone(M, srv, zs, which)
    for i, (a, w) in enumerate(zip(alone, want)):
        assert np.array_equal(a, w), f"request {i} {SIZES[i]} bank {which[i]} alone differs"
    outs = [z.new_empty(z.shape).pin_memory() for z in zs]
    reqs = [M.Server.request(z, b, o) for z, b, o in zip(zs, which, outs)]
    done = srv.replay(reqs, synth.poisson_arrivals(5000.0, len(zs), 5300))
    assert all(c["status"] == M.MDN_OK for c in done), done
    for i, (o, w) in enumerate(zip(outs, want)):
        assert np.array_equal(o.numpy(), w), f"request {i} {SIZES[i]} bank {which[i]} differs in the mix"
    srv.close()


def test_server_mixes_luma_and_colour_selector_banks():
    """A luma-selector bank (its selection pass a launch of its own at the level's filtering stage)
    served beside colour-selector banks (their selection pass in the pyramid step's launch): every
    request equals the plain per-image denoiser bit for bit, alone and in the mix."""
    import torch
    import paper_1802_06130_amd as M
    colour = _banks(M, torch)[:2]
    luma = gpu_bank(trained_bank_multiscale(levels=3, selector="luma"), 3, coeff_dtype=torch.float16)
    banks = colour + [luma]
    zs = _inputs(torch, np.float16)
    which = [(i * 2) % 3 for i in range(len(zs))]
    want = _plain(M, banks, zs, which, M.F16)
    srv = M.Server(banks, storage=M.F16, max_slots=4, stages_per_tick=2, hbm_budget=1 << 30)
    alone = _alone(M, srv, zs, which)
    for i, (a, w) in enumerate(zip(alone, want)):
        assert np.array_equal(a, w), f"request {i} {SIZES[i]} bank {which[i]} alone differs"
    outs = [z.new_empty(z.shape).pin_memory() for z in zs]
    for o in outs:
        o.fill_(-7.0)
    reqs = [M.Server.request(z, b, o) for z, b, o in zip(zs, which, outs)]
    done = srv.replay(reqs, synth.poisson_arrivals(5000.0, len(zs), 5400))
    assert all(c["status"] == M.MDN_OK for c in done), done
    for i, (o, w) in enumerate(zip(outs, want)):
        assert np.array_equal(o.numpy(), w), f"request {i} {SIZES[i]} bank {which[i]} differs in the mix"
    srv.close()
