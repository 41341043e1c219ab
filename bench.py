"""Benchmark: megapixels/s denoised on the 4-level RGB 7x7 path (216 buckets per level).

Workload (synthetic, seeded): 64 RGB images, width and height uniform over {480, 488, ..., 4032}
with at most 4032*3024 pixels each (about 296 MP per batch), noise sigma 25/255 quantised to 8
bits, stored as float16; a 4-level pyramid (3 trained levels) with 7x7 upscale and 7x7 denoise
filters and 24 x 3 x 3 buckets per level, float16 storage and float32 accumulation. One step
denoises the whole batch with one mdn_denoise call per image, back to back on one stream (the
plain per-image form). Inputs are resident in HBM before timing starts.

The batched form (the headline value) denoises the same batch with one persistent launch per kernel
and level over all 64 images (per level the pyramid step with the selection pass, then the
filtering: 6 launches), captured once as a hipGraph and replayed each step, with strip heights
chosen by the plan's autotuner; its outputs are checked to be bitwise equal to the plain per-image
form's.

The quality block runs a stand-in for the paper's evaluation set (68 seeded scenes of 481x321, half
of them transposed, 8-bit noisy input at sigma 15, 25 and 50) through the served banks and through
banks of the paper's sizing trained on 256 pairs with their eight symmetries, and reports the mean
PSNR beside the noisy input's.

The filter bank is trained on the GPU by the library's own training path (32 seeded 256x256
pairs at the same noise level, GPU equal-population thresholds, ridge 1e-3, float16 coefficients)
before timing. A float32-storage run of the same batch (float32 filters, float32 arithmetic) is
reported beside it.

The served form replays open-loop Poisson request traces (2,000 requests at each of 50, 200 and
800 requests/s, arrival seed 5000 + rate) through the library's serving loop: sizes uniform over
{1280x720, 1920x1080, 4032x3024}, noise sigma uniform over {15, 25, 50}/255 selecting one of three
GPU-trained banks, float16 host images in pinned memory, results copied back into per-slot pinned
staging buffers. It reports p50/p99 latency (arrival to device done, arrival to host done) and
completed megapixels/s beside the offered load. Its latencies include both PCIe copies.

The roofline object reports the dominant kernel, the batched form's level-0 filtering launch,
against the HBM roofline (algorithmic bytes per launch / its HIP-event duration), with the unit that
actually limits it (the LDS coefficient gathers) and the dot2 issue rate beside it.

Beside them: the single-level grey method of Eq. (1) on 256x256 (latency), and the 3-level float32
RGB cascade on 1024x768 (MP/s and its HBM roofline at 52.5 algorithmic bytes per pixel).

The paper's own configuration at sigma 25 (16 x 16 x 16 buckets, 7x7 / 5x5 filters, 5 levels,
float16) runs the same batch in the batched form beside it (paper_config_batched).

The CPU leg times the FP64 oracle on the leading crops of the batch and then reports the accuracy of
the GPU results on that sample against it: bucket flips, max-abs at the GPU's maps, max-abs and
|dPSNR| against pure FP64, and the training normal equations and coefficients of both Gram
precisions against FP64 on two training pairs.

Prints one JSON line. Run: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

N_IMAGES = 64
LEVELS = 3            # trained levels; the pyramid has 4
Q_THETA, Q_S, Q_C = 24, 3, 3
RADIUS = 3
SIGMA = 25.0
HBM_PEAK_GBS = 8000.0
# dot2 (2 FP16 MACs per lane) issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2 MACs x 2 FLOP x 2.4 GHz
ALU_PEAK_TFLOPS = 157.3
FLOP_PER_PX = 2 * 3 * 98          # 3 channels x (49 upscale + 49 denoise) MACs per output pixel
ALG_BYTES_F16 = 27.5625           # whole 4-level path, float16 storage and I/O, per level-0 pixel
WALK_BYTES_PX_F16 = 13.5          # level-0 filter pass: read z (6) + coarser output (1.5) + write (6)
# LDS bytes the filter pass gathers per pixel: 3 channels x 14 rows (7 upscale + 7 denoise) x 16 bytes
WALK_LDS_BYTES_PX = 3 * 14 * 16
# random 16-byte LDS gathers, measured at about 81 bytes per clock per CU: 256 CUs x 2.4 GHz
LDS_GATHER_PEAK_GBS = 81 * 256 * 2.4


ACC_CROPS, CROP = 8, 1024   # leading images, cropped, that the CPU baseline and the accuracy check run


def _make_image(args):
    seed, w, h, dt, keep_clean = args
    z, u = synth.noisy_pair(seed, h, w, 3, SIGMA, dtype=dt)
    return z, (np.ascontiguousarray(u[:, :CROP, :CROP]) if keep_clean else None)


def make_inputs(n: int, dtype):
    """The batch (noisy images) and the clean crops of its leading images, made in worker processes
    before the GPU is touched."""
    sizes = synth.ragged_sizes(4, n)
    jobs = [(4001 + i, w, h, dtype, i < ACC_CROPS) for i, (w, h) in enumerate(sizes)]
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_make_image, jobs, chunksize=1)
    return sizes, [z for z, _ in res], [u for _, u in res if u is not None]


def train_bank(M, torch, n_pairs=32, size=256, sigma=SIGMA):
    pairs = [synth.noisy_pair(7000 + i, size, size, 3, sigma) for i in range(n_pairs)]
    dev = torch.device("cuda:0")
    pairs = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
    bank, _, fbs = M.train_multiscale(pairs, LEVELS, Q_THETA, Q_S, Q_C, RADIUS, RADIUS, 1e-3)
    torch.cuda.synchronize()
    return bank, fbs


def as_dtype(M, bank, dt):
    return M.Bank([M.Level(lv.q_theta, lv.t_s, lv.t_c, lv.radius_g, lv.radius_f, lv.coeffs.to(dt), 3)
                   for lv in bank.levels])


def spread(ms, what=None, nd=3):
    """p10 / p50 / p90 / p99 of a list of timings."""
    a = np.asarray(ms, dtype=np.float64)
    d = {f"p{q}": round(float(np.percentile(a, q)), nd) for q in (10, 50, 90, 99)}
    if what is not None:
        d["what"] = what
    return d


def copy_bandwidth(torch, nbytes=1 << 30, reps=20, warmup=5):
    """Device-to-device copy rate of an nbytes buffer (torch's copy kernel, read plus write counted),
    HIP events around each copy on the current stream: the HBM rate a streaming kernel reaches in
    practice, beside the 8 TB/s of the data sheet."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        dst.copy_(src)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
    torch.cuda.synchronize()
    gbs = np.array([2.0 * nbytes / (a.elapsed_time(b) * 1e-3) / 1e9 for a, b in evs])
    del src, dst
    return {"GBs": round(float(np.median(gbs)), 1), "p10_GBs": round(float(np.percentile(gbs, 10)), 1),
            "p90_GBs": round(float(np.percentile(gbs, 90)), 1), "bytes_per_copy": 2 * nbytes, "reps": reps,
            "what": "device-to-device copy of a 1 GiB buffer (read + write), median of HIP-event-timed copies"}


def run_form(M, torch, zs, bank, storage, steps, warmup):
    """Plain per-image form: returns (wall seconds for `steps`, per-image latencies ms, step ms)."""
    dev = zs[0].device
    outs = [torch.empty_like(z) for z in zs]
    ws_bytes = max(M.denoise_workspace_size(z.shape[2], z.shape[1], 3, LEVELS, storage) for z in zs)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        for i, z in enumerate(zs):
            if ev is not None:
                ev[i][0].record(stream)
            M.denoise(z, bank, storage, ws=ws, out=outs[i])
            if ev is not None:
                ev[i][1].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev_img = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in zs]
              for _ in range(steps)]
    ev_step = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev_step[k][0].record(stream)
        step(ev_img[k])
        ev_step[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([[a.elapsed_time(b) for a, b in row] for row in ev_img]).ravel()
    ms_steps = [a.elapsed_time(b) for a, b in ev_step]
    return wall, lat, ms_steps, outs


def run_batched(M, torch, zs, bank, steps, warmup):
    """Batched form: one plan, autotuned, graph replay; returns (wall s, batch latencies ms, rows, outs,
    per-launch kernel times). The kernel times come after the timed steps: the same launches, one at
    a time between HIP events on the plan's stream."""
    plan = M.Plan(bank, M.F16, max_images=len(zs))
    outs = [torch.empty_like(z) for z in zs]
    rows = plan.autotune(zs, outs)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.denoise_batch(zs, outs, use_graph=True)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k][0].record(stream)
        plan.denoise_batch(zs, outs, use_graph=True)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    ktimes = plan.kernel_times(zs, outs, reps=3)
    plan.close()
    return wall, lat, rows, outs, ktimes


SERVE_SIZES = [(1280, 720), (1920, 1080), (4032, 3024)]
SERVE_SIGMAS = [15.0, 25.0, 50.0]


def _make_serve_image(args):
    k, w, h, sigma = args
    z, _ = synth.noisy_pair(8100 + k, h, w, 3, sigma, dtype=np.float16)
    return z


def make_serve_images():
    """The served form's nine request images (size x sigma), made in worker processes before the GPU
    is touched: a process forked after the HIP runtime started could inherit its held locks."""
    jobs = [(3 * si + gi, w, h, g) for si, (w, h) in enumerate(SERVE_SIZES) for gi, g in enumerate(SERVE_SIGMAS)]
    workers = max(1, min(9, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_make_serve_image, jobs, chunksize=1)


def run_served(M, torch, banks16, rates, n_requests, imgs):
    """Open-loop Poisson traces through the serving loop; returns the per-rate report. Each request
    size is also served alone once more and compared with the plain per-image form bit for bit."""
    host = [torch.from_numpy(z).pin_memory() for z in imgs]          # [size * 3 + sigma]
    staging = max(z.numel() for z in host) * 2
    srv = M.Server(banks16, storage=M.F16, max_slots=16, stages_per_tick=1, max_ticks_in_flight=2,
                   hbm_budget=8 << 30, staging_bytes=staging)
    px_of = [w * h for w, h in SERVE_SIZES]
    # latency of each size alone (no other request in the server)
    alone = {}
    for si, (w, h) in enumerate(SERVE_SIZES):
        lat = []
        for rep in range(4):
            srv.submit(host[si * 3 + 1], 1, None, tag=rep)
            (c,) = srv.wait_all()
            lat.append((c["t_host_done"] - c["t_arrival"]) * 1e3)
        alone[f"{w}x{h}"] = round(float(np.median(lat[1:])), 3)
    report = {"alone_host_ms": alone}
    same = {}
    for si, (w, h) in enumerate(SERVE_SIZES):
        out_host = torch.empty_like(host[si * 3 + 1]).pin_memory()
        srv.submit(host[si * 3 + 1], 1, out_host, tag=100 + si)
        (c,) = srv.wait_all()
        ref = M.denoise(host[si * 3 + 1].to("cuda:0"), banks16[1], M.F16).cpu()
        same[f"{w}x{h}"] = bool(c["status"] == M.MDN_OK and torch.equal(out_host, ref))
    report["bitwise_equal_to_plain"] = same
    # unmeasured warm-up at the highest rate: the first busy trace of a process pays one-time costs
    # (seen as a p99 of 11-17 ms against 6 ms for the same trace replayed afterwards)
    wrate = float(max(rates))
    wrng = np.random.default_rng(4999)
    warr = synth.poisson_arrivals(wrate, 400, 4999)
    srv.replay([M.Server.request(host[int(a) * 3 + int(b)], int(b))
                for a, b in zip(wrng.integers(0, 3, 400), wrng.integers(0, 3, 400))], warr)
    for rate in rates:
        rng = np.random.default_rng(5000 + rate)
        arrivals = synth.poisson_arrivals(float(rate), n_requests, 5000 + rate)
        size = rng.integers(0, 3, n_requests)
        sig = rng.integers(0, 3, n_requests)
        reqs = [M.Server.request(host[int(a) * 3 + int(b)], int(b)) for a, b in zip(size, sig)]
        before = srv.stats()
        t0 = time.perf_counter()
        done = srv.replay(reqs, arrivals)
        wall = time.perf_counter() - t0
        st = srv.stats()
        ok = [c for c in done if c["status"] == M.MDN_OK]
        px = np.array([px_of[s] for s, c in zip(size, done) if c["status"] == M.MDN_OK], dtype=np.float64)
        dev = np.array([(c["t_device_done"] - c["t_arrival"]) * 1e3 for c in ok])
        hst = np.array([(c["t_host_done"] - c["t_arrival"]) * 1e3 for c in ok])
        span = max(c["t_host_done"] for c in ok) - min(c["t_arrival"] for c in done)
        ticks = st["ticks"] - before["ticks"]
        report[str(rate)] = {
            "requests": n_requests, "completed": len(ok), "failed_or_rejected": n_requests - len(ok),
            "offered_MP_s": round(float(sum(px_of[s] for s in size) / 1e6 / arrivals[-1]), 1),
            "completed_MP_s": round(float(px.sum() / 1e6 / span), 1),
            "device_done_ms": {"p50": round(float(np.percentile(dev, 50)), 3),
                               "p99": round(float(np.percentile(dev, 99)), 3)},
            "host_done_ms": {"p50": round(float(np.percentile(hst, 50)), 3),
                             "p99": round(float(np.percentile(hst, 99)), 3)},
            "ticks": int(ticks), "launches": int(st["launches"] - before["launches"]),
            "stages_per_tick_mean": round((st["tick_items"] - before["tick_items"]) / max(1, ticks), 2),
            "wall_s": round(wall, 2)}
        print(f"# served {rate} req/s: {report[str(rate)]}", file=sys.stderr, flush=True)
    report["config"] = ("16 slots, 8 GiB device budget, 1 stage per tick, 2 ticks ahead; sizes uniform over "
                        "1280x720/1920x1080/4032x3024, sigma uniform over 15/25/50 of 255 (one bank each), "
                        "float16 pinned host images, Poisson arrivals seed 5000+rate, after an unmeasured "
                        "warm-up trace of 400 requests at the highest rate")
    srv.close()
    return report


TRAIN_PAIRS, TRAIN_SIZE = 256, 512
ACC_TRAIN_PAIRS = 2       # training pairs whose normal equations are checked against FP64
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


def _make_train_pair(args):
    seed, sigma = args
    z, u = synth.noisy_pair(seed, TRAIN_SIZE, TRAIN_SIZE, 3, sigma)
    return z, u


def make_train_pairs(n_pairs=TRAIN_PAIRS, pool=True):
    """256 seeded 512x512 RGB training pairs (sigma per pair from {15, 25, 50}/255, rng(3)); the
    profiler probe takes the first n_pairs. Worker processes are forked before the GPU is touched."""
    rng = np.random.default_rng(3)
    sig = rng.choice([15.0, 25.0, 50.0], TRAIN_PAIRS)[:n_pairs]
    jobs = [(1 + i, float(g)) for i, g in enumerate(sig)]
    if pool:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
        with mp.get_context("fork").Pool(workers) as pool_:
            return pool_.map(_make_train_pair, jobs, chunksize=8)
    return [_make_train_pair(j) for j in jobs]


def gram_mfma_flop(D, C, samples):
    """FLOP the Gram kernel issues on the matrix cores: the feature vector plus the target (which
    rides along as one more feature) is padded to T tiles of 32, and only the T(T+1)/2 tiles on and
    above the diagonal are multiplied, 2 x 32 x 32 FLOP per tile and sample."""
    T = -(-(D + 1) // 32)
    return 2.0 * (T * (T + 1) // 2) * 32 * 32 * C * samples


def run_training(M, torch, pairs):
    """Training throughput, 3-level pyramid: accumulation of the level-0 normal equations (D = 98 per
    channel; 67.1 M samples on the 256 pairs) in both Gram precisions, then the level's FP64 solve
    (648 systems)."""
    n_pairs = len(pairs)
    dev = torch.device("cuda:0")
    zs = [torch.from_numpy(z).to(dev) for z, _ in pairs]
    us = [torch.from_numpy(u).to(dev) for _, u in pairs]
    del pairs
    coarse = [M.pyramid_build(z, 1)[0] for z in zs]
    t_s, t_c = M.level_thresholds(zs[:32], Q_S, Q_C)
    K, C, D = Q_THETA * Q_S * Q_C, 3, 98
    sel = M.Level(Q_THETA, t_s, t_c, RADIUS, RADIUS, torch.zeros((K, C, D), device=dev), 3)
    stream = torch.cuda.current_stream()
    samples = n_pairs * TRAIN_SIZE * TRAIN_SIZE
    useful = 2.0 * (D * D + D) * C * samples          # G and b products per sample and channel
    issued = gram_mfma_flop(D, C, samples)
    out = {"workload": f"{n_pairs} RGB pairs {TRAIN_SIZE}x{TRAIN_SIZE}, level 0 of a 3-level pyramid, "
                       f"D = 98 per channel, {K} buckets, {samples / 1e6:.1f} M samples"}
    g = None
    for name, prec, peak, mult in (("fp32_mfma", M.GRAM_F32, FP32_MFMA_PEAK_TFLOPS, 1),
                                   ("bf16x3_mfma", M.GRAM_BF16X3, BF16_MFMA_PEAK_TFLOPS, 3)):
        g = M.Gram(K, C, RADIUS, RADIUS, device=dev)
        ws = M.train_accumulate(g, zs[0], us[0], sel, u_coarse=coarse[0], coarse_color=M.RGB, precision=prec)
        g.zero()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for z, u, c in zip(zs, us, coarse):
            M.train_accumulate(g, z, u, sel, u_coarse=c, coarse_color=M.RGB, precision=prec, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
        out[name] = {"accumulate_ms": round(sec * 1e3, 2), "samples_per_s": round(samples / sec / 1e9, 3),
                     "samples_unit": "G/s", "useful_TFLOPs": round(useful / sec / 1e12, 2),
                     "mfma_issued_TFLOPs": round(issued * mult / sec / 1e12, 2),
                     "mfma_frac": round(issued * mult / sec / 1e12 / peak, 4), "peak_TFLOPs": peak}
        print(f"# training {name}: {out[name]}", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    co, nfb = M.train_solve(g, 1e-3)
    e1.record(stream)
    torch.cuda.synchronize()
    out["solve_ms"] = round(e0.elapsed_time(e1), 3)
    out["solve_systems"] = K * C
    out["fallback_systems"] = nfb
    # accuracy sample: the first ACC_TRAIN_PAIRS pairs accumulated in both precisions and solved; the
    # CPU leg compares them with the FP64 normal equations over the same selector maps
    sub = []
    for z, u, c in list(zip(zs, us, coarse))[:ACC_TRAIN_PAIRS]:
        sub.append({"z": z.cpu().numpy(), "u": u.cpu().numpy(), "coarse": c.cpu().numpy(),
                    "s": M.select_filters(z, sel).cpu().numpy()})
    res = {}
    for name, prec in (("fp32_mfma", M.GRAM_F32), ("bf16x3_mfma", M.GRAM_BF16X3)):
        g = M.Gram(K, C, RADIUS, RADIUS, device=dev)
        for z, u, c in list(zip(zs, us, coarse))[:ACC_TRAIN_PAIRS]:
            M.train_accumulate(g, z, u, sel, u_coarse=c, coarse_color=M.RGB, precision=prec)
        co, nfb = M.train_solve(g, 1e-3)
        res[name] = {"G": g.G.cpu().numpy().reshape(K, C, D, D), "n": g.n.cpu().numpy(),
                     "h": co.double().cpu().numpy(), "fallback": nfb}
    # cross-channel layout (x = the 7x7 taps of all three channels, D = 147, one Gram per bucket and
    # three right-hand sides), single scale on the same pairs and thresholds
    selx = M.Level(Q_THETA, t_s, t_c, RADIUS, None, torch.zeros((K, C, 49), device=dev), 3)
    resx = {}
    for name, prec in (("fp32_mfma", M.GRAM_F32), ("bf16x3_mfma", M.GRAM_BF16X3)):
        g = M.Gram(K, C, RADIUS, None, layout=M.X_CROSS_CHANNEL, device=dev)
        for z, u, _ in list(zip(zs, us, coarse))[:ACC_TRAIN_PAIRS]:
            M.train_accumulate(g, z, u, selx, precision=prec)
        co, nfb = M.train_solve(g, 1e-3)
        resx[name] = {"G": g.G.cpu().numpy().reshape(K, 147, 147), "n": g.n.cpu().numpy(),
                      "h": co.double().cpu().numpy(), "fallback": nfb}
    for p, (z, _, _) in zip(sub, list(zip(zs, us, coarse))[:ACC_TRAIN_PAIRS]):
        p["s0"] = M.select_filters(z, selx).cpu().numpy()
    sample = {"pairs": sub, "results": res, "results_cross": resx, "t_s": np.asarray(t_s), "t_c": np.asarray(t_c),
              "K": K, "C": C, "D": D}
    return out, sample


def run_paper_config_batched(M, torch, zs, steps, warmup, sigma=25):
    """The paper's own configuration (Section 5) at sigma 25 on the same batch: 16 x 16 x 16 buckets,
    7x7 denoise and 5x5 upscale filters, 5 pyramid levels, trained on the GPU from the bench's 32
    training pairs (most of the 4096 buckets take the pooled solution with this little data), float16
    coefficients and storage; batched form (one tiled launch per level, selection inline, hipGraph
    replay). Returns its rate and whether it equals the per-image form on the first images."""
    L, rf, rg = PAPER_CONFIG[sigma]
    pairs = [synth.noisy_pair(7000 + i, 256, 256, 3, float(sigma)) for i in range(32)]
    dev = torch.device("cuda:0")
    pairs = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
    b32, _, fbs = M.train_multiscale(pairs, L, 16, 16, 16, rf, rg, 1e-3)
    bank = M.Bank([M.Level(lv.q_theta, lv.t_s, lv.t_c, lv.radius_g, lv.radius_f, lv.coeffs.half(), 3)
                   for lv in b32.levels])
    plan = M.Plan(bank, M.F16, max_images=len(zs))
    outs = [torch.empty_like(z) for z in zs]
    plan.autotune(zs, outs)
    for _ in range(warmup):
        plan.denoise_batch(zs, outs, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.denoise_batch(zs, outs, use_graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = plan.kernel_times(zs, outs, reps=1)
    plan.close()
    same = all(torch.equal(outs[i], M.denoise(zs[i], bank, storage=M.F16)) for i in range(4))
    px = sum(z.shape[1] * z.shape[2] for z in zs)
    return {"value": round(px * steps / wall / 1e6, 2), "unit": "MP/s", "ms_per_step": round(wall * 1e3 / steps, 3),
            "steps": steps, "levels": L + 1, "buckets": 4096, "radius_f": rf, "radius_g": rg,
            "fallback_systems": fbs, "bitwise_equal_to_plain_first4": bool(same),
            "kernel_us_per_level": [[round(t, 1) for t in lv] for lv in kt],
            "what": "paper configuration at sigma 25 (16x16x16 buckets, 7x7 g / 5x5 f, 5 levels), float16, "
                    "batched form on the same 64 images: tiled select-and-filter kernel, one launch per level"}


QUALITY_SIGMAS = (15, 25, 50)
QUALITY_SCENES = 68          # test scenes 481 x 321, every other one transposed
QUALITY_TRAIN = 256          # training pairs 256 x 256 per noise level for the paper-sized bank


def _make_quality_item(args):
    seed, h, w = args
    u = synth.synth_scene(seed, h, w, 3)
    return u, [synth.add_noise(u, float(g), seed) for g in QUALITY_SIGMAS]


def make_quality_inputs():
    """A test set shaped like the paper's evaluation set (Section 5: 68 images of 481 x 321 or
    321 x 481, 8-bit noisy input) and, per noise level, 256 training pairs of 256 x 256; made in
    worker processes before the GPU is touched."""
    test = [(8001 + i, 321, 481) if i % 2 == 0 else (8001 + i, 481, 321) for i in range(QUALITY_SCENES)]
    train = [(9001 + i, 256, 256) for i in range(QUALITY_TRAIN)]
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_make_quality_item, test + train, chunksize=8)
    return res[:QUALITY_SCENES], res[QUALITY_SCENES:]


def _psnr(est, ref):
    e = np.clip(est.astype(np.float64), 0.0, 1.0) - ref.astype(np.float64)
    return 10.0 * np.log10(1.0 / float(np.mean(e * e)))


def run_quality(M, torch, data, served32):
    """PSNR on the synthetic stand-in for the paper's evaluation set, per noise level, of two banks:
    the served one (24 x 3 x 3 buckets, 7x7 / 7x7, 4 pyramid levels, 32 training pairs) and one of
    the paper's sizing (16 x 16 x 16 buckets, 5x5 upscale / 7x7 denoise filters, as many levels as
    bring the coarsest level's noise below 2; 256 pairs, each with its eight symmetries). Float16
    storage and I/O, mean of the per-image PSNR against the clean scene (peak 1)."""
    test, train = data
    dev = torch.device("cuda:0")
    out = {}
    for gi, g in enumerate(QUALITY_SIGMAS):
        t0 = time.perf_counter()
        L, rf, rg = PAPER_CONFIG[g]
        pairs = [(torch.from_numpy(zz[gi]).to(dev), torch.from_numpy(u).to(dev)) for u, zz in train]
        b32, _, fbs = M.train_multiscale(pairs, L, 16, 16, 16, rf, rg, 1e-3, augment=True)
        del pairs
        paper16 = as_dtype(M, b32, torch.float16)
        served16 = as_dtype(M, served32[gi], torch.float16)
        noisy, den_s, den_p = [], [], []
        for u, zz in test:
            z = torch.from_numpy(zz[gi]).to(dev).half()
            noisy.append(_psnr(zz[gi], u))
            den_s.append(_psnr(M.denoise(z, served16, M.F16).float().cpu().numpy(), u))
            den_p.append(_psnr(M.denoise(z, paper16, M.F16).float().cpu().numpy(), u))
        out[str(g)] = {"psnr_noisy_db": round(float(np.mean(noisy)), 3),
                       "psnr_served_bank_db": round(float(np.mean(den_s)), 3),
                       "psnr_paper_sized_bank_db": round(float(np.mean(den_p)), 3),
                       "paper_sized_levels": L + 1, "paper_sized_fallback_systems": fbs,
                       "seconds": round(time.perf_counter() - t0, 1)}
        print(f"# quality sigma {g}: {out[str(g)]}", file=sys.stderr, flush=True)
        del b32, paper16
        torch.cuda.empty_cache()
    out["test_set"] = (f"{QUALITY_SCENES} seeded scenes 481x321, every other one transposed, seeds 8001.., "
                       "noise quantised to 8 bits and clamped; stand-in for the paper's 68 Berkeley test images")
    out["training"] = (f"paper-sized bank: {QUALITY_TRAIN} seeded pairs 256x256 per noise level (seeds 9001..), "
                       "eight symmetries each, lambda 1e-3; served bank: 32 pairs 256x256, no symmetries")
    out["paper_table1_db"] = {"15": 32.46, "25": 29.58, "50": 25.92,
                              "what": "the paper's own figures on the Berkeley set with its 2.23e9-pixel corpus: "
                                      "context only, neither the images nor the corpus are here"}
    return out


def _time_calls(torch, fn, reps=50, warmup=5):
    """Device time of each of `reps` calls (HIP events on the current stream), in microseconds."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) * 1e3 for a, b in evs])


def run_single_level_grey(M, torch):
    """Single-level plain method (Eq. (1)) on a grey 256x256 float32 image: 16 x 3 x 3 buckets of 5x5
    filters trained on the GPU from 8 seeded 128x128 pairs at sigma 25; one mdn_denoise call per
    image, latency-bound at this size. Algorithmic HBM bytes: read 4 + write 4 per pixel."""
    dev = torch.device("cuda:0")
    pairs = [synth.noisy_pair(1 + i, 128, 128, 1, SIGMA) for i in range(8)]
    pairs = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
    bank, _, _ = M.train_single(pairs, 16, 3, 3, 2, 1e-3)
    z, u = synth.noisy_pair(1001, 256, 256, 1, SIGMA)
    zt = torch.from_numpy(z).to(dev)
    out = torch.empty_like(zt)
    us = _time_calls(torch, lambda: M.denoise(zt, bank, M.F32, out=out))
    med = float(np.median(us))
    return {"latency_us": {"p50": round(med, 2), "p99": round(float(np.percentile(us, 99)), 2)},
            "MP_s": round(256 * 256 / med, 1), "hbm_GB_s": round(8.0 * 256 * 256 / med * 1e-3, 1),
            "what": "grey 256x256 float32, 16x3x3 buckets, 5x5 filters (Eq. (1)), one mdn_denoise call; "
                    "latency-bound (65k pixels)"}, (z, u, bank, out.cpu().numpy())


def run_three_level_f32(M, torch):
    """3-level RGB 1024x768 float32 cascade, 7x7 upscale and denoise filters, 24 x 3 x 3 buckets,
    trained on the GPU from 64 seeded 256x256 pairs with sigma drawn from {15, 25, 50}/255 (rng(2));
    one seeded test image at sigma 25. Algorithmic HBM bytes 52.5 per pixel in float32."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(2)
    sig = rng.choice([15.0, 25.0, 50.0], 64)
    pairs = [synth.noisy_pair(1 + i, 256, 256, 3, float(g)) for i, g in enumerate(sig)]
    pairs = [(torch.from_numpy(z).to(dev), torch.from_numpy(u).to(dev)) for z, u in pairs]
    bank, _, _ = M.train_multiscale(pairs, 2, Q_THETA, Q_S, Q_C, RADIUS, RADIUS, 1e-3)
    z, u = synth.noisy_pair(2001, 768, 1024, 3, SIGMA)
    zt = torch.from_numpy(z).to(dev)
    out = torch.empty_like(zt)
    ws = torch.empty(M.denoise_workspace_size(1024, 768, 3, 2, M.F32), dtype=torch.uint8, device=dev)
    us = _time_calls(torch, lambda: M.denoise(zt, bank, M.F32, ws=ws, out=out))
    med = float(np.median(us))
    px = 1024 * 768
    hbm = 52.5 * px / med * 1e-3
    pyr = [zt] + M.pyramid_build(zt, 2, storage=torch.float32)
    maps = [M.select_filters(pyr[l], bank.levels[l]).cpu().numpy().astype(np.int64) for l in range(2)]
    return {"MP_s": round(px / med, 1), "latency_us": {"p50": round(med, 2), "p99": round(float(np.percentile(us, 99)), 2)},
            "roofline": {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(hbm / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_px": 52.5},
            "what": "RGB 1024x768 float32, 3 levels, 7x7/7x7, 24x3x3 buckets, one mdn_denoise call (per level "
                    "the pyramid step with the selection pass, then LDS-bank filtering)"}, (z, u, bank, out.cpu().numpy(), maps)


def time_level0_filter(M, torch, zs, bank, n=16, reps=3):
    """The dominant kernel, the level-0 filtering pass, timed alone with HIP events on its stream
    (the selector map and the coarser output are prepared first)."""
    stream = torch.cuda.current_stream()
    lv0, lv1 = bank.levels[0], bank.levels[1]
    prep = []
    for z in zs[:n]:
        p = M.pyramid_build(z, 2)
        s1 = torch.empty(p[0].shape[1:], dtype=torch.uint8, device=z.device)
        uc = M.apply_level(p[0], lv1, u_coarse=p[1], coarse_color=M.RGB, s_out=s1)
        s0 = M.select_filters(z, lv0)
        prep.append((z, uc, s0, torch.empty_like(z)))
    torch.cuda.synchronize()
    evs, px = [], []
    for rep in range(reps):
        for z, uc, s0, o in prep:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            M.apply_level(z, lv0, u_coarse=uc, s=s0, out=o, out_color=M.RGB)
            e1.record(stream)
            evs.append((e0, e1))
            if rep == 0:
                px.append(z.shape[1] * z.shape[2])
    torch.cuda.synchronize()
    durs = np.array([a.elapsed_time(b) for a, b in evs]) * 1e-3
    return float(np.mean(px)), float(np.mean(durs))


def walk_source_sha():
    p = os.path.join(ROOT, "paper_1802_06130_amd", "csrc", "walk.hip")
    with open(p, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per level-0 pixel of the filtering pass from the committed PMC summary, if it was
    taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "walk_level0_traffic.json")
    try:
        with open(p) as fh:
            d = json.load(fh)
    except OSError:
        return None
    if d.get("walk_hip_sha256_16") != walk_source_sha():
        return None
    return d


def pmc_probe():
    """For hardware-counter runs: one copy kernel of known size (512 MiB read + written), then the
    bench's batch of images through the batched form (autotuned strip heights), its launches once
    more one at a time: the last six dispatches are the pyramid steps with their levels' selection
    passes (levels 0 -> 1 -> 2 -> 3, one launch each), then the filtering of levels 2, 1 and 0. The
    bank has random coefficients."""
    sizes, imgs, _ = make_inputs(N_IMAGES, np.float16)     # before the GPU is touched (worker pool)
    import torch
    import paper_1802_06130_amd as M
    dev = torch.device("cuda:0")
    src = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    zs = [torch.from_numpy(z).to(dev) for z in imgs]
    outs = [torch.empty_like(z) for z in zs]
    bank = M.Bank([M.Level(Q_THETA, [0.02, 0.05], [0.25, 0.5], RADIUS, RADIUS,
                           torch.tensor(synth.random_bank_coeffs(100 + i, Q_THETA * Q_S * Q_C, 3, 49, 49),
                                        dtype=torch.float16, device=dev), 3)
                   for i in range(LEVELS)])
    plan = M.Plan(bank, M.F16, max_images=len(zs))
    plan.autotune(zs, outs)
    plan.kernel_times(zs, outs, reps=1)
    torch.cuda.synchronize()
    plan.close()
    print(f"pmc probe done: {len(zs)} images, {sum(w * h for w, h in sizes)} level-0 pixels", flush=True)


# The paper's own configuration (Section 5): 16 x 16 x 16 buckets at every level; 7x7 denoise and
# 5x5 upscale filters (5x5 and 3x3 below sigma 10); as many pyramid levels as bring the coarsest
# level's noise below 2 (noise sigma -> trained levels, radius_f, radius_g).
PAPER_CONFIG = {5: (2, 1, 2), 15: (3, 2, 3), 25: (4, 2, 3), 50: (5, 2, 3)}


def paper_frame_probe(sigma: int):
    """The cascade of the paper's configuration at noise sigma on one seeded 4032x3024 float16 frame:
    seeded stand-in float16 coefficients, thresholds at the equal-population quantiles of a
    1024x1024 crop of the frame, 3 untimed and 5 timed mdn_denoise calls. For the profiler."""
    if sigma not in PAPER_CONFIG:
        raise SystemExit(f"--paper-frame: sigma one of {sorted(PAPER_CONFIG)}")
    L, rf, rg = PAPER_CONFIG[sigma]
    qt = qs = qc = 16
    noisy = synth.noisy_pair(7, 3024, 4032, 3, float(sigma))[0]
    import torch
    import paper_1802_06130_amd as M
    dev = torch.device("cuda:0")
    frame = torch.from_numpy(noisy).to(dev).half()
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
                      "frame_ms_f16": round(ms, 3), "MP_s_f16": round(3024 * 4032 / ms * 1e-3, 1)}), flush=True)


def accuracy_crops(imgs):
    """The leading images of the batch cropped to at most CROP x CROP: the sample both the CPU
    baseline and the accuracy check run."""
    return [np.ascontiguousarray(z[:, :CROP, :CROP]) for z in imgs[:ACC_CROPS]]


def gpu_crop_outputs(M, torch, crops, bank16):
    """The crops through the headline (batched) form, and every level's selector map as the selection
    walk writes it on the float16 pyramid."""
    dev = torch.device("cuda:0")
    zs = [torch.from_numpy(c).to(dev) for c in crops]
    plan = M.Plan(bank16, M.F16, max_images=len(zs))
    outs = plan.denoise_batch(zs, use_graph=True)
    torch.cuda.synchronize()
    plan.close()
    res = []
    for z, o in zip(zs, outs):
        pyr = [z] + M.pyramid_build(z, LEVELS, storage=torch.float16)
        maps = [M.select_filters(pyr[lev], bank16.levels[lev]).cpu().numpy().astype(np.int64)
                for lev in range(LEVELS)]
        res.append((o.float().cpu().numpy().astype(np.float64), maps))
    return res


def cpu_baseline_leg(crops, clean_crops, gpu_crops, bank16_dev, bank32_dev, train_sample, c1=None, c2=None,
                     budget_s=20.0):
    """The FP64 oracle on a bounded sample of the same workload (the leading crops), timed; then the
    accuracy of the GPU results on that sample against it:
    * inference (the crops through the batched form): bucket flips per level against the oracle's
      selection on the same float16 pyramid, all of them near a boundary (oracle margin < 1e-6);
      max-abs over every pixel against the oracle's float16-storage mode run on the GPU's maps with
      the same float16 coefficients; and max-abs and |dPSNR| against the pure FP64 oracle with the
      bank as trained (float32 coefficients, no storage rounding);
    * training (ACC_TRAIN_PAIRS pairs of the training workload): the worst Gram entry error relative
      to sqrt(G_pp G_qq), the coefficient max-abs and the output-space error
      sqrt(sum dh^T G dh / sum y^2) of both Gram precisions against the FP64 normal equations
      accumulated over the same selector maps and solved in FP64."""
    import oracle as O

    def host_bank(b):
        return O.Bank([O.LevelBank(lv.q_theta, lv.t_s, lv.t_c, lv.radius_g, None if lv.radius_f < 0 else lv.radius_f,
                                   lv.coeffs.double().cpu().numpy()) for lv in b.levels])
    bank, bank64 = host_bank(bank16_dev), host_bank(bank32_dev)
    from threadpoolctl import threadpool_limits
    done_px, n = 0, 0
    own = []
    with threadpool_limits(limits=1):       # one core: the oracle is timed as a single process
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s * 0.6 and n < len(crops):
            own.append(O.denoise(crops[n], bank, storage=np.float16, return_index_maps=True))
            done_px += crops[n].shape[1] * crops[n].shape[2]
            n += 1
        dt = time.perf_counter() - t0
    base = {"value": round(done_px / dt / 1e6, 4), "unit": "MP/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} leading image(s) of the batch cropped to at most {CROP}x{CROP} "
                      f"({done_px / 1e6:.2f} MP), 4-level FP64 NumPy oracle in float16-storage mode, "
                      f"one process, BLAS and OpenMP pools limited to one thread",
            "host_cpus": {"affinity": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()},
            "paper_context": "Section 5, Table 1: 0.038 s per 1 MP image on a Xeon E5-1650 3.5 GHz (about 26 MP/s); "
                             "Section 4: 18 MP/s on CPU and 188 MP/s on GPU of a Pixel 2017 phone"}
    acc = {"inference": {"crops": n, "form": "batched (plan, hipGraph), float16 storage and filters",
                         "flips_per_level": [0] * LEVELS, "near_boundary_per_level": [0] * LEVELS,
                         "flips_away_from_boundary": 0,
                         "max_abs_vs_fp16_mode_at_gpu_maps": 0.0, "max_abs_vs_fp64": 0.0, "dpsnr_vs_fp64_db": 0.0}}
    inf = acc["inference"]
    for i in range(n):
        ref16, omaps = own[i]
        got, gmaps = gpu_crops[i]
        pyr = O.build_pyramid(crops[i], LEVELS + 1, storage=np.float16)
        flipped = False
        for lev in range(LEVELS):
            lb = bank.levels[lev]
            _, margin = O.select(np.asarray(pyr[lev], np.float64), lb.q_theta, lb.t_s, lb.t_c, return_margin=True)
            mism = gmaps[lev] != omaps[lev]
            near = margin < 1e-6
            inf["flips_per_level"][lev] += int(mism.sum())
            inf["near_boundary_per_level"][lev] += int(near.sum())
            inf["flips_away_from_boundary"] += int((mism & ~near).sum())
            flipped |= bool(mism.any())
        at = O.denoise(crops[i], bank, storage=np.float16, maps=gmaps) if flipped else ref16
        ref64 = O.denoise(np.asarray(crops[i], np.float64), bank64)
        clean = np.asarray(clean_crops[i], np.float64)
        inf["max_abs_vs_fp16_mode_at_gpu_maps"] = max(inf["max_abs_vs_fp16_mode_at_gpu_maps"],
                                                     float(np.max(np.abs(got - at))))
        inf["max_abs_vs_fp64"] = max(inf["max_abs_vs_fp64"], float(np.max(np.abs(got - ref64))))
        inf["dpsnr_vs_fp64_db"] = max(inf["dpsnr_vs_fp64_db"], abs(O.psnr(got, clean) - O.psnr(ref64, clean)))
    for k in ("max_abs_vs_fp16_mode_at_gpu_maps", "max_abs_vs_fp64"):
        inf[k] = float(f"{inf[k]:.3g}")
    inf["dpsnr_vs_fp64_db"] = round(float(inf["dpsnr_vs_fp64_db"]), 5)
    if train_sample is not None:
        ts = train_sample
        K, C, D = ts["K"], ts["C"], ts["D"]
        st = O.GramStats.zeros(K, C, D)
        for p in ts["pairs"]:
            O.accumulate_level(st, p["s"].astype(np.int64), O.to_filter_space(np.asarray(p["z"], np.float64)),
                               O.to_filter_space(np.asarray(p["u"], np.float64)), RADIUS, RADIUS,
                               O.to_filter_space(np.asarray(p["coarse"], np.float64)))
        href, _ = O.solve_level(st, 1e-3)
        d = np.sqrt(np.maximum(np.einsum("kcii->kci", st.G), 0.0))
        tr = {"pairs": len(ts["pairs"]), "samples": int(st.n.sum()), "lambda": 1e-3}
        for name, r in ts["results"].items():
            dh = r["h"] - href
            e = np.einsum("kcd,kcde,kce->", dh, st.G, dh)
            tr[name] = {"counts_equal": bool(np.array_equal(r["n"], st.n)),
                        "gram_worst_rel": float(f"{np.max(np.abs(r['G'] - st.G) / (d[..., :, None] * d[..., None, :] + 1e-300)):.3g}"),
                        "coeff_max_abs": float(f"{np.max(np.abs(dh)):.3g}"),
                        "output_space_rel": float(f"{np.sqrt(max(e, 0.0) / st.yy.sum()):.3g}")}
        stx = O.CrossGramStats.zeros(K, C, 147)
        for p in ts["pairs"]:
            O.accumulate_level_cross(stx, p["s0"].astype(np.int64), O.to_filter_space(np.asarray(p["z"], np.float64)),
                                     O.to_filter_space(np.asarray(p["u"], np.float64)), RADIUS)
        hx, _ = O.solve_level_cross(stx, 1e-3)
        dx = np.sqrt(np.maximum(np.einsum("kii->ki", stx.G), 0.0))
        trx = {"layout": "cross-channel, D = 147 (single scale, level 0)"}
        for name, r in ts["results_cross"].items():
            dh = r["h"] - hx
            e = np.einsum("kcd,kde,kce->", dh, stx.G, dh)
            trx[name] = {"counts_equal": bool(np.array_equal(r["n"], stx.n)),
                         "gram_worst_rel": float(f"{np.max(np.abs(r['G'] - stx.G) / (dx[:, :, None] * dx[:, None, :] + 1e-300)):.3g}"),
                         "coeff_max_abs": float(f"{np.max(np.abs(dh)):.3g}"),
                         "output_space_rel": float(f"{np.sqrt(max(e, 0.0) / stx.yy.sum()):.3g}")}
        tr["cross_D147"] = trx
        acc["training"] = tr
    if c1 is not None:
        z, u, bank_dev, got = c1
        lb = bank_dev.levels[0]
        b1 = O.Bank([O.LevelBank(lb.q_theta, lb.t_s, lb.t_c, lb.radius_g, None, lb.coeffs.double().cpu().numpy())])
        ref = O.denoise(np.asarray(z, np.float64), b1, storage=np.float32)
        acc["single_level_grey"] = {"max_abs_vs_fp64_fp32_mode": float(f"{np.max(np.abs(got - ref)):.3g}"),
                                    "psnr_noisy_db": round(O.psnr(np.asarray(z, np.float64), u), 3),
                                    "psnr_gpu_db": round(O.psnr(np.asarray(got, np.float64), u), 3)}
    if c2 is not None:
        z, u, bank_dev, got, maps = c2
        b2 = host_bank(bank_dev)
        at = O.denoise(np.asarray(z, np.float64), b2, storage=np.float32, maps=maps)
        ref64 = O.denoise(np.asarray(z, np.float64), b2)
        acc["three_level_f32"] = {"max_abs_vs_fp32_mode_at_gpu_maps": float(f"{np.max(np.abs(got - at)):.3g}"),
                                  "max_abs_vs_fp64": float(f"{np.max(np.abs(got - ref64)):.3g}"),
                                  "psnr_noisy_db": round(O.psnr(np.asarray(z, np.float64), u), 3),
                                  "psnr_gpu_db": round(O.psnr(np.asarray(got, np.float64), u), 3)}
    return base, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--images", type=int, default=N_IMAGES)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true", help="run only the hardware-counter probe")
    ap.add_argument("--train-probe", action="store_true",
                    help="run only the training measurement on 64 pairs, without worker processes (for the profiler)")
    ap.add_argument("--paper-frame", type=int, default=None, metavar="SIGMA",
                    help="run only the paper-configuration frame probe at this noise level (for the profiler)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-paper-config", action="store_true")
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    args = ap.parse_args()
    if args.pmc_probe:
        pmc_probe()
        return
    if args.paper_frame is not None:
        paper_frame_probe(args.paper_frame)
        return
    if args.train_probe:
        pairs = make_train_pairs(64, pool=False)
        import torch
        import paper_1802_06130_amd as M
        print(json.dumps(run_training(M, torch, pairs)[0]), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; the library has no multi-GPU path (images are independent "
              "and would be routed to GPUs one by one).", file=sys.stderr)
        sys.exit(2)

    # every worker pool runs before the GPU is touched
    t_gen = time.perf_counter()
    sizes, imgs, clean_crops = make_inputs(args.images, np.float16)
    train_pairs = None if args.no_train else make_train_pairs()
    serve_imgs = None if args.no_serve else make_serve_images()
    quality_data = None if args.no_quality else make_quality_inputs()
    print(f"# generated {len(imgs)} images ({sum(w * h for w, h in sizes) / 1e6:.1f} MP) and the training and "
          f"serving inputs in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)

    import torch
    import paper_1802_06130_amd as M
    dev = torch.device("cuda:0")
    t_tr = time.perf_counter()
    bank32, fbs = train_bank(M, torch)
    bank16 = as_dtype(M, bank32, torch.float16)
    print(f"# trained bank on the GPU in {time.perf_counter() - t_tr:.1f}s (fallback systems {fbs})",
          file=sys.stderr, flush=True)
    zs = [torch.from_numpy(z).to(dev) for z in imgs]
    total_px = sum(z.shape[1] * z.shape[2] for z in zs)

    wall_p, lat_p, ms_steps, outs_p = run_form(M, torch, zs, bank16, M.F16, args.steps, args.warmup)
    plain = total_px * args.steps / wall_p / 1e6
    print(f"# plain per-image f16: {plain:.1f} MP/s", file=sys.stderr, flush=True)
    wall, lat_b, rows, outs_b, ktimes = run_batched(M, torch, zs, bank16, args.steps, args.warmup)
    value = total_px * args.steps / wall / 1e6
    same = all(torch.equal(a, b) for a, b in zip(outs_p, outs_b))
    print(f"# batched f16: {value:.1f} MP/s, rows {rows}, bitwise equal to plain: {same}", file=sys.stderr, flush=True)
    del outs_p, outs_b

    f32 = None
    if not args.no_f32:
        zs32 = [z.float() for z in zs]
        steps32 = max(2, args.steps // 3)
        w32, lat32, _, _ = run_form(M, torch, zs32, bank32, M.F32, steps32, 1)
        f32 = {"value": round(total_px * steps32 / w32 / 1e6, 2), "unit": "MP/s",
               "p99_ms": round(float(np.percentile(lat32, 99)), 3), "steps": steps32,
               "what": "same batch, float32 storage/filters/arithmetic (parity-grade path)"}
        del zs32

    # the dominant kernel: the batched form's level-0 filtering launch (all images, one launch)
    avg_px, avg_dur = float(total_px), ktimes[0][2] * 1e-6
    img_px, img_dur = time_level0_filter(M, torch, zs, bank16)
    flops = FLOP_PER_PX * avg_px / avg_dur / 1e12
    hbm = WALK_BYTES_PX_F16 * avg_px / avg_dur / 1e9
    lds = WALK_LDS_BYTES_PX * avg_px / avg_dur / 1e9
    tr = measured_traffic()
    copy = copy_bandwidth(torch)
    print(f"# copy kernel: {copy}", file=sys.stderr, flush=True)
    line = {
        "metric": "megapixels/s denoised (4-level RGB 7x7) + p99 latency; batched vs plain per-image",
        "value": round(value, 2),
        "unit": "MP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": f"{len(zs)} seeded RGB images, sides uniform in [480, 4032] step 8, <= 12.19 MP "
                               f"each ({total_px / 1e6:.1f} MP/step), sigma 25/255, 4-level pyramid, 7x7 upscale "
                               f"and 7x7 denoise filters, 24x3x3 buckets, float16 storage, float32 accumulation",
                   "form": "batched (one persistent launch per kernel and level, hipGraph replay, autotuned)",
                   "levels": LEVELS + 1, "buckets": Q_THETA * Q_S * Q_C, "storage": "f16"},
        "latency_ms": spread(lat_b, "batched: whole-batch device time per step (HIP events)"),
        "batched": {"value": round(value, 2), "unit": "MP/s", "tuned_rows_per_level": rows,
                    "bitwise_equal_to_plain": bool(same)},
        "plain_per_image": {"value": round(plain, 2), "unit": "MP/s",
                            "ms_per_step": round(wall_p * 1e3 / args.steps, 3),
                            "latency_ms": spread(lat_p, "per-image mdn_denoise device time (HIP events)"),
                            "step_ms_events": spread(ms_steps, "whole step, HIP events")},
        "whole_path_hbm": {"algorithmic_bytes_per_px": ALG_BYTES_F16,
                           "frac": round(value * 1e6 * ALG_BYTES_F16 / (HBM_PEAK_GBS * 1e9), 4),
                           "frac_vs_copy": round(value * 1e6 * ALG_BYTES_F16 / (copy["GBs"] * 1e9), 4)},
        "copy_kernel": copy,
        "roofline": {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(hbm / HBM_PEAK_GBS, 4),
                     "frac_vs_copy": round(hbm / copy["GBs"], 4),
                     "traffic": None if tr is None else round(tr["hbm_bytes_per_px"] * avg_px),
                     "traffic_GBs": None if tr is None else round(tr["hbm_bytes_per_px"] * avg_px / avg_dur / 1e9, 1),
                     "traffic_source": None if tr is None else
                     ("profiles/walk_level0_traffic.json: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE of this launch, "
                      "scaled by a copy kernel of known size, taken at the current walk.hip (sha256 "
                      f"{tr['walk_hip_sha256_16']}); carried from that file, not measured in this run"),
                     "kernel": "k_walk, level-0 filtering launch of the batched form (all images of the step)",
                     "algorithmic_bytes_per_launch": round(WALK_BYTES_PX_F16 * avg_px),
                     "algorithmic_bytes_per_px": WALK_BYTES_PX_F16,
                     "avg_launch_us": round(avg_dur * 1e6, 2),
                     "limiter": {
                         "unit": "lds",
                         "what": "the kernel is bound by its LDS coefficient gathers, not by HBM: the same launch "
                                 "against each unit's ceiling",
                         "lds_gather_GBs": round(lds, 1), "lds_gather_bytes_per_px": WALK_LDS_BYTES_PX,
                         "lds_random_gather_ceiling_GBs": LDS_GATHER_PEAK_GBS,
                         "lds_frac": round(lds / LDS_GATHER_PEAK_GBS, 4),
                         "dot2_TFLOPs": round(flops, 2), "dot2_peak_TFLOPs": ALU_PEAK_TFLOPS,
                         "dot2_frac": round(flops / ALU_PEAK_TFLOPS, 4),
                         "algorithmic_flop_per_px": FLOP_PER_PX,
                         "hbm_frac": round(hbm / HBM_PEAK_GBS, 4)},
                     "kernel_us_per_level": [[round(t, 1) for t in lv] for lv in ktimes],
                     "kernel_us_order": "per level 0, 1, 2: pyramid step (level l -> l+1; where the level has one column-walk bank its selection pass runs in the same launch and the selection entry is 0), selection, filtering",
                     "per_image_launch": {"mean_px": round(img_px), "avg_launch_us": round(img_dur * 1e6, 2),
                                          "TFLOP/s": round(FLOP_PER_PX * img_px / img_dur / 1e12, 2),
                                          "what": "the same kernel launched per image on the first 16 images"}},
    }
    if f32 is not None:
        line["plain_f32"] = f32
    line["single_level_grey"], c1 = run_single_level_grey(M, torch)
    line["three_level_f32"], c2 = run_three_level_f32(M, torch)
    print(f"# single level grey: {line['single_level_grey']}\n# three level f32: {line['three_level_f32']}",
          file=sys.stderr, flush=True)
    if not args.no_paper_config:
        line["paper_config_batched"] = run_paper_config_batched(M, torch, zs, max(2, args.steps // 2), 1)
        print(f"# paper configuration batched: {line['paper_config_batched']}", file=sys.stderr, flush=True)
    crops = accuracy_crops(imgs)
    gpu_crops = gpu_crop_outputs(M, torch, crops, bank16) if not args.no_cpu_baseline else None
    train_sample = None
    if not args.no_train:
        line["training"], train_sample = run_training(M, torch, train_pairs)
        del train_pairs
    del zs
    torch.cuda.empty_cache()
    if not (args.no_serve and args.no_quality):
        banks32 = [bank32 if g == SIGMA else train_bank(M, torch, sigma=g)[0] for g in SERVE_SIGMAS]
    if not args.no_serve:
        banks = [as_dtype(M, b, torch.float16) for b in banks32]
        line["served"] = run_served(M, torch, banks, (50, 200, 800), args.serve_requests, serve_imgs)
        del banks
    if not args.no_quality:
        line["quality"] = run_quality(M, torch, quality_data, banks32)
        del quality_data
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["accuracy"] = cpu_baseline_leg(crops, clean_crops, gpu_crops, bank16, bank32,
                                                                  train_sample, c1, c2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
