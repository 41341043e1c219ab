"""Serving-loop scheduler on the virtual-clock executor (no device): admission by device
footprint, slots, first-come-first-served order, continuous batching of cascade stages,
time-outs, cancellation and injected failures. Expected times follow the executor's stated cost
model (copies at a fixed bandwidth, a fixed cost per launch, stage work proportional to the
pixels of the stage's level)."""

import math

import numpy as np
import pytest
import torch

import paper_1802_06130_amd as M
from paper_1802_06130_amd import _lib as B
from synth import poisson_arrivals

H2D, D2H, GPX, LAUNCH_US = 10.0, 10.0, 1.0, 10.0     # GB/s, GB/s, Gpixel/s, microseconds
LEVELS = 4


def _bank(levels=LEVELS, q_theta=24):
    K = q_theta * 3 * 3
    lv = [M.Level(q_theta, [0.01, 0.02], [0.3, 0.6], 3, 3, torch.zeros(K, 3, 98, dtype=torch.float16), 3)
          for _ in range(levels)]
    return M.Bank(lv)


def _server(**kw):
    args = dict(storage=M.F16, max_slots=4, stages_per_tick=1, max_ticks_in_flight=2, hbm_budget=1 << 30,
                executor=M.EXEC_FAKE, fake_model=(H2D, D2H, GPX, LAUNCH_US))
    banks = kw.pop("banks", None) or [_bank()]
    args.update(kw)
    return M.Server(banks, **args)


def _req(w, h, tag=0, bank=0, dtype=M.F16):
    # the fake executor never touches host memory: any non-null addresses do
    return B.MdnRequest(0x1000, 0x2000, w, h, dtype, bank, tag)


def _bytes(w, h, dtype=M.F16):
    return w * h * 3 * (2 if dtype == M.F16 else 4)


def _cascade_time(w, h, levels=LEVELS, stages_per_tick=1):
    """Compute-engine time of one request alone under the cost model."""
    px = []
    for _ in range(levels + 1):
        px.append(w * h)
        w, h = (w + 1) // 2, (h + 1) // 2
    t = 0.0
    for l in range(levels):                          # pyramid stages with the level's selection, one launch each
        t += LAUNCH_US * 1e-6 + 0.075 * px[l] / (GPX * 1e9)
    for l in range(levels - 1, -1, -1):              # filtering, one launch each
        t += LAUNCH_US * 1e-6 + 0.675 * px[l] / (GPX * 1e9)
    return t


def _run(srv, max_wait=10.0):
    return sorted(srv.wait_all(max_wait), key=lambda c: c["tag"])


def test_single_request_timeline():
    srv = _server()
    w, h = 1000, 1000
    srv.submit_request(_req(w, h, tag=7))
    (c,) = _run(srv)
    assert c["status"] == M.MDN_OK and c["tag"] == 7
    up = _bytes(w, h) / (H2D * 1e9)
    dev = up + _cascade_time(w, h)
    assert c["t_arrival"] == 0.0 and c["t_admit"] == 0.0
    assert c["t_device_done"] == pytest.approx(dev, rel=1e-9)
    assert c["t_host_done"] == pytest.approx(dev + _bytes(w, h) / (D2H * 1e9), rel=1e-9)
    assert c["tick_last"] - c["tick_first"] == 2 * LEVELS - 1
    st = srv.stats()
    assert st["ticks"] == 2 * LEVELS and st["launches"] == 2 * LEVELS and st["tick_items"] == 2 * LEVELS
    assert st["completed"] == 1 and st["arena_used"] == 0 and st["active"] == 0


def test_footprint_matches_layout():
    srv = _server()
    w, h = 1001, 777
    fp = srv.footprint(_req(w, h))
    al = lambda v: (v + 255) // 256 * 256
    want = 2 * al(_bytes(w, h))
    for l in range(1, LEVELS + 1):
        w, h = (w + 1) // 2, (h + 1) // 2
        lvl = al((w + 63) // 64 * 64 * h * 3 * 2)
        want += lvl * (2 if l < LEVELS else 1)
    w, h = 1001, 777
    for l in range(LEVELS):                 # one uint8 selector map per trained level
        want += al(w * h)
        w, h = (w + 1) // 2, (h + 1) // 2
    assert fp == want


def test_admission_by_footprint():
    srv = _server(max_slots=8)
    fp = srv.footprint(_req(640, 480))
    srv.close()
    srv = _server(max_slots=8, hbm_budget=int(2.5 * fp))
    for i in range(6):
        srv.submit_request(_req(640, 480, tag=i))
    done = _run(srv)
    assert [c["status"] for c in done] == [M.MDN_OK] * 6
    events = sorted([(c["t_admit"], 1) for c in done] + [(c["t_host_done"], -1) for c in done],
                    key=lambda e: (e[0], e[1]))
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak == 2
    st = srv.stats()
    assert st["arena_peak"] == 2 * fp and st["arena_used"] == 0


def test_slot_limit_serialises():
    srv = _server(max_slots=1)
    for i in range(3):
        srv.submit_request(_req(300, 200, tag=i))
    done = _run(srv)
    assert all(c["slot"] == 0 for c in done)
    for a, b in zip(done, done[1:]):
        assert b["t_admit"] >= a["t_host_done"]


def test_oversize_rejected_others_proceed():
    srv = _server(hbm_budget=64 << 20)
    with pytest.raises(M.MdnError) as e:
        srv.submit_request(_req(4032, 3024, tag=1))
    assert e.value.status == M.MDN_ENOMEM
    srv.submit_request(_req(256, 256, tag=2))
    (c,) = _run(srv)
    assert c["status"] == M.MDN_OK
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 1


def test_first_come_first_served_no_overtaking():
    srv = _server(max_slots=8)
    big = srv.footprint(_req(2000, 2000))
    small = srv.footprint(_req(64, 64))
    srv.close()
    srv = _server(max_slots=8, hbm_budget=big + small + 4096)
    srv.submit_request(_req(2000, 2000, tag=0))
    srv.submit_request(_req(2000, 2000, tag=1))    # waits for memory
    srv.submit_request(_req(64, 64, tag=2))        # would fit now, but may not overtake tag 1
    done = _run(srv)
    assert done[2]["t_admit"] >= done[1]["t_admit"] >= done[0]["t_host_done"]


def test_continuous_batching_joins_mid_cascade():
    srv = _server()
    srv.submit_request(_req(2000, 2000, tag=0))
    up = _bytes(2000, 2000) / (H2D * 1e9)
    srv.poll(max_wait=up + 0.05 * _cascade_time(2000, 2000))   # request 0 is mid-cascade
    srv.submit_request(_req(200, 200, tag=1))
    done = _run(srv)
    a, b = done
    assert a["status"] == b["status"] == M.MDN_OK
    assert a["tick_first"] < b["tick_first"] <= a["tick_last"]          # joined while 0 was running
    # its stages rode in request 0's ticks: it ends a few short ticks after request 0, sooner than
    # a whole cascade of its own queued behind request 0
    assert b["t_device_done"] < a["t_device_done"] + _cascade_time(200, 200)
    st = srv.stats()
    assert st["tick_items"] > st["ticks"]                               # some ticks held both


def test_stages_per_tick_whole_cascade():
    srv = _server(stages_per_tick=2 * LEVELS)
    srv.submit_request(_req(500, 400, tag=0))
    (c,) = _run(srv)
    assert c["status"] == M.MDN_OK and c["tick_first"] == c["tick_last"]
    assert srv.stats()["launches"] == 2 * LEVELS


def test_injected_launch_failure_only_fails_that_request():
    srv = _server()
    srv.fake_inject(M.FAKE_FAIL_LAUNCH, 1)
    for i in range(4):
        srv.submit_request(_req(320, 240, tag=i))
    done = _run(srv)
    assert [c["status"] for c in done] == [M.MDN_OK, M.MDN_EDEVICE, M.MDN_OK, M.MDN_OK]
    assert done[1]["host_out"] is None
    st = srv.stats()
    assert st["failed"] == 1 and st["completed"] == 3 and st["arena_used"] == 0


def test_injected_tick_failure_fails_its_tick_then_recovers():
    srv = _server()
    srv.submit_request(_req(320, 240, tag=0))
    assert _run(srv)[0]["status"] == M.MDN_OK
    srv.fake_inject(M.FAKE_FAIL_TICK, 2)
    srv.submit_request(_req(320, 240, tag=2))
    srv.submit_request(_req(320, 240, tag=3))
    done = _run(srv)
    assert done[0]["status"] == M.MDN_EDEVICE
    # tag 3 shared the failing tick only if it was already active; either way it completes
    assert done[1]["status"] in (M.MDN_OK, M.MDN_EDEVICE)
    srv.submit_request(_req(320, 240, tag=4))
    assert _run(srv)[0]["status"] == M.MDN_OK
    assert srv.stats()["arena_used"] == 0


def test_injected_copy_failures():
    srv = _server()
    srv.fake_inject(M.FAKE_FAIL_UPLOAD, 5)
    srv.fake_inject(M.FAKE_FAIL_DOWNLOAD, 6)
    for t in (5, 6, 7):
        srv.submit_request(_req(128, 96, tag=t))
    done = _run(srv)
    assert [c["status"] for c in done] == [M.MDN_EDEVICE, M.MDN_EDEVICE, M.MDN_OK]
    assert done[0]["tick_first"] == -1                 # never reached the device
    assert srv.stats()["arena_used"] == 0


def test_queue_timeout():
    srv = _server(max_slots=1, queue_timeout=1e-3)
    srv.fake_inject(M.FAKE_STALL, 0, 10e-3)
    srv.submit_request(_req(128, 128, tag=0))
    srv.submit_request(_req(128, 128, tag=1))
    done = _run(srv)
    assert done[0]["status"] == M.MDN_OK
    assert done[1]["status"] == M.MDN_ETIMEOUT and done[1]["t_admit"] < 0 and done[1]["slot"] == -1


def test_cancel_waiting_and_running():
    srv = _server(max_slots=1)
    ids = [srv.submit_request(_req(1500, 1500, tag=i)) for i in range(3)]
    srv.cancel(ids[2])
    got = srv.poll(0.0)
    assert [c["tag"] for c in got] == [2] and got[0]["status"] == M.MDN_ECANCELED and got[0]["t_admit"] < 0
    up = _bytes(1500, 1500) / (H2D * 1e9)
    srv.poll(max_wait=up + 0.02 * _cascade_time(1500, 1500))
    srv.cancel(ids[0])
    done = _run(srv)
    assert [(c["tag"], c["status"]) for c in done] == [(0, M.MDN_ECANCELED), (1, M.MDN_OK)]
    assert 0 <= done[0]["tick_last"] - done[0]["tick_first"] < 2 * LEVELS - 1
    assert srv.stats()["arena_used"] == 0


def test_bad_configurations():
    with pytest.raises(M.MdnError):
        _server(max_slots=0)
    with pytest.raises(M.MdnError):
        _server(stages_per_tick=0)
    with pytest.raises(M.MdnError):
        _server(max_ticks_in_flight=9)
    lv = M.Level(24, [0.01, 0.02], [0.3, 0.6], 3, 3, torch.zeros(216, 3, 98, dtype=torch.float32), 3)
    with pytest.raises(M.MdnError) as e:
        _server(banks=[M.Bank([lv])])
    assert e.value.status == M.MDN_ENOTSUP
    # float16 7x7/7x7 levels that select on the coarser output, and banks that run the LDS-bank kernel
    # per image (this phase-aware bank of 216 buckets), are refused
    co = torch.zeros(216, 3, 98, dtype=torch.float16)
    for lvx in (M.Level(24, [0.01, 0.02], [0.3, 0.6], 3, 3, co, 3, M.SELECT_COARSE),
                M.Level(6, [0.01, 0.02], [0.3, 0.6], 3, 3, co, 3, M.SELECT_RGB, 4)):
        with pytest.raises(M.MdnError) as e:
            _server(banks=[M.Bank([lvx] * LEVELS)])
        assert e.value.status == M.MDN_ENOTSUP
    srv = _server()
    with pytest.raises(M.MdnError):
        srv.submit_request(_req(64, 64, bank=3))
    with pytest.raises(M.MdnError):
        srv.submit_request(B.MdnRequest(0x1000, None, 64, 64, M.F16, 0, 0))   # no host_out, no staging
    srv.close()
    srv = _server(storage=M.F32)
    with pytest.raises(M.MdnError) as e:
        srv.submit_request(_req(64, 64, dtype=M.F16))
    assert e.value.status == M.MDN_ENOTSUP


def test_tiled_bank_levels_take_one_launch_each():
    """Levels of the tiled kernel (the paper's 16 x 16 x 16 buckets, 7x7 / 5x5 filters) select inline:
    a request alone takes L pyramid launches and L filtering launches, no selection launch."""
    lv = M.Level(16, list(np.linspace(0.01, 0.2, 15)), list(np.linspace(0.05, 0.9, 15)), 3, 2,
                 torch.zeros(4096, 3, 74, dtype=torch.float16), 3)
    srv = _server(banks=[M.Bank([lv] * LEVELS)])
    srv.submit_request(_req(640, 480))
    (c,) = _run(srv)
    assert c["status"] == M.MDN_OK
    assert srv.stats()["launches"] == 2 * LEVELS
    srv.close()


SIZES = [(1280, 720), (1920, 1080), (4032, 3024)]


def _trace(seed, rate, n):
    rng = np.random.default_rng(seed)
    arr = poisson_arrivals(rate, n, seed)
    size = rng.integers(0, 3, n)
    bank = rng.integers(0, 3, n)
    reqs = [_req(*SIZES[s], tag=100 + i, bank=int(b)) for i, (s, b) in enumerate(zip(size, bank))]
    return reqs, arr, size


def test_replay_open_loop_trace():
    srv = _server(banks=[_bank(), _bank(), _bank()], max_slots=16, hbm_budget=4 << 30,
                  fake_model=(25.0, 25.0, 20.0, 5.0))
    reqs, arr, size = _trace(5000 + 200, 200.0, 400)
    done = srv.replay(reqs, arr)
    assert all(c["status"] == M.MDN_OK for c in done)
    assert [c["tag"] for c in done] == [r.tag for r in reqs]
    lat = np.array([c["t_host_done"] - c["t_arrival"] for c in done])
    assert np.all(lat > 0)
    for c, a in zip(done, arr):
        assert c["t_arrival"] == pytest.approx(a)
        assert c["t_arrival"] <= c["t_admit"] <= c["t_device_done"] <= c["t_host_done"]
    st = srv.stats()
    assert st["completed"] == 400 and st["arena_used"] == 0 and st["arena_peak"] <= 4 << 30
    # at a light load most requests see no queueing: the median is near the alone latency
    srv.close()
    srv = _server(banks=[_bank(), _bank(), _bank()], max_slots=16, hbm_budget=4 << 30,
                  fake_model=(25.0, 25.0, 20.0, 5.0))
    reqs, arr, size = _trace(5000 + 5, 5.0, 60)
    done = srv.replay(reqs, arr)
    alone = {}
    for s, (w, h) in enumerate(SIZES):
        alone[s] = 2 * _bytes(w, h) / 25e9
    lat = np.array([c["t_host_done"] - c["t_arrival"] for c in done])
    ratio = lat / np.array([alone[s] for s in size])
    assert np.median(ratio) < 1.5


def test_replay_needs_idle_server_and_sorted_arrivals():
    srv = _server()
    reqs = [_req(64, 64, tag=i) for i in range(3)]
    with pytest.raises(M.MdnError):
        srv.replay(reqs, [0.0, 0.2, 0.1])
    srv.submit_request(_req(64, 64))
    with pytest.raises(M.MdnError):
        srv.replay(reqs, [0.0, 0.1, 0.2])


def test_staging_slot_lent_until_next_poll():
    srv = _server(max_slots=1, staging_bytes=1 << 20)
    srv.submit_request(B.MdnRequest(0x1000, None, 64, 64, M.F16, 0, 0))
    srv.submit_request(B.MdnRequest(0x1000, None, 64, 64, M.F16, 0, 1))
    first = srv.poll(10.0)
    assert [c["tag"] for c in first] == [0]
    assert srv.stats()["active"] == 0          # the slot is still lent: request 1 is not admitted yet
    second = srv.wait_all()
    assert [c["tag"] for c in second] == [1]
    assert second[0]["t_admit"] >= first[0]["t_host_done"]
