// Serving loop: requests of any sizes, each naming one of several on-device banks (one per
// noise level, the level being known), arrive over time. A request is admitted once a slot is free
// and its device-memory footprint (input, output, pyramid and selector map) fits the budget;
// admission is first come, first served, with no overtaking. The input is copied to the device on
// a copy stream; once it is there the request joins the next scheduling tick. A tick advances
// every active request by one or more cascade stages (pyramid levels 0..L-1, then selection and
// filtering of levels L-1..0) with one persistent launch per kernel, level, bank and dtype over
// all requests at that point, so requests that arrive while others are mid-cascade share the
// next launches with them. Ticks are queued on one compute stream, a bounded number ahead of the
// device; the copy back (second copy stream) waits on the tick that ran the request's last stage.
//
// Every result is produced by the same per-pixel arithmetic as the plain and batched forms (no
// atomics, no dependence on batch position), so a request's output does not depend on what it
// was batched with.
//
// Device work goes through an executor interface: a HIP executor (three streams, an event per
// enqueued piece of work, one device allocation for the whole budget), or a virtual-clock executor with a simple cost model that runs on any host and lets the scheduler's admission,
// ordering, time-outs, cancellation and failure handling be exercised without a device.

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "walk_types.h"

using namespace mdn;

namespace {

constexpr int kMaxBanks = 16;
constexpr int kMaxSlots = 256;

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

using Token = int64_t;   // executor handle of an enqueued piece of work (0: none)

// ---------------------------------------------------------------- device-memory arena
// First fit over byte offsets; freed ranges merge with their neighbours.
class Arena {
public:
    void reset(size_t cap) {
        cap_ = cap;
        used_ = peak_ = 0;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, after = it->first + n;
            free_.erase(it);
            if (rest) free_[after] = rest;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
        used_ -= n;
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

enum State { QUEUED, UPLOADING, ACTIVE, DOWNLOADING };

struct Bank {
    int L;
    mdn_level lv[kMaxLevels];
    double thr[kMaxLevels][2][kMaxThr];
    SelWalkArgs selc[kMaxLevels];
    bool tiled[kMaxLevels];    // level filtered by the tiled kernel (selection inline, one launch)
};

struct Request {
    uint64_t id = 0;
    mdn_request q;
    State state = QUEUED;
    int L = 0;
    int status = MDN_OK;
    bool cancel = false, failed = false;
    int slot = -1;
    size_t off = 0, bytes = 0, in_bytes = 0, out_bytes = 0;
    int stage = 0;             // next cascade stage to issue (0 .. 2L)
    int in_ticks = 0;          // ticks in flight that hold a stage of this request
    Token up = 0, down = 0;
    int tick_first = -1, tick_last = -1;
    double t_arrival = 0, t_admit = -1, t_device_done = -1, t_host_done = -1;
    void* host_out = nullptr;  // destination of the copy back
    // device descriptors of the cascade (HIP executor)
    D2Image d2[kMaxLevels];
    SelImage sel[kMaxLevels];
    WalkImage walk[kMaxLevels];
    TileImage tile[kMaxLevels];
    int64_t px[kMaxLevels + 1];
};

// One cascade stage of one request, with its position among that request's stages in the tick.
struct Item {
    Request* r;
    int stage;
    int round;
};

int level_dtype(const Request& r, int level, int storage) { return level == 0 ? r.q.dtype : storage; }

// Launch groups of one round: stages that can share a launch (same kernel, level, bank, dtypes).
struct GroupKey {
    int kind, bank, level, zd, od;
    bool operator<(const GroupKey& o) const {
        return std::tie(kind, bank, level, zd, od) < std::tie(o.kind, o.bank, o.level, o.zd, o.od);
    }
};

// Levels of a tiled bank level have no selection launch: the tiled kernel selects inline. The
// selection pass of a column-walk level runs in the launch of that level's pyramid step (kind 3,
// one launch per bank and level), long before the level's filtering stage.
bool selects_with_pyramid(const Bank& bk, int l) { return !bk.tiled[l] && pyr_sel_fusable(bk.selc[l]); }

template <typename F>
void for_each_group(const std::vector<Item>& items, int round, int storage, const Bank* banks, F&& f) {
    std::map<GroupKey, std::vector<const Item*>> g;
    for (const Item& it : items) {
        if (it.round != round) continue;
        const Request& r = *it.r;
        const int L = r.L;
        const Bank& bk = banks[r.q.bank];
        if (it.stage < L) {
            const int l = it.stage;
            if (selects_with_pyramid(bk, l)) g[{3, r.q.bank, l, level_dtype(r, l, storage), storage}].push_back(&it);
            else g[{0, 0, 0, level_dtype(r, l, storage), storage}].push_back(&it);
        } else {
            const int l = 2 * L - 1 - it.stage;
            if (!bk.tiled[l] && !selects_with_pyramid(bk, l))
                g[{1, r.q.bank, l, level_dtype(r, l, storage), 0}].push_back(&it);
            g[{2, r.q.bank, l, level_dtype(r, l, storage), level_dtype(r, l, storage)}].push_back(&it);
        }
    }
    // kind 0 (pyramid) < 1 (selection) < 2 (filtering) < 3 (pyramid with selection); the groups of a
    // round hold different requests, so their order does not matter
    for (auto& kv : g) f(kv.first, kv.second);
}

// ---------------------------------------------------------------- executors
class Executor {
public:
    virtual ~Executor() = default;
    virtual mdn_status init(const mdn_server_config& c, const Bank* banks) = 0;
    virtual double now() = 0;
    virtual void prepare(Request& r) = 0;                        // after admission: device addresses
    virtual void* staging(int slot) = 0;
    virtual mdn_status upload(Request& r, Token* t) = 0;
    // Enqueue the stages; items whose launch failed get their request marked failed.
    virtual mdn_status tick(const std::vector<Item>& items, int rounds, uint64_t seq, Token* t, int* launches) = 0;
    virtual mdn_status download(Request& r, Token after, Token* t) = 0;
    virtual int query(Token t) = 0;                               // 1 done, 0 pending, -1 failed
    virtual void release(Token t) = 0;
    virtual void drain() = 0;
};

class HipExecutor final : public Executor {
public:
    ~HipExecutor() override {
        drain();
        for (hipEvent_t e : events_) hipEventDestroy(e);
        for (int i = 0; i < (int)tab_host_.size(); ++i) {
            if (tab_host_[i]) hipHostFree(tab_host_[i]);
            if (tab_dev_[i]) hipFree(tab_dev_[i]);
        }
        for (void* p : staging_) hipHostFree(p);
        if (arena_) hipFree(arena_);
        for (hipStream_t s : {h2d_, d2h_, comp_})
            if (s) hipStreamDestroy(s);
    }

    mdn_status init(const mdn_server_config& c, const Bank* banks) override {
        banks_ = banks;
        storage_ = c.storage;
        t0_ = std::chrono::steady_clock::now();
        mdn_status st = init_walk_kernels();
        if (st) return st;
        ncu_ = device_cus();
        if (hipStreamCreateWithFlags(&h2d_, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&d2h_, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&comp_, hipStreamNonBlocking) != hipSuccess)
            return fail(MDN_EDEVICE, "server: stream creation failed");
        if (hipMalloc((void**)&arena_, c.hbm_budget) != hipSuccess)
            return fail(MDN_ENOMEM, "server: cannot allocate the %llu-byte device budget",
                        (unsigned long long)c.hbm_budget);
        // one table region per tick that can be in flight, plus one being filled
        const size_t items = (size_t)c.max_slots * c.stages_per_tick;
        tab_cap_ = items * (sizeof(D2Image) + sizeof(SelImage) + sizeof(WalkImage) + sizeof(TileImage)) +
                   3 * 256 * (items + 4);
        const int ring = c.max_ticks_in_flight + 1;
        tab_host_.assign(ring, nullptr);
        tab_dev_.assign(ring, nullptr);
        for (int i = 0; i < ring; ++i)
            if (hipHostMalloc((void**)&tab_host_[i], tab_cap_, hipHostMallocDefault) != hipSuccess ||
                hipMalloc((void**)&tab_dev_[i], tab_cap_) != hipSuccess)
                return fail(MDN_ENOMEM, "server: table allocation failed");
        if (c.staging_bytes) {
            staging_.assign(c.max_slots, nullptr);
            for (int i = 0; i < c.max_slots; ++i)
                if (hipHostMalloc(&staging_[i], c.staging_bytes, hipHostMallocDefault) != hipSuccess)
                    return fail(MDN_ENOMEM, "server: pinned staging allocation failed");
        }
        return MDN_OK;
    }

    double now() override {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
    }

    void prepare(Request& r) override {
        char* in = arena_ + r.off;
        char* out = in + al256(r.in_bytes);
        char* ws = out + al256(r.out_bytes);
        mdn_image a, b;
        memset(&a, 0, sizeof(a));
        a.data = in;
        a.width = r.q.width;
        a.height = r.q.height;
        a.channels = 3;
        a.dtype = r.q.dtype;
        a.color = MDN_RGB;
        a.row_pitch = r.q.width;
        a.plane_pitch = (int64_t)r.q.width * r.q.height;
        b = a;
        b.data = out;
        describe_cascade(a, b, ws, r.L, storage_, nullptr, ncu_, r.d2, r.sel, r.walk, r.tile);
    }

    void* staging(int slot) override { return staging_.empty() ? nullptr : staging_[slot]; }

    mdn_status upload(Request& r, Token* t) override {
        if (hipMemcpyAsync(arena_ + r.off, r.q.host_in, r.in_bytes, hipMemcpyHostToDevice, h2d_) != hipSuccess)
            return fail(MDN_EDEVICE, "server: upload failed");
        return record(h2d_, t);
    }

    mdn_status tick(const std::vector<Item>& items, int rounds, uint64_t seq, Token* t, int* launches) override {
        char* th = tab_host_[seq % tab_host_.size()];
        char* td = tab_dev_[seq % tab_dev_.size()];
        size_t used = 0;
        struct Launch {
            GroupKey k;
            size_t off;
            int n, strips;
            std::vector<Request*> reqs;
            size_t off2 = 0;      // kind 3: the selection table after the pyramid table
            int strips2 = 0;
        };
        std::vector<Launch> ls;
        for (int round = 0; round < rounds; ++round) {
            for_each_group(items, round, storage_, banks_, [&](const GroupKey& k, const std::vector<const Item*>& its) {
                Launch L{k, used, (int)its.size(), 0, {}, 0, 0};
                int begin = 0;
                auto put = [&](const void* d, size_t n) {
                    if (used + n <= tab_cap_) memcpy(th + used, d, n);
                    used += n;
                };
                for (const Item* it : its) {
                    const Request& r = *it->r;
                    const int l = (k.kind == 0 || k.kind == 3) ? it->stage : 2 * r.L - 1 - it->stage;
                    if (k.kind == 0 || k.kind == 3) {
                        D2Image d = r.d2[l];
                        d.strip_begin = begin;
                        begin += strips_of(d);
                        put(&d, sizeof(d));
                    } else if (k.kind == 1) {
                        SelImage d = r.sel[l];
                        d.strip_begin = begin;
                        begin += strips_of(d);
                        put(&d, sizeof(d));
                    } else if (banks_[k.bank].tiled[l]) {
                        TileImage d = r.tile[l];
                        d.tile_begin = begin;
                        begin += tiles_of(d);
                        put(&d, sizeof(d));
                    } else {
                        WalkImage d = r.walk[l];
                        d.strip_begin = begin;
                        begin += strips_of(d);
                        put(&d, sizeof(d));
                    }
                    L.reqs.push_back(it->r);
                }
                L.strips = begin;
                used = al256(used);
                if (k.kind == 3) {
                    L.off2 = used;
                    begin = 0;
                    for (const Item* it : its) {
                        SelImage d = it->r->sel[it->stage];
                        d.strip_begin = begin;
                        begin += strips_of(d);
                        put(&d, sizeof(d));
                    }
                    L.strips2 = begin;
                    used = al256(used);
                }
                ls.push_back(std::move(L));
            });
        }
        if (used > tab_cap_) return fail(MDN_ENOMEM, "server: tick tables exceed their buffer");
        if (used && hipMemcpyAsync(td, th, used, hipMemcpyHostToDevice, comp_) != hipSuccess)
            return fail(MDN_EDEVICE, "server: table upload failed");
        for (const Launch& L : ls) {
            mdn_status st = MDN_OK;
            const Bank& bk = banks_[L.k.bank];
            if (L.k.kind == 0) {
                D2Args a;
                memset(&a, 0, sizeof(a));
                a.imgs = reinterpret_cast<const D2Image*>(td + L.off);
                a.n_imgs = L.n;
                a.n_strips = L.strips;
                st = launch_down2_args(a, 3, L.k.zd, storage_, comp_);
            } else if (L.k.kind == 3) {
                D2Args a;
                memset(&a, 0, sizeof(a));
                a.imgs = reinterpret_cast<const D2Image*>(td + L.off);
                a.n_imgs = L.n;
                a.n_strips = L.strips;
                SelWalkArgs sa = bk.selc[L.k.level];
                sa.imgs = reinterpret_cast<const SelImage*>(td + L.off2);
                sa.n_imgs = L.n;
                sa.n_strips = L.strips2;
                st = launch_pyr_sel_args(a, sa, L.k.zd, storage_, comp_);
            } else if (L.k.kind == 1) {
                SelWalkArgs a = bk.selc[L.k.level];
                a.imgs = reinterpret_cast<const SelImage*>(td + L.off);
                a.n_imgs = L.n;
                a.n_strips = L.strips;
                st = launch_select_args(a, 3, L.k.zd, comp_);
            } else if (bk.tiled[L.k.level]) {
                const int l = L.k.level;
                st = launch_select_apply_table(bk.lv[l], reinterpret_cast<const TileImage*>(td + L.off), L.n, L.strips, 3,
                                               L.k.zd, storage_, l == bk.L - 1 ? MDN_RGB : MDN_YCC, L.k.od,
                                               l == 0 ? MDN_RGB : MDN_YCC, comp_);
            } else {
                const mdn_level& lv = bk.lv[L.k.level];
                WalkArgs a;
                memset(&a, 0, sizeof(a));
                a.imgs = reinterpret_cast<const WalkImage*>(td + L.off);
                a.n_imgs = L.n;
                a.n_strips = L.strips;
                a.coeffs = lv.coeffs;
                a.coeff_dtype = lv.coeff_dtype;
                a.K = level_buckets(lv);
                st = launch_walk_args(a, L.k.zd, storage_, L.k.od, comp_);
            }
            if (st)
                for (Request* r : L.reqs) {
                    r->failed = true;
                    r->status = MDN_EDEVICE;
                }
        }
        *launches = (int)ls.size();
        return record(comp_, t);
    }

    mdn_status download(Request& r, Token after, Token* t) override {
        if (hipStreamWaitEvent(d2h_, events_[after - 1], 0) != hipSuccess)
            return fail(MDN_EDEVICE, "server: stream ordering failed");
        char* out = arena_ + r.off + al256(r.in_bytes);
        if (hipMemcpyAsync(r.host_out, out, r.out_bytes, hipMemcpyDeviceToHost, d2h_) != hipSuccess)
            return fail(MDN_EDEVICE, "server: download failed");
        return record(d2h_, t);
    }

    int query(Token t) override {
        const hipError_t e = hipEventQuery(events_[t - 1]);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        return -1;
    }

    void release(Token t) override {
        if (t > 0) free_events_.push_back(t);
    }

    void drain() override {
        for (hipStream_t s : {h2d_, comp_, d2h_})
            if (s) hipStreamSynchronize(s);
    }

private:
    mdn_status record(hipStream_t s, Token* t) {
        Token k;
        if (!free_events_.empty()) {
            k = free_events_.back();
            free_events_.pop_back();
        } else {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return fail(MDN_EDEVICE, "server: event creation failed");
            events_.push_back(e);
            k = (Token)events_.size();
        }
        if (hipEventRecord(events_[k - 1], s) != hipSuccess) {
            free_events_.push_back(k);
            return fail(MDN_EDEVICE, "server: event record failed");
        }
        *t = k;
        return MDN_OK;
    }

    const Bank* banks_ = nullptr;
    int storage_ = MDN_F16;
    int ncu_ = 256;
    std::chrono::steady_clock::time_point t0_;
    hipStream_t h2d_ = nullptr, d2h_ = nullptr, comp_ = nullptr;
    char* arena_ = nullptr;
    size_t tab_cap_ = 0;
    std::vector<char*> tab_host_, tab_dev_;
    std::vector<void*> staging_;
    std::vector<hipEvent_t> events_;
    std::vector<Token> free_events_;
};

// Virtual clock; three in-order engines (host-to-device copy, compute, device-to-host copy). A
// copy takes bytes / bandwidth; a tick takes fake_launch_us per launch plus, per stage, the
// pixels of its level over the pixel rate, weighted so that a whole cascade of P pixels costs
// about P / rate (pyramid stages 0.075, selection and filtering 0.675 of their level's pixels).
class FakeExecutor final : public Executor {
public:
    mdn_status init(const mdn_server_config& c, const Bank* banks) override {
        banks_ = banks;
        storage_ = c.storage;
        h2d_ = c.fake_h2d_gbps > 0 ? c.fake_h2d_gbps * 1e9 : 25e9;
        d2h_ = c.fake_d2h_gbps > 0 ? c.fake_d2h_gbps * 1e9 : 25e9;
        rate_ = c.fake_gpx_per_s > 0 ? c.fake_gpx_per_s * 1e9 : 20e9;
        launch_ = c.fake_launch_us >= 0 ? c.fake_launch_us * 1e-6 : 5e-6;
        return MDN_OK;
    }
    double now() override { return clock_; }
    void prepare(Request&) override {}
    void* staging(int) override { return nullptr; }

    mdn_status upload(Request& r, Token* t) override {
        if (fail_upload_.count(r.q.tag)) return fail(MDN_EDEVICE, "server: injected upload failure");
        const double start = std::max(clock_, h2d_free_);
        h2d_free_ = start + (double)r.in_bytes / h2d_;
        *t = add(h2d_free_, false);
        return MDN_OK;
    }

    mdn_status tick(const std::vector<Item>& items, int rounds, uint64_t, Token* t, int* launches) override {
        int n = 0;
        double work = 0.0, stall = 0.0;
        bool async_fail = false;
        for (int round = 0; round < rounds; ++round)
            for_each_group(items, round, storage_, banks_, [&](const GroupKey&, const std::vector<const Item*>& its) {
                ++n;
                for (const Item* it : its) {
                    Request& r = *it->r;
                    if (fail_launch_.count(r.q.tag)) {
                        r.failed = true;
                        r.status = MDN_EDEVICE;
                    }
                }
            });
        for (const Item& it : items) {
            const Request& r = *it.r;
            const int L = r.L;
            const int l = it.stage < L ? it.stage : 2 * L - 1 - it.stage;
            work += (double)r.px[l] * (it.stage < L ? 0.075 : 0.675);
            auto s = stall_.find(r.q.tag);
            if (s != stall_.end()) {
                stall += s->second;
                stall_.erase(s);
            }
            if (fail_async_.count(r.q.tag)) async_fail = true;
        }
        const double start = std::max(clock_, comp_free_);
        comp_free_ = start + n * launch_ + work / rate_ + stall;
        *t = add(comp_free_, async_fail);
        *launches = n;
        return MDN_OK;
    }

    mdn_status download(Request& r, Token after, Token* t) override {
        const double start = std::max({clock_, d2h_free_, toks_[after].done});
        d2h_free_ = start + (double)r.out_bytes / d2h_;
        *t = add(d2h_free_, fail_download_.count(r.q.tag) > 0);
        return MDN_OK;
    }

    int query(Token t) override {
        const Tok& k = toks_.at(t);
        if (k.done > clock_) return 0;
        return k.fail ? -1 : 1;
    }
    void release(Token t) override { toks_.erase(t); }
    void drain() override {}

    void advance(double t) { clock_ = std::max(clock_, t); }
    // earliest completion still ahead of the clock (infinity if none)
    double next_event() const {
        double t = INFINITY;
        for (auto& kv : toks_)
            if (kv.second.done > clock_) t = std::min(t, kv.second.done);
        return t;
    }
    void inject(int what, uint64_t tag, double value) {
        switch (what) {
            case MDN_FAKE_FAIL_UPLOAD: fail_upload_[tag] = 1; break;
            case MDN_FAKE_FAIL_LAUNCH: fail_launch_[tag] = 1; break;
            case MDN_FAKE_FAIL_TICK: fail_async_[tag] = 1; break;
            case MDN_FAKE_FAIL_DOWNLOAD: fail_download_[tag] = 1; break;
            case MDN_FAKE_STALL: stall_[tag] = value; break;
            default: break;
        }
    }

private:
    struct Tok {
        double done;
        bool fail;
    };
    Token add(double done, bool f) {
        toks_[next_] = Tok{done, f};
        return next_++;
    }
    const Bank* banks_ = nullptr;
    int storage_ = MDN_F16;
    double h2d_ = 0, d2h_ = 0, rate_ = 0, launch_ = 0;
    double clock_ = 0, h2d_free_ = 0, d2h_free_ = 0, comp_free_ = 0;
    std::unordered_map<Token, Tok> toks_;
    Token next_ = 1;
    std::unordered_map<uint64_t, int> fail_upload_, fail_launch_, fail_async_, fail_download_;
    std::unordered_map<uint64_t, double> stall_;
};

struct Tick {
    uint64_t seq;
    Token tok;
    std::vector<uint64_t> ids;        // requests with a stage in this tick
    std::vector<uint64_t> finishing;  // requests whose last stage is in this tick
};

}  // namespace

struct mdn_server {
    mdn_server_config cfg;
    Bank banks[kMaxBanks];
    std::unique_ptr<Executor> ex;
    FakeExecutor* fake = nullptr;
    Arena arena;

    std::mutex inbox_mu;                       // submit and cancel may come from other threads
    std::vector<std::unique_ptr<Request>> inbox;
    std::vector<uint64_t> cancels;
    std::atomic<uint64_t> next_id{1};

    std::unordered_map<uint64_t, std::unique_ptr<Request>> live;
    std::deque<Request*> queue;                // waiting for admission, in arrival order
    std::vector<Request*> admitted;            // uploading, active or downloading
    std::deque<Tick> ticks;                    // in flight, in issue order
    std::vector<int> free_slots;
    // completions not yet returned; a slot whose staging buffer holds a result is lent to the
    // caller until the poll after the one that returned it
    std::deque<std::pair<mdn_completion, bool>> done;
    std::vector<int> lent;
    uint64_t tick_seq = 0;
    mdn_server_counters st{};
};

namespace {

mdn_status check_request(mdn_server* s, const mdn_request* q) {
    if (!q) return fail(MDN_EINVAL, "server: null request");
    if (q->width < 1 || q->height < 1) return fail(MDN_EINVAL, "server: sizes must be positive");
    if (q->dtype != MDN_F16 && q->dtype != MDN_F32) return fail(MDN_EINVAL, "server: unknown dtype");
    if (q->dtype == MDN_F16 && s->cfg.storage != MDN_F16)
        return fail(MDN_ENOTSUP, "server: float16 requests need float16 storage");
    if (q->bank < 0 || q->bank >= s->cfg.n_banks) return fail(MDN_EINVAL, "server: bank %d out of range", q->bank);
    if (!q->host_in) return fail(MDN_EINVAL, "server: null host_in");
    if ((int64_t)q->width * q->height * 3 > 0x7fffffffLL) return fail(MDN_ENOTSUP, "server: image exceeds 2^31 elements");
    const size_t ob = (size_t)q->width * q->height * 3 * (q->dtype == MDN_F16 ? 2 : 4);
    if (!q->host_out && ob > s->cfg.staging_bytes)
        return fail(MDN_EINVAL, "server: no host_out and the output exceeds the staging buffer");
    return MDN_OK;
}

size_t footprint(const Request& r, int storage) {
    return al256(r.in_bytes) + al256(r.out_bytes) + batch_image_ws(r.q.width, r.q.height, r.L, storage);
}

void complete(mdn_server* s, Request* r, int status) {
    mdn_completion c;
    memset(&c, 0, sizeof(c));
    c.id = r->id;
    c.tag = r->q.tag;
    c.status = status;
    c.slot = r->slot;
    c.tick_first = r->tick_first;
    c.tick_last = r->tick_last;
    c.t_arrival = r->t_arrival;
    c.t_admit = r->t_admit;
    c.t_device_done = r->t_device_done;
    c.t_host_done = r->t_host_done;
    c.host_out = status == MDN_OK ? r->host_out : nullptr;
    const bool staged = r->slot >= 0 && !r->q.host_out;
    s->done.push_back({c, staged});
    if (r->slot >= 0) {
        if (!staged) s->free_slots.push_back(r->slot);
        s->arena.release(r->off, r->bytes);
    }
    s->ex->release(r->up);
    s->ex->release(r->down);
    if (status == MDN_OK) ++s->st.completed;
    else ++s->st.failed;
    s->admitted.erase(std::remove(s->admitted.begin(), s->admitted.end(), r), s->admitted.end());
    s->live.erase(r->id);
}

Request* find(mdn_server* s, uint64_t id) {
    auto it = s->live.find(id);
    return it == s->live.end() ? nullptr : it->second.get();
}

// One pass over the schedule at the executor's current time; returns whether anything changed.
bool step(mdn_server* s) {
    bool changed = false;
    const double now = s->ex->now();
    {
        std::lock_guard<std::mutex> g(s->inbox_mu);
        for (auto& p : s->inbox) {
            s->queue.push_back(p.get());
            s->live.emplace(p->id, std::move(p));
            changed = true;
        }
        s->inbox.clear();
        for (uint64_t id : s->cancels)
            if (Request* r = find(s, id)) r->cancel = true;
        s->cancels.clear();
    }
    // waiting requests: cancellation and time-out
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request* r = *it;
        const bool late = s->cfg.queue_timeout > 0 && now - r->t_arrival >= s->cfg.queue_timeout;
        if (r->cancel || late) {
            it = s->queue.erase(it);
            complete(s, r, r->cancel ? MDN_ECANCELED : MDN_ETIMEOUT);
            changed = true;
        } else {
            ++it;
        }
    }
    // retire ticks in issue order
    while (!s->ticks.empty()) {
        Tick& t = s->ticks.front();
        const int q = s->ex->query(t.tok);
        if (q == 0) break;
        for (uint64_t id : t.ids)
            if (Request* r = find(s, id)) {
                --r->in_ticks;
                if (q < 0 && !r->failed) {
                    r->failed = true;
                    r->status = MDN_EDEVICE;
                }
            }
        for (uint64_t id : t.finishing)
            if (Request* r = find(s, id))
                if (r->t_device_done < 0) r->t_device_done = now;
        s->ex->release(t.tok);
        s->ticks.pop_front();
        changed = true;
    }
    // copies
    for (size_t i = 0; i < s->admitted.size();) {
        Request* r = s->admitted[i];
        if (r->state == UPLOADING) {
            const int q = s->ex->query(r->up);
            if (q != 0) {
                r->state = ACTIVE;
                if (q < 0) {
                    r->failed = true;
                    r->status = MDN_EDEVICE;
                }
                changed = true;
            }
        } else if (r->state == DOWNLOADING && r->in_ticks == 0) {
            const int q = s->ex->query(r->down);
            if (q != 0) {
                if (r->t_device_done < 0) r->t_device_done = now;
                r->t_host_done = now;
                complete(s, r, q > 0 && !r->failed ? MDN_OK : (r->failed ? r->status : MDN_EDEVICE));
                changed = true;
                continue;
            }
        }
        // failed or cancelled mid-cascade: finish once no work of it is in flight
        if ((r->failed || r->cancel) && r->state == ACTIVE && r->in_ticks == 0) {
            complete(s, r, r->failed ? r->status : MDN_ECANCELED);
            changed = true;
            continue;
        }
        ++i;
    }
    // admission: first come, first served, no overtaking
    while (!s->queue.empty() && !s->free_slots.empty()) {
        Request* r = s->queue.front();
        size_t off;
        if (!s->arena.alloc(r->bytes, &off)) break;
        s->queue.pop_front();
        r->off = off;
        r->slot = s->free_slots.back();
        s->free_slots.pop_back();
        r->t_admit = now;
        r->host_out = r->q.host_out ? r->q.host_out : s->ex->staging(r->slot);
        s->ex->prepare(*r);
        s->admitted.push_back(r);
        r->state = UPLOADING;
        ++s->st.admitted;
        if (s->ex->upload(*r, &r->up)) {
            r->state = ACTIVE;
            r->failed = true;
            r->status = MDN_EDEVICE;
        }
        changed = true;
    }
    // one tick: every active request advances by up to stages_per_tick stages
    if ((int)s->ticks.size() < s->cfg.max_ticks_in_flight) {
        std::vector<Item> items;
        std::vector<Request*> in_tick;
        int rounds = 0;
        for (Request* r : s->admitted) {
            if (r->state != ACTIVE || r->failed || r->cancel || r->stage >= 2 * r->L) continue;
            const int k = std::min(s->cfg.stages_per_tick, 2 * r->L - r->stage);
            for (int j = 0; j < k; ++j) items.push_back(Item{r, r->stage + j, j});
            in_tick.push_back(r);
            rounds = std::max(rounds, k);
        }
        if (!items.empty()) {
            Tick t;
            t.seq = s->tick_seq++;
            int launches = 0;
            const mdn_status e = s->ex->tick(items, rounds, t.seq, &t.tok, &launches);
            ++s->st.ticks;
            s->st.launches += launches;
            s->st.tick_items += items.size();
            if (e) {
                // the tick could not be enqueued whole: wait for whatever did start, then fail its requests
                s->ex->drain();
                for (Request* r : in_tick) {
                    r->failed = true;
                    r->status = MDN_EDEVICE;
                }
            } else {
                for (Request* r : in_tick) {
                    // a request whose launch failed still holds the tick: other launches of the tick may use its memory
                    ++r->in_ticks;
                    t.ids.push_back(r->id);
                    if (r->tick_first < 0) r->tick_first = (int)t.seq;
                    r->tick_last = (int)t.seq;
                    if (r->failed) continue;
                    r->stage = std::min(r->stage + s->cfg.stages_per_tick, 2 * r->L);
                    if (r->stage == 2 * r->L) {
                        t.finishing.push_back(r->id);
                        if (s->ex->download(*r, t.tok, &r->down)) {
                            r->failed = true;
                            r->status = MDN_EDEVICE;
                        } else {
                            r->state = DOWNLOADING;
                        }
                    }
                }
                s->ticks.push_back(std::move(t));
            }
            changed = true;
        }
    }
    return changed;
}

void progress(mdn_server* s) {
    for (int i = 0; i < 64 && step(s); ++i) {
    }
}

// earliest future time at which the fake schedule can change (a completion or a time-out)
double fake_next(mdn_server* s) {
    double t = s->fake->next_event();
    if (s->cfg.queue_timeout > 0)
        for (Request* r : s->queue) t = std::min(t, r->t_arrival + s->cfg.queue_timeout);
    return t;
}

mdn_status submit_at(mdn_server* s, const mdn_request* q, double t_arrival, uint64_t* id) {
    mdn_status e = check_request(s, q);
    if (e) return e;
    auto r = std::make_unique<Request>();
    r->q = *q;
    r->L = s->banks[q->bank].L;
    r->in_bytes = r->out_bytes = (size_t)q->width * q->height * 3 * (q->dtype == MDN_F16 ? 2 : 4);
    r->bytes = footprint(*r, s->cfg.storage);
    if (r->bytes > s->arena.capacity())
        return fail(MDN_ENOMEM, "server: request footprint %zu exceeds the %zu-byte budget", r->bytes,
                    s->arena.capacity());
    int64_t w = q->width, h = q->height;
    for (int l = 0; l <= r->L; ++l) {
        r->px[l] = w * h;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    r->t_arrival = t_arrival;
    r->id = s->next_id++;
    if (id) *id = r->id;
    std::lock_guard<std::mutex> g(s->inbox_mu);
    s->inbox.push_back(std::move(r));
    ++s->st.submitted;
    return MDN_OK;
}

int take(mdn_server* s, mdn_completion* out, int max_out) {
    int n = 0;
    while (n < max_out && !s->done.empty()) {
        out[n++] = s->done.front().first;
        if (s->done.front().second) s->lent.push_back(s->done.front().first.slot);
        s->done.pop_front();
    }
    return n;
}

bool idle(mdn_server* s) {
    std::lock_guard<std::mutex> g(s->inbox_mu);
    return s->inbox.empty() && s->live.empty();
}

}  // namespace

extern "C" {

mdn_status mdn_server_create(const mdn_server_config* cfg, mdn_server** out) {
    clear_error();
    if (!out || !cfg) return fail(MDN_EINVAL, "server: null argument");
    *out = nullptr;
    mdn_server_config c = *cfg;
    if (c.n_banks < 1 || c.n_banks > kMaxBanks || !c.banks)
        return fail(MDN_EINVAL, "server: need 1..%d banks", kMaxBanks);
    if (c.storage != MDN_F16 && c.storage != MDN_F32) return fail(MDN_EINVAL, "server: unknown storage dtype");
    if (c.max_slots < 1 || c.max_slots > kMaxSlots) return fail(MDN_EINVAL, "server: max_slots must be 1..%d", kMaxSlots);
    if (c.stages_per_tick < 1) return fail(MDN_EINVAL, "server: stages_per_tick must be >= 1");
    if (c.max_ticks_in_flight < 1 || c.max_ticks_in_flight > 8)
        return fail(MDN_EINVAL, "server: max_ticks_in_flight must be 1..8");
    if (c.executor != MDN_EXEC_HIP && c.executor != MDN_EXEC_FAKE) return fail(MDN_EINVAL, "server: unknown executor");
    if (c.hbm_budget < 4096) return fail(MDN_EINVAL, "server: hbm_budget too small");
    if (c.reserved[0] || c.reserved[1]) return fail(MDN_EINVAL, "server: reserved fields must be zero");
    auto s = std::make_unique<mdn_server>();
    s->cfg = c;
    for (int b = 0; b < c.n_banks; ++b) {
        const mdn_bank& bk = c.banks[b];
        if (bk.levels < 1 || bk.levels > kMaxLevels || !bk.level)
            return fail(MDN_EINVAL, "server: bank %d needs 1..%d levels", b, kMaxLevels);
        Bank& B = s->banks[b];
        B.L = bk.levels;
        for (int l = 0; l < B.L; ++l) {
            const mdn_level& lv = bk.level[l];
            mdn_status e = validate_level(&lv, 3);
            if (!e && !lv.t_s && lv.q_s > 1) e = fail(MDN_EINVAL, "server: null thresholds");
            if (e) return e;
            if (lv.radius_f < 1) return fail(MDN_ENOTSUP, "server: banks must be multiscale");
            const bool walk = lv.coeff_dtype == MDN_F16 && walk_supported(lv, 3);
            if (walk && lv.selector == MDN_SELECT_COARSE)
                return fail(MDN_ENOTSUP, "server: float16 7x7/7x7 levels that select on the coarser output are not served");
            if (!walk && !level_runs_tiled(lv, 3))
                return fail(MDN_ENOTSUP, "server: float32 banks that fit in LDS one channel at a time are not served");
            B.tiled[l] = !walk;
            B.lv[l] = lv;
            for (int j = 0; j < lv.q_s - 1; ++j) B.thr[l][0][j] = lv.t_s[j];
            for (int j = 0; j < lv.q_c - 1; ++j) B.thr[l][1][j] = lv.t_c[j];
            B.lv[l].t_s = B.thr[l][0];
            B.lv[l].t_c = B.thr[l][1];
            memset(&B.selc[l], 0, sizeof(SelWalkArgs));
            fill_sel_consts(B.lv[l], B.selc[l]);
        }
    }
    if (c.executor == MDN_EXEC_FAKE) {
        auto f = std::make_unique<FakeExecutor>();
        s->fake = f.get();
        s->ex = std::move(f);
    } else {
        s->ex = std::make_unique<HipExecutor>();
    }
    mdn_status e = s->ex->init(c, s->banks);
    if (e) return e;
    s->arena.reset(c.hbm_budget);
    s->st.arena_bytes = c.hbm_budget;
    for (int i = c.max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    *out = s.release();
    return MDN_OK;
}

mdn_status mdn_server_destroy(mdn_server* s) {
    if (!s) return MDN_OK;
    s->ex->drain();
    delete s;
    return MDN_OK;
}

mdn_status mdn_server_submit(mdn_server* s, const mdn_request* q, uint64_t* id) {
    clear_error();
    if (!s) return fail(MDN_EINVAL, "server: null");
    const mdn_status e = submit_at(s, q, s->ex->now(), id);
    if (e) {
        std::lock_guard<std::mutex> g(s->inbox_mu);
        ++s->st.rejected;
    }
    return e;
}

mdn_status mdn_server_cancel(mdn_server* s, uint64_t id) {
    clear_error();
    if (!s) return fail(MDN_EINVAL, "server: null");
    std::lock_guard<std::mutex> g(s->inbox_mu);
    s->cancels.push_back(id);
    return MDN_OK;
}

mdn_status mdn_server_poll(mdn_server* s, double max_wait, mdn_completion* out, int32_t max_out, int32_t* n_out) {
    clear_error();
    if (!s || !n_out || (max_out > 0 && !out)) return fail(MDN_EINVAL, "server: bad poll arguments");
    *n_out = 0;
    s->free_slots.insert(s->free_slots.end(), s->lent.begin(), s->lent.end());
    s->lent.clear();
    const double until = s->ex->now() + std::max(0.0, max_wait);
    for (;;) {
        progress(s);
        if (!s->done.empty() || idle(s)) break;
        if (s->fake) {
            const double t = fake_next(s);
            if (!(t <= until)) {
                s->fake->advance(until);
                progress(s);
                break;
            }
            s->fake->advance(t);
        } else {
            if (s->ex->now() >= until) break;
            std::this_thread::yield();
        }
    }
    *n_out = take(s, out, max_out);
    return MDN_OK;
}

mdn_status mdn_server_replay(mdn_server* s, const mdn_request* reqs, const double* arrival, int32_t n,
                             mdn_completion* out) {
    clear_error();
    if (!s || n < 0 || (n > 0 && (!reqs || !arrival || !out))) return fail(MDN_EINVAL, "server: bad replay arguments");
    if (!idle(s) || !s->done.empty()) return fail(MDN_EINVAL, "server: replay needs an idle server");
    s->free_slots.insert(s->free_slots.end(), s->lent.begin(), s->lent.end());
    s->lent.clear();
    for (int i = 1; i < n; ++i)
        if (arrival[i] < arrival[i - 1]) return fail(MDN_EINVAL, "server: arrivals must be non-decreasing");
    std::vector<char> have(n, 0);
    int got = 0;
    std::atomic<int> rejected{0};
    auto record_reject = [&](int i, int status) {
        memset(&out[i], 0, sizeof(mdn_completion));
        out[i].tag = reqs[i].tag;
        out[i].status = status;
        out[i].slot = -1;
        out[i].tick_first = out[i].tick_last = -1;
        out[i].t_arrival = arrival[i];
        out[i].t_admit = out[i].t_device_done = out[i].t_host_done = -1;
    };
    auto harvest = [&] {
        while (!s->done.empty()) {
            const mdn_completion c = s->done.front().first;
            if (s->done.front().second) s->free_slots.push_back(c.slot);   // replay keeps no staged result
            s->done.pop_front();
            const uint64_t i = c.tag;
            if (i < (uint64_t)n && !have[i]) {
                out[i] = c;
                out[i].tag = reqs[i].tag;
                have[i] = 1;
                ++got;
            }
        }
    };
    // requests carry their index as tag inside the replay
    if (s->fake) {
        const double base = s->ex->now();
        int next = 0;
        while (got + rejected.load() < n) {
            while (next < n && base + arrival[next] <= s->ex->now()) {
                mdn_request q = reqs[next];
                q.tag = (uint64_t)next;
                const mdn_status e = submit_at(s, &q, base + arrival[next], nullptr);
                if (e) {
                    record_reject(next, e);
                    have[next] = 1;
                    ++s->st.rejected;
                    rejected.fetch_add(1);
                }
                ++next;
            }
            progress(s);
            harvest();
            if (got + rejected.load() >= n) break;
            double t = fake_next(s);
            if (next < n) t = std::min(t, base + arrival[next]);
            if (!std::isfinite(t)) return fail(MDN_EDEVICE, "server: replay stalled");
            s->fake->advance(t);
        }
        return MDN_OK;
    }
    const double base = s->ex->now();
    std::atomic<bool> stop{false};
    std::thread arrivals([&] {
        for (int i = 0; i < n && !stop.load(); ++i) {
            const double t = base + arrival[i];
            for (;;) {
                const double d = t - s->ex->now();
                if (d <= 0) break;
                if (d > 500e-6) std::this_thread::sleep_for(std::chrono::duration<double>(d - 300e-6));
                else std::this_thread::yield();
            }
            mdn_request q = reqs[i];
            q.tag = (uint64_t)i;
            const mdn_status e = submit_at(s, &q, t, nullptr);
            if (e) {
                record_reject(i, e);
                {
                    std::lock_guard<std::mutex> g(s->inbox_mu);
                    ++s->st.rejected;
                }
                rejected.fetch_add(1);
            }
        }
    });
    while (got + rejected.load() < n) {
        const uint64_t before = s->st.completed + s->st.failed;
        progress(s);
        harvest();
        if (s->st.completed + s->st.failed == before) std::this_thread::yield();
    }
    stop.store(true);
    arrivals.join();
    return MDN_OK;
}

mdn_status mdn_server_stats(mdn_server* s, mdn_server_counters* out) {
    clear_error();
    if (!s || !out) return fail(MDN_EINVAL, "server: null argument");
    std::lock_guard<std::mutex> g(s->inbox_mu);
    *out = s->st;
    out->arena_used = s->arena.used();
    out->arena_peak = s->arena.peak();
    out->queued = (int32_t)(s->queue.size() + s->inbox.size());
    out->active = (int32_t)s->admitted.size();
    return MDN_OK;
}

mdn_status mdn_server_footprint(mdn_server* s, const mdn_request* q, uint64_t* bytes) {
    clear_error();
    if (!s || !bytes) return fail(MDN_EINVAL, "server: null argument");
    mdn_status e = check_request(s, q);
    if (e) return e;
    Request r;
    r.q = *q;
    r.L = s->banks[q->bank].L;
    r.in_bytes = r.out_bytes = (size_t)q->width * q->height * 3 * (q->dtype == MDN_F16 ? 2 : 4);
    *bytes = footprint(r, s->cfg.storage);
    return MDN_OK;
}

mdn_status mdn_server_now(mdn_server* s, double* t) {
    clear_error();
    if (!s || !t) return fail(MDN_EINVAL, "server: null argument");
    *t = s->ex->now();
    return MDN_OK;
}

mdn_status mdn_server_fake_advance(mdn_server* s, double t) {
    clear_error();
    if (!s || !s->fake) return fail(MDN_EINVAL, "server: not a fake-executor server");
    s->fake->advance(t);
    return MDN_OK;
}

mdn_status mdn_server_fake_inject(mdn_server* s, int32_t what, uint64_t tag, double value) {
    clear_error();
    if (!s || !s->fake) return fail(MDN_EINVAL, "server: not a fake-executor server");
    if (what < MDN_FAKE_FAIL_UPLOAD || what > MDN_FAKE_STALL) return fail(MDN_EINVAL, "server: unknown injection");
    s->fake->inject(what, tag, value);
    return MDN_OK;
}

}  // extern "C"
