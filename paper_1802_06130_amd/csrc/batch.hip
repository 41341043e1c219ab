// Batched form of the cascade: a list of images of any sizes is denoised level by level with one
// persistent launch per kernel and level over all images (pyramid levels, selection pass,
// filtering pass), from device-resident image tables. A plan owns the per-image pyramids, the
// tables and an internal stream; with graphs enabled the launches of a batch are captured once
// and replayed while the same batch (same images, sizes and buffers) comes back. The strip height
// of every kernel and level comes from the plan's autotuner (timed candidates) or a default.

#include <stdio.h>
#include <string.h>

#include <vector>

#include "walk_types.h"

using namespace mdn;

namespace {

constexpr int kMaxLevels = 8;

size_t al256(size_t v) { return (v + 255) / 256 * 256; }
int64_t pitch64(int w) { return ((int64_t)w + 63) / 64 * 64; }

mdn_image mk_image(void* data, int w, int h, int dtype, int color) {
    mdn_image im;
    memset(&im, 0, sizeof(im));
    im.data = data;
    im.width = w;
    im.height = h;
    im.channels = 3;
    im.dtype = dtype;
    im.color = color;
    im.row_pitch = pitch64(w);
    im.plane_pitch = im.row_pitch * h;
    return im;
}

size_t image_ws(int w, int h, int L, int storage) {
    const size_t es = storage == MDN_F16 ? 2 : 4;
    size_t total = 0;
    for (int l = 1; l <= L; ++l) {
        w = (w + 1) / 2;
        h = (h + 1) / 2;
        const size_t b = al256((size_t)pitch64(w) * h * 3 * es);
        total += b;
        if (l < L) total += b;
    }
    return total;
}

}  // namespace

struct mdn_plan {
    int device = 0;
    int storage = MDN_F16;
    int L = 0;
    mdn_level lv[kMaxLevels];
    double thr[kMaxLevels][2][kMaxThr];
    SelWalkArgs selc[kMaxLevels];
    int max_images = 0;
    char* ws = nullptr;
    size_t ws_cap = 0;
    char* tab_dev = nullptr;
    char* tab_host = nullptr;
    size_t tab_cap = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<uint64_t> sig;          // batch of the captured graph / uploaded tables
    bool tables_valid = false;
    int rows_d2[kMaxLevels], rows_sel[kMaxLevels], rows_walk[kMaxLevels];
    bool tuned = false;
    // prepared launch arguments (tables point into tab_dev)
    D2Args d2[kMaxLevels];
    SelWalkArgs sel[kMaxLevels];
    WalkArgs walk[kMaxLevels];
    int in_dtype = MDN_F16, out_dtype = MDN_F16;
    std::vector<mdn_image> zl, ul;      // [image * (L+1) + level]
    std::vector<uint8_t*> smap;
};

namespace {

std::vector<uint64_t> signature(const mdn_image* in, const mdn_image* out, int n) {
    std::vector<uint64_t> s;
    s.reserve(n * 8 + 1);
    s.push_back((uint64_t)n);
    for (int i = 0; i < n; ++i) {
        s.push_back((uint64_t)in[i].data);
        s.push_back((uint64_t)out[i].data);
        s.push_back(((uint64_t)in[i].width << 32) | (uint32_t)in[i].height);
        s.push_back((uint64_t)in[i].row_pitch);
        s.push_back((uint64_t)in[i].plane_pitch);
        s.push_back((uint64_t)out[i].row_pitch ^ ((uint64_t)out[i].plane_pitch << 20));
        s.push_back(((uint64_t)in[i].dtype << 8) | (uint64_t)out[i].dtype);
    }
    return s;
}

mdn_status ensure_ws(mdn_plan* p, size_t need) {
    if (need <= p->ws_cap) return MDN_OK;
    if (p->ws) {
        if (hipStreamSynchronize(p->stream) != hipSuccess) return fail(MDN_EDEVICE, "plan: sync failed");
        hipFree(p->ws);
        p->ws = nullptr;
    }
    if (hipMalloc((void**)&p->ws, need) != hipSuccess) {
        p->ws_cap = 0;
        return fail(MDN_ENOMEM, "plan: cannot allocate %zu bytes of workspace", need);
    }
    p->ws_cap = need;
    return MDN_OK;
}

mdn_status ensure_tables(mdn_plan* p, size_t need) {
    if (need <= p->tab_cap) return MDN_OK;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return fail(MDN_EDEVICE, "plan: sync failed");
    if (p->tab_dev) hipFree(p->tab_dev);
    if (p->tab_host) hipHostFree(p->tab_host);
    p->tab_dev = nullptr;
    p->tab_host = nullptr;
    p->tab_cap = 0;
    if (hipMalloc((void**)&p->tab_dev, need) != hipSuccess) return fail(MDN_ENOMEM, "plan: table allocation failed");
    if (hipHostMalloc((void**)&p->tab_host, need, hipHostMallocDefault) != hipSuccess)
        return fail(MDN_ENOMEM, "plan: pinned table allocation failed");
    p->tab_cap = need;
    return MDN_OK;
}

// Carve the per-image pyramids out of the workspace and build the launch tables for `n` images.
mdn_status prepare(mdn_plan* p, const mdn_image* in, const mdn_image* out, int n) {
    const int L = p->L;
    size_t need = 0;
    for (int i = 0; i < n; ++i) need += image_ws(in[i].width, in[i].height, L, p->storage) + al256((size_t)in[i].width * in[i].height);
    mdn_status st;
    if ((st = ensure_ws(p, need))) return st;
    const size_t tab_need = al256(sizeof(D2Image) * n) * L + al256(sizeof(SelImage) * n) * L + al256(sizeof(WalkImage) * n) * L;
    if ((st = ensure_tables(p, tab_need))) return st;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return fail(MDN_EDEVICE, "plan: sync failed");

    p->zl.assign((size_t)n * (L + 1), mdn_image{});
    p->ul.assign((size_t)n * (L + 1), mdn_image{});
    p->smap.assign(n, nullptr);
    char* w = p->ws;
    for (int i = 0; i < n; ++i) {
        int W = in[i].width, H = in[i].height;
        p->zl[(size_t)i * (L + 1)] = in[i];
        for (int l = 1; l <= L; ++l) {
            W = (W + 1) / 2;
            H = (H + 1) / 2;
            const size_t b = al256((size_t)pitch64(W) * H * 3 * (p->storage == MDN_F16 ? 2 : 4));
            p->zl[(size_t)i * (L + 1) + l] = mk_image(w, W, H, p->storage, MDN_RGB);
            w += b;
            if (l < L) {
                p->ul[(size_t)i * (L + 1) + l] = mk_image(w, W, H, p->storage, MDN_YCC);
                w += b;
            }
        }
        p->smap[i] = reinterpret_cast<uint8_t*>(w);
        w += al256((size_t)in[i].width * in[i].height);
        p->ul[(size_t)i * (L + 1)] = out[i];
    }

    const int ncu = device_cus();
    char* th = p->tab_host;
    char* td = p->tab_dev;
    for (int l = 0; l < L; ++l) {
        D2Image* t = reinterpret_cast<D2Image*>(th);
        int begin = 0;
        for (int i = 0; i < n; ++i) {
            const mdn_image& a = p->zl[(size_t)i * (L + 1) + l];
            const mdn_image& b = p->zl[(size_t)i * (L + 1) + l + 1];
            D2Image& d = t[i];
            memset(&d, 0, sizeof(d));
            d.in = a.data;
            d.out = b.data;
            d.i_row = a.row_pitch;
            d.i_plane = a.plane_pitch;
            d.o_row = b.row_pitch;
            d.o_plane = b.plane_pitch;
            d.Wi = a.width;
            d.Hi = a.height;
            d.Wo = b.width;
            d.Ho = b.height;
            d.nsx = (b.width + kD2LanesOut - 1) / kD2LanesOut;
            d.rows = p->tuned ? p->rows_d2[l] : down2_rows(b.width, b.height, ncu);
            d.strip_begin = begin;
            begin += d.nsx * ((b.height + d.rows - 1) / d.rows);
        }
        memset(&p->d2[l], 0, sizeof(D2Args));
        p->d2[l].imgs = reinterpret_cast<const D2Image*>(td);
        p->d2[l].n_imgs = n;
        p->d2[l].n_strips = begin;
        th += al256(sizeof(D2Image) * n);
        td += al256(sizeof(D2Image) * n);
    }
    for (int l = 0; l < L; ++l) {
        SelImage* t = reinterpret_cast<SelImage*>(th);
        int begin = 0;
        for (int i = 0; i < n; ++i) {
            const mdn_image& z = p->zl[(size_t)i * (L + 1) + l];
            SelImage& d = t[i];
            memset(&d, 0, sizeof(d));
            d.z = z.data;
            d.s = p->smap[i];
            d.z_row = z.row_pitch;
            d.z_plane = z.plane_pitch;
            d.s_pitch = z.width;
            d.W = z.width;
            d.H = z.height;
            d.C = 3;
            d.nsx = (z.width + kSelLanesOut - 1) / kSelLanesOut;
            d.rows = p->tuned ? p->rows_sel[l] : select_walk_rows(z.width, z.height, ncu);
            d.strip_begin = begin;
            begin += d.nsx * ((z.height + d.rows - 1) / d.rows);
        }
        p->sel[l] = p->selc[l];
        p->sel[l].imgs = reinterpret_cast<const SelImage*>(td);
        p->sel[l].n_imgs = n;
        p->sel[l].n_strips = begin;
        th += al256(sizeof(SelImage) * n);
        td += al256(sizeof(SelImage) * n);
    }
    for (int l = 0; l < L; ++l) {
        WalkImage* t = reinterpret_cast<WalkImage*>(th);
        int begin = 0;
        for (int i = 0; i < n; ++i) {
            const mdn_image& z = p->zl[(size_t)i * (L + 1) + l];
            const mdn_image& uc = (l == L - 1) ? p->zl[(size_t)i * (L + 1) + L] : p->ul[(size_t)i * (L + 1) + l + 1];
            const mdn_image& o = p->ul[(size_t)i * (L + 1) + l];
            fill_walk_image(t[i], z, uc, o, begin);
            t[i].s_map = p->smap[i];
            t[i].s_pitch = z.width;
            t[i].rows = p->tuned ? p->rows_walk[l] : walk_rows(z.width, z.height, ncu * 4);
            begin += t[i].nsx * ((z.height + t[i].rows - 1) / t[i].rows);
        }
        memset(&p->walk[l], 0, sizeof(WalkArgs));
        p->walk[l].imgs = reinterpret_cast<const WalkImage*>(td);
        p->walk[l].n_imgs = n;
        p->walk[l].n_strips = begin;
        p->walk[l].coeffs = p->lv[l].coeffs;
        p->walk[l].coeff_dtype = p->lv[l].coeff_dtype;
        p->walk[l].K = p->lv[l].q_theta * p->lv[l].q_s * p->lv[l].q_c;
        th += al256(sizeof(WalkImage) * n);
        td += al256(sizeof(WalkImage) * n);
    }
    if (hipMemcpyAsync(p->tab_dev, p->tab_host, (size_t)(th - p->tab_host), hipMemcpyHostToDevice, p->stream) !=
        hipSuccess)
        return fail(MDN_EDEVICE, "plan: table upload failed");
    p->in_dtype = in[0].dtype;
    p->out_dtype = out[0].dtype;
    p->tables_valid = true;
    return MDN_OK;
}

mdn_status run_d2(mdn_plan* p, int l) {
    const int ind = l == 0 ? p->in_dtype : p->storage;
    return launch_down2_args(p->d2[l], 3, ind, p->storage, p->stream);
}
mdn_status run_sel(mdn_plan* p, int l) {
    return launch_select_args(p->sel[l], 3, l == 0 ? p->in_dtype : p->storage, p->stream);
}
mdn_status run_walk(mdn_plan* p, int l) {
    const int zd = l == 0 ? p->in_dtype : p->storage;
    const int od = l == 0 ? p->out_dtype : p->storage;
    return launch_walk_args(p->walk[l], zd, p->storage, od, p->stream);
}

mdn_status launch_all(mdn_plan* p) {
    mdn_status st;
    for (int l = 0; l < p->L; ++l)
        if ((st = run_d2(p, l))) return st;
    for (int l = p->L - 1; l >= 0; --l) {
        if ((st = run_sel(p, l))) return st;
        if ((st = run_walk(p, l))) return st;
    }
    return MDN_OK;
}

void drop_graph(mdn_plan* p) {
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

mdn_status check_batch(const mdn_plan* p, const mdn_image* in, const mdn_image* out, int n) {
    if (n < 1 || n > p->max_images) return fail(MDN_EINVAL, "batch: n must be 1..%d", p->max_images);
    if (!in || !out) return fail(MDN_EINVAL, "batch: null image arrays");
    for (int i = 0; i < n; ++i) {
        const mdn_image& a = in[i];
        const mdn_image& b = out[i];
        if (a.channels != 3 || a.color != MDN_RGB || b.channels != 3 || b.color != MDN_RGB)
            return fail(MDN_EINVAL, "batch: images must be RGB");
        if (a.width < 1 || a.height < 1 || a.width != b.width || a.height != b.height)
            return fail(MDN_EINVAL, "batch: image %d: sizes must be positive and equal for input and output", i);
        if (!a.data || !b.data || a.reserved || b.reserved) return fail(MDN_EINVAL, "batch: image %d: bad descriptor", i);
        if (a.row_pitch < a.width || a.plane_pitch < a.row_pitch * a.height || b.row_pitch < b.width ||
            b.plane_pitch < b.row_pitch * b.height)
            return fail(MDN_EINVAL, "batch: image %d: bad pitches", i);
        if (a.plane_pitch * 3 > 0x7fffffffLL || b.plane_pitch * 3 > 0x7fffffffLL)
            return fail(MDN_ENOTSUP, "batch: image %d exceeds 2^31 elements", i);
        if (a.dtype != in[0].dtype || b.dtype != out[0].dtype) return fail(MDN_EINVAL, "batch: mixed dtypes");
    }
    const bool zh = in[0].dtype == MDN_F16, oh = out[0].dtype == MDN_F16, sh = p->storage == MDN_F16;
    if (zh != oh) return fail(MDN_ENOTSUP, "batch: input and output dtypes must match");
    if (zh && !sh) return fail(MDN_ENOTSUP, "batch: float16 images need float16 storage");
    return MDN_OK;
}

}  // namespace

extern "C" {

mdn_status mdn_plan_create(const mdn_bank* bank, int32_t storage, int32_t max_images, mdn_plan** out) {
    clear_error();
    if (!out) return fail(MDN_EINVAL, "plan: null out");
    *out = nullptr;
    if (!bank || bank->levels < 1 || bank->levels > kMaxLevels || !bank->level)
        return fail(MDN_EINVAL, "plan: need 1..%d bank levels", kMaxLevels);
    if (storage != MDN_F16 && storage != MDN_F32) return fail(MDN_EINVAL, "plan: unknown storage dtype");
    if (max_images < 1 || max_images > 4096) return fail(MDN_EINVAL, "plan: max_images must be 1..4096");
    for (int l = 0; l < bank->levels; ++l) {
        const mdn_level& lv = bank->level[l];
        mdn_status st = validate_level(&lv, 3);
        if (!st && !lv.t_s && lv.q_s > 1) st = fail(MDN_EINVAL, "plan: null thresholds");
        if (st) return st;
        if (lv.coeff_dtype != MDN_F16 || !walk_supported(lv, 3))
            return fail(MDN_ENOTSUP, "plan: the batched form runs float16 7x7/7x7 colour banks (K <= 243)");
    }
    mdn_status ist = init_walk_kernels();
    if (ist) return ist;
    mdn_plan* p = new mdn_plan();
    hipGetDevice(&p->device);
    p->storage = storage;
    p->L = bank->levels;
    p->max_images = max_images;
    for (int l = 0; l < p->L; ++l) {
        p->lv[l] = bank->level[l];
        for (int j = 0; j < p->lv[l].q_s - 1; ++j) p->thr[l][0][j] = p->lv[l].t_s[j];
        for (int j = 0; j < p->lv[l].q_c - 1; ++j) p->thr[l][1][j] = p->lv[l].t_c[j];
        p->lv[l].t_s = p->thr[l][0];
        p->lv[l].t_c = p->thr[l][1];
        memset(&p->selc[l], 0, sizeof(SelWalkArgs));
        fill_sel_consts(p->lv[l], p->selc[l]);
    }
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming) != hipSuccess) {
        mdn_plan_destroy(p);
        return fail(MDN_EDEVICE, "plan: stream/event creation failed");
    }
    *out = p;
    return MDN_OK;
}

mdn_status mdn_plan_destroy(mdn_plan* p) {
    if (!p) return MDN_OK;
    if (p->stream) hipStreamSynchronize(p->stream);
    drop_graph(p);
    if (p->ws) hipFree(p->ws);
    if (p->tab_dev) hipFree(p->tab_dev);
    if (p->tab_host) hipHostFree(p->tab_host);
    if (p->ev_in) hipEventDestroy(p->ev_in);
    if (p->ev_out) hipEventDestroy(p->ev_out);
    if (p->stream) hipStreamDestroy(p->stream);
    delete p;
    return MDN_OK;
}

mdn_status mdn_plan_autotune(mdn_plan* p, const mdn_image* in, const mdn_image* out, int32_t n, int32_t* rows_out,
                             void* stream) {
    clear_error();
    if (!p) return fail(MDN_EINVAL, "plan: null");
    mdn_status st = check_batch(p, in, out, n);
    if (st) return st;
    hipStream_t cs = static_cast<hipStream_t>(stream);
    if (hipEventRecord(p->ev_in, cs) != hipSuccess || hipStreamWaitEvent(p->stream, p->ev_in, 0) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: stream ordering failed");
    drop_graph(p);
    p->tuned = false;
    if ((st = prepare(p, in, out, n))) return st;
    const int L = p->L;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    auto time_it = [&](auto&& fn) -> float {
        fn();
        hipEventRecord(e0, p->stream);
        fn();
        hipEventRecord(e1, p->stream);
        hipEventSynchronize(e1);
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    // every candidate re-prepares the tables of that kernel and level only through `tuned` rows
    const int c_d2[] = {8, 16, 32, 64}, c_sel[] = {10, 20, 30, 60}, c_walk[] = {14, 28, 42, 56};
    int best_d2[kMaxLevels], best_sel[kMaxLevels], best_walk[kMaxLevels];
    const int ncu = device_cus();
    for (int l = 0; l < L; ++l) {
        best_d2[l] = down2_rows(p->zl[l + 1].width, p->zl[l + 1].height, ncu);
        best_sel[l] = 20;
        best_walk[l] = 56;
    }
    p->tuned = true;
    for (int l = 0; l < L; ++l) {
        p->rows_d2[l] = best_d2[l];
        p->rows_sel[l] = best_sel[l];
        p->rows_walk[l] = best_walk[l];
    }
    // pyramid, finest first (each level's input exists once the previous one ran)
    for (int l = 0; l < L && !st; ++l) {
        float best = 1e30f;
        for (int c : c_d2) {
            p->rows_d2[l] = c;
            if ((st = prepare(p, in, out, n))) break;
            const float ms = time_it([&] { run_d2(p, l); });
            if (ms < best) {
                best = ms;
                best_d2[l] = c;
            }
        }
        p->rows_d2[l] = best_d2[l];
        if (!st) st = prepare(p, in, out, n);
        if (!st) st = run_d2(p, l);
    }
    for (int l = L - 1; l >= 0 && !st; --l) {
        float best = 1e30f;
        for (int c : c_sel) {
            p->rows_sel[l] = c;
            if ((st = prepare(p, in, out, n))) break;
            const float ms = time_it([&] { run_sel(p, l); });
            if (ms < best) {
                best = ms;
                best_sel[l] = c;
            }
        }
        p->rows_sel[l] = best_sel[l];
        if (st) break;
        best = 1e30f;
        for (int c : c_walk) {
            p->rows_walk[l] = c;
            if ((st = prepare(p, in, out, n))) break;
            const float ms = time_it([&] { run_walk(p, l); });
            if (ms < best) {
                best = ms;
                best_walk[l] = c;
            }
        }
        p->rows_walk[l] = best_walk[l];
        if (!st) st = prepare(p, in, out, n);
        if (!st) st = run_sel(p, l);
        if (!st) st = run_walk(p, l);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    if (rows_out)
        for (int l = 0; l < L; ++l) {
            rows_out[3 * l] = best_d2[l];
            rows_out[3 * l + 1] = best_sel[l];
            rows_out[3 * l + 2] = best_walk[l];
        }
    p->tables_valid = false;
    p->sig.clear();
    if (hipEventRecord(p->ev_out, p->stream) != hipSuccess || hipStreamWaitEvent(cs, p->ev_out, 0) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: stream ordering failed");
    return check_launch("autotune");
}

mdn_status mdn_denoise_batch(mdn_plan* p, const mdn_image* in, const mdn_image* out, int32_t n, int32_t use_graph,
                             void* stream) {
    clear_error();
    if (!p) return fail(MDN_EINVAL, "plan: null");
    mdn_status st = check_batch(p, in, out, n);
    if (st) return st;
    hipStream_t cs = static_cast<hipStream_t>(stream);
    if (hipEventRecord(p->ev_in, cs) != hipSuccess || hipStreamWaitEvent(p->stream, p->ev_in, 0) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: stream ordering failed");
    std::vector<uint64_t> sig = signature(in, out, n);
    const bool same = p->tables_valid && sig == p->sig;
    if (!same) {
        drop_graph(p);
        if ((st = prepare(p, in, out, n))) return st;
        p->sig = sig;
    }
    if (use_graph) {
        if (!p->exec) {
            if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return fail(MDN_EDEVICE, "plan: graph capture failed to start");
            st = launch_all(p);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(p->stream, &g);
            if (st) {
                if (g) hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess || !g) return fail(MDN_EDEVICE, "plan: graph capture failed");
            p->graph = g;
            if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
                drop_graph(p);
                return fail(MDN_EDEVICE, "plan: graph instantiation failed");
            }
        }
        if (hipGraphLaunch(p->exec, p->stream) != hipSuccess) return fail(MDN_EDEVICE, "plan: graph launch failed");
    } else {
        if ((st = launch_all(p))) return st;
    }
    if (hipEventRecord(p->ev_out, p->stream) != hipSuccess || hipStreamWaitEvent(cs, p->ev_out, 0) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: stream ordering failed");
    return check_launch("denoise_batch");
}

}  // extern "C"
