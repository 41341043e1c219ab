// Batched form of the cascade: a list of images of any sizes, each with one of the plan's banks, is
// denoised level by level with one persistent launch per kernel, level and bank over all the images
// concerned (pyramid levels over every image deep enough; selection and filtering over the images
// of one bank), from device-resident image tables. A plan owns the per-image pyramids, the tables
// and an internal stream; with graphs enabled the launches of a batch are captured once and
// replayed while the same batch (same images, sizes, banks and buffers) comes back. The strip
// height of every kernel and level comes from the plan's autotuner (timed candidates) or a default.

#include <stdio.h>
#include <string.h>

#include <vector>

#include "walk_types.h"

// 0: the pyramid steps and selection passes of a batch always run as launches of their own
#ifndef MDN_FUSE_PYR_SEL
#define MDN_FUSE_PYR_SEL 1
#endif

using namespace mdn;

namespace {

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

struct PlanBank {
    int L = 0;
    mdn_level lv[kMaxLevels];
    double thr[kMaxLevels][2][kMaxThr];
    SelWalkArgs selc[kMaxLevels];
};

struct mdn_plan {
    int device = 0;
    int storage = MDN_F16;
    int n_banks = 0;
    int Lmax = 0;
    PlanBank bank[kMaxPlanBanks];
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
    BatchLaunch bl;                     // prepared launch arguments (tables in tab_dev)
};

namespace {

std::vector<uint64_t> signature(const mdn_image* in, const mdn_image* out, const int32_t* bank, int n) {
    std::vector<uint64_t> s;
    s.reserve(n * 9 + 1);
    s.push_back((uint64_t)n);
    for (int i = 0; i < n; ++i) {
        s.push_back(bank ? (uint64_t)(uint32_t)bank[i] : 0);
        // every field that the tables or the captured launches depend on, each in a word of its own
        s.push_back((uint64_t)in[i].data);
        s.push_back((uint64_t)out[i].data);
        s.push_back(((uint64_t)(uint32_t)in[i].width << 32) | (uint32_t)in[i].height);
        s.push_back((uint64_t)in[i].row_pitch);
        s.push_back((uint64_t)in[i].plane_pitch);
        s.push_back((uint64_t)out[i].row_pitch);
        s.push_back((uint64_t)out[i].plane_pitch);
        s.push_back(((uint64_t)(uint32_t)in[i].dtype << 8) | (uint32_t)out[i].dtype);
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

}  // namespace

namespace mdn {

// the selector maps of levels 0 .. L-1, one each: a level's selection may run long before its
// filtering (beside a pyramid step), so the levels cannot share one map
size_t batch_maps_bytes(int w, int h, int L) {
    size_t b = 0;
    for (int l = 0; l < L; ++l) {
        b += al256((size_t)w * h);
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    return b;
}

size_t batch_image_ws(int w, int h, int L, int storage) { return image_ws(w, h, L, storage) + batch_maps_bytes(w, h, L); }

// Per-level descriptors of one image's cascade, each with strip_begin = 0: d2[l] makes z^{l+1}
// from z^l, sel[l] and walk[l] run level l (walk[0] writes `out`). ws (batch_image_ws bytes,
// 256-aligned) holds z^1..z^L, u^1..u^{L-1} and the selector maps of levels 0..L-1.
void describe_cascade(const mdn_image& in, const mdn_image& out, void* ws, int L, int storage, const int (*rows)[3],
                      int ncu, D2Image* d2, SelImage* sel, WalkImage* walk, TileImage* tile) {
    mdn_image zl[kMaxLevels + 1], ul[kMaxLevels + 1];
    char* w = static_cast<char*>(ws);
    int W = in.width, H = in.height;
    zl[0] = in;
    ul[0] = out;
    for (int l = 1; l <= L; ++l) {
        W = (W + 1) / 2;
        H = (H + 1) / 2;
        const size_t b = al256((size_t)pitch64(W) * H * 3 * (storage == MDN_F16 ? 2 : 4));
        zl[l] = mk_image(w, W, H, storage, MDN_RGB);
        w += b;
        if (l < L) {
            ul[l] = mk_image(w, W, H, storage, MDN_YCC);
            w += b;
        }
    }
    for (int l = 0; l < L; ++l) {
        const mdn_image& a = zl[l];
        const mdn_image& o = zl[l + 1];
        uint8_t* smap = reinterpret_cast<uint8_t*>(w);
        w += al256((size_t)a.width * a.height);
        D2Image& d = d2[l];
        memset(&d, 0, sizeof(d));
        d.in = a.data;
        d.out = o.data;
        d.i_row = a.row_pitch;
        d.i_plane = a.plane_pitch;
        d.o_row = o.row_pitch;
        d.o_plane = o.plane_pitch;
        d.Wi = a.width;
        d.Hi = a.height;
        d.Wo = o.width;
        d.Ho = o.height;
        d.nsx = (o.width + kD2LanesOut - 1) / kD2LanesOut;
        d.rows = rows ? rows[l][0] : down2_rows(o.width, o.height, ncu);

        SelImage& e = sel[l];
        memset(&e, 0, sizeof(e));
        e.z = a.data;
        e.s = smap;
        e.z_row = a.row_pitch;
        e.z_plane = a.plane_pitch;
        e.s_pitch = a.width;
        e.W = a.width;
        e.H = a.height;
        e.C = 3;
        e.nsx = (a.width + kSelLanesOut - 1) / kSelLanesOut;
        e.rows = rows ? rows[l][1] : select_walk_rows(a.width, a.height, ncu);

        fill_walk_image(walk[l], a, l == L - 1 ? zl[L] : ul[l + 1], ul[l], 0);
        walk[l].s_map = smap;
        walk[l].s_pitch = a.width;
        walk[l].rows = rows ? rows[l][2] : walk_rows(a.width, a.height, ncu * kWalkWaves);

        if (tile) {
            // the coarser output (z^L in RGB at the coarsest trained level) is also the image the
            // coarse selector analyses
            const mdn_image& c = l == L - 1 ? zl[L] : ul[l + 1];
            const mdn_image& u = ul[l];
            TileImage& t = tile[l];
            memset(&t, 0, sizeof(t));
            t.z = ImageArg{a.data, a.row_pitch, a.plane_pitch, a.width, a.height};
            t.uc = ImageArg{c.data, c.row_pitch, c.plane_pitch, c.width, c.height};
            t.su = t.uc;
            t.out = u.data;
            t.out_row = u.row_pitch;
            t.out_plane = u.plane_pitch;
            int ty = 0;
            tiled_grid(a.width, a.height, &t.tiles_x, &ty);
        }
    }
}

int tiles_of(const TileImage& t) {
    int tx = 0, ty = 0;
    tiled_grid(t.z.w, t.z.h, &tx, &ty);
    return tx * ty;
}

int strips_of(const D2Image& d) { return d.nsx * ((d.Ho + d.rows - 1) / d.rows); }
int strips_of(const SelImage& d) { return d.nsx * ((d.H + d.rows - 1) / d.rows); }
int strips_of(const WalkImage& d) { return d.nsx * ((d.H + d.rows - 1) / d.rows); }

}  // namespace mdn

namespace {

int image_bank(const int32_t* bank, int i) { return bank ? bank[i] : 0; }

// Launch list and tables of one batch: image i, of bank bank[i], uses the workspace ws[i]
// (batch_image_ws bytes for its bank's depth, 256-aligned). The tables are appended to `tab` (host
// bytes, every table 256-aligned) and each launch keeps its table's offset.
void build_batch(const mdn_plan* p, const mdn_image* in, const mdn_image* out, const int32_t* bank,
                 void* const* ws, int n, const int (*rows)[3], std::vector<char>& tab, BatchLaunch* bl) {
    const int ncu = device_cus();
    const int storage = p->storage;
    std::vector<D2Image> d2((size_t)n * kMaxLevels);
    std::vector<SelImage> sel((size_t)n * kMaxLevels);
    std::vector<WalkImage> walk((size_t)n * kMaxLevels);
    std::vector<TileImage> tile((size_t)n * kMaxLevels);
    for (int i = 0; i < n; ++i) {
        const size_t o = (size_t)i * kMaxLevels;
        describe_cascade(in[i], out[i], ws[i], p->bank[image_bank(bank, i)].L, storage, rows, ncu, &d2[o], &sel[o],
                         &walk[o], &tile[o]);
    }
    tab.clear();
    bl->items.clear();
    auto put = [&](const void* d, size_t bytes) {
        const char* c = static_cast<const char*>(d);
        tab.insert(tab.end(), c, c + bytes);
    };
    auto item = [&](int kind, int level, int b) {
        BatchItem it;
        memset(&it, 0, sizeof(it));
        it.kind = kind;
        it.level = level;
        it.bank = b;
        it.tab_off = tab.size();
        it.z_dtype = level == 0 ? in[0].dtype : storage;
        it.out_dtype = level == 0 ? out[0].dtype : storage;
        it.out_color = level == 0 ? MDN_RGB : MDN_YCC;
        return it;
    };
    auto close = [&](BatchItem& it) {
        bl->items.push_back(it);
        tab.resize(al256(tab.size()));
    };
    // pyramid steps l -> l + 1 over every image whose bank is deeper than l
    for (int l = 0; l < p->Lmax; ++l) {
        BatchItem it = item(0, l, -1);
        int begin = 0, cnt = 0;
        for (int i = 0; i < n; ++i) {
            if (p->bank[image_bank(bank, i)].L <= l) continue;
            D2Image d = d2[(size_t)i * kMaxLevels + l];
            d.strip_begin = begin;
            begin += strips_of(d);
            put(&d, sizeof(d));
            ++cnt;
        }
        if (!cnt) continue;
        it.d2.n_imgs = cnt;
        it.d2.n_strips = begin;
        close(it);
    }
    // levels from the coarsest trained one down, bank by bank: an image's level l runs after its
    // level l + 1, whatever the depth of its bank
    for (int l = p->Lmax - 1; l >= 0; --l) {
        for (int b = 0; b < p->n_banks; ++b) {
            const PlanBank& pb = p->bank[b];
            if (pb.L <= l) continue;
            std::vector<int> imgs;
            for (int i = 0; i < n; ++i)
                if (image_bank(bank, i) == b) imgs.push_back(i);
            if (imgs.empty()) continue;
            const mdn_level& lv = pb.lv[l];
            if (level_runs_tiled(lv, 3)) {
                BatchItem it = item(3, l, b);
                int begin = 0;
                for (int i : imgs) {
                    TileImage t = tile[(size_t)i * kMaxLevels + l];
                    t.tile_begin = begin;
                    begin += tiles_of(t);
                    put(&t, sizeof(t));
                }
                it.lv = lv;
                it.n_imgs = (int)imgs.size();
                it.n_tiles = begin;
                it.uc_color = l == pb.L - 1 ? MDN_RGB : MDN_YCC;
                close(it);
                continue;
            }
            BatchItem si = item(1, l, b);
            int begin = 0;
            for (int i : imgs) {
                SelImage e = sel[(size_t)i * kMaxLevels + l];
                e.strip_begin = begin;
                begin += strips_of(e);
                put(&e, sizeof(e));
            }
            si.sel = pb.selc[l];
            si.sel.n_imgs = (int)imgs.size();
            si.sel.n_strips = begin;
            close(si);
            BatchItem wi = item(2, l, b);
            begin = 0;
            for (int i : imgs) {
                WalkImage w = walk[(size_t)i * kMaxLevels + l];
                w.strip_begin = begin;
                begin += strips_of(w);
                put(&w, sizeof(w));
            }
            wi.walk.n_imgs = (int)imgs.size();
            wi.walk.n_strips = begin;
            wi.walk.coeffs = lv.coeffs;
            wi.walk.coeff_dtype = lv.coeff_dtype;
            wi.walk.K = level_buckets(lv);
            close(wi);
        }
    }
    bl->Lmax = p->Lmax;
    bl->storage = storage;
    bl->in_dtype = in[0].dtype;
    bl->out_dtype = out[0].dtype;
    bl->table_bytes = tab.size();
}

mdn_status launch_item(const BatchLaunch& bl, const BatchItem& it, hipStream_t st) {
    const char* t = bl.tab_dev + it.tab_off;
    switch (it.kind) {
    case 0: {
        D2Args a = it.d2;
        a.imgs = reinterpret_cast<const D2Image*>(t);
        return launch_down2_args(a, 3, it.z_dtype, bl.storage, st);
    }
    case 1: {
        SelWalkArgs a = it.sel;
        a.imgs = reinterpret_cast<const SelImage*>(t);
        return launch_select_args(a, 3, it.z_dtype, st);
    }
    case 2: {
        WalkArgs a = it.walk;
        a.imgs = reinterpret_cast<const WalkImage*>(t);
        return launch_walk_args(a, it.z_dtype, bl.storage, it.out_dtype, st);
    }
    default:
        return launch_select_apply_table(it.lv, reinterpret_cast<const TileImage*>(t), it.n_imgs, it.n_tiles, 3,
                                         it.z_dtype, bl.storage, it.uc_color, it.out_dtype, it.out_color, st);
    }
}

// the launches of one kind group at level l: pyramid (0), selection (1), filtering (2: walk or tiled)
mdn_status run_group(mdn_plan* p, int group, int l) {
    for (const BatchItem& it : p->bl.items) {
        if (it.level != l) continue;
        const bool in = group == 0 ? it.kind == 0 : group == 1 ? it.kind == 1 : (it.kind == 2 || it.kind == 3);
        if (!in) continue;
        mdn_status e = launch_item(p->bl, it, p->stream);
        if (e) return e;
    }
    return MDN_OK;
}
bool level_has_selection(const mdn_plan* p, int l) {
    for (const BatchItem& it : p->bl.items)
        if (it.level == l && it.kind == 1) return true;
    return false;
}

// Carve the per-image workspaces out of the plan's workspace and build the launch tables.
mdn_status prepare(mdn_plan* p, const mdn_image* in, const mdn_image* out, const int32_t* bank, int n) {
    size_t need = 0;
    for (int i = 0; i < n; ++i) need += batch_image_ws(in[i].width, in[i].height, p->bank[image_bank(bank, i)].L, p->storage);
    mdn_status st;
    if ((st = ensure_ws(p, need))) return st;
    std::vector<void*> ws(n);
    char* w = p->ws;
    for (int i = 0; i < n; ++i) {
        ws[i] = w;
        w += batch_image_ws(in[i].width, in[i].height, p->bank[image_bank(bank, i)].L, p->storage);
    }
    int rows[kMaxLevels][3];
    for (int l = 0; l < p->Lmax; ++l) {
        rows[l][0] = p->rows_d2[l];
        rows[l][1] = p->rows_sel[l];
        rows[l][2] = p->rows_walk[l];
    }
    std::vector<char> tab;
    build_batch(p, in, out, bank, ws.data(), n, p->tuned ? rows : nullptr, tab, &p->bl);
    if ((st = ensure_tables(p, tab.size() ? tab.size() : 256))) return st;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return fail(MDN_EDEVICE, "plan: sync failed");
    memcpy(p->tab_host, tab.data(), tab.size());
    p->bl.tab_dev = p->tab_dev;
    if (tab.size() && hipMemcpyAsync(p->tab_dev, p->tab_host, tab.size(), hipMemcpyHostToDevice, p->stream) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: table upload failed");
    p->tables_valid = true;
    return MDN_OK;
}

mdn_status run_d2(mdn_plan* p, int l) { return run_group(p, 0, l); }
mdn_status run_sel(mdn_plan* p, int l) { return run_group(p, 1, l); }
mdn_status run_walk(mdn_plan* p, int l) { return run_group(p, 2, l); }
// The selection item that runs in the launch of pyramid item `d2` (same level): the level's only
// selection pass, when its bank allows it; items.size() when none does.
size_t fused_selection(const std::vector<BatchItem>& items, const BatchItem& d2) {
    size_t sel = items.size();
    int nsel = 0;
    for (size_t j = 0; j < items.size(); ++j)
        if (items[j].kind == 1 && items[j].level == d2.level) {
            sel = j;
            ++nsel;
        }
    return (MDN_FUSE_PYR_SEL && nsel == 1 && pyr_sel_fusable(items[sel].sel)) ? sel : items.size();
}
mdn_status launch_fused(const BatchLaunch& bl, const BatchItem& d2, const BatchItem& si, hipStream_t st) {
    D2Args d = d2.d2;
    d.imgs = reinterpret_cast<const D2Image*>(bl.tab_dev + d2.tab_off);
    SelWalkArgs a = si.sel;
    a.imgs = reinterpret_cast<const SelImage*>(bl.tab_dev + si.tab_off);
    return launch_pyr_sel_args(d, a, d2.z_dtype, bl.storage, st);
}
// The pyramid step of level l, with the level's selection pass in the same launch where possible;
// *fused tells whether it was.
mdn_status run_d2_fused(mdn_plan* p, int l, bool* fused) {
    const std::vector<BatchItem>& items = p->bl.items;
    *fused = false;
    for (const BatchItem& it : items) {
        if (it.kind != 0 || it.level != l) continue;
        const size_t sel = fused_selection(items, it);
        mdn_status e;
        if (sel < items.size()) {
            e = launch_fused(p->bl, it, items[sel], p->stream);
            *fused = true;
        } else {
            e = launch_item(p->bl, it, p->stream);
        }
        if (e) return e;
    }
    return MDN_OK;
}

// The batch's launches: the pyramid steps first, each together with its level's selection pass in
// one launch where the level has exactly one selection pass that allows it (one column-walk bank
// over the images); then, from the coarsest level down, the remaining selection passes and the
// filtering launches.
mdn_status launch_all(mdn_plan* p) {
    const std::vector<BatchItem>& items = p->bl.items;
    std::vector<char> done(items.size(), 0);
    for (size_t i = 0; i < items.size(); ++i) {
        const BatchItem& it = items[i];
        if (it.kind != 0) continue;
        done[i] = 1;
        const size_t sel = fused_selection(items, it);
        mdn_status e;
        if (sel < items.size()) {
            e = launch_fused(p->bl, it, items[sel], p->stream);
            done[sel] = 1;
        } else {
            e = launch_item(p->bl, it, p->stream);
        }
        if (e) return e;
    }
    for (size_t i = 0; i < items.size(); ++i) {
        if (done[i]) continue;
        mdn_status e = launch_item(p->bl, items[i], p->stream);
        if (e) return e;
    }
    return MDN_OK;
}

void drop_graph(mdn_plan* p) {
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

mdn_status check_batch(const mdn_plan* p, const mdn_image* in, const mdn_image* out, const int32_t* bank, int n) {
    if (n < 1 || n > p->max_images) return fail(MDN_EINVAL, "batch: n must be 1..%d", p->max_images);
    if (!in || !out) return fail(MDN_EINVAL, "batch: null image arrays");
    for (int i = 0; i < n; ++i) {
        const mdn_image& a = in[i];
        const mdn_image& b = out[i];
        if (bank && (bank[i] < 0 || bank[i] >= p->n_banks))
            return fail(MDN_EINVAL, "batch: image %d: bank %d, the plan has %d", i, bank[i], p->n_banks);
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

mdn_status mdn_plan_create_banks(const mdn_bank* banks, int32_t n_banks, int32_t storage, int32_t max_images,
                                 mdn_plan** out) {
    clear_error();
    if (!out) return fail(MDN_EINVAL, "plan: null out");
    *out = nullptr;
    if (!banks || n_banks < 1 || n_banks > kMaxPlanBanks) return fail(MDN_EINVAL, "plan: need 1..%d banks", kMaxPlanBanks);
    if (storage != MDN_F16 && storage != MDN_F32) return fail(MDN_EINVAL, "plan: unknown storage dtype");
    if (max_images < 1 || max_images > 4096) return fail(MDN_EINVAL, "plan: max_images must be 1..4096");
    for (int b = 0; b < n_banks; ++b) {
        const mdn_bank* bank = &banks[b];
        if (bank->levels < 1 || bank->levels > kMaxLevels || !bank->level)
            return fail(MDN_EINVAL, "plan: bank %d: need 1..%d levels", b, kMaxLevels);
        for (int l = 0; l < bank->levels; ++l) {
            const mdn_level& lv = bank->level[l];
            mdn_status st = validate_level(&lv, 3);
            if (!st && !lv.t_s && lv.q_s > 1) st = fail(MDN_EINVAL, "plan: null thresholds");
            if (st) return st;
            if (lv.radius_f < 1) return fail(MDN_ENOTSUP, "plan: the batched form runs multiscale banks");
            const bool walk = lv.coeff_dtype == MDN_F16 && walk_supported(lv, 3);
            if (walk && lv.selector == MDN_SELECT_COARSE)
                return fail(MDN_ENOTSUP, "plan: float16 7x7/7x7 levels that select on the coarser output are not batched");
            if (!walk && !level_runs_tiled(lv, 3))
                return fail(MDN_ENOTSUP, "plan: float32 banks that fit in LDS one channel at a time are not batched");
        }
    }
    mdn_status ist = init_walk_kernels();
    if (ist) return ist;
    mdn_plan* p = new mdn_plan();
    hipGetDevice(&p->device);
    p->storage = storage;
    p->n_banks = n_banks;
    p->max_images = max_images;
    for (int b = 0; b < n_banks; ++b) {
        PlanBank& pb = p->bank[b];
        pb.L = banks[b].levels;
        p->Lmax = pb.L > p->Lmax ? pb.L : p->Lmax;
        for (int l = 0; l < pb.L; ++l) {
            pb.lv[l] = banks[b].level[l];
            for (int j = 0; j < pb.lv[l].q_s - 1; ++j) pb.thr[l][0][j] = pb.lv[l].t_s[j];
            for (int j = 0; j < pb.lv[l].q_c - 1; ++j) pb.thr[l][1][j] = pb.lv[l].t_c[j];
            pb.lv[l].t_s = pb.thr[l][0];
            pb.lv[l].t_c = pb.thr[l][1];
            memset(&pb.selc[l], 0, sizeof(SelWalkArgs));
            fill_sel_consts(pb.lv[l], pb.selc[l]);
        }
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

mdn_status mdn_plan_create(const mdn_bank* bank, int32_t storage, int32_t max_images, mdn_plan** out) {
    return mdn_plan_create_banks(bank, 1, storage, max_images, out);
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

mdn_status mdn_plan_autotune(mdn_plan* p, const mdn_image* in, const mdn_image* out, const int32_t* bank, int32_t n,
                             int32_t* rows_out, void* stream) {
    clear_error();
    if (!p) return fail(MDN_EINVAL, "plan: null");
    mdn_status st = check_batch(p, in, out, bank, n);
    if (st) return st;
    hipStream_t cs = static_cast<hipStream_t>(stream);
    if (hipEventRecord(p->ev_in, cs) != hipSuccess || hipStreamWaitEvent(p->stream, p->ev_in, 0) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: stream ordering failed");
    drop_graph(p);
    p->tuned = false;
    if ((st = prepare(p, in, out, bank, n))) return st;
    const int L = p->Lmax;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    // one warm-up launch, then one timed launch started on an idle stream: events recorded between
    // back-to-back launches have been seen to miss part of the second launch
    auto time_it = [&](auto&& fn) -> float {
        fn();
        hipStreamSynchronize(p->stream);
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
    for (int l = 0; l < L; ++l) {
        best_d2[l] = 32;
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
            if ((st = prepare(p, in, out, bank, n))) break;
            const float ms = time_it([&] { run_d2(p, l); });
            if (ms < best) {
                best = ms;
                best_d2[l] = c;
            }
        }
        p->rows_d2[l] = best_d2[l];
        if (!st) st = prepare(p, in, out, bank, n);
        if (!st) st = run_d2(p, l);
    }
    for (int l = L - 1; l >= 0 && !st; --l) {
        if (!level_has_selection(p, l)) {
            // every bank's level runs the tiled kernel (fixed 64 x 16 tiles, selection inline):
            // nothing to tune, run the level once
            st = run_walk(p, l);
            continue;
        }
        float best = 1e30f;
        for (int c : c_sel) {
            p->rows_sel[l] = c;
            if ((st = prepare(p, in, out, bank, n))) break;
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
            if ((st = prepare(p, in, out, bank, n))) break;
            const float ms = time_it([&] { run_walk(p, l); });
            if (ms < best) {
                best = ms;
                best_walk[l] = c;
            }
        }
        p->rows_walk[l] = best_walk[l];
        if (!st) st = prepare(p, in, out, bank, n);
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

mdn_status mdn_plan_kernel_times(mdn_plan* p, const mdn_image* in, const mdn_image* out, const int32_t* bank,
                                 int32_t n, int32_t reps, float* us_out, void* stream) {
    clear_error();
    if (!p) return fail(MDN_EINVAL, "plan: null");
    mdn_status st = check_batch(p, in, out, bank, n);
    if (st) return st;
    if (reps < 1 || reps > 1000) return fail(MDN_EINVAL, "plan: reps must be 1..1000");
    if (!us_out) return fail(MDN_EINVAL, "plan: null output");
    hipStream_t cs = static_cast<hipStream_t>(stream);
    if (hipEventRecord(p->ev_in, cs) != hipSuccess || hipStreamWaitEvent(p->stream, p->ev_in, 0) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: stream ordering failed");
    std::vector<uint64_t> sig = signature(in, out, bank, n);
    if (!(p->tables_valid && sig == p->sig)) {
        drop_graph(p);
        if ((st = prepare(p, in, out, bank, n))) return st;
        p->sig = sig;
    }
    // the launches of one batch in their usual order, each between two events on the plan's stream
    // and started on an idle stream (events recorded between back-to-back launches have been seen to
    // miss part of the second launch)
    const int L = p->Lmax, nk = 3 * L;
    std::vector<hipEvent_t> ev(2 * (size_t)nk * reps, nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            st = fail(MDN_EDEVICE, "plan: event creation failed");
            break;
        }
    auto slot = [&](int r, int l, int k) { return 2 * ((size_t)r * nk + 3 * l + k); };
    auto timed = [&](size_t i, auto&& fn) -> mdn_status {
        if (hipEventRecord(ev[i], p->stream) != hipSuccess) return fail(MDN_EDEVICE, "plan: event record failed");
        mdn_status e = fn();
        if (e) return e;
        if (hipEventRecord(ev[i + 1], p->stream) != hipSuccess) return fail(MDN_EDEVICE, "plan: event record failed");
        if (hipEventSynchronize(ev[i + 1]) != hipSuccess) return fail(MDN_EDEVICE, "plan: event wait failed");
        return MDN_OK;
    };
    std::vector<char> fused(L, 0);
    for (int r = 0; r < reps && !st; ++r) {
        for (int l = 0; l < L && !st; ++l)
            st = timed(slot(r, l, 0), [&] {
                bool f = false;
                const mdn_status e = run_d2_fused(p, l, &f);
                fused[l] = f;
                return e;
            });
        for (int l = L - 1; l >= 0 && !st; --l) {
            if (!fused[l]) st = timed(slot(r, l, 1), [&] { return run_sel(p, l); });
            if (!st) st = timed(slot(r, l, 2), [&] { return run_walk(p, l); });
        }
    }
    if (!st && hipEventSynchronize(ev.back()) != hipSuccess) st = fail(MDN_EDEVICE, "plan: event wait failed");
    for (int l = 0; l < L && !st; ++l)
        for (int k = 0; k < 3; ++k) {
            if (k == 1 && fused[l]) {
                us_out[3 * l + k] = 0.0f;       // the selection ran in the pyramid step's launch
                continue;
            }
            double sum = 0.0;
            for (int r = 0; r < reps; ++r) {
                float ms = 0.0f;
                hipEventElapsedTime(&ms, ev[slot(r, l, k)], ev[slot(r, l, k) + 1]);
                sum += ms;
            }
            us_out[3 * l + k] = (float)(sum * 1e3 / reps);
        }
    for (auto& e : ev)
        if (e) hipEventDestroy(e);
    if (st) return st;
    if (hipEventRecord(p->ev_out, p->stream) != hipSuccess || hipStreamWaitEvent(cs, p->ev_out, 0) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: stream ordering failed");
    return check_launch("kernel_times");
}

mdn_status mdn_denoise_batch(mdn_plan* p, const mdn_image* in, const mdn_image* out, const int32_t* bank, int32_t n,
                             int32_t use_graph, void* stream) {
    clear_error();
    if (!p) return fail(MDN_EINVAL, "plan: null");
    mdn_status st = check_batch(p, in, out, bank, n);
    if (st) return st;
    hipStream_t cs = static_cast<hipStream_t>(stream);
    if (hipEventRecord(p->ev_in, cs) != hipSuccess || hipStreamWaitEvent(p->stream, p->ev_in, 0) != hipSuccess)
        return fail(MDN_EDEVICE, "plan: stream ordering failed");
    std::vector<uint64_t> sig = signature(in, out, bank, n);
    const bool same = p->tables_valid && sig == p->sig;
    if (!same) {
        drop_graph(p);
        if ((st = prepare(p, in, out, bank, n))) return st;
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
