// C ABI entry points: argument validation, workspace carving and launch sequencing.

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "mdn_internal.h"

namespace mdn {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

mdn_status fail(mdn_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

mdn_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MDN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return MDN_OK;
}

int64_t elem_size(int32_t dtype) { return dtype == MDN_F16 ? 2 : 4; }

void clear_error() { g_err[0] = 0; }

namespace {

bool empty(const mdn_image& im) { return im.width == 0 || im.height == 0; }

mdn_status check_image(const mdn_image* im, const char* name) {
    if (!im) return fail(MDN_EINVAL, "%s: null image", name);
    if (im->width < 0 || im->height < 0) return fail(MDN_EINVAL, "%s: negative size", name);
    if (im->channels != 1 && im->channels != 3) return fail(MDN_EINVAL, "%s: channels must be 1 or 3", name);
    if (im->dtype != MDN_F32 && im->dtype != MDN_F16) return fail(MDN_EINVAL, "%s: unknown dtype", name);
    if (im->color != MDN_GRAY && im->color != MDN_RGB && im->color != MDN_YCC)
        return fail(MDN_EINVAL, "%s: unknown colour", name);
    if ((im->channels == 1) != (im->color == MDN_GRAY))
        return fail(MDN_EINVAL, "%s: colour does not match channel count", name);
    if (im->reserved != 0) return fail(MDN_EINVAL, "%s: reserved field must be 0", name);
    if (empty(*im)) return MDN_OK;
    if (!im->data) return fail(MDN_EINVAL, "%s: null data", name);
    if (im->row_pitch < im->width) return fail(MDN_EINVAL, "%s: row_pitch < width", name);
    if (im->channels > 1 && im->plane_pitch < im->row_pitch * im->height)
        return fail(MDN_EINVAL, "%s: plane_pitch < height*row_pitch", name);
    // kernels address an image with 32-bit byte offsets from its base
    const int64_t extent = ((int64_t)(im->channels - 1) * im->plane_pitch + (int64_t)(im->height - 1) * im->row_pitch +
                            im->width) * (im->dtype == MDN_F16 ? 2 : 4);
    if (extent >= ((int64_t)1 << 31)) return fail(MDN_ENOTSUP, "%s: image spans 2 GiB or more", name);
    return MDN_OK;
}

mdn_status check_level(const mdn_level* lv, int channels) {
    if (!lv) return fail(MDN_EINVAL, "level: null");
    if (lv->selector != MDN_SELECT_RGB && lv->selector != MDN_SELECT_LUMA && lv->selector != MDN_SELECT_COARSE)
        return fail(MDN_EINVAL, "level: selector must be MDN_SELECT_RGB, MDN_SELECT_LUMA or MDN_SELECT_COARSE");
    if (lv->selector == MDN_SELECT_COARSE && lv->radius_f < 1)
        return fail(MDN_EINVAL, "level: a single-scale level has no coarser output to select on");
    if (lv->q_theta < 2 || lv->q_theta > kMaxTheta || (lv->q_theta & 1))
        return fail(MDN_EINVAL, "level: q_theta must be even in [2, %d]", kMaxTheta);
    if (lv->q_s < 1 || lv->q_s > kMaxThr || lv->q_c < 1 || lv->q_c > kMaxThr)
        return fail(MDN_EINVAL, "level: q_s and q_c must be in [1, %d]", kMaxThr);
    if (lv->phases != 1 && lv->phases != 4) return fail(MDN_EINVAL, "level: phases must be 1 or 4");
    if (lv->reserved != 0) return fail(MDN_EINVAL, "level: reserved field must be 0");
    const int K = level_buckets(*lv);
    if (K > 65536) return fail(MDN_ENOTSUP, "level: K = %d > 65536 buckets is not supported (uint16 selector)", K);
    if (lv->channels != channels) return fail(MDN_EINVAL, "level: channels %d != image channels %d", lv->channels, channels);
    if (lv->coeff_dtype != MDN_F32 && lv->coeff_dtype != MDN_F16) return fail(MDN_EINVAL, "level: unknown coeff dtype");
    if (lv->radius_g < 1 || lv->radius_g > 3) return fail(MDN_ENOTSUP, "level: radius_g must be 1..3");
    if (lv->radius_f > 3) return fail(MDN_ENOTSUP, "level: radius_f must be -1 or 1..3");
    if (lv->radius_f == 0) return fail(MDN_ENOTSUP, "level: radius_f must be -1 or 1..3");
    if (!lv->coeffs) return fail(MDN_EINVAL, "level: null coeffs");
    if (lv->q_s > 1 && !lv->t_s) return fail(MDN_EINVAL, "level: null t_s");
    if (lv->q_c > 1 && !lv->t_c) return fail(MDN_EINVAL, "level: null t_c");
    for (int j = 1; j < lv->q_s - 1; ++j)
        if (!(lv->t_s[j] >= lv->t_s[j - 1])) return fail(MDN_EINVAL, "level: t_s not ascending");
    for (int j = 1; j < lv->q_c - 1; ++j)
        if (!(lv->t_c[j] >= lv->t_c[j - 1])) return fail(MDN_EINVAL, "level: t_c not ascending");
    return MDN_OK;
}

int half_up(int v) { return (v + 1) / 2; }

int64_t pitch_for(int w) { return ((int64_t)w + 63) / 64 * 64; }

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

mdn_image plane_image(void* data, int w, int h, int c, int dtype, int color) {
    mdn_image im;
    memset(&im, 0, sizeof(im));
    im.data = data;
    im.width = w;
    im.height = h;
    im.channels = c;
    im.dtype = dtype;
    im.color = color;
    im.row_pitch = pitch_for(w);
    im.plane_pitch = im.row_pitch * h;
    return im;
}

size_t image_bytes(int w, int h, int c, int dtype) {
    return align256((size_t)pitch_for(w) * (size_t)h * (size_t)c * (size_t)elem_size(dtype));
}


mdn_status check_gram(const mdn_gram* g) {
    if (!g) return fail(MDN_EINVAL, "gram: null");
    if (g->reserved != 0) return fail(MDN_EINVAL, "gram: reserved field must be 0");
    if (g->K < 1 || g->K > 65536) return fail(MDN_EINVAL, "gram: K must be 1..65536");
    if (g->channels != 1 && g->channels != 3) return fail(MDN_EINVAL, "gram: channels must be 1 or 3");
    if (g->layout != MDN_X_PER_CHANNEL && g->layout != MDN_X_CROSS_CHANNEL) return fail(MDN_EINVAL, "gram: layout");
    if (g->radius_g < 1 || g->radius_g > 3) return fail(MDN_ENOTSUP, "gram: radius_g must be 1..3");
    if (!(g->radius_f == -1 || (g->radius_f >= 1 && g->radius_f <= 3))) return fail(MDN_ENOTSUP, "gram: radius_f");
    if (g->layout == MDN_X_CROSS_CHANNEL && g->radius_f != -1) return fail(MDN_EINVAL, "gram: cross layout has no upscale block");
    int D, nrhs, spk;
    gram_dims(*g, &D, &nrhs, &spk);
    if (D + nrhs > kMaxFeat) return fail(MDN_ENOTSUP, "gram: %d features exceed %d", D + nrhs, kMaxFeat);
    if (!g->G || !g->b || !g->n || !g->yy) return fail(MDN_EINVAL, "gram: null accumulator");
    return MDN_OK;
}

}  // namespace

mdn_status validate_level(const mdn_level* lv, int channels) { return check_level(lv, channels); }

}  // namespace mdn

using namespace mdn;

extern "C" {

const char* mdn_last_error(void) { return g_err; }

const char* mdn_version(void) { return "mdn 0.1 (gfx950)"; }

mdn_status mdn_pyramid_build(const mdn_image* level0, int32_t n_out, const mdn_image* out, void* stream) {
    g_err[0] = 0;
    mdn_status st = check_image(level0, "level0");
    if (st) return st;
    if (n_out < 0) return fail(MDN_EINVAL, "n_out < 0");
    if (n_out > 0 && !out) return fail(MDN_EINVAL, "null out");
    int w = level0->width, h = level0->height;
    for (int i = 0; i < n_out; ++i) {
        if ((st = check_image(&out[i], "out"))) return st;
        w = half_up(w);
        h = half_up(h);
        if (out[i].width != w || out[i].height != h)
            return fail(MDN_EINVAL, "out[%d] must be %d x %d, got %d x %d", i, w, h, out[i].width, out[i].height);
        if (out[i].channels != level0->channels || out[i].color != level0->color)
            return fail(MDN_EINVAL, "out[%d]: channels/colour differ from level 0", i);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const mdn_image* prev = level0;
    for (int i = 0; i < n_out; ++i) {
        if (empty(*prev)) break;
        if ((st = launch_down2(*prev, out[i], s))) return st;
        prev = &out[i];
    }
    return MDN_OK;
}

mdn_status mdn_dihedral(const mdn_image* in, int32_t transform, const mdn_image* out, void* stream) {
    g_err[0] = 0;
    mdn_status st = check_image(in, "in");
    if (st) return st;
    if ((st = check_image(out, "out"))) return st;
    if (transform < 0 || transform > 7) return fail(MDN_EINVAL, "transform must be in [0, 7], got %d", transform);
    const int w = (transform & 4) ? in->height : in->width, h = (transform & 4) ? in->width : in->height;
    if (out->width != w || out->height != h)
        return fail(MDN_EINVAL, "out must be %d x %d, got %d x %d", w, h, out->width, out->height);
    if (out->channels != in->channels || out->dtype != in->dtype || out->color != in->color)
        return fail(MDN_EINVAL, "out: channels, dtype and colour must equal the input's");
    if (!empty(*in) && in->data == out->data) return fail(MDN_EINVAL, "out must not alias in");
    return launch_dihedral(*in, *out, transform, static_cast<hipStream_t>(stream));
}

mdn_status mdn_select_filters(const mdn_image* z, const mdn_level* lvl, void* s_out, int64_t s_pitch,
                              void* stream) {
    g_err[0] = 0;
    mdn_status st = check_image(z, "z");
    if (st) return st;
    if (z->color == MDN_YCC) return fail(MDN_EINVAL, "z: the selector reads RGB or grey images");
    if ((st = check_level(lvl, z->channels))) return st;
    if (lvl->selector == MDN_SELECT_COARSE)
        return fail(MDN_EINVAL, "level selects on the coarser output: use mdn_select_filters_coarse");
    if (empty(*z)) return MDN_OK;
    if (!s_out) return fail(MDN_EINVAL, "null s_out");
    if (s_pitch < z->width) return fail(MDN_EINVAL, "s_pitch < width");
    return launch_select_apply(*z, nullptr, nullptr, s_pitch, s_out, *lvl, nullptr, static_cast<hipStream_t>(stream));
}

// The fine level's size, as an image without data (the coarse selector reads only u_coarse).
static mdn_status coarse_target(const mdn_image* u_coarse, int32_t width, int32_t height, mdn_image* z) {
    mdn_status st = check_image(u_coarse, "u_coarse");
    if (st) return st;
    if (width < 0 || height < 0) return fail(MDN_EINVAL, "negative size");
    if (u_coarse->width != half_up(width) || u_coarse->height != half_up(height))
        return fail(MDN_EINVAL, "u_coarse must be ceil(width/2) x ceil(height/2)");
    memset(z, 0, sizeof(*z));
    z->width = width;
    z->height = height;
    z->channels = u_coarse->channels;
    z->dtype = MDN_F32;
    z->color = u_coarse->channels == 3 ? MDN_RGB : MDN_GRAY;
    z->row_pitch = width;
    z->plane_pitch = (int64_t)width * height;
    return MDN_OK;
}

mdn_status mdn_select_filters_coarse(const mdn_image* u_coarse, int32_t width, int32_t height, const mdn_level* lvl,
                                     void* s_out, int64_t s_pitch, void* stream) {
    g_err[0] = 0;
    mdn_image z;
    mdn_status st = coarse_target(u_coarse, width, height, &z);
    if (st) return st;
    if ((st = check_level(lvl, u_coarse->channels))) return st;
    if (lvl->selector != MDN_SELECT_COARSE) return fail(MDN_EINVAL, "level does not select on the coarser output");
    if (width == 0 || height == 0) return MDN_OK;
    if (!s_out) return fail(MDN_EINVAL, "null s_out");
    if (s_pitch < width) return fail(MDN_EINVAL, "s_pitch < width");
    return launch_select_apply(z, u_coarse, nullptr, s_pitch, s_out, *lvl, nullptr, static_cast<hipStream_t>(stream));
}

mdn_status mdn_apply_level(const mdn_image* z, const mdn_image* u_coarse, const void* s, int64_t s_pitch,
                           const mdn_level* lvl, const mdn_image* u_out, void* s_out, void* stream) {
    g_err[0] = 0;
    mdn_status st = check_image(z, "z");
    if (st) return st;
    if (z->color == MDN_YCC) return fail(MDN_EINVAL, "z: pass the level as RGB or grey");
    if ((st = check_level(lvl, z->channels))) return st;
    if ((st = check_image(u_out, "u_out"))) return st;
    if (u_out->width != z->width || u_out->height != z->height || u_out->channels != z->channels)
        return fail(MDN_EINVAL, "u_out must match z in size and channels");
    if (lvl->radius_f >= 1) {
        if ((st = check_image(u_coarse, "u_coarse"))) return st;
        if (u_coarse->width != half_up(z->width) || u_coarse->height != half_up(z->height))
            return fail(MDN_EINVAL, "u_coarse must be ceil(w/2) x ceil(h/2)");
        if (u_coarse->channels != z->channels) return fail(MDN_EINVAL, "u_coarse channels differ");
    } else if (u_coarse) {
        return fail(MDN_EINVAL, "u_coarse given for a single-scale level");
    }
    if (empty(*z)) return MDN_OK;
    if ((s || s_out) && s_pitch < z->width) return fail(MDN_EINVAL, "s_pitch < width");
    if (s && s_out) return fail(MDN_EINVAL, "give either a selector or a selector output, not both");
    return launch_select_apply(*z, lvl->radius_f >= 1 ? u_coarse : nullptr, s, s_pitch, s_out, *lvl, u_out,
                               static_cast<hipStream_t>(stream));
}

mdn_status mdn_denoise_workspace_size(int32_t width, int32_t height, int32_t channels, int32_t levels,
                                      int32_t storage, size_t* bytes) {
    g_err[0] = 0;
    if (!bytes) return fail(MDN_EINVAL, "null bytes");
    if (width < 0 || height < 0) return fail(MDN_EINVAL, "negative size");
    if (channels != 1 && channels != 3) return fail(MDN_EINVAL, "channels must be 1 or 3");
    if (levels < 1 || levels > 16) return fail(MDN_EINVAL, "levels must be 1..16");
    if (storage != MDN_F32 && storage != MDN_F16) return fail(MDN_EINVAL, "unknown storage dtype");
    size_t total = 0;
    int w = width, h = height;
    for (int l = 1; l <= levels; ++l) {
        w = half_up(w);
        h = half_up(h);
        total += image_bytes(w, h, channels, storage);                 // z^l
        if (l < levels) total += image_bytes(w, h, channels, storage); // u^l
    }
    w = width;
    h = height;
    for (int l = 0; l < levels; ++l) {                                   // selector map of level l
        total += align256((size_t)w * (size_t)h);
        w = half_up(w);
        h = half_up(h);
    }
    *bytes = total;
    return MDN_OK;
}

mdn_status mdn_denoise(const mdn_image* in, const mdn_bank* bank, int32_t storage, void* ws, size_t ws_bytes,
                       const mdn_image* out, void* stream) {
    g_err[0] = 0;
    mdn_status st = check_image(in, "in");
    if (st) return st;
    if (in->color == MDN_YCC) return fail(MDN_EINVAL, "in: pass RGB or grey");
    if ((st = check_image(out, "out"))) return st;
    if (out->width != in->width || out->height != in->height || out->channels != in->channels ||
        out->color != in->color)
        return fail(MDN_EINVAL, "out must match in");
    if (!bank || bank->levels < 1 || bank->levels > 16 || !bank->level)
        return fail(MDN_EINVAL, "bank: need 1..16 levels");
    const int L = bank->levels;
    for (int l = 0; l < L; ++l) {
        if ((st = check_level(&bank->level[l], in->channels))) return st;
        const bool ms = bank->level[l].radius_f >= 1;
        if (ms != (bank->level[0].radius_f >= 1)) return fail(MDN_EINVAL, "bank: mixed single/multiscale levels");
    }
    const bool multiscale = bank->level[0].radius_f >= 1;
    if (!multiscale && L != 1) return fail(MDN_EINVAL, "bank: a single-scale bank has exactly one level");
    if (storage != MDN_F32 && storage != MDN_F16) return fail(MDN_EINVAL, "unknown storage dtype");
    if (empty(*in)) return MDN_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!multiscale) return launch_select_apply(*in, nullptr, nullptr, 0, nullptr, bank->level[0], out, s);

    size_t need = 0;
    if ((st = mdn_denoise_workspace_size(in->width, in->height, in->channels, L, storage, &need))) return st;
    if (!ws || ws_bytes < need) return fail(MDN_ENOMEM, "workspace: need %zu bytes, got %zu", need, ws_bytes);
    if (((uintptr_t)ws) & 255) return fail(MDN_EINVAL, "workspace must be 256-byte aligned");

    const int C = in->channels;
    const int sel_color = in->color;
    const int filt_color = C == 3 ? MDN_YCC : MDN_GRAY;
    mdn_image zl[17], ul[17];
    char* p = static_cast<char*>(ws);
    int w = in->width, h = in->height;
    for (int l = 1; l <= L; ++l) {
        w = half_up(w);
        h = half_up(h);
        zl[l] = plane_image(p, w, h, C, storage, sel_color);
        p += image_bytes(w, h, C, storage);
        if (l < L) {
            ul[l] = plane_image(p, w, h, C, storage, filt_color);
            p += image_bytes(w, h, C, storage);
        }
    }
    zl[0] = *in;
    // uint8 selector maps, one per level: they serve the column walk and the LDS-bank kernel
    uint8_t* smap[17];
    for (int l = 0; l < L; ++l) {
        smap[l] = reinterpret_cast<uint8_t*>(p);
        p += align256((size_t)zl[l].width * (size_t)zl[l].height);
    }
    auto uses_map = [&](int l) {
        const mdn_level& lv = bank->level[l];
        return (lv.coeff_dtype == MDN_F16 && walk_supported(lv, C)) || (!wide_selector(lv) && apply_lds_supported(lv, C));
    };
    // pyramid steps; a level whose filtering reads a map has its selection pass in the same launch
    bool selected[17] = {};
    for (int l = 0; l < L; ++l) {
        const mdn_level& lv = bank->level[l];
        if (uses_map(l) && pyr_sel_fits(lv, C)) {
            st = launch_pyr_sel(zl[l], zl[l + 1], lv, smap[l], zl[l].width, s);
            selected[l] = true;
        } else {
            st = launch_down2(zl[l], zl[l + 1], s);
        }
        if (st) return st;
    }
    // u^L = z^L (read as RGB and converted by the level L-1 step)
    const mdn_image* coarse = &zl[L];
    for (int l = L - 1; l >= 0; --l) {
        const mdn_image* dst = l == 0 ? out : &ul[l];
        const mdn_level& lv = bank->level[l];
        const bool map = uses_map(l);
        if ((st = launch_select_apply(zl[l], coarse, selected[l] ? smap[l] : nullptr, zl[l].width,
                                      map && !selected[l] ? smap[l] : nullptr, lv, dst, s)))
            return st;
        coarse = dst;
    }
    return MDN_OK;
}


mdn_status mdn_gram_dims(const mdn_gram* g, int32_t* D, int32_t* nrhs, int32_t* systems) {
    g_err[0] = 0;
    mdn_status st = check_gram(g);
    if (st && st != MDN_EINVAL) return st;
    if (!g) return st;
    if (!D || !nrhs || !systems) return fail(MDN_EINVAL, "null output");
    int d, r, spk;
    gram_dims(*g, &d, &r, &spk);
    *D = d;
    *nrhs = r;
    *systems = g->K * spk;
    return MDN_OK;
}

mdn_status mdn_gram_zero(const mdn_gram* g, void* stream) {
    g_err[0] = 0;
    mdn_status st = check_gram(g);
    if (st) return st;
    return gram_zero(*g, static_cast<hipStream_t>(stream));
}

mdn_status mdn_train_workspace_size(const mdn_gram* g, int32_t width, int32_t height, size_t* bytes) {
    g_err[0] = 0;
    if (!bytes) return fail(MDN_EINVAL, "null bytes");
    mdn_status st = check_gram(g);
    if (st) return st;
    if (width < 0 || height < 0) return fail(MDN_EINVAL, "negative size");
    *bytes = train_ws_bytes(*g, width, height);
    return MDN_OK;
}

mdn_status mdn_train_accumulate(const mdn_gram* g, const mdn_image* z, const mdn_image* u_coarse,
                                const mdn_image* target, const mdn_level* sel, int32_t precision, void* ws,
                                size_t ws_bytes, void* stream) {
    g_err[0] = 0;
    mdn_status st = check_gram(g);
    if (st) return st;
    if ((st = check_image(z, "z"))) return st;
    if (z->color == MDN_YCC) return fail(MDN_EINVAL, "z: pass RGB or grey");
    if ((st = check_image(target, "target"))) return st;
    if (target->width != z->width || target->height != z->height || target->channels != z->channels ||
        target->color == MDN_YCC)
        return fail(MDN_EINVAL, "target must match z (RGB or grey)");
    if (z->channels != g->channels) return fail(MDN_EINVAL, "gram channels differ from the image's");
    if ((st = check_level(sel, z->channels))) return st;
    if (level_buckets(*sel) != g->K) return fail(MDN_EINVAL, "selector K differs from gram K");
    if (sel->selector == MDN_SELECT_COARSE && g->radius_f < 1)
        return fail(MDN_EINVAL, "the coarse selector needs a layout with the coarser output");
    if (precision != MDN_GRAM_F32 && precision != MDN_GRAM_BF16X3) return fail(MDN_EINVAL, "unknown precision");
    if (g->radius_f >= 1) {
        if ((st = check_image(u_coarse, "u_coarse"))) return st;
        if (u_coarse->width != half_up(z->width) || u_coarse->height != half_up(z->height) ||
            u_coarse->channels != z->channels)
            return fail(MDN_EINVAL, "u_coarse must be ceil(w/2) x ceil(h/2) with the same channels");
    } else if (u_coarse) {
        return fail(MDN_EINVAL, "u_coarse given for a layout without upscale block");
    }
    if (empty(*z)) return MDN_OK;
    {
        // the sample gathers address the float32 planes with 32-bit element offsets
        const int64_t px = (int64_t)z->width * z->height;
        const int64_t elems = 2 * px * z->channels + (int64_t)half_up(z->width) * half_up(z->height) * z->channels + 256;
        if (elems > 0x7fffffffLL) return fail(MDN_ENOTSUP, "train_accumulate: image too large (2^31 elements)");
    }
    if (!ws || ws_bytes < train_ws_bytes(*g, z->width, z->height))
        return fail(MDN_ENOMEM, "workspace too small (need %zu)", train_ws_bytes(*g, z->width, z->height));
    if (((uintptr_t)ws) & 255) return fail(MDN_EINVAL, "workspace must be 256-byte aligned");
    return train_accumulate(*g, *z, g->radius_f >= 1 ? u_coarse : nullptr, *target, *sel, precision, ws,
                            static_cast<hipStream_t>(stream));
}

mdn_status mdn_train_solve_workspace_size(const mdn_gram* g, size_t* bytes) {
    g_err[0] = 0;
    mdn_status st = check_gram(g);
    if (st) return st;
    if (!bytes) return fail(MDN_EINVAL, "null bytes");
    *bytes = solve_ws_bytes(*g);
    return MDN_OK;
}

mdn_status mdn_train_solve(const mdn_gram* g, double lambda, int64_t min_count, void* coeffs, int32_t coeff_dtype,
                           int32_t* n_fallback, void* ws, size_t ws_bytes, void* stream) {
    g_err[0] = 0;
    mdn_status st = check_gram(g);
    if (st) return st;
    if (!(lambda >= 0.0)) return fail(MDN_EINVAL, "lambda must be >= 0");
    if (!coeffs) return fail(MDN_EINVAL, "null coeffs");
    if (coeff_dtype != MDN_F32 && coeff_dtype != MDN_F16) return fail(MDN_EINVAL, "unknown coeff dtype");
    if (!ws || ws_bytes < solve_ws_bytes(*g)) return fail(MDN_ENOMEM, "workspace too small (need %zu)", solve_ws_bytes(*g));
    if (((uintptr_t)ws) & 255) return fail(MDN_EINVAL, "workspace must be 256-byte aligned");
    return train_solve(*g, lambda, min_count, coeffs, coeff_dtype, n_fallback, ws, static_cast<hipStream_t>(stream));
}

mdn_status mdn_level_features(const mdn_image* z, int32_t selector, double* strength, double* coherence,
                              void* stream) {
    g_err[0] = 0;
    mdn_status st = check_image(z, "z");
    if (st) return st;
    if (selector == MDN_SELECT_COARSE)
        return fail(MDN_EINVAL, "features of the coarser output: use mdn_level_features_coarse");
    if (selector != MDN_SELECT_RGB && selector != MDN_SELECT_LUMA)
        return fail(MDN_EINVAL, "selector must be MDN_SELECT_RGB or MDN_SELECT_LUMA");
    if (z->color == MDN_YCC) return fail(MDN_EINVAL, "z: pass RGB or grey");
    if (empty(*z)) return MDN_OK;
    if (!strength || !coherence) return fail(MDN_EINVAL, "null output");
    return launch_features(*z, selector == MDN_SELECT_LUMA, nullptr, strength, coherence,
                           static_cast<hipStream_t>(stream));
}

mdn_status mdn_level_features_coarse(const mdn_image* u_coarse, int32_t width, int32_t height, double* strength,
                                     double* coherence, void* stream) {
    g_err[0] = 0;
    mdn_image z;
    mdn_status st = coarse_target(u_coarse, width, height, &z);
    if (st) return st;
    if (width == 0 || height == 0) return MDN_OK;
    if (!strength || !coherence) return fail(MDN_EINVAL, "null output");
    return launch_features(z, 0, u_coarse, strength, coherence, static_cast<hipStream_t>(stream));
}

mdn_status mdn_quantiles_workspace_size(int64_t n, size_t* bytes) {
    g_err[0] = 0;
    if (!bytes) return fail(MDN_EINVAL, "null bytes");
    if (n < 1 || n > 2000000000LL) return fail(MDN_EINVAL, "n must be 1..2e9");
    *bytes = quantile_ws_bytes(n);
    return MDN_OK;
}

mdn_status mdn_quantiles(const double* values, int64_t n, int32_t q, double* out_host, void* ws, size_t ws_bytes,
                         void* stream) {
    g_err[0] = 0;
    if (!values || !out_host) return fail(MDN_EINVAL, "null pointer");
    if (n < 1 || n > 2000000000LL) return fail(MDN_EINVAL, "n must be 1..2e9");
    if (q < 2 || q > 64) return fail(MDN_EINVAL, "q must be 2..64");
    if (!ws || ws_bytes < quantile_ws_bytes(n)) return fail(MDN_ENOMEM, "workspace too small");
    return quantiles(values, n, q, out_host, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"
