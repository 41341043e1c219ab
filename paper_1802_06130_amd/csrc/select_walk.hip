// Selection launches: the persistent column-walk kernel over a list of strips (the strip's work is
// in select_walk.h), its strip heights, the per-level constants and the launcher. The kernel is
// held to 128 registers per lane so that four waves share each SIMD and hide one another's
// latencies.

#include "select_walk.h"

#include <string.h>

namespace mdn {

namespace {

#ifndef MDN_SEL_WAVES_PER_SIMD
#define MDN_SEL_WAVES_PER_SIMD 4
#endif
constexpr int kWaves = 4;
using sw::kLanesOut;

template <typename TZ, typename TS, int C, bool LUMA, int QS, int QC, int MQ, int NSTEP>
__global__ __launch_bounds__(64 * kWaves, MDN_SEL_WAVES_PER_SIMD) void k_select_walk(SelWalkArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    __shared__ sw::BoundaryTable bt;
    // per wave: one row of A, B and C products with two zero pads on each side, for the 5-wide
    // horizontal box sums (lanes exchange through LDS: no barrier is needed within a wave)
    __shared__ double hbox[kWaves][3][sw::kHboxW];
    sw::prologue(a, bt, &hbox[0][0][0], kWaves * 3 * sw::kHboxW, 64 * kWaves);
    __syncthreads();
    for (int strip = blockIdx.x * kWaves + wave; strip < a.n_strips; strip += gridDim.x * kWaves)
        sw::strip<TZ, TS, C, LUMA, QS, QC, MQ, NSTEP>(a, strip, lane, bt, &hbox[wave][0][0]);
}

}  // namespace

int select_walk_rows(int w, int h, int ncu) {
    // enough strips to give every SIMD a few waves, at most 60 rows (a multiple of 10)
    const int nsx = (w + kLanesOut - 1) / kLanesOut;
    int rows = 60;
    while (rows > 10 && (int64_t)nsx * ((h + rows - 1) / rows) < (int64_t)ncu * 4 * 3) rows -= 10;
    return rows;
}

void fill_sel_consts(const mdn_level& lvl, SelWalkArgs& a) {
    a.q_theta = lvl.q_theta;
    a.q_s = lvl.q_s;
    a.q_c = lvl.q_c;
    a.half = lvl.q_theta / 2;
    a.luma = lvl.selector == MDN_SELECT_LUMA && lvl.channels == 3;
    a.phases = lvl.phases;
    for (int j = 0; j < lvl.q_s - 1; ++j) {
        const double t = lvl.t_s[j] > 0.0 ? lvl.t_s[j] : 0.0;
        a.s_lim[j] = 100.0 * t * t;
    }
    for (int j = 0; j < lvl.q_c - 1; ++j) {
        const double t = lvl.t_c[j];
        if (t <= 0.0) {
            a.c_k2[j] = -1.0;
        } else {
            const double k = 2.0 * t / (1.0 + t * t);
            a.c_k2[j] = k * k;
        }
    }
    orientation_boundaries(lvl.q_theta, a.bcos, a.bsin);
}

mdn_status launch_select_args(const SelWalkArgs& a, int channels, int z_dtype, hipStream_t st) {
    if (a.n_strips <= 0) return MDN_OK;
    const int ncu = device_cus();
    const int blocks = (a.n_strips + kWaves - 1) / kWaves;
    const int grid = blocks < 8 * ncu ? blocks : 8 * ncu;
    // 3 x 3 strength/coherence bins with 24 or 16 orientation bins get fixed-count instances
    const bool wide = a.q_theta * a.q_s * a.q_c * a.phases > 256;      // uint16 selector map
    const int spec = (!wide && a.q_s == 3 && a.q_c == 3) ? (a.q_theta == 24 ? 1 : a.q_theta == 16 ? 2 : 0) : 0;
#define MDN_SEL_LAUNCH(TZ_, C_, L_)                                                                 \
    do {                                                                                               \
        if (spec == 1) k_select_walk<TZ_, uint8_t, C_, L_, 3, 3, 5, 0><<<grid, 64 * kWaves, 0, st>>>(a);         \
        else if (spec == 2) k_select_walk<TZ_, uint8_t, C_, L_, 3, 3, 3, 0><<<grid, 64 * kWaves, 0, st>>>(a);    \
        else if (wide) k_select_walk<TZ_, uint16_t, C_, L_, 0, 0, 0, 5><<<grid, 64 * kWaves, 0, st>>>(a);        \
        else k_select_walk<TZ_, uint8_t, C_, L_, 0, 0, 0, 5><<<grid, 64 * kWaves, 0, st>>>(a);                   \
    } while (0)
    if (channels == 3 && a.luma) {
        if (z_dtype == MDN_F16) MDN_SEL_LAUNCH(_Float16, 3, true);
        else MDN_SEL_LAUNCH(float, 3, true);
    } else if (channels == 3) {
        if (z_dtype == MDN_F16) MDN_SEL_LAUNCH(_Float16, 3, false);
        else MDN_SEL_LAUNCH(float, 3, false);
    } else {
        if (z_dtype == MDN_F16) MDN_SEL_LAUNCH(_Float16, 1, false);
        else MDN_SEL_LAUNCH(float, 1, false);
    }
#undef MDN_SEL_LAUNCH
    return check_launch("select_walk");
}

void fill_select_single(const mdn_image& z, const mdn_level& lvl, void* s, int64_t s_pitch, SelWalkArgs& a) {
    memset(&a, 0, sizeof(a));
    SelImage& im = a.single;
    im.z = z.data;
    im.s = s;
    im.z_row = z.row_pitch;
    im.z_plane = z.plane_pitch;
    im.s_pitch = s_pitch;
    im.W = z.width;
    im.H = z.height;
    im.C = z.channels;
    im.nsx = (z.width + kLanesOut - 1) / kLanesOut;
    im.rows = select_walk_rows(z.width, z.height, device_cus());
    im.strip_begin = 0;
    a.imgs = nullptr;
    a.n_imgs = 1;
    a.n_strips = im.nsx * ((z.height + im.rows - 1) / im.rows);
    fill_sel_consts(lvl, a);
}

mdn_status launch_select_walk(const mdn_image& z, const mdn_level& lvl, void* s, int64_t s_pitch, hipStream_t st) {
    if (z.width == 0 || z.height == 0) return MDN_OK;
    SelWalkArgs a;
    fill_select_single(z, lvl, s, s_pitch, a);
    return launch_select_args(a, z.channels, z.dtype, st);
}

}  // namespace mdn
