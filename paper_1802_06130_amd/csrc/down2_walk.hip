// Pyramid launches: the persistent column-walk kernel over a list of strips (the strip's work is in
// down2_walk.h), its strip heights and its launcher.

#include "down2_walk.h"

#include <string.h>

namespace mdn {

namespace {

constexpr int kWaves = 4;

template <typename TI, typename TO, int C>
__global__ __launch_bounds__(64 * kWaves) void k_down2_walk(D2Args a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int strip = blockIdx.x * kWaves + wave; strip < a.n_strips; strip += gridDim.x * kWaves)
        d2w::strip<TI, TO, C>(a, strip, lane);
}

}  // namespace

int down2_rows(int wo, int ho, int ncu) {
    const int nsx = (wo + kD2LanesOut - 1) / kD2LanesOut;
    int rows = 64;
    while (rows > 8 && (int64_t)nsx * ((ho + rows - 1) / rows) < (int64_t)ncu * kWaves * 4) rows -= 8;
    return rows;
}

mdn_status launch_down2_args(const D2Args& a, int C, int in_dtype, int out_dtype, hipStream_t st) {
    if (a.n_strips <= 0) return MDN_OK;
    const int ncu = device_cus();
    const int blocks = (a.n_strips + kWaves - 1) / kWaves;
    const int grid = blocks < 8 * ncu ? blocks : 8 * ncu;
#define MDN_D2(TI_, TO_, DI_, DO_)                                                        \
    if (in_dtype == DI_ && out_dtype == DO_) {                                            \
        if (C == 3) k_down2_walk<TI_, TO_, 3><<<grid, 64 * kWaves, 0, st>>>(a);           \
        else k_down2_walk<TI_, TO_, 1><<<grid, 64 * kWaves, 0, st>>>(a);                  \
        return check_launch("down2_walk");                                                \
    }
    MDN_D2(float, float, MDN_F32, MDN_F32)
    MDN_D2(float, _Float16, MDN_F32, MDN_F16)
    MDN_D2(_Float16, _Float16, MDN_F16, MDN_F16)
    MDN_D2(_Float16, float, MDN_F16, MDN_F32)
#undef MDN_D2
    return fail(MDN_EINVAL, "down2: unsupported dtype pair");
}

void fill_down2_single(const mdn_image& in, const mdn_image& out, D2Args& a) {
    memset(&a, 0, sizeof(a));
    D2Image& im = a.single;
    im.in = in.data;
    im.out = out.data;
    im.i_row = in.row_pitch;
    im.i_plane = in.plane_pitch;
    im.o_row = out.row_pitch;
    im.o_plane = out.plane_pitch;
    im.Wi = in.width;
    im.Hi = in.height;
    im.Wo = out.width;
    im.Ho = out.height;
    im.nsx = (out.width + kD2LanesOut - 1) / kD2LanesOut;
    im.rows = down2_rows(out.width, out.height, device_cus());
    a.n_imgs = 1;
    a.n_strips = im.nsx * ((out.height + im.rows - 1) / im.rows);
}

mdn_status launch_down2_walk(const mdn_image& in, const mdn_image& out, hipStream_t st) {
    if (out.width == 0 || out.height == 0) return MDN_OK;
    D2Args a;
    fill_down2_single(in, out, a);
    return launch_down2_args(a, in.channels, in.dtype, out.dtype, st);
}

}  // namespace mdn
