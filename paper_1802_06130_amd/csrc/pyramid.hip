// Factor-two bicubic downsampling (Section 4, "Multiscale filtering").
//
// Keys' cubic kernel with a = -1/2, stretched by two (anti-aliased) and centred at 2m + 1/2,
// sampled at the eight input offsets 2m-3 .. 2m+4: weights (-12, -36, 116, 444, 444, 116, -36,
// -12) / 1024. The separable filter runs rows first, then columns, in float64 with the integer
// weights; the 1/1024^2 scale is an exact power of two and the result is rounded once to the
// output type. For float32 or float16 inputs both passes are exact in float64 except in rare
// wide-exponent cases, so the stored level is the correctly rounded value of the exact filter.
//
// Layout: one 256-thread block makes a 16 x 64 output tile; the 39 x 135 input window (clamped
// at the borders) is staged in LDS, the horizontal pass writes 39 x 64 float64 partial rows to
// LDS, the vertical pass reads them and stores coalesced output rows.

#include "mdn_internal.h"

namespace mdn {

namespace {

constexpr int kTW = 64;               // output tile width
constexpr int kTH = 16;               // output tile height
constexpr int kIW = 2 * kTW + 7;      // input columns 2*ox0-3 .. 2*(ox0+kTW-1)+4
constexpr int kIH = 2 * kTH + 7;      // input rows

__device__ __forceinline__ double down2_w(int t) {
    // t = 0..7 <-> input offset t-3
    return t == 0 || t == 7 ? -12.0 : (t == 1 || t == 6 ? -36.0 : (t == 2 || t == 5 ? 116.0 : 444.0));
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_down2(ImageArg in, TO* out, int64_t out_row, int64_t out_plane,
                                               int32_t wo, int32_t ho, int32_t channels) {
    __shared__ float xs[kIH][kIW + 1];
    __shared__ double hs[kIH][kTW];
    const int tid = threadIdx.x;
    const int ox0 = blockIdx.x * kTW, oy0 = blockIdx.y * kTH;
    const int ix0 = 2 * ox0 - 3, iy0 = 2 * oy0 - 3;
    const TI* src = static_cast<const TI*>(in.data);
    for (int c = 0; c < channels; ++c) {
        const TI* plane = src + (int64_t)c * in.plane;
        for (int i = tid; i < kIH * kIW; i += 256) {
            const int r = i / kIW, q = i - r * kIW;
            const int gy = clampi(iy0 + r, 0, in.h - 1);
            const int gx = clampi(ix0 + q, 0, in.w - 1);
            xs[r][q] = load_f(plane + (int64_t)gy * in.row + gx);
        }
        __syncthreads();
        for (int i = tid; i < kIH * kTW; i += 256) {
            const int r = i / kTW, oc = i - r * kTW;
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < 8; ++t) acc += down2_w(t) * (double)xs[r][2 * oc + t];
            hs[r][oc] = acc;
        }
        __syncthreads();
        for (int i = tid; i < kTH * kTW; i += 256) {
            const int orow = i / kTW, oc = i - orow * kTW;
            const int oy = oy0 + orow, ox = ox0 + oc;
            if (oy < ho && ox < wo) {
                double acc = 0.0;
#pragma unroll
                for (int t = 0; t < 8; ++t) acc += down2_w(t) * hs[2 * orow + t][oc];
                store_d(out + (int64_t)c * out_plane + (int64_t)oy * out_row + ox, acc * (1.0 / 1048576.0));
            }
        }
        __syncthreads();
    }
}

template <typename TI, typename TO>
mdn_status launch_typed(const mdn_image& in, const mdn_image& out, hipStream_t st) {
    ImageArg a{in.data, in.row_pitch, in.plane_pitch, in.width, in.height};
    dim3 grid((out.width + kTW - 1) / kTW, (out.height + kTH - 1) / kTH);
    k_down2<TI, TO><<<grid, 256, 0, st>>>(a, static_cast<TO*>(out.data), out.row_pitch, out.plane_pitch,
                                          out.width, out.height, in.channels);
    return check_launch("down2");
}

}  // namespace

mdn_status launch_down2_tiled(const mdn_image& in, const mdn_image& out, hipStream_t st) {
    if (out.width == 0 || out.height == 0) return MDN_OK;
    if (in.dtype == MDN_F32 && out.dtype == MDN_F32) return launch_typed<float, float>(in, out, st);
    if (in.dtype == MDN_F32 && out.dtype == MDN_F16) return launch_typed<float, __half>(in, out, st);
    if (in.dtype == MDN_F16 && out.dtype == MDN_F16) return launch_typed<__half, __half>(in, out, st);
    if (in.dtype == MDN_F16 && out.dtype == MDN_F32) return launch_typed<__half, float>(in, out, st);
    return fail(MDN_EINVAL, "down2: unsupported dtype pair %d -> %d", in.dtype, out.dtype);
}

}  // namespace mdn
