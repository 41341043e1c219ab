// Column-walk factor-two bicubic downsampling (Section 4, "Multiscale filtering").
//
// Same arithmetic as the tiled kernel: Keys cubic (a = -1/2) stretched by two and centred at
// 2m + 1/2, integer weights (-12, -36, 116, 444, 444, 116, -36, -12) over input samples 2m-3 ..
// 2m+4, rows first, float64 accumulation (exact for float16/float32 inputs), one scaling by
// 2^-20 and a single rounding to the output type.
//
// A wavefront owns 60 output columns (64 lanes, 2 halo lanes each side) and walks down a strip
// of output rows. Each lane loads the input pair (2m, 2m+1) of its output column m; the other six
// horizontal taps come from lanes m-2 .. m+2 by DPP wave shifts. The horizontally filtered rows
// sit in an 8-row register ring (fixed slots, the 4-row step body is expanded at compile time);
// each output row consumes two new input rows. (Walking each channel of a strip in its own wave,
// 64 registers and eight waves per SIMD instead of 156 and three, measured 4-6% slower on the
// level-0 step: neighbouring waves then read different planes instead of neighbouring bands.)

#include "walk_types.h"

#include <string.h>

#include <type_traits>
#include <utility>

namespace mdn {

namespace {

constexpr int kOut = kD2LanesOut;
constexpr int kWaves = 4;

__device__ __forceinline__ uint32_t shl1(uint32_t v) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ uint32_t shr1(uint32_t v) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ double shl1d(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return __longlong_as_double((long long)(((uint64_t)shl1((uint32_t)(u >> 32)) << 32) | shl1((uint32_t)u)));
}
__device__ __forceinline__ double shr1d(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return __longlong_as_double((long long)(((uint64_t)shr1((uint32_t)(u >> 32)) << 32) | shr1((uint32_t)u)));
}

#define MDN_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ float ldo(const void* base, uint32_t elem) {
    const MDN_GLOBAL char* b = (const MDN_GLOBAL char*)(base);
    return (float)*(const MDN_GLOBAL T*)(b + elem * (uint32_t)sizeof(T));
}
// float64 -> storage type with a single rounding to nearest even
__device__ __forceinline__ float round_to(double v, float*) { return (float)v; }
__device__ __forceinline__ _Float16 round_to(double v, _Float16*) {
    // round to odd into float (24 bits >= 11 + 2), then one correct rounding to half. Of the two
    // floats around an inexact v, round to odd takes the one whose last bit is odd: the nearest
    // float when its last bit is odd, else its neighbour on v's side (last bit flipped).
    const float t = (float)v;
    const double d = (double)t;
    uint32_t b = __float_as_uint(t);
    if (d != v && !(b & 1u) && t != 0.0f) b += ((v > d) == (t > 0.0f)) ? 1u : 0xffffffffu;
    return (_Float16)__uint_as_float(b);
}
template <typename T> __device__ __forceinline__ void sto_d(void* base, uint32_t elem, double v) {
    MDN_GLOBAL char* b = (MDN_GLOBAL char*)(base);
    *(MDN_GLOBAL T*)(b + elem * (uint32_t)sizeof(T)) = round_to(v, (T*)nullptr);
}

// a pointer every lane holds alike, moved to scalar registers
template <typename T> __device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t u = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

template <int I>
using IC = std::integral_constant<int, I>;
template <typename F, int... Is>
__device__ __forceinline__ void unroll(F&& f, std::integer_sequence<int, Is...>) {
    (f(IC<Is>{}), ...);
}

template <typename TI, typename TO, int C>
__global__ __launch_bounds__(64 * kWaves) void k_down2_walk(D2Args a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int strip = blockIdx.x * kWaves + wave; strip < a.n_strips; strip += gridDim.x * kWaves) {
        D2Image im;
        if (a.imgs == nullptr) {
            im = a.single;
        } else {
            int lo = 0, hi = a.n_imgs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.imgs[mid].strip_begin <= strip) lo = mid; else hi = mid - 1;
            }
            im = a.imgs[lo];
        }
        const int local = strip - im.strip_begin;
        const int sy = local / im.nsx, sx = local - sy * im.nsx;
        const int m = sx * kOut - 2 + lane;                 // output column of this lane
        const int oy0 = sy * im.rows;
        const int oy1 = min(oy0 + im.rows, im.Ho);
        const bool out_lane = lane >= 2 && lane < 2 + kOut && m < im.Wo;
        const uint32_t c0 = (uint32_t)clampi(2 * m, 0, im.Wi - 1), c1 = (uint32_t)clampi(2 * m + 1, 0, im.Wi - 1);
        const uint32_t irow = (uint32_t)im.i_row, ipl = (uint32_t)im.i_plane;
        // the image's planes are wave-uniform: scalar registers
        im.in = uniform_ptr(im.in);
        im.out = uniform_ptr(im.out);

        // raw input pair (2m, 2m+1) of one input row (clamped), all channels
        auto load = [&](int r, float e[C], float o[C]) {
            const uint32_t ro = (uint32_t)clampi(r, 0, im.Hi - 1) * irow;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                e[c] = ldo<TI>(im.in, ro + c * ipl + c0);    // column 2m
                o[c] = ldo<TI>(im.in, ro + c * ipl + c1);    // column 2m+1
            }
        };
        // horizontal pass of one loaded row -> float64 (integer weights, exact). Lane k holds
        // x(2k) = e and x(2k+1) = o, converted once. Output m takes -12 x(2m-3) - 36 x(2m-2) +
        // 116 x(2m-1) from lanes m-2 and m-1, 444 (x(2m) + x(2m+1)) from its own lane, and 116 x(2m+2)
        // - 36 x(2m+3) - 12 x(2m+4) from lanes m+1 and m+2; each side is gathered into one value
        // before its last move, so four float64 moves (two DPP each) bring in the six neighbours.
        auto hrow = [&](const float ev[C], const float ov[C], double h[C]) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double e = (double)ev[c], o = (double)ov[c];
                const double lsd = 116.0 * o - 36.0 * e - 12.0 * shr1d(o);   // lane m-1's part of output m
                const double rsd = 116.0 * e - 36.0 * o - 12.0 * shl1d(e);   // lane m+1's part
                h[c] = shr1d(lsd) + 444.0 * (e + o) + shl1d(rsd);
            }
        };
        // ring: input row 2*oy0 - 3 + k in slot k mod 8; the next output row's two input rows are
        // loaded one step ahead of their use
        double ring[8][C];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float e[C], o[C];
            load(2 * oy0 - 3 + k, e, o);
            hrow(e, o, ring[k]);
        }
        float ea[C], oa[C], eb[C], ob[C];
        load(2 * oy0 + 3, ea, oa);
        load(2 * oy0 + 4, eb, ob);
        for (int y0 = oy0; y0 < oy1; y0 += 4) {
            unroll([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                const int oy = y0 + I;
                float en[C], on[C], fn[C], pn[C];
                load(2 * oy + 5, en, on);
                load(2 * oy + 6, fn, pn);
                hrow(ea, oa, ring[(2 * I + 6) % 8]);
                hrow(eb, ob, ring[(2 * I + 7) % 8]);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    ea[c] = en[c];
                    oa[c] = on[c];
                    eb[c] = fn[c];
                    ob[c] = pn[c];
                }
                if (out_lane && oy < oy1) {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const double v = -12.0 * ring[(2 * I) % 8][c] - 36.0 * ring[(2 * I + 1) % 8][c] +
                                         116.0 * ring[(2 * I + 2) % 8][c] + 444.0 * ring[(2 * I + 3) % 8][c] +
                                         444.0 * ring[(2 * I + 4) % 8][c] + 116.0 * ring[(2 * I + 5) % 8][c] -
                                         36.0 * ring[(2 * I + 6) % 8][c] - 12.0 * ring[(2 * I + 7) % 8][c];
                        sto_d<TO>(im.out, (uint32_t)oy * (uint32_t)im.o_row + c * (uint32_t)im.o_plane + (uint32_t)m,
                                  v * (1.0 / 1048576.0));
                    }
                }
            }, std::make_integer_sequence<int, 4>{});
        }
    }
}

}  // namespace

int down2_rows(int wo, int ho, int ncu) {
    const int nsx = (wo + kOut - 1) / kOut;
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

mdn_status launch_down2_walk(const mdn_image& in, const mdn_image& out, hipStream_t st) {
    if (out.width == 0 || out.height == 0) return MDN_OK;
    D2Args a;
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
    im.nsx = (out.width + kOut - 1) / kOut;
    im.rows = down2_rows(out.width, out.height, device_cus());
    a.n_imgs = 1;
    a.n_strips = im.nsx * ((out.height + im.rows - 1) / im.rows);
    return launch_down2_args(a, in.channels, in.dtype, out.dtype, st);
}

}  // namespace mdn
