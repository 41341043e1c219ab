// Column-walk factor-two bicubic downsampling (Section 4, "Multiscale filtering"): the work of one
// strip, shared by the pyramid launch and the launch that runs it beside the selection pass.
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
// 64 registers and eight waves per SIMD instead of 156 and three (an earlier form of this body), measured 4-6% slower on the
// level-0 step: neighbouring waves then read different planes instead of neighbouring bands.)

#pragma once

#include "walk_types.h"

#include <type_traits>
#include <utility>

namespace mdn {
namespace d2w {

constexpr int kOut = kD2LanesOut;

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

// One strip of a pyramid step, walked by the calling wave (lane = its lane number).
template <typename TI, typename TO, int C>
__device__ __forceinline__ void strip(const D2Args& a, int strip, int lane) {
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
    im = wave_uniform(im);
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
            // a buffer resource on the plane row (scalar registers); lanes add byte offsets
            const char* rowb = (const char*)im.in + (size_t)(ro + c * ipl) * sizeof(TI);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)rowb, 0, 0x7fffffff, 0x00020000);
            if constexpr (sizeof(TI) == 2) {
                e[c] = (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs, c0 * 2u, 0, 0));
                o[c] = (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs, c1 * 2u, 0, 0));
            } else {
                e[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, c0 * 4u, 0, 0));
                o[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, c1 * 4u, 0, 0));
            }
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
    // ring: input row 2*oy0 - 3 + k in slot k mod 8; the input rows of an output row are loaded two
    // steps ahead of their use
    double ring[8][C];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float e[C], o[C];
        load(2 * oy0 - 3 + k, e, o);
        hrow(e, o, ring[k]);
    }
    // input rows 2 oy + 3 + k (k = 0..3) in flight: the pair of step oy in slot oy mod 2
    float be[2][2][C], bo[2][2][C];
    load(2 * oy0 + 3, be[0][0], bo[0][0]);
    load(2 * oy0 + 4, be[0][1], bo[0][1]);
    load(2 * oy0 + 5, be[1][0], bo[1][0]);
    load(2 * oy0 + 6, be[1][1], bo[1][1]);
    for (int y0 = oy0; y0 < oy1; y0 += 4) {
        unroll([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            constexpr int P = I % 2;
            const int oy = y0 + I;
            float en[C], on[C], fn[C], pn[C];
            load(2 * oy + 7, en, on);
            load(2 * oy + 8, fn, pn);
            hrow(be[P][0], bo[P][0], ring[(2 * I + 6) % 8]);
            hrow(be[P][1], bo[P][1], ring[(2 * I + 7) % 8]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                be[P][0][c] = en[c];
                bo[P][0][c] = on[c];
                be[P][1][c] = fn[c];
                bo[P][1][c] = pn[c];
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

}  // namespace d2w
}  // namespace mdn
