// Filtering (Eq. (9)-(10), float32 arithmetic) from a precomputed selector map, with the level's
// bank staged in LDS one channel at a time.
//
// The tiled select-and-apply kernel gathers every coefficient from the L2-resident bank: each lane
// reads its own bucket's row, so one load instruction touches up to 64 cache lines, and its waves
// spend most of their time waiting on those gathers. A float32 bank of 7x7/7x7 colour filters does
// not fit in LDS whole (216 buckets x 3 channels x 98 taps x 4 bytes = 254 KB), but one channel of
// it does (85 KB). So one 512-thread block owns a 64 x 64 tile (its windows and one channel of the
// bank fill the LDS) and
//  1. stages the tile's input window (g radius halo, clamped) converted to YCbCr, and the coarser
//     output's window at floor(i/2) + j (clamped, converted from RGB at the coarsest level);
//  2. per channel, copies that channel's K rows of D taps (padded to a multiple of four) into LDS
//     with 8-byte loads, each block starting at another row, and lets every thread accumulate the
//     f and g taps of its eight pixels, consecutive rows of one column: the window rows are read
//     from LDS once into registers and reused down the column, and each pixel's bucket row comes
//     in with 16-byte LDS loads.
// The taps are summed in the order of the tiled kernel (f taps row-major, then g taps, one fused
// multiply-add each), so for the same selector the two kernels give the same float32 result.
// Colour levels only: grey multiscale levels keep the tiled kernel.

#include "mdn_internal.h"

#include <string.h>

namespace mdn {

namespace {

constexpr int kLTW = 64;                  // tile width (one wave spans a row)
constexpr int kLTH = 64;                  // tile height: 8 waves x 8 rows
constexpr int kLRows = kLTH / 8;          // rows (pixels) per thread
constexpr int kLThreads = 512;
constexpr size_t kLdsBytes = 160 * 1024;

template <int C, int RF, int RG>
struct LdsShape {
    // rows are read along x by consecutive lanes, so they need no padding against bank conflicts
    static constexpr int ZH = kLTH + 2 * RG, ZW = kLTW + 2 * RG, ZP = ZW;
    static constexpr int UH = kLTH / 2 + 2 * RF, UW = kLTW / 2 + 2 * RF, UP = UW;
    static constexpr int TF = (2 * RF + 1) * (2 * RF + 1);
    static constexpr int TG = (2 * RG + 1) * (2 * RG + 1);
    static constexpr int D = TF + TG;
    static constexpr int DP = (D + 3) & ~3;   // LDS row of one bucket, 16-byte aligned
    static_assert(D % 2 == 0, "taps per channel come in pairs");
    // the windows, rounded up to the 16-byte alignment of the bank that follows them
    static constexpr size_t static_bytes = (sizeof(float) * (size_t)C * (ZH * ZP + UH * UP) + 15) & ~(size_t)15;
};

struct ApplyLdsArgs {
    ImageArg z;                 // RGB or grey input of the level
    int32_t z_dtype;
    ImageArg uc;                // coarser output
    int32_t uc_dtype, uc_rgb;
    const void* s;              // selector map, uint8 or uint16
    int64_t s_pitch;
    int32_t s16;
    void* out;
    int64_t out_row, out_plane;
    int32_t out_dtype, out_rgb;
    const void* coeffs;         // [K][C][D], float32 or float16
    int32_t coeff_dtype, K;
};

__device__ __forceinline__ float ld_any(const void* base, int32_t dtype, int64_t off) {
    return dtype == MDN_F16 ? __half2float(static_cast<const __half*>(base)[off])
                            : static_cast<const float*>(base)[off];
}

template <int C, int RF, int RG>
__global__ __launch_bounds__(kLThreads, 2) void k_apply_lds(ApplyLdsArgs a) {
    using S = LdsShape<C, RF, RG>;
    __shared__ float zs[C][S::ZH][S::ZP];
    __shared__ float us[C][S::UH][S::UP];
    extern __shared__ __attribute__((aligned(16))) float bank[];     // [K][DP], one channel

    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    const int x0 = blockIdx.x * kLTW, y0 = blockIdx.y * kLTH;
    const int W = a.z.w, H = a.z.h;

    // 1. windows: this level's input (YCbCr) and the coarser output, clamped at the borders (loop
    //    unrolled so that several iterations' loads are in flight together)
#pragma unroll 4
    for (int i = tid; i < S::ZH * S::ZW; i += kLThreads) {
        const int r = i / S::ZW, q = i - r * S::ZW;
        const int gy = clampi(y0 - RG + r, 0, H - 1);
        const int gx = clampi(x0 - RG + q, 0, W - 1);
        const int64_t off = (int64_t)gy * a.z.row + gx;
        float v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = ld_any(a.z.data, a.z_dtype, off + (int64_t)c * a.z.plane);
        if constexpr (C == 3) Ycc::from_rgb(v[0], v[1], v[2], v[0], v[1], v[2]);
#pragma unroll
        for (int c = 0; c < C; ++c) zs[c][r][q] = v[c];
    }
    const int cy0 = y0 / 2 - RF, cx0 = x0 / 2 - RF;
#pragma unroll 4
    for (int i = tid; i < S::UH * S::UW; i += kLThreads) {
        const int r = i / S::UW, q = i - r * S::UW;
        const int gy = clampi(cy0 + r, 0, a.uc.h - 1);
        const int gx = clampi(cx0 + q, 0, a.uc.w - 1);
        const int64_t off = (int64_t)gy * a.uc.row + gx;
        float v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = ld_any(a.uc.data, a.uc_dtype, off + (int64_t)c * a.uc.plane);
        if constexpr (C == 3) {
            if (a.uc_rgb) Ycc::from_rgb(v[0], v[1], v[2], v[0], v[1], v[2]);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) us[c][r][q] = v[c];
    }

    // 2. the selector of this thread's pixels: rows kLRows * ty .. kLRows * ty + 7 of column tx.
    //    Vertical neighbours share all but one row of their g window and, in pairs, their whole f
    //    window, so the window rows are loaded once into registers and reused down the column.
    int sv[kLRows];
#pragma unroll
    for (int j = 0; j < kLRows; ++j) {
        const int y = y0 + kLRows * ty + j, x = x0 + tx;
        const int64_t o = (int64_t)y * a.s_pitch + x;
        sv[j] = (y < H && x < W) ? (a.s16 ? (int)static_cast<const uint16_t*>(a.s)[o]
                                          : (int)static_cast<const uint8_t*>(a.s)[o])
                                 : 0;
    }

    constexpr int NG = 2 * RG + 1, NF = 2 * RF + 1;
    // per-channel results, indexed by compile-time pixel and channel only (so they stay in registers)
    float acc0[kLRows], acc1[kLRows], acc2[kLRows];
    const int K = a.K;
    const int py0 = kLRows * ty, px = tx;
#pragma unroll 1
    for (int c = 0; c < C; ++c) {
        __syncthreads();        // windows staged; the previous channel's rows are no longer read
        // D is even (a sum of two odd squares) and rows start at even offsets: pairs of taps are
        // copied with 8-byte loads; blocks start at different rows so that they do not all read
        // the same lines of the bank at once
        constexpr int D2 = S::D / 2;
        const int n2 = K * D2;
        const int rot = (int)((blockIdx.x * 7u + blockIdx.y * 13u) % (unsigned)K) * D2;
        if (a.coeff_dtype == MDN_F16) {
            const __half2* src = static_cast<const __half2*>(a.coeffs);
#pragma unroll 8
            for (int i = tid; i < n2; i += kLThreads) {
                int e = i + rot;
                e = e >= n2 ? e - n2 : e;
                const int k = e / D2, t2 = e - k * D2;
                const float2 v = __half22float2(src[((int64_t)k * C + c) * D2 + t2]);
                *reinterpret_cast<float2*>(bank + (size_t)k * S::DP + 2 * t2) = v;
            }
        } else {
            const float2* src = static_cast<const float2*>(a.coeffs);
#pragma unroll 8
            for (int i = tid; i < n2; i += kLThreads) {
                int e = i + rot;
                e = e >= n2 ? e - n2 : e;
                const int k = e / D2, t2 = e - k * D2;
                *reinterpret_cast<float2*>(bank + (size_t)k * S::DP + 2 * t2) = src[((int64_t)k * C + c) * D2 + t2];
            }
        }
        __syncthreads();
        float gw[kLRows + 2 * RG][NG];          // g window rows py0 .. py0 + 7 + 2 RG (loaded on first use)
        float fw[kLRows / 2 + 2 * RF][NF];      // f window rows py0/2 .. py0/2 + 3 + 2 RF
#pragma unroll
        for (int j = 0; j < kLRows; ++j) {
            // rows entering the windows at this pixel
#pragma unroll
            for (int r = (j == 0 ? 0 : j + 2 * RG); r <= j + 2 * RG; ++r)
#pragma unroll
                for (int dx = 0; dx < NG; ++dx) gw[r][dx] = zs[c][py0 + r][px + dx];
            if (j % 2 == 0) {
#pragma unroll
                for (int r = (j == 0 ? 0 : j / 2 + 2 * RF); r <= j / 2 + 2 * RF; ++r)
#pragma unroll
                    for (int dx = 0; dx < NF; ++dx) fw[r][dx] = us[c][py0 / 2 + r][px / 2 + dx];
            }
            const int s = sv[j] < K ? sv[j] : 0;       // a selector outside the bank yields NaN below
            const float4* h4 = reinterpret_cast<const float4*>(bank + (size_t)s * S::DP);
            float sum = 0.0f;
#pragma unroll
            for (int t4 = 0; t4 < S::DP / 4; ++t4) {
                const float4 q = h4[t4];
                const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int t = 4 * t4 + e;
                    if (t < S::TF) {
                        sum += qv[e] * fw[j / 2 + t / NF][t % NF];
                    } else if (t < S::D) {
                        const int tg = t - S::TF;
                        sum += qv[e] * gw[j + tg / NG][tg % NG];
                    }
                }
            }
            if (sv[j] >= K) sum = __builtin_nanf("");
            if (c == 0) acc0[j] = sum;
            else if (c == 1) acc1[j] = sum;
            else acc2[j] = sum;
        }
    }

    // 3. store (back to RGB at the finest level)
#pragma unroll
    for (int j = 0; j < kLRows; ++j) {
        const int y = y0 + kLRows * ty + j, x = x0 + tx;
        if (y >= H || x >= W) continue;
        float o[C];
        o[0] = acc0[j];
        if constexpr (C == 3) {
            o[1] = acc1[j];
            o[2] = acc2[j];
        }
        if constexpr (C == 3) {
            if (a.out_rgb) Ycc::to_rgb(o[0], o[1], o[2], o[0], o[1], o[2]);
        }
        const int64_t off = (int64_t)y * a.out_row + x;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (a.out_dtype == MDN_F16)
                static_cast<__half*>(a.out)[off + (int64_t)c * a.out_plane] = __float2half_rn(o[c]);
            else
                static_cast<float*>(a.out)[off + (int64_t)c * a.out_plane] = o[c];
        }
    }
}

template <int C, int RF, int RG>
size_t lds_need(int K) {
    using S = LdsShape<C, RF, RG>;
    return S::static_bytes + (size_t)K * S::DP * sizeof(float);
}

template <int C, int RF, int RG>
mdn_status launch_typed(const ApplyLdsArgs& a, hipStream_t st) {
    using S = LdsShape<C, RF, RG>;
    static size_t static_lds = 0;     // per instance, once per process: the compiled static LDS size
    const void* fn = (const void*)k_apply_lds<C, RF, RG>;
    if (!static_lds) {
        hipFuncAttributes attr;
        if (hipFuncGetAttributes(&attr, fn) != hipSuccess) return fail(MDN_EDEVICE, "apply: kernel attributes");
        const size_t st_b = (attr.sharedSizeBytes + 15) & ~(size_t)15;
        if (st_b >= kLdsBytes) return fail(MDN_ENOTSUP, "apply: %zu bytes of static LDS", st_b);
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsBytes - st_b));
        if (e != hipSuccess)
            return fail(MDN_EDEVICE, "apply: cannot reserve %zu bytes of LDS beside %zu static (%s)", kLdsBytes - st_b,
                        st_b, hipGetErrorString(e));
        static_lds = st_b;
    }
    const size_t dyn = (size_t)a.K * S::DP * sizeof(float);
    if (static_lds + dyn > kLdsBytes) return fail(MDN_ENOTSUP, "apply: bank does not fit in LDS");
    dim3 grid((a.z.w + kLTW - 1) / kLTW, (a.z.h + kLTH - 1) / kLTH);
    k_apply_lds<C, RF, RG><<<grid, kLThreads, dyn, st>>>(a);
    return check_launch("apply (bank in LDS)");
}

// need: LDS bytes of the (C, RF, RG) instance for K buckets, or 0 when there is no instance
size_t lds_bytes_for(int C, int rf, int rg, int K) {
#define MDN_LDS_NEED(C_, RF_, RG_) \
    if (C == C_ && rf == RF_ && rg == RG_) return lds_need<C_, RF_, RG_>(K);
    MDN_LDS_NEED(3, 3, 3)
    MDN_LDS_NEED(3, 2, 3)
    MDN_LDS_NEED(3, 2, 2)
    MDN_LDS_NEED(3, 1, 2)
    MDN_LDS_NEED(3, 1, 1)
#undef MDN_LDS_NEED
    return 0;
}

}  // namespace

bool apply_lds_supported(const mdn_level& lvl, int channels) {
    // the bank is copied in pairs of taps: 8-byte (float32) or 4-byte (float16) aligned rows
    const uintptr_t align = lvl.coeff_dtype == MDN_F16 ? 3 : 7;
    if (lvl.radius_f < 1 || ((uintptr_t)lvl.coeffs & align)) return false;
    const size_t need = lds_bytes_for(channels, lvl.radius_f, lvl.radius_g, level_buckets(lvl));
    return need > 0 && need <= kLdsBytes;
}

mdn_status launch_apply_lds(const mdn_image& z, const mdn_image& uc, const void* s, int64_t s_pitch,
                            const mdn_level& lvl, const mdn_image& out, hipStream_t st) {
    if (z.width == 0 || z.height == 0) return MDN_OK;
    if (!apply_lds_supported(lvl, z.channels)) return fail(MDN_ENOTSUP, "apply: bank does not fit in LDS");
    ApplyLdsArgs a;
    memset(&a, 0, sizeof(a));
    a.z = ImageArg{z.data, z.row_pitch, z.plane_pitch, z.width, z.height};
    a.z_dtype = z.dtype;
    a.uc = ImageArg{uc.data, uc.row_pitch, uc.plane_pitch, uc.width, uc.height};
    a.uc_dtype = uc.dtype;
    a.uc_rgb = uc.color == MDN_RGB;
    a.s = s;
    a.s_pitch = s_pitch;
    a.s16 = wide_selector(lvl);
    a.out = out.data;
    a.out_row = out.row_pitch;
    a.out_plane = out.plane_pitch;
    a.out_dtype = out.dtype;
    a.out_rgb = out.color == MDN_RGB;
    a.coeffs = lvl.coeffs;
    a.coeff_dtype = lvl.coeff_dtype;
    a.K = level_buckets(lvl);
    const int rf = lvl.radius_f, rg = lvl.radius_g;
#define MDN_LDS_LAUNCH(C_, RF_, RG_) \
    if (z.channels == C_ && rf == RF_ && rg == RG_) return launch_typed<C_, RF_, RG_>(a, st);
    MDN_LDS_LAUNCH(3, 3, 3)
    MDN_LDS_LAUNCH(3, 2, 3)
    MDN_LDS_LAUNCH(3, 2, 2)
    MDN_LDS_LAUNCH(3, 1, 2)
    MDN_LDS_LAUNCH(3, 1, 1)
#undef MDN_LDS_LAUNCH
    return fail(MDN_ENOTSUP, "apply: radii (f=%d, g=%d) have no LDS-bank instance", rf, rg);
}

}  // namespace mdn
