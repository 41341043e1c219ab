// Filter selection (Section 3, Eq. (3)-(6)) and adaptive filtering (Eq. (1), Eq. (9)-(10)).
//
// One 256-thread block owns a 16 x 64 tile of output pixels.
//  1. The tile's input window plus a 3-pixel halo (clamped at the image border) is staged in
//     LDS as float32 (RGB or grey).
//  2. Selection, in float64: per position of the tile plus a 2-pixel halo, the central-difference
//     gradients of every channel (or of the luma alone, for luma-selector levels) give
//     A = sum_c gx^2, B = sum_c gx gy, C = sum_c gy^2 (evaluated at
//     the clamped position, so the box reads replicated border values); a 5 x 5 box mean (a
//     horizontal then a vertical 5-sum in LDS) gives the tensor (a, b, c); its eigen-features are
//     binned into s(i). The orientation bin is found without atan2: the doubled-angle vector of
//     the minor eigenvector, (c - a, -2b), is tested against the bin-boundary unit vectors with
//     cross products.
//     Levels that select on the coarser output (MDN_SELECT_COARSE) stage that level's window instead,
//     in float64 and taken back to RGB, and form the gradients of its linear factor-two upsampling
//     onto this level's grid (fine pixel 2m: 3/4 of coarse m and 1/4 of m-1; 2m+1: 3/4 of m and 1/4
//     of m+1; rows, then columns), evaluated where the gradient stencil needs it.
//  3. Filtering, in float32: the staged window is converted to YCbCr in place, the coarser level's
//     window (for Eq. (9)) is staged too, and every pixel accumulates its bucket's f taps over the
//     coarse window at floor(i/2) + j and g taps over the fine window at i + j, per channel. The
//     result is written in YCbCr or converted back to RGB.

#include "mdn_internal.h"

#include <math.h>
#include <string.h>

namespace mdn {

namespace {

constexpr int kTW = 64;
constexpr int kTH = 16;
constexpr int kHalo = 3;                     // gradient (1) + box (2); also the max filter radius
constexpr int kZW = kTW + 2 * kHalo;         // 70
constexpr int kZH = kTH + 2 * kHalo;         // 22
constexpr int kPW = kTW + 4;                 // tensor-product field: tile + 2-pixel halo
constexpr int kPH = kTH + 4;
// Coarse window of the coarse selector: the gradient stencil reads fine pixels y0-3 .. y0+kTH+2,
// whose interpolation reads coarse rows y0/2-3 .. y0/2+kTH/2+2 (likewise for columns).
constexpr int kCH = kTH / 2 + 6;             // 14
constexpr int kCW = kTW / 2 + 6;             // 38

struct FilterArgs {
    ImageArg z;                 // RGB or grey input of this level
    int32_t z_dtype;
    ImageArg uc;                // coarser output (may be empty)
    int32_t uc_dtype, uc_rgb;
    const void* s_in;           // precomputed selector or null
    int64_t s_pitch;
    void* s_out;                // selector output or null
    int32_t s16;                // selector maps hold uint16 (K > 256) instead of uint8
    void* out;
    int64_t out_row, out_plane;
    int32_t out_dtype, out_rgb;
    const void* coeffs;
    int32_t K;
    double* feat_s;             // features mode: strength and coherence per pixel (row pitch W)
    double* feat_c;
    ImageArg su;                // coarse selector: the coarser output whose upsampling is analysed
    int32_t su_dtype, su_ycc;
    const TileImage* imgs;      // batched launch: per-image fields (z, uc, su, out, maps), or null
    int32_t n_imgs;
    SelectArg sel;
};

// YCbCr -> RGB in float64 (the exact algebraic inverse of the BT.601 matrix).
__device__ __forceinline__ void ycc_to_rgb_d(double& c0, double& c1, double& c2) {
    const double y = c0, cb = c1 - 0.5, cr = c2 - 0.5;
    const double r = y + 1.402 * cr;
    const double b = y + 1.772 * cb;
    c0 = r;
    c1 = (y - kLumaR * r - kLumaB * b) / kLumaG;
    c2 = b;
}

__device__ __forceinline__ float load_any(const void* base, int32_t dtype, int64_t off) {
    return dtype == MDN_F16 ? __half2float(static_cast<const __half*>(base)[off])
                            : static_cast<const float*>(base)[off];
}

__device__ __forceinline__ void store_any(void* base, int32_t dtype, int64_t off, float v) {
    if (dtype == MDN_F16)
        static_cast<__half*>(base)[off] = __float2half_rn(v);
    else
        static_cast<float*>(base)[off] = v;
}

// Strength sqrt(lambda1) and coherence (sqrt(l1) - sqrt(l2)) / (sqrt(l1) + sqrt(l2)) of the
// smoothed tensor [[a, b], [b, c]], float64.
__device__ __forceinline__ void strength_coherence(double a, double b, double c, double& s1, double& coh) {
    const double tr = a + c;
    const double dd = a - c;
    const double mu = sqrt(dd * dd + 4.0 * b * b);
    const double l1 = 0.5 * (tr + mu);
    const double l2 = fmax(0.5 * (tr - mu), 0.0);
    s1 = sqrt(fmax(l1, 0.0));
    const double s2 = sqrt(l2);
    coh = (s1 + s2 > 0.0) ? (s1 - s2) / (s1 + s2) : 0.0;
}

// Bucket index from the smoothed tensor (a, b, c), float64 throughout.
__device__ __forceinline__ int bucket_of(double a, double b, double c, const SelectArg& sp) {
    double s1, coh;
    strength_coherence(a, b, c, s1, coh);
    // Orientation: the minor eigenvector's angle theta in [0, pi) doubled is the angle of
    // (c - a, -2b) in [0, 2 pi); bin = floor(angle * q_theta / (2 pi)). An isotropic tensor has
    // theta = pi/2 by convention.
    const double X = c - a, Y = -2.0 * b;
    int qt;
    const int half = sp.q_theta >> 1;
    if (X == 0.0 && Y == 0.0) {
        qt = half;
    } else {
        const bool upper = (Y > 0.0) || (Y == 0.0 && X > 0.0);
        const double px = upper ? X : -X, py = upper ? Y : -Y;
        int k = 0;
        // both products rounded alone (no fused multiply-add): an exact tie compares equal
        for (int j = 0; j < half - 1; ++j) k += (__dmul_rn(sp.bcos[j], py) >= __dmul_rn(sp.bsin[j], px)) ? 1 : 0;
        qt = k + (upper ? 0 : half);
    }
    int qs = 0;
    for (int j = 0; j < sp.q_s - 1; ++j) qs += (s1 >= sp.t_s[j]) ? 1 : 0;
    int qc = 0;
    for (int j = 0; j < sp.q_c - 1; ++j) qc += (coh >= sp.t_c[j]) ? 1 : 0;
    return (qt * sp.q_s + qs) * sp.q_c + qc;
}

// MODE 0: selector only; 1: selector + filtering; 2: strength/coherence features only.
// SU: the structure tensor is taken on the upsampled coarser output (a.su) instead of a.z.
template <int C, int RF, int RG, typename TC, int MODE, bool SU>
__global__ __launch_bounds__(256) void k_select_apply(FilterArgs a) {
    constexpr bool APPLY = MODE == 1;
    constexpr int kUH = kTH / 2 + 2 * (RF > 0 ? RF : 0);
    constexpr int kUW = kTW / 2 + 2 * (RF > 0 ? RF : 0);
    constexpr int kTF = RF >= 0 ? (2 * RF + 1) * (2 * RF + 1) : 0;
    constexpr int kTG = (2 * RG + 1) * (2 * RG + 1);
    constexpr int kD = kTF + kTG;

    __shared__ float zs[C][kZH][kZW + 1];
    __shared__ double pa[kPH][kPW], pb[kPH][kPW], pc[kPH][kPW];
    // The coarser output's window is staged after the selection has read its last tensor product,
    // in the storage of pa: the block's LDS then admits three blocks per CU.
    using UsRows = float[RF >= 0 ? kUH : 1][RF >= 0 ? kUW + 1 : 1];
    static_assert(sizeof(float) * C * (RF >= 0 ? kUH : 1) * (RF >= 0 ? kUW + 1 : 1) <= sizeof(pa),
                  "the coarse window fits in the tensor-product field");
    UsRows* us = reinterpret_cast<UsRows*>(&pa[0][0]);
    __shared__ double ucs[SU ? C : 1][SU ? kCH : 1][SU ? kCW : 1];

    // the image of this block: the launch's own, or (batched launches) the one whose tile range holds
    // blockIdx.x, found by binary search over the image table
    ImageArg Z = a.z, UC = a.uc, SUI = a.su;
    void* OUT = a.out;
    int64_t OROW = a.out_row, OPL = a.out_plane, SP = a.s_pitch;
    const void* SIN = a.s_in;
    void* SOUT = a.s_out;
    int bx = blockIdx.x, by = blockIdx.y;
    if (a.imgs != nullptr) {
        const int t = blockIdx.x;
        int lo = 0, hi = a.n_imgs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.imgs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
        }
        const TileImage& ti = a.imgs[lo];
        Z = ti.z;
        UC = ti.uc;
        SUI = ti.su;
        OUT = ti.out;
        OROW = ti.out_row;
        OPL = ti.out_plane;
        SIN = ti.s_in;
        SOUT = ti.s_out;
        SP = ti.s_pitch;
        const int local = t - ti.tile_begin;
        by = local / ti.tiles_x;
        bx = local - by * ti.tiles_x;
    }
    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    const int x0 = bx * kTW, y0 = by * kTH;
    const int W = Z.w, H = Z.h;

    // 1. stage the input window (clamped); the coarse selector without filtering never reads it
    if constexpr (!SU || APPLY) {
        for (int i = tid; i < C * kZH * kZW; i += 256) {
            const int c = i / (kZH * kZW);
            const int rem = i - c * kZH * kZW;
            const int r = rem / kZW, q = rem - r * kZW;
            const int gy = clampi(y0 - kHalo + r, 0, H - 1);
            const int gx = clampi(x0 - kHalo + q, 0, W - 1);
            zs[c][r][q] = load_any(Z.data, a.z_dtype, (int64_t)c * Z.plane + (int64_t)gy * Z.row + gx);
        }
    }
    const int cy0 = (y0 >> 1) - 3, cx0 = (x0 >> 1) - 3;
    if constexpr (SU) {
        // the coarser output's window, float64 RGB (or grey), at clamped coarse positions
        for (int i = tid; i < kCH * kCW; i += 256) {
            const int r = i / kCW, q = i - r * kCW;
            const int gy = clampi(cy0 + r, 0, SUI.h - 1);
            const int gx = clampi(cx0 + q, 0, SUI.w - 1);
            const int64_t off = (int64_t)gy * SUI.row + gx;
            double v[C];
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = (double)load_any(SUI.data, a.su_dtype, off + (int64_t)c * SUI.plane);
            if constexpr (C == 3) {
                if (a.su_ycc) ycc_to_rgb_d(v[0], v[1], v[2]);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) ucs[c][r][q] = v[c];
        }
    }
    __syncthreads();

    // 2. selector
    int sv[4];
    if (SIN == nullptr) {
        for (int i = tid; i < kPH * kPW; i += 256) {
            const int r = i / kPW, q = i - r * kPW;
            const int yc = clampi(y0 - 2 + r, 0, H - 1);
            const int xc = clampi(x0 - 2 + q, 0, W - 1);
            const int ly = yc - (y0 - kHalo), lx = xc - (x0 - kHalo);
            const int lxr = clampi(xc + 1, 0, W - 1) - (x0 - kHalo);
            const int lxl = clampi(xc - 1, 0, W - 1) - (x0 - kHalo);
            const int lyd = clampi(yc + 1, 0, H - 1) - (y0 - kHalo);
            const int lyu = clampi(yc - 1, 0, H - 1) - (y0 - kHalo);
            double A = 0.0, B = 0.0, Cc = 0.0;
            if constexpr (SU) {
                // linear factor-two upsampling of the coarse window at fine (fy, fx), both clamped
                const int Hc = SUI.h, Wc = SUI.w;
                auto up = [&](int c, int fy, int fx) {
                    const int my = fy >> 1, mx = fx >> 1;
                    const int ny = (fy & 1) ? min(my + 1, Hc - 1) : max(my - 1, 0);
                    const int nx = (fx & 1) ? min(mx + 1, Wc - 1) : max(mx - 1, 0);
                    const int ly = my - cy0, lny = ny - cy0, lx = mx - cx0, lnx = nx - cx0;
                    const double r0 = 0.75 * ucs[c][ly][lx] + 0.25 * ucs[c][lny][lx];
                    const double r1 = 0.75 * ucs[c][ly][lnx] + 0.25 * ucs[c][lny][lnx];
                    return 0.75 * r0 + 0.25 * r1;
                };
                const int xr = clampi(xc + 1, 0, W - 1), xl = clampi(xc - 1, 0, W - 1);
                const int yd = clampi(yc + 1, 0, H - 1), yu = clampi(yc - 1, 0, H - 1);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const double gx = (up(c, yc, xr) - up(c, yc, xl)) * 0.5;
                    const double gy = (up(c, yd, xc) - up(c, yu, xc)) * 0.5;
                    A += gx * gx;
                    B += gx * gy;
                    Cc += gy * gy;
                }
            } else if (C == 3 && a.sel.luma) {
                // luma-only structure tensor: gradients of Y at the four neighbours
                auto Y = [&](int yy, int xx) { return luma_d(zs[0][yy][xx], zs[C > 1 ? 1 : 0][yy][xx], zs[C - 1][yy][xx]); };
                const double gx = (Y(ly, lxr) - Y(ly, lxl)) * 0.5;
                const double gy = (Y(lyd, lx) - Y(lyu, lx)) * 0.5;
                A = gx * gx;
                B = gx * gy;
                Cc = gy * gy;
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const double gx = ((double)zs[c][ly][lxr] - (double)zs[c][ly][lxl]) * 0.5;
                    const double gy = ((double)zs[c][lyd][lx] - (double)zs[c][lyu][lx]) * 0.5;
                    A += gx * gx;
                    B += gx * gy;
                    Cc += gy * gy;
                }
            }
            pa[r][q] = A;
            pb[r][q] = B;
            pc[r][q] = Cc;
        }
        __syncthreads();
        // horizontal 5-sums, written back in place (columns 0 .. kTW-1)
        constexpr int kHN = (kPH * kTW + 255) / 256;
        double ha[kHN], hb[kHN], hc[kHN];
#pragma unroll
        for (int k = 0; k < kHN; ++k) {
            const int i = tid + k * 256;
            if (i < kPH * kTW) {
                const int r = i / kTW, q = i - r * kTW;
                double sa = 0.0, sb = 0.0, sc = 0.0;
#pragma unroll
                for (int d = 0; d < 5; ++d) {
                    sa += pa[r][q + d];
                    sb += pb[r][q + d];
                    sc += pc[r][q + d];
                }
                ha[k] = sa;
                hb[k] = sb;
                hc[k] = sc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kHN; ++k) {
            const int i = tid + k * 256;
            if (i < kPH * kTW) {
                const int r = i / kTW, q = i - r * kTW;
                pa[r][q] = ha[k];
                pb[r][q] = hb[k];
                pc[r][q] = hc[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int py = ty + 4 * k;
            double sa = 0.0, sb = 0.0, sc = 0.0;
#pragma unroll
            for (int d = 0; d < 5; ++d) {
                sa += pa[py + d][tx];
                sb += pb[py + d][tx];
                sc += pc[py + d][tx];
            }
            if constexpr (MODE == 2) {
                const int y = y0 + py, x = x0 + tx;
                if (y < H && x < W) {
                    double s1, coh;
                    strength_coherence(sa / 25.0, sb / 25.0, sc / 25.0, s1, coh);
                    a.feat_s[(int64_t)y * W + x] = s1;
                    a.feat_c[(int64_t)y * W + x] = coh;
                }
                sv[k] = 0;
            } else {
                sv[k] = bucket_of(sa / 25.0, sb / 25.0, sc / 25.0, a.sel);
                if (a.sel.phases == 4) sv[k] = 4 * sv[k] + (((y0 + py) & 1) << 1) + ((x0 + tx) & 1);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int y = y0 + ty + 4 * k, x = x0 + tx;
            const int64_t o = (int64_t)y * SP + x;
            sv[k] = (y < H && x < W) ? (a.s16 ? (int)static_cast<const uint16_t*>(SIN)[o]
                                              : (int)static_cast<const uint8_t*>(SIN)[o])
                                     : 0;
        }
    }
    if (SOUT != nullptr) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int y = y0 + ty + 4 * k, x = x0 + tx;
            const int64_t o = (int64_t)y * SP + x;
            if (y < H && x < W) {
                if (a.s16) static_cast<uint16_t*>(SOUT)[o] = (uint16_t)sv[k];
                else static_cast<uint8_t*>(SOUT)[o] = (uint8_t)sv[k];
            }
        }
    }
    if constexpr (!APPLY) return;

    // 3. filtering
    __syncthreads();
    if constexpr (C == 3) {
        for (int i = tid; i < kZH * kZW; i += 256) {
            const int r = i / kZW, q = i - r * kZW;
            float yv, cb, cr;
            Ycc::from_rgb(zs[0][r][q], zs[1][r][q], zs[2][r][q], yv, cb, cr);
            zs[0][r][q] = yv;
            zs[1][r][q] = cb;
            zs[2][r][q] = cr;
        }
    }
    if constexpr (RF >= 0) {
        const int cy0 = y0 / 2 - RF, cx0 = x0 / 2 - RF;
        for (int i = tid; i < kUH * kUW; i += 256) {
            const int r = i / kUW, q = i - r * kUW;
            const int gy = clampi(cy0 + r, 0, UC.h - 1);
            const int gx = clampi(cx0 + q, 0, UC.w - 1);
            const int64_t off = (int64_t)gy * UC.row + gx;
            float v[C];
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = load_any(UC.data, a.uc_dtype, off + (int64_t)c * UC.plane);
            if constexpr (C == 3) {
                if (a.uc_rgb) Ycc::from_rgb(v[0], v[1], v[2], v[0], v[1], v[2]);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) us[c][r][q] = v[c];
        }
    }
    __syncthreads();

    const TC* coef = static_cast<const TC*>(a.coeffs);
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        const int py = ty + 4 * k, px = tx;
        const int y = y0 + py, x = x0 + px;
        if (y >= H || x >= W) continue;
        const int s = sv[k];
        float acc[C];
        if (s >= a.K) {
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = __builtin_nanf("");
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const TC* h = coef + ((int64_t)s * C + c) * kD;
                float sum = 0.0f;
                if constexpr (RF >= 0) {
                    const int uy = py / 2, ux = px / 2;
#pragma unroll
                    for (int dy = 0; dy < 2 * RF + 1; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 2 * RF + 1; ++dx)
                            sum += load_f(h + dy * (2 * RF + 1) + dx) * us[c][uy + dy][ux + dx];
                }
#pragma unroll
                for (int dy = 0; dy < 2 * RG + 1; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2 * RG + 1; ++dx)
                        sum += load_f(h + kTF + dy * (2 * RG + 1) + dx) *
                               zs[c][py + kHalo - RG + dy][px + kHalo - RG + dx];
                acc[c] = sum;
            }
        }
        const int64_t off = (int64_t)y * OROW + x;
        if constexpr (C == 3) {
            if (a.out_rgb) Ycc::to_rgb(acc[0], acc[1], acc[2], acc[0], acc[1], acc[2]);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) store_any(OUT, a.out_dtype, off + (int64_t)c * OPL, acc[c]);
    }
}

template <int C, int RF, int RG, typename TC>
mdn_status launch_kernel(const FilterArgs& fa, bool apply, bool su, int w, int h, hipStream_t st) {
    dim3 grid((w + kTW - 1) / kTW, (h + kTH - 1) / kTH);
    if constexpr (RF >= 1) {
        if (su && apply) {
            k_select_apply<C, RF, RG, TC, 1, true><<<grid, 256, 0, st>>>(fa);
            return check_launch("select_apply (coarse selector)");
        }
    }
    if (su) {
        if (apply) return fail(MDN_EINVAL, "the coarse selector needs a multiscale level");
        k_select_apply<C, 1, 1, float, 0, true><<<grid, 256, 0, st>>>(fa);
        return check_launch("select (coarse selector)");
    }
    if (apply)
        k_select_apply<C, RF, RG, TC, 1, false><<<grid, 256, 0, st>>>(fa);
    else
        k_select_apply<C, RF, RG, TC, 0, false><<<grid, 256, 0, st>>>(fa);
    return check_launch(apply ? "select_apply" : "select");
}

template <int C, typename TC>
mdn_status dispatch_radii(const FilterArgs& fa, bool apply, bool su, int rf, int rg, int w, int h, hipStream_t st) {
#define MDN_RADII(RF_, RG_) \
    if (rf == RF_ && rg == RG_) return launch_kernel<C, RF_, RG_, TC>(fa, apply, su, w, h, st);
    MDN_RADII(-1, 1)
    MDN_RADII(-1, 2)
    MDN_RADII(-1, 3)
    MDN_RADII(1, 1)
    MDN_RADII(2, 2)
    MDN_RADII(3, 3)
    MDN_RADII(2, 3)
    MDN_RADII(1, 2)
#undef MDN_RADII
    return fail(MDN_ENOTSUP, "filter radii (f=%d, g=%d) not supported", rf, rg);
}

}  // namespace

void set_coarse_source(FilterArgs& fa, const mdn_image& uc) {
    fa.su = ImageArg{uc.data, uc.row_pitch, uc.plane_pitch, uc.width, uc.height};
    fa.su_dtype = uc.dtype;
    fa.su_ycc = uc.color == MDN_YCC;
}

mdn_status launch_features(const mdn_image& z, int luma, const mdn_image* su, double* strength, double* coherence,
                           hipStream_t st) {
    if (z.width == 0 || z.height == 0) return MDN_OK;
    FilterArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.sel.luma = luma && z.channels == 3;
    fa.z = ImageArg{z.data, z.row_pitch, z.plane_pitch, z.width, z.height};
    fa.z_dtype = z.dtype;
    if (su) set_coarse_source(fa, *su);
    fa.feat_s = strength;
    fa.feat_c = coherence;
    fa.sel.q_theta = 2;
    fa.sel.q_s = 1;
    fa.sel.q_c = 1;
    dim3 grid((z.width + kTW - 1) / kTW, (z.height + kTH - 1) / kTH);
    if (su) {
        if (z.channels == 3)
            k_select_apply<3, -1, 1, float, 2, true><<<grid, 256, 0, st>>>(fa);
        else
            k_select_apply<1, -1, 1, float, 2, true><<<grid, 256, 0, st>>>(fa);
    } else if (z.channels == 3) {
        k_select_apply<3, -1, 1, float, 2, false><<<grid, 256, 0, st>>>(fa);
    } else {
        k_select_apply<1, -1, 1, float, 2, false><<<grid, 256, 0, st>>>(fa);
    }
    return check_launch("features");
}

void fill_select_arg(const mdn_level& lvl, SelectArg& sa) {
    memset(&sa, 0, sizeof(sa));
    sa.q_theta = lvl.q_theta;
    sa.q_s = lvl.q_s;
    sa.q_c = lvl.q_c;
    sa.luma = lvl.selector == MDN_SELECT_LUMA && lvl.channels == 3;
    sa.phases = lvl.phases;
    for (int j = 0; j < lvl.q_s - 1; ++j) sa.t_s[j] = lvl.t_s[j];
    for (int j = 0; j < lvl.q_c - 1; ++j) sa.t_c[j] = lvl.t_c[j];
    orientation_boundaries(lvl.q_theta, sa.bcos, sa.bsin);
}

void orientation_boundaries(int q_theta, double* bcos, double* bsin) {
    const double two_pi = 6.283185307179586476925286766559;
    const int half = q_theta / 2;
    for (int k = 1; k < half; ++k) {
        const int m = half - k;             // mirror partner: angle pi - 2 pi k / q_theta
        const int r = k < m ? k : m;        // the partner below the vertical
        double c, s;
        if (2 * k == half) {
            c = 0.0;
            s = 1.0;
        } else if (4 * r == half) {
            c = s = sqrt(0.5);
        } else {
            const double ang = two_pi * (double)r / (double)q_theta;
            c = cos(ang);
            s = sin(ang);
        }
        bcos[k - 1] = k < m ? c : -c;
        bsin[k - 1] = s;
    }
}

void tiled_grid(int w, int h, int* tiles_x, int* tiles_y) {
    *tiles_x = (w + kTW - 1) / kTW;
    *tiles_y = (h + kTH - 1) / kTH;
}

bool level_runs_tiled(const mdn_level& lvl, int channels) {
    if (lvl.radius_f < 1) return true;                       // single scale
    if (lvl.coeff_dtype == MDN_F16 && walk_supported(lvl, channels)) return false;
    return wide_selector(lvl) || !apply_lds_supported(lvl, channels);
}

mdn_status launch_select_apply_table(const mdn_level& lvl, const TileImage* imgs, int n_imgs, int n_tiles, int C,
                                     int z_dtype, int uc_dtype, int uc_color, int out_dtype, int out_color,
                                     hipStream_t st) {
    if (n_tiles <= 0) return MDN_OK;
    FilterArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.imgs = imgs;
    fa.n_imgs = n_imgs;
    fa.z_dtype = z_dtype;
    fa.uc_dtype = uc_dtype;
    fa.uc_rgb = uc_color == MDN_RGB;
    fa.out_dtype = out_dtype;
    fa.out_rgb = out_color == MDN_RGB;
    fa.s16 = wide_selector(lvl);
    fa.coeffs = lvl.coeffs;
    fa.K = level_buckets(lvl);
    fill_select_arg(lvl, fa.sel);
    const bool su = lvl.selector == MDN_SELECT_COARSE;
    if (su) {
        fa.su_dtype = uc_dtype;
        fa.su_ycc = uc_color == MDN_YCC;
    }
    const int rf = lvl.radius_f < 0 ? -1 : lvl.radius_f;
    // one block per tile: a grid of n_tiles x 1 tiles
    const int w = n_tiles * kTW, h = 1;
    if (C == 3 && lvl.coeff_dtype == MDN_F32) return dispatch_radii<3, float>(fa, true, su, rf, lvl.radius_g, w, h, st);
    if (C == 3 && lvl.coeff_dtype == MDN_F16) return dispatch_radii<3, __half>(fa, true, su, rf, lvl.radius_g, w, h, st);
    if (C == 1 && lvl.coeff_dtype == MDN_F32) return dispatch_radii<1, float>(fa, true, su, rf, lvl.radius_g, w, h, st);
    if (C == 1 && lvl.coeff_dtype == MDN_F16) return dispatch_radii<1, __half>(fa, true, su, rf, lvl.radius_g, w, h, st);
    return fail(MDN_EINVAL, "unsupported channels/coeff dtype");
}

mdn_status launch_select_apply(const mdn_image& z, const mdn_image* uc, const void* s_in, int64_t s_pitch,
                               void* s_out, const mdn_level& lvl, const mdn_image* out, hipStream_t st) {
    if (z.width == 0 || z.height == 0) return MDN_OK;
    const bool su = lvl.selector == MDN_SELECT_COARSE;
    if (su && !uc) return fail(MDN_EINVAL, "a level that selects on the coarser output needs u_coarse");
    // selector only: column-walk float64 selection pass (the coarse selector runs the tiled kernel)
    if (!out && s_out && !s_in && !su) return launch_select_walk(z, lvl, s_out, s_pitch, st);
    // float16 filter banks of 7x7/7x7 colour filters run on the persistent column-walk kernel
    if (out && uc && lvl.coeff_dtype == MDN_F16 && walk_supported(lvl, z.channels)) {
        if (!s_in && !s_out) return fail(MDN_EINVAL, "float16 levels need a selector map (s) or a buffer for it (s_out)");
        return launch_walk(z, *uc, lvl, *out, static_cast<const uint8_t*>(s_in), static_cast<uint8_t*>(s_out), s_pitch, st);
    }
    // other multiscale banks that fit in LDS one channel at a time: selection pass, then filtering
    // with the bank in LDS (without a map or a buffer for one, the fused kernel below runs)
    if (out && uc && (s_in || s_out) && apply_lds_supported(lvl, z.channels)) {
        if (!s_in) {
            mdn_status e = launch_select_apply(z, uc, nullptr, s_pitch, s_out, lvl, nullptr, st);
            if (e) return e;
            s_in = s_out;
        }
        return launch_apply_lds(z, *uc, s_in, s_pitch, lvl, *out, st);
    }
    FilterArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.z = ImageArg{z.data, z.row_pitch, z.plane_pitch, z.width, z.height};
    fa.z_dtype = z.dtype;
    if (uc) {
        fa.uc = ImageArg{uc->data, uc->row_pitch, uc->plane_pitch, uc->width, uc->height};
        fa.uc_dtype = uc->dtype;
        fa.uc_rgb = uc->color == MDN_RGB;
    }
    fa.s_in = s_in;
    fa.s16 = wide_selector(lvl);
    fa.s_pitch = s_pitch;
    fa.s_out = s_out;
    if (out) {
        fa.out = out->data;
        fa.out_row = out->row_pitch;
        fa.out_plane = out->plane_pitch;
        fa.out_dtype = out->dtype;
        fa.out_rgb = out->color == MDN_RGB;
    }
    fa.coeffs = lvl.coeffs;
    fa.K = level_buckets(lvl);
    fill_select_arg(lvl, fa.sel);
    if (su) set_coarse_source(fa, *uc);
    const bool apply = out != nullptr;
    const bool su_sel = su && !s_in;        // a given map leaves nothing to select
    const int C = z.channels;
    const int rf = lvl.radius_f < 0 ? -1 : lvl.radius_f;
    const int rg = lvl.radius_g;
    if (C == 3 && lvl.coeff_dtype == MDN_F32) return dispatch_radii<3, float>(fa, apply, su_sel, rf, rg, z.width, z.height, st);
    if (C == 3 && lvl.coeff_dtype == MDN_F16) return dispatch_radii<3, __half>(fa, apply, su_sel, rf, rg, z.width, z.height, st);
    if (C == 1 && lvl.coeff_dtype == MDN_F32) return dispatch_radii<1, float>(fa, apply, su_sel, rf, rg, z.width, z.height, st);
    if (C == 1 && lvl.coeff_dtype == MDN_F16) return dispatch_radii<1, __half>(fa, apply, su_sel, rf, rg, z.width, z.height, st);
    return fail(MDN_EINVAL, "unsupported channels/coeff dtype");
}

}  // namespace mdn
