// Internal declarations shared by the HIP translation units of libmdn.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "mdn.h"

namespace mdn {

// ------------------------------------------------------------------------ error state
void set_error(const char* fmt, ...);
void clear_error();
mdn_status validate_level(const mdn_level* lv, int channels);
mdn_status fail(mdn_status st, const char* fmt, ...);
mdn_status check_launch(const char* what);

// ------------------------------------------------------------------------ element access
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <typename T> __device__ __forceinline__ float load_f(const T* p);
template <> __device__ __forceinline__ float load_f<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float load_f<__half>(const __half* p) { return __half2float(*p); }

template <typename T> __device__ __forceinline__ void store_f(T* p, float v);
template <> __device__ __forceinline__ void store_f<float>(float* p, float v) { *p = v; }
template <> __device__ __forceinline__ void store_f<__half>(__half* p, float v) { *p = __float2half_rn(v); }

// float64 -> storage type with a single rounding (round to nearest even).
template <typename T> __device__ __forceinline__ void store_d(T* p, double v);
template <> __device__ __forceinline__ void store_d<float>(float* p, double v) { *p = (float)v; }
template <> __device__ __forceinline__ void store_d<__half>(__half* p, double v) {
    // Round to odd into float (24 bits >= 11 + 2), then float -> half rounds once correctly.
    float t = __double2float_rz(v);
    if ((double)t != v) t = __uint_as_float(__float_as_uint(t) | 1u);
    *p = __float2half_rn(t);
}

// ------------------------------------------------------------------------ BT.601 full range
// Y = Kr R + Kg G + Kb B, Cb = (B - Y) / (2 (1 - Kb)) + 1/2, Cr = (R - Y) / (2 (1 - Kr)) + 1/2.
struct Ycc {
    static constexpr float kr = 0.299f, kb = 0.114f, kg = 1.0f - 0.299f - 0.114f;
    static constexpr float cb_s = 1.0f / 1.772f, cr_s = 1.0f / 1.402f;
    __device__ __forceinline__ static void from_rgb(float r, float g, float b, float& y, float& cb, float& cr) {
        y = 0.299f * r + 0.587f * g + 0.114f * b;
        cb = (b - y) * (1.0f / 1.772f) + 0.5f;
        cr = (r - y) * (1.0f / 1.402f) + 0.5f;
    }
    // Exact algebraic inverse: R = Y + 1.402 (Cr - 1/2), B = Y + 1.772 (Cb - 1/2),
    // G = (Y - Kr R - Kb B) / Kg.
    __device__ __forceinline__ static void to_rgb(float y, float cb, float cr, float& r, float& g, float& b) {
        r = y + 1.402f * (cr - 0.5f);
        b = y + 1.772f * (cb - 0.5f);
        g = (y - 0.299f * r - 0.114f * b) * (1.0f / 0.587f);
    }
};

// ------------------------------------------------------------------------ kernel parameters
struct ImageArg {
    const void* data;
    int64_t row, plane;
    int32_t w, h;
};

constexpr int kMaxThr = 16;       // max thresholds per feature (q_s, q_c <= 16)
constexpr int kMaxTheta = 64;     // max orientation bins
constexpr int kMaxFeat = 160;     // max regression features incl. targets (training)

// Selector constants, passed by value.
// BT.601 luma in float64, products and sums rounded one at a time in a fixed order
// ((Kr R + Kg G) + Kb B), so every kernel gets the same value for the same pixel.
constexpr double kLumaR = 0.299, kLumaB = 0.114, kLumaG = 1.0 - kLumaR - kLumaB;
__device__ __forceinline__ double luma_d(double r, double g, double b) {
    return __dadd_rn(__dadd_rn(__dmul_rn(kLumaR, r), __dmul_rn(kLumaG, g)), __dmul_rn(kLumaB, b));
}

struct SelectArg {
    int32_t q_theta, q_s, q_c;
    int32_t luma;               // colour input: structure tensor of the luma only
    int32_t phases, pad;        // 4: bucket s' = 4 s + 2 (y mod 2) + (x mod 2)
    double t_s[kMaxThr];
    double t_c[kMaxThr];
    // Unit vectors at the orientation-bin boundaries of the doubled angle, k = 1 .. q_theta/2 - 1,
    // i.e. (cos(2 pi k / q_theta), sin(2 pi k / q_theta)).
    double bcos[kMaxTheta / 2];
    double bsin[kMaxTheta / 2];
};

void fill_select_arg(const mdn_level& lvl, SelectArg& a);
// Directions (cos, sin) of the orientation-bin boundaries k = 1 .. q_theta/2 - 1 in the doubled-angle
// plane (angle 2 pi k / q_theta), made exactly mirror-symmetric about the vertical: the boundary at
// pi - x is (-cos x, sin x) bit for bit, the vertical one is (0, 1) and a diagonal one has equal
// components. A vector lying exactly on a boundary then has a zero cross product with it and goes
// to the upper bin, on either side of the vertical.
void orientation_boundaries(int q_theta, double* bcos, double* bsin);

// Launchers (stream work only; arguments already validated).
mdn_status launch_down2_walk(const mdn_image& in, const mdn_image& out, hipStream_t st);
inline mdn_status launch_down2(const mdn_image& in, const mdn_image& out, hipStream_t st) {
    return launch_down2_walk(in, out, st);
}
// Selector maps hold uint8 when K <= 256 and uint16 otherwise (s_pitch in elements).
inline int level_buckets(const mdn_level& lvl) { return lvl.q_theta * lvl.q_s * lvl.q_c * lvl.phases; }
inline bool wide_selector(const mdn_level& lvl) { return level_buckets(lvl) > 256; }
// uc: the coarser output, read by the Eq. (9) upscale taps and by levels that select on it
// (MDN_SELECT_COARSE; with them a selector-only call needs only z's size).
mdn_status launch_select_apply(const mdn_image& z, const mdn_image* uc, const void* s_in,
                               int64_t s_pitch, void* s_out, const mdn_level& lvl,
                               const mdn_image* out, hipStream_t st);

// One image of a batched launch of the tiled select-and-filter kernel (the kernel of the levels
// that run neither the column walk nor the LDS-bank kernel): its 64 x 16 output tiles are the
// launch's tiles [tile_begin, tile_begin + tiles_x * ceil(h / 16)).
struct TileImage {
    ImageArg z, uc, su;         // level input (RGB), coarser output, image the selector analyses
    void* out;
    int64_t out_row, out_plane;
    const void* s_in;           // selector map to filter with, or null (select inline)
    void* s_out;                // receives the selector used, or null
    int64_t s_pitch;
    int32_t tiles_x, tile_begin;
};
// tiles across and down of a w x h level for the tiled kernel
void tiled_grid(int w, int h, int* tiles_x, int* tiles_y);
// Batched launch over `n_imgs` images (device table, `n_tiles` tiles in all) of one level: the
// colours and dtypes are those of the launch, as for launch_select_apply.
mdn_status launch_select_apply_table(const mdn_level& lvl, const TileImage* imgs, int n_imgs, int n_tiles, int C,
                                     int z_dtype, int uc_dtype, int uc_color, int out_dtype, int out_color,
                                     hipStream_t st);
// true when the cascade filters this level with the tiled kernel (selection inline, no map)
bool level_runs_tiled(const mdn_level& lvl, int channels);

bool walk_supported(const mdn_level& lvl, int channels);
// Multiscale levels whose bank, one channel at a time, fits in LDS beside the tile windows
// (colour levels; float32 7x7/7x7 banks up to 219 buckets) filter from a selector map with the bank in LDS.
bool apply_lds_supported(const mdn_level& lvl, int channels);
mdn_status launch_apply_lds(const mdn_image& z, const mdn_image& uc, const void* s, int64_t s_pitch,
                            const mdn_level& lvl, const mdn_image& out, hipStream_t st);
mdn_status launch_walk(const mdn_image& z, const mdn_image& uc, const mdn_level& lvl, const mdn_image& out,
                       const uint8_t* s_in, uint8_t* s_buf, int64_t s_pitch, hipStream_t st);
mdn_status launch_select_walk(const mdn_image& z, const mdn_level& lvl, void* s, int64_t s_pitch, hipStream_t st);
// The pyramid step z -> next and the selection pass of z (uint8 map s) in one launch; for RGB levels
// with the colour selector, one phase and at most 256 buckets (pyr_sel_fits).
bool pyr_sel_fits(const mdn_level& lvl, int channels);
mdn_status launch_pyr_sel(const mdn_image& z, const mdn_image& next, const mdn_level& lvl, void* s, int64_t s_pitch,
                          hipStream_t st);
mdn_status launch_dihedral(const mdn_image& in, const mdn_image& out, int t, hipStream_t st);
// su: select on the upsampled coarser output su instead of z (z then only gives the size)
mdn_status launch_features(const mdn_image& z, int luma, const mdn_image* su, double* strength, double* coherence,
                           hipStream_t st);

// training
int gram_dims(const mdn_gram& g, int* D, int* nrhs, int* sys_per_k);
mdn_status gram_zero(const mdn_gram& g, hipStream_t st);
size_t train_ws_bytes(const mdn_gram& g, int w, int h);
mdn_status train_accumulate(const mdn_gram& g, const mdn_image& z, const mdn_image* uc, const mdn_image& target,
                            const mdn_level& sel, int precision, void* ws, hipStream_t st);
size_t solve_ws_bytes(const mdn_gram& g);
mdn_status train_solve(const mdn_gram& g, double lam, int64_t min_count, void* coeffs, int out_dtype,
                       int32_t* n_fallback, void* ws, hipStream_t st);
size_t quantile_ws_bytes(int64_t n);
mdn_status quantiles(const double* values, int64_t n, int q, double* out_host, void* ws, size_t ws_bytes,
                     hipStream_t st);

int64_t elem_size(int32_t dtype);

}  // namespace mdn
