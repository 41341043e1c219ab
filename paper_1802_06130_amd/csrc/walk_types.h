// Descriptor tables of the persistent column-walk kernels (pyramid, selection, filtering).
// A launch walks a list of strips that may span many images: image i owns the strips
// [strip_begin_i, strip_begin_i + nsx_i * ceil(height_i / rows_i)), found by binary search.
#pragma once

#include "mdn_internal.h"

#include <vector>

namespace mdn {

constexpr int kWalkLanesOut = 58;   // filtering: output columns per wave (3-column halo each side)
constexpr int kSelLanesOut = 58;    // selection: output columns per wave
constexpr int kD2LanesOut = 60;     // pyramid: output columns per wave (2-column halo each side)
#ifndef MDN_WALK_WAVES
#define MDN_WALK_WAVES 8
#endif
constexpr int kWalkWaves = MDN_WALK_WAVES;   // filtering: waves per workgroup (one workgroup per CU)

// A value every lane holds alike, moved to scalar registers word by word. A strip's image descriptor
// is read either from the kernel arguments or from the launch's table; the compiler may read both
// through one generic pointer, which would leave the descriptor and all addressing derived from it
// in vector registers.
template <typename T> __device__ __forceinline__ T wave_uniform(const T& v) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T r;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&v);
    uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)s[i]);
    return r;
}

struct WalkImage {
    const void* z;          // RGB input of the level
    const void* uc;         // coarser output (YCbCr, or RGB at the coarsest level)
    void* out;
    int64_t z_row, z_plane, uc_row, uc_plane, o_row, o_plane;
    int32_t W, H, Wc, Hc;
    int32_t z_dtype, uc_dtype, uc_rgb, o_dtype, o_rgb;
    int32_t nsx;            // strips across
    int32_t strip_begin;    // first strip index of this image in the list
    int32_t rows;           // output rows per strip (a multiple of 14)
    const uint8_t* s_map;   // selector of this level (from the selection pass)
    int64_t s_pitch;
};

struct WalkArgs {
    WalkImage single;           // used when imgs == nullptr
    const WalkImage* imgs;      // device array (batch) or null
    int32_t n_imgs, n_strips;
    const void* coeffs;         // [K][3][98], float16 or float32
    int32_t coeff_dtype, K;
    int32_t bank_stride;        // bytes between buckets in LDS (set by the launcher)
    int32_t sync_rounds;        // the block's waves start their strips together (set by the launcher)
};

struct SelImage {
    const void* z;
    void* s;                    // selector map: uint8, or uint16 when K > 256
    int64_t z_row, z_plane, s_pitch;
    int32_t W, H, C;
    int32_t nsx, strip_begin, rows;     // strips across, first strip, rows per strip (multiple of 10)
};

struct SelWalkArgs {
    SelImage single;
    const SelImage* imgs;
    int32_t n_imgs, n_strips;
    int32_t q_theta, q_s, q_c, half;
    int32_t luma;               // RGB input: structure tensor of its float64 luma only
    int32_t phases;             // 4: bucket s' = 4 s + 2 (y mod 2) + (x mod 2)
    double s_lim[kMaxThr];      // 100 t^2: box sums of squared differences are 100 x the box mean
    double c_k2[kMaxThr];       // (2t/(1+t^2))^2, or -1 when t <= 0 (always reached)
    double bcos[kMaxTheta / 2], bsin[kMaxTheta / 2];
};

struct D2Image {
    const void* in;
    void* out;
    int64_t i_row, i_plane, o_row, o_plane;
    int32_t Wi, Hi, Wo, Ho;
    int32_t nsx, strip_begin, rows;     // rows: output rows per strip (multiple of 4)
    int32_t pad;
};

struct D2Args {
    D2Image single;
    const D2Image* imgs;
    int32_t n_imgs, n_strips;
};

// strip heights chosen from the number of wave slots when not tuned
int walk_rows(int w, int h, int wave_slots);
int select_walk_rows(int w, int h, int ncu);
int down2_rows(int wo, int ho, int ncu);

void fill_walk_image(WalkImage& wi, const mdn_image& z, const mdn_image& uc, const mdn_image& out, int begin);
void fill_sel_consts(const mdn_level& lvl, SelWalkArgs& a);
size_t walk_lds_bytes(int K);
int device_cus();

mdn_status init_walk_kernels();

// launches over prepared arguments (dtypes select the template instance)
mdn_status launch_walk_args(const WalkArgs& a, int z_dtype, int uc_dtype, int o_dtype, hipStream_t st);
mdn_status launch_select_args(const SelWalkArgs& a, int channels, int z_dtype, hipStream_t st);
mdn_status launch_down2_args(const D2Args& a, int channels, int in_dtype, int out_dtype, hipStream_t st);
// a pyramid step and the selection pass of the same level (RGB, uint8 map, colour selector) in one
// launch; pyr_sel_fusable tells whether the selection's bank allows it
bool pyr_sel_fusable(const SelWalkArgs& s);
mdn_status launch_pyr_sel_args(const D2Args& d, const SelWalkArgs& s, int level_dtype, int next_dtype, hipStream_t st);
// single-image arguments of the pyramid step in -> out and of the selection pass of z
void fill_down2_single(const mdn_image& in, const mdn_image& out, D2Args& a);
void fill_select_single(const mdn_image& z, const mdn_level& lvl, void* s, int64_t s_pitch, SelWalkArgs& a);


// ---------------------------------------------------------------- batched cascade
constexpr int kMaxLevels = 8;
constexpr int kMaxPlanBanks = 8;

// One launch of a batch: a pyramid step (level l -> l+1, every image deep enough), or the selection
// pass, the filtering walk or the tiled select-and-filter kernel of level l for the images of one
// bank. The table of the launch sits at tab_off in the batch's table buffer.
struct BatchItem {
    int kind;                    // 0 pyramid, 1 selection, 2 filtering walk, 3 tiled
    int level, bank;
    size_t tab_off;              // table of the launch in the batch's table buffer
    D2Args d2;
    SelWalkArgs sel;
    WalkArgs walk;
    mdn_level lv;                // tiled launches
    const TileImage* tiles;
    int32_t n_imgs, n_tiles, z_dtype, uc_color, out_dtype, out_color;
};

struct BatchLaunch {
    int Lmax, storage, in_dtype, out_dtype;
    size_t table_bytes;
    const char* tab_dev;               // device copy of the tables
    std::vector<BatchItem> items;      // in launch order
};

size_t batch_image_ws(int w, int h, int L, int storage);
// tile: per-level descriptors for the tiled kernel, or null when not wanted
void describe_cascade(const mdn_image& in, const mdn_image& out, void* ws, int L, int storage, const int (*rows)[3],
                      int ncu, D2Image* d2, SelImage* sel, WalkImage* walk, TileImage* tile = nullptr);
int tiles_of(const TileImage& t);
int strips_of(const D2Image& d);
int strips_of(const SelImage& d);
int strips_of(const WalkImage& d);

}  // namespace mdn
