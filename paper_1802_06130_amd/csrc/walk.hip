// Persistent column-walk filtering kernel for the multiscale step (Eq. (9)) with 7x7 upscale and
// 7x7 denoise filters on colour images, float16 filter coefficients resident in LDS and float32
// accumulation. The selector s(i) comes from the float64 selection pass as a uint8 map.
//
// Work decomposition. A wavefront owns a strip of 58 output columns and 14-56 output rows; its 64
// lanes hold the columns x0-3 .. x0+60 (a 3-column halo on each side) and walk down the strip one
// output row per step. Persistent 512-thread workgroups (one per CU, two waves per SIMD; the bank
// fills 145 KB of the 160 KB LDS) take strips round-robin from a list that may span many images.
//
// Per step (output row y) every lane
//  - converts the prefetched RGB pixel (y+3, x) to YCbCr and float16 and forms the new row of the
//    7x7 fine window, the neighbouring columns coming from DPP wave shifts (wave_shl / wave_shr)
//    instead of LDS, and prefetches row y+4 and s(y+1);
//  - after odd rows, adds a row to the 7x7 window of the coarser output around floor(x/2), built
//    from three loads per lane (columns floor(x/2) - 3, floor(x/2), floor(x/2) + 3) and DPP shifts
//    by two lanes;
//  - accumulates, per channel, 14 coefficient rows of its bucket (one ds_read_b128 each: 7 taps
//    and a zero as float16 pairs) against the window pairs with v_dot2_f32_f16.
// Window rows live in fixed register slots (row r in slot r mod 7); the 14-row step body is
// expanded at compile time, so no register ever moves when the windows slide.

#include "walk_types.h"

#include <string.h>

#include <type_traits>
#include <utility>

namespace mdn {

namespace {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int kLanesOut = kWalkLanesOut;
constexpr int kWaves = kWalkWaves;     // waves per workgroup
constexpr int kRows = 14;              // coefficient rows per (bucket, channel): 7 f + 7 g
constexpr int kRowBytes = 16;          // 8 halves per row (7 taps + 0)
constexpr int kBucketBytes = 3 * kRows * kRowBytes;   // 672
constexpr int kMaxK = 160 * 1024 / kBucketBytes;      // 243 buckets fit in LDS
// Bucket stride in LDS: 43 rows of 16 bytes (one padding row) when the bank still fits. All lanes
// of a wave read the same (channel, row) of their own buckets; with an odd stride in 16-byte
// units those reads spread over every group of four banks instead of half of them.
constexpr int kPaddedBucketBytes = kBucketBytes + kRowBytes;   // 688
int bank_stride(int K) { return (size_t)K * kPaddedBucketBytes <= 160 * 1024 ? kPaddedBucketBytes : kBucketBytes; }

// lane i <- lane i+1 (shl) / lane i-1 (shr); the lane without a source reads 0 (bound_ctrl)
__device__ __forceinline__ uint32_t shl1(uint32_t v) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ uint32_t shr1(uint32_t v) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ float shl1f(float v) { return __uint_as_float(shl1(__float_as_uint(v))); }
__device__ __forceinline__ float shr1f(float v) { return __uint_as_float(shr1(__float_as_uint(v))); }
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    const h2 v = {(_Float16)lo, (_Float16)hi};
    return __builtin_bit_cast(uint32_t, v);
}
// (lo half of a, lo half of b), (hi of a, hi of b)
__device__ __forceinline__ uint32_t lolo(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x05040100u); }
__device__ __forceinline__ uint32_t hihi(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x07060302u); }
__device__ __forceinline__ float dot2(uint32_t c, uint32_t w, float acc) {
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, c), __builtin_bit_cast(h2, w), acc, false);
}


template <int I>
using IC = std::integral_constant<int, I>;

template <typename F, int... Is>
__device__ __forceinline__ void unroll(F&& f, std::integer_sequence<int, Is...>) {
    (f(IC<Is>{}), ...);
}

// element access through a wave-uniform global base and a 32-bit byte offset (saddr + voffset)
#define MDN_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ float ldo(const T* base, uint32_t elem) {
    const MDN_GLOBAL char* b = (const MDN_GLOBAL char*)(base);
    return (float)*(const MDN_GLOBAL T*)(b + elem * (uint32_t)sizeof(T));
}
template <typename T> __device__ __forceinline__ void sto(T* base, uint32_t elem, float v) {
    MDN_GLOBAL char* b = (MDN_GLOBAL char*)(base);
    *(MDN_GLOBAL T*)(b + elem * (uint32_t)sizeof(T)) = (T)v;
}
__device__ __forceinline__ int ldo_u8(const uint8_t* base, uint32_t elem) {
    return *((const MDN_GLOBAL uint8_t*)base + elem);
}

// Filtering pass of the column walk (the selector map comes from the selection pass).
// TZ: input storage, TU: coarser-output storage, TO: output storage.
template <typename TZ, typename TU, typename TO>
__global__ __launch_bounds__(64 * MDN_WALK_WAVES) void k_walk(WalkArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char bank[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);     // wave-uniform

    const int bstride = __builtin_amdgcn_readfirstlane(a.bank_stride);
    // ---- bank into LDS: row (k, c, r) = 7 taps + 0, float16. One thread takes a whole (bucket,
    // channel) vector of 98 taps: all of its loads are issued before the first row is packed, so a
    // launch pays one memory latency for the fill (per-tap loads in a loop paid one per row).
    {
        const int nvec = a.K * 3;
        for (int i = tid; i < nvec; i += 64 * kWaves) {
            const int k = i / 3, c = i - 3 * k;
            float v[98];
            if (a.coeff_dtype == MDN_F16) {
                // 98 halves at a 196-byte multiple: 49 aligned words
                const uint32_t* src = reinterpret_cast<const uint32_t*>(static_cast<const __half*>(a.coeffs)) +
                                      (int64_t)i * 49;
                uint32_t w[49];
#pragma unroll
                for (int d = 0; d < 49; ++d) w[d] = src[d];
#pragma unroll
                for (int d = 0; d < 49; ++d) {
                    v[2 * d] = __half2float(__ushort_as_half((unsigned short)(w[d] & 0xffffu)));
                    v[2 * d + 1] = __half2float(__ushort_as_half((unsigned short)(w[d] >> 16)));
                }
            } else {
                const float* src = static_cast<const float*>(a.coeffs) + (int64_t)i * 98;
#pragma unroll
                for (int t = 0; t < 98; ++t) v[t] = src[t];
            }
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                // the 7th tap meets the shared pair (x+3 of Y | x+3 of Cb) for Y and Cb, (x+3 of Cr | 0) for Cr
                u4 q;
                q.x = pack2(v[7 * r], v[7 * r + 1]);
                q.y = pack2(v[7 * r + 2], v[7 * r + 3]);
                q.z = pack2(v[7 * r + 4], v[7 * r + 5]);
                q.w = c == 1 ? pack2(0.0f, v[7 * r + 6]) : pack2(v[7 * r + 6], 0.0f);
                *reinterpret_cast<u4*>(bank + (size_t)k * bstride + (size_t)(c * kRows + r) * kRowBytes) = q;
            }
        }
    }
    __syncthreads();

    // The block's waves take neighbouring strips. When each wave has many strips to walk (a.sync_rounds)
    // they move on to their next strips together (a barrier per round): neighbouring strips then read
    // the cache lines they share at about the same time, and L2 serves the second read. Left to drift
    // apart over 44 strips each, the waves fetched half as many bytes again from HBM. With a few
    // strips per wave the barrier's waits cost more time than the drift.
    // XCD-aware order: blocks go to the 8 XCDs round-robin; give each XCD a contiguous run of
    // logical block numbers so that neighbouring strip groups share an L2
    const int G = gridDim.x, b = blockIdx.x, xq = G / 8, xr = G % 8, xcd = b % 8;
    const int lb = (xcd < xr ? xcd * (xq + 1) : xr * (xq + 1) + (xcd - xr) * xq) + b / 8;
    for (int base = lb * kWaves; base < a.n_strips; base += gridDim.x * kWaves) {
      const int strip = base + wave;
      if (strip < a.n_strips) {
        WalkImage im;
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
        const int W = im.W, H = im.H;
        const int xs = sx * kLanesOut, ys = sy * im.rows;
        const int x = xs - 3 + lane;
        const int xc = clampi(x, 0, W - 1);
        const bool out_lane = lane >= 3 && lane < 3 + kLanesOut && x < W;
        const int cxq = x >> 1;
        // element offsets fit in 32 bits (validated on the host); bases stay wave-uniform
        const TZ* zb = static_cast<const TZ*>(im.z);
        const uint32_t zpl = (uint32_t)im.z_plane, zrow = (uint32_t)im.z_row;
        const TU* ub = static_cast<const TU*>(im.uc);
        const uint32_t upl = (uint32_t)im.uc_plane, urow = (uint32_t)im.uc_row;
        const uint32_t uc0 = clampi(cxq - 3, 0, im.Wc - 1), uc1 = clampi(cxq, 0, im.Wc - 1),
                       uc2 = clampi(cxq + 3, 0, im.Wc - 1);
        const uint8_t* sb = im.s_map;
        const uint32_t spitch = (uint32_t)im.s_pitch;

        auto load_rgb = [&](int row, float v[3]) {
            const uint32_t o = (uint32_t)clampi(row, 0, H - 1) * zrow + (uint32_t)xc;
            v[0] = ldo(zb, o);
            v[1] = ldo(zb, o + zpl);
            v[2] = ldo(zb, o + 2 * zpl);
        };
        // a window row: w[c][0..2] = pairs (x-3,x-2) (x-1,x) (x+1,x+2) of channel c,
        // w[0][3] = (Y(x+3), Cb(x+3)) and w[2][3] = (Cr(x+3), 0) shared by the three channels.
        // Y and Cb travel packed in one register, Cr in another, through the DPP shifts.
        auto fine_row = [&](const float rgb[3], uint32_t w[3][4]) {
            float yv, cb, cr;
            Ycc::from_rgb(rgb[0], rgb[1], rgb[2], yv, cb, cr);
            const uint32_t a0 = pack2(yv, cb), b0 = pack2(cr, 0.0f);
            const uint32_t a1 = shl1(a0), a2 = shl1(a1), a3 = shl1(a2);
            const uint32_t am1 = shr1(a0), am2 = shr1(am1), am3 = shr1(am2);
            const uint32_t b1 = shl1(b0), b2 = shl1(b1), b3 = shl1(b2);
            const uint32_t bm1 = shr1(b0), bm2 = shr1(bm1), bm3 = shr1(bm2);
            w[0][0] = lolo(am3, am2);
            w[0][1] = lolo(am1, a0);
            w[0][2] = lolo(a1, a2);
            w[1][0] = hihi(am3, am2);
            w[1][1] = hihi(am1, a0);
            w[1][2] = hihi(a1, a2);
            w[2][0] = lolo(bm3, bm2);
            w[2][1] = lolo(bm1, b0);
            w[2][2] = lolo(b1, b2);
            w[0][3] = a3;
            w[2][3] = b3;
        };
        auto load_coarse = [&](int cr, float u[3][3]) {
            const uint32_t r0 = (uint32_t)clampi(cr, 0, im.Hc - 1) * urow;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u[0][c] = ldo(ub, r0 + c * upl + uc0);
                u[1][c] = ldo(ub, r0 + c * upl + uc1);
                u[2][c] = ldo(ub, r0 + c * upl + uc2);
            }
        };
        auto coarse_row = [&](float u[3][3], uint32_t w[3][4]) {
            if (im.uc_rgb) {
#pragma unroll
                for (int j = 0; j < 3; ++j) Ycc::from_rgb(u[j][0], u[j][1], u[j][2], u[j][0], u[j][1], u[j][2]);
            }
            // u[0], u[1], u[2]: columns floor(x/2) - 3, floor(x/2), floor(x/2) + 3
            const uint32_t a0 = pack2(u[0][0], u[0][1]), b0 = pack2(u[0][2], 0.0f);
            const uint32_t a1 = pack2(u[1][0], u[1][1]), b1 = pack2(u[1][2], 0.0f);
            const uint32_t a2 = pack2(u[2][0], u[2][1]), b2 = pack2(u[2][2], 0.0f);
            // lane x+2 holds floor(x/2)+1, lane x-2 floor(x/2)-1
            const uint32_t am2 = shl1(shl1(a0)), bm2 = shl1(shl1(b0));     // floor(x/2) - 2
            const uint32_t ap1 = shl1(shl1(a1)), bp1 = shl1(shl1(b1));     // floor(x/2) + 1
            const uint32_t am1 = shr1(shr1(a1)), bm1 = shr1(shr1(b1));     // floor(x/2) - 1
            const uint32_t ap2 = shr1(shr1(a2)), bp2 = shr1(shr1(b2));     // floor(x/2) + 2
            w[0][0] = lolo(a0, am2);
            w[0][1] = lolo(am1, a1);
            w[0][2] = lolo(ap1, ap2);
            w[1][0] = hihi(a0, am2);
            w[1][1] = hihi(am1, a1);
            w[1][2] = hihi(ap1, ap2);
            w[2][0] = lolo(b0, bm2);
            w[2][1] = lolo(bm1, b1);
            w[2][2] = lolo(bp1, bp2);
            w[0][3] = a2;
            w[2][3] = b2;
        };

        // ring slots: fine row r sits in fw[r mod 7], coarse row cr in cw[cr mod 7] (ys = 0 mod 14)
        uint32_t fw[7][3][4];
        uint32_t cw[7][3][4];
        float znext[3];
        int snext;
        {
            float t[3];
#pragma unroll
            for (int d = -3; d <= 2; ++d) {
                load_rgb(ys + d, t);
                fine_row(t, fw[(d + 7) % 7]);
            }
            const int cy = ys >> 1;
#pragma unroll
            for (int d = -3; d <= 3; ++d) {
                float u[3][3];
                load_coarse(cy + d, u);
                coarse_row(u, cw[(d + 7) % 7]);
            }
            load_rgb(ys + 3, znext);
            snext = ldo_u8(sb, (uint32_t)clampi(ys, 0, H - 1) * spitch + (uint32_t)xc);
        }
        for (int y0 = ys; y0 < ys + im.rows && y0 < H; y0 += 14) {
            unroll([&](auto ic) {
                constexpr int I = decltype(ic)::value;
                const int y = y0 + I;
                // the prefetched row y+3 enters the fine window; prefetch row y+4 and s(y+1)
                fine_row(znext, fw[(I + 3) % 7]);
                // a selector value outside the bank reads bucket 0 and yields NaN (memory-safe)
                const bool s_ok = snext < a.K;
                const int s = s_ok ? snext : 0;
                load_rgb(y + 4, znext);
                snext = ldo_u8(sb, (uint32_t)clampi(y + 1, 0, H - 1) * spitch + (uint32_t)xc);
                float unext[3][3];
                if constexpr (I & 1) load_coarse(((y + 1) >> 1) + 3, unext);
                const uint8_t* bp = bank + (size_t)s * bstride;
                float acc[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float af = 0.0f, ag = 0.0f;
#pragma unroll
                    for (int r = 0; r < 7; ++r) {
                        const u4 q = *reinterpret_cast<const u4*>(bp + (c * kRows + r) * kRowBytes);
                        const uint32_t (*w)[4] = cw[(I / 2 + r + 4) % 7];
                        af = dot2(q.x, w[c][0], af);
                        af = dot2(q.y, w[c][1], af);
                        af = dot2(q.z, w[c][2], af);
                        af = dot2(q.w, w[c == 2 ? 2 : 0][3], af);
                    }
#pragma unroll
                    for (int r = 0; r < 7; ++r) {
                        const u4 q = *reinterpret_cast<const u4*>(bp + (c * kRows + 7 + r) * kRowBytes);
                        const uint32_t (*w)[4] = fw[(I + r + 4) % 7];
                        ag = dot2(q.x, w[c][0], ag);
                        ag = dot2(q.y, w[c][1], ag);
                        ag = dot2(q.z, w[c][2], ag);
                        ag = dot2(q.w, w[c == 2 ? 2 : 0][3], ag);
                    }
                    acc[c] = af + ag;
                }
                if (out_lane && y < H) {
                    if (!s_ok) acc[0] = acc[1] = acc[2] = __builtin_nanf("");
                    if (im.o_rgb) Ycc::to_rgb(acc[0], acc[1], acc[2], acc[0], acc[1], acc[2]);
                    const uint32_t off = (uint32_t)y * (uint32_t)im.o_row + (uint32_t)x;
#pragma unroll
                    for (int c = 0; c < 3; ++c) sto(static_cast<TO*>(im.out), off + c * (uint32_t)im.o_plane, acc[c]);
                }
                // after an odd row the next row has a new floor(y/2): the coarse row floor/2 + 3 enters
                if constexpr (I & 1) coarse_row(unext, cw[((I + 1) / 2 + 3) % 7]);
            }, std::make_integer_sequence<int, 14>{});
        }
      }
      if (a.sync_rounds) __syncthreads();   // uniform: every wave reaches it once per round
    }
}

}  // namespace

bool walk_supported(const mdn_level& lvl, int channels) {
    // the bank is copied a word at a time: 4-byte aligned coefficients
    return channels == 3 && lvl.radius_f == 3 && lvl.radius_g == 3 && lvl.phases == 1 && level_buckets(lvl) <= kMaxK &&
           ((uintptr_t)lvl.coeffs & 3) == 0;
}

size_t walk_lds_bytes(int K) { return (size_t)K * bank_stride(K); }

int device_cus() {
    int dev = 0, ncu = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return ncu;
}

void fill_walk_image(WalkImage& wi, const mdn_image& z, const mdn_image& uc, const mdn_image& out, int begin) {
    memset(&wi, 0, sizeof(wi));
    wi.z = z.data;
    wi.uc = uc.data;
    wi.out = out.data;
    wi.z_row = z.row_pitch;
    wi.z_plane = z.plane_pitch;
    wi.uc_row = uc.row_pitch;
    wi.uc_plane = uc.plane_pitch;
    wi.o_row = out.row_pitch;
    wi.o_plane = out.plane_pitch;
    wi.W = z.width;
    wi.H = z.height;
    wi.Wc = uc.width;
    wi.Hc = uc.height;
    wi.z_dtype = z.dtype;
    wi.uc_dtype = uc.dtype;
    wi.uc_rgb = uc.color == MDN_RGB;
    wi.o_dtype = out.dtype;
    wi.o_rgb = out.color == MDN_RGB;
    wi.nsx = (z.width + kLanesOut - 1) / kLanesOut;
    wi.strip_begin = begin;
}

// rows per strip: 56 when the image gives every wave slot a few strips, else down to 14
int walk_rows(int w, int h, int wave_slots) {
    const int nsx = (w + kLanesOut - 1) / kLanesOut;
    int rows = 56;
    while (rows > 14 && (int64_t)nsx * ((h + rows - 1) / rows) < (int64_t)wave_slots * 3) rows -= 14;
    return rows;
}

static int g_walk_init = 0;

// Allow every filtering-kernel instance the whole LDS (once per process; before any graph capture).
mdn_status init_walk_kernels() {
    if (g_walk_init) return MDN_OK;
    const void* fns[] = {(const void*)k_walk<_Float16, _Float16, _Float16>, (const void*)k_walk<float, _Float16, float>,
                         (const void*)k_walk<float, float, float>, (const void*)k_walk<_Float16, float, _Float16>};
    for (const void* f : fns)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
            return fail(MDN_EDEVICE, "walk: cannot reserve LDS");
    g_walk_init = 1;
    return MDN_OK;
}

template <typename TZ, typename TU, typename TO>
static mdn_status launch_typed_walk(const WalkArgs& a, int grid, size_t lds, hipStream_t st) {
    mdn_status e = init_walk_kernels();
    if (e) return e;
    k_walk<TZ, TU, TO><<<grid, 64 * kWaves, lds, st>>>(a);
    return check_launch("walk");
}

mdn_status launch_walk_args(const WalkArgs& args, int zd, int ud, int od, hipStream_t st) {
    if (args.n_strips <= 0) return MDN_OK;
    WalkArgs a = args;
    a.bank_stride = bank_stride(a.K);
    const size_t lds = walk_lds_bytes(a.K);
    const int ncu = device_cus();
    const int blocks = (a.n_strips + kWaves - 1) / kWaves;
    const int grid = blocks < ncu ? blocks : ncu;
    a.sync_rounds = (int64_t)a.n_strips >= 24LL * grid * kWaves;     // 24 or more strips per wave
    const bool zh = zd == MDN_F16, uh = ud == MDN_F16, oh = od == MDN_F16;
    if (zh && uh && oh) return launch_typed_walk<_Float16, _Float16, _Float16>(a, grid, lds, st);
    if (!zh && uh && !oh) return launch_typed_walk<float, _Float16, float>(a, grid, lds, st);
    if (!zh && !uh && !oh) return launch_typed_walk<float, float, float>(a, grid, lds, st);
    if (zh && !uh && oh) return launch_typed_walk<_Float16, float, _Float16>(a, grid, lds, st);
    return fail(MDN_ENOTSUP, "walk: input/coarse/output dtype combination not supported");
}

// Selection pass (float64 tensor, uint8 map) followed by the filtering pass.
mdn_status launch_walk(const mdn_image& z, const mdn_image& uc, const mdn_level& lvl, const mdn_image& out,
                       const uint8_t* s_in, uint8_t* s_buf, int64_t s_pitch, hipStream_t st) {
    if (z.width == 0 || z.height == 0) return MDN_OK;
    mdn_status e;
    const uint8_t* smap = s_in;
    if (!smap) {
        if ((e = launch_select_apply(z, &uc, nullptr, s_pitch, s_buf, lvl, nullptr, st))) return e;
        smap = s_buf;
    }
    WalkArgs a;
    memset(&a, 0, sizeof(a));
    fill_walk_image(a.single, z, uc, out, 0);
    a.single.s_map = smap;
    a.single.s_pitch = s_pitch;
    a.single.rows = walk_rows(z.width, z.height, device_cus() * kWaves);
    a.imgs = nullptr;
    a.n_imgs = 1;
    a.n_strips = a.single.nsx * ((z.height + a.single.rows - 1) / a.single.rows);
    a.coeffs = lvl.coeffs;
    a.coeff_dtype = lvl.coeff_dtype;
    a.K = level_buckets(lvl);
    return launch_walk_args(a, z.dtype, uc.dtype, out.dtype, st);
}

}  // namespace mdn
