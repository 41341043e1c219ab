// Per-bucket least-squares filter training (Eq. (7)-(8)).
//
// For every bucket k the filters minimise the squared error over the pixels with s(i) = k,
// which is one linear regression per bucket (and per YCbCr channel, footnote of Section 3).
// The normal equations are accumulated here and solved with a ridge term.
//
// Grouping: the pixel indices of the level are sorted by bucket with a stable radix sort of the
// selector map (8-bit keys), so every bucket's pixels form one contiguous run in raster order,
// and the run boundaries come from a binary search per bucket.
//
// Accumulation (k_gram): one workgroup per (bucket, system, segment). A bucket's run is cut into
// up to kMaxSeg equal segments of whole 64-sample chunks, so that large buckets do not leave the
// rest of the device idle. A workgroup gathers 64 samples at a time into LDS as a feature-major
// matrix X^T (regression taps followed by the target value(s), zero padded to a multiple of 32;
// the gathers of the next chunk are in flight while the current one is multiplied). The planes
// are float32 copies with a replicated margin of kPad pixels, so every tap row of a sample is
// consecutive floats of one plane row: a wave takes whole tap rows, one sample per lane, each
// row one contiguous load,
// and accumulates the upper-triangle 32x32 tiles of X^T X on MFMA with FP32 accumulators. The
// target value rides along as an extra feature, so the same tiles yield G = sum x x^T,
// b = sum x y and yy = sum y^2. Two products are offered:
//   MDN_GRAM_F32    : v_mfma_f32_32x32x2_f32 - exact FP32 products, FP32 accumulation;
//   MDN_GRAM_BF16X3 : v_mfma_f32_32x32x16_bf16 on a hi/lo split x = hi + lo (hi = bf16(x),
//                     lo = bf16(x - hi)); x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y.
// Each workgroup writes its FP32 tiles to a partial buffer; k_gram_reduce then adds the segments
// of each system in segment order into the FP64 accumulators (fixed order: bitwise reproducible).
//
// Solve (k_solve): one workgroup per system, (G/n + lambda I) h = b/n by Cholesky in float64,
// the lower triangle packed in LDS. Buckets with fewer than min_count samples (or a failed
// factorisation) take the pooled solution of the level (sums over all buckets).

#include <hipcub/hipcub.hpp>

#include "mdn_internal.h"

#include <string.h>

#include <type_traits>

namespace mdn {

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kChunk = 64;                 // samples per MFMA chunk
constexpr int kPad = 3;                    // replicated margin of the gather planes (radius <= 3)
constexpr int kMaxRows = 24;               // tap rows per sample: 3 planes x 7 rows + 3 targets
constexpr int kMaxSeg = 16;                // segments per bucket run
constexpr int kMinSegChunks = 8;           // chunks per segment, at least

// chunks per segment of a run of `chunks` chunks (segments after the run's end stay idle)
__host__ __device__ inline int seg_chunks(int chunks, int nseg) {
    const int per = (chunks + nseg - 1) / nseg;
    return per > kMinSegChunks ? per : kMinSegChunks;
}
// LDS row stride (elements) of X^T: bf16 rows keep 16-byte aligned 8-element reads; f32 rows
// use a stride of 2 mod 64 dwords so that the 64 lanes of an MFMA operand read (32 rows x 2
// columns) fall in 64 distinct banks.
template <int PREC> struct Ldw { static constexpr int v = PREC == 0 ? kChunk + 2 : kChunk + 8; };

// Segments per bucket: enough to spread a big bucket over several workgroups, fewer when the
// buckets are many (and so small on average), which also bounds the partial-sum buffer.
int gram_segments(int64_t npx, int K) {
    const int64_t s = (npx + 16383) / 16384;
    const int cap = K <= 256 ? kMaxSeg : (kMaxSeg * 256 / K > 1 ? kMaxSeg * 256 / K : 1);
    return (int)(s < 1 ? 1 : (s > cap ? cap : s));
}

// tap-row descriptor: source (0 fine, 1 coarse, 2 target), plane, row offset dy, first column
// offset dx0, length, index of its first feature
__host__ __device__ inline int row_pack(int src, int plane, int dy, int dx0, int len, int fbase) {
    return (src << 28) | (plane << 26) | ((dy + 8) << 22) | ((dx0 + 8) << 18) | (len << 14) | fbase;
}

struct GramArgs {
    // YCbCr (or grey) planes of z^l, of the clean level u^l and of the coarser output u^{l+1},
    // float32 with a replicated margin of kPad pixels on every side, in one buffer: target and
    // coarse planes start at the given element offsets; pitches are those of the padded planes
    const float* planes;
    int32_t target_off, coarse_off;
    int32_t f_row, f_plane, c_row, c_plane;
    int32_t W, H, Wc, Hc;
    const int32_t* idx;     // pixel indices sorted by bucket (raster order within a bucket)
    const int32_t* off;     // [K+1] start of each bucket's run in idx
    int32_t D, Daug, nrhs, per_channel;
    int32_t nseg;           // segments per bucket run
    int32_t nrows;          // tap rows per sample
    int32_t rows[kMaxRows];
    float* part;            // [K][systems per bucket][nseg][tiles][1024] partial tiles
    double* G;
    double* b;
    int64_t* n;
    double* yy;
};

// float -> bfloat16, round to nearest even (v_cvt_pk_bf16_f32 on gfx950; inputs are finite).
__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

__device__ __forceinline__ float from_bf16(__bf16 h) {
    return __uint_as_float((uint32_t)__builtin_bit_cast(unsigned short, h) << 16);
}

// Tile t of the upper triangle (P <= Q, row-major over P) -> (P, Q).
__host__ __device__ inline void tile_pq(int T, int t, int* P, int* Q) {
    int p = 0;
    while (t >= T - p) {
        t -= T - p;
        ++p;
    }
    *P = p;
    *Q = p + t;
}

// Sum the segment partials of one system in segment order (float64) and add them to the
// accumulators (256 threads); the result does not depend on timing.
__device__ void add_partials(const GramArgs& a, int T, int k, int sys_c, int sys, int nseg) {
    const int NT = T * (T + 1) / 2;
    if (sys_c == 0 && threadIdx.x == 0) a.n[k] += a.off[k + 1] - a.off[k];
    const float* part = a.part + (int64_t)sys * a.nseg * NT * 1024;
    const int D = a.D;
    double* G = a.G + (int64_t)sys * D * D;
    double* bvec = a.b + (int64_t)sys * a.nrhs * D;
    double* yy = a.yy + (int64_t)sys * a.nrhs;
    for (int e = threadIdx.x; e < NT * 1024; e += 256) {
        // every segment's partial is loaded at once (idle segments re-read segment 0), then
        // summed in segment order
        float pv[kMaxSeg];
#pragma unroll
        for (int sg = 0; sg < kMaxSeg; ++sg) pv[sg] = part[(int64_t)(sg < nseg ? sg : 0) * NT * 1024 + e];
        double v = 0.0;
#pragma unroll
        for (int sg = 0; sg < kMaxSeg; ++sg)
            if (sg < nseg) v += (double)pv[sg];
        const int t = e >> 10, r = (e >> 6) & 15, lane = e & 63;
        int P, Q;
        tile_pq(T, t, &P, &Q);
        const int p = P * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int q = Q * 32 + (lane & 31);
        if (p >= a.Daug || q >= a.Daug) continue;
        if (p < D && q < D) {
            G[(int64_t)p * D + q] += v;
            if (P != Q) G[(int64_t)q * D + p] += v;
        } else if (p < D && q >= D) {
            bvec[(int64_t)(q - D) * D + p] += v;
        } else if (p >= D && q >= D && p == q) {
            yy[p - D] += v;
        }
    }
}

// RPW: tap rows per wave (the sample's rows are dealt to the four waves), at least ceil(nrows / 4).
template <int PREC, int T, int RPW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_gram(GramArgs a) {
    constexpr int DPAD = 32 * T;
    constexpr int NT = T * (T + 1) / 2;
    constexpr int TPW = (NT + 3) / 4;
    constexpr int LDW = Ldw<PREC>::v;
    using XT = typename std::conditional<PREC == 0, float, __bf16>::type;
    __shared__ XT xhi[DPAD][LDW];
    __shared__ XT xlo[PREC == 0 ? 1 : DPAD][PREC == 0 ? 1 : LDW];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: row decoding is scalar
    const int k = blockIdx.x;
    const int sys_c = blockIdx.y;                      // channel (per-channel systems) or 0
    const int seg = blockIdx.z;
    const int plane_off = a.per_channel ? sys_c : 0;
    const int W = a.W;

    // this segment's chunks of the bucket's run
    const int beg = a.off[k], end = a.off[k + 1];
    const int chunks = (end - beg + kChunk - 1) / kChunk;
    const int per = seg_chunks(chunks, a.nseg);
    const int c0 = seg * per, c1 = min(chunks, c0 + per);
    if (c0 >= c1) return;

    const float* planes = a.planes;
    const int nrows = __builtin_amdgcn_readfirstlane(a.nrows);
    const int daug = __builtin_amdgcn_readfirstlane(a.Daug);
    // feature rows past the last feature stay zero
    for (int e = tid; e < (DPAD - daug) * LDW; e += 256) {
        const int f = daug + e / LDW, col = e - (e / LDW) * LDW;
        xhi[f][col] = XT(0.0f);
        if constexpr (PREC != 0) xlo[f][col] = XT(0.0f);
    }

    // tiles owned by this wave: t = wave, wave + 4, ...
    int tP[TPW], tQ[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) tile_pq(T, min(wave + 4 * i, NT - 1), &tP[i], &tQ[i]);
    const int my_tiles = (NT - wave + 3) / 4;
    f16v acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][r] = 0.0f;

    // Gather: wave w takes tap rows w, w + 4, ... of every sample, one sample per lane; a row's
    // taps are consecutive floats of a padded plane row, loaded together. The next chunk's loads
    // are in flight while the current chunk is multiplied from LDS, and are consumed only when
    // that chunk is stored to LDS. (Two chunks in flight measured the same.)
    struct Buf {
        float v[RPW][8];
        bool live;
    };
    Buf buf;
    auto load = [&](int chunk, Buf& b) {
        const int base = beg + chunk * kChunk;
        b.live = base + lane < end;
        const int pix = b.live ? a.idx[base + lane] : 0;
        const int y = pix / W, x = pix - y * W;
        float (&v)[RPW][8] = b.v;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wave + 4 * i;
            if (r >= nrows) break;
            const int e = a.rows[r];
            const int src = e >> 28, pl = ((e >> 26) & 3) + plane_off;
            const int dy = ((e >> 22) & 15) - 8, dx0 = ((e >> 18) & 15) - 8, len = (e >> 14) & 15;
            const bool cs = src == 1;
            const int yb = (cs ? (y >> 1) : y) + kPad + dy, xb = (cs ? (x >> 1) : x) + kPad + dx0;
            const int start = src == 0 ? 0 : (cs ? a.coarse_off : a.target_off);
            const float* q = planes + start + pl * (cs ? a.c_plane : a.f_plane) + yb * (cs ? a.c_row : a.f_row) + xb;
            // the row length is the same on every lane (wave-uniform branch)
            if (len == 7) {
                __builtin_memcpy(&v[i][0], q, 7 * sizeof(float));
            } else if (len == 5) {
                __builtin_memcpy(&v[i][0], q, 5 * sizeof(float));
            } else if (len == 3) {
                __builtin_memcpy(&v[i][0], q, 3 * sizeof(float));
            } else {
                v[i][0] = *q;
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // keep every load ahead of the first use
    };
    auto store = [&](const Buf& b) {
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wave + 4 * i;
            if (r >= nrows) break;
            const int e = a.rows[r];
            const int len = (e >> 14) & 15, fb = e & 0x3fff;
#pragma unroll
            for (int j = 0; j < 7; ++j) {
                if (j >= len) break;
                const float w = b.live ? b.v[i][j] : 0.0f;
                if constexpr (PREC == 0) {
                    xhi[fb + j][lane] = w;
                } else {
                    const __bf16 h = to_bf16(w);
                    xhi[fb + j][lane] = h;
                    xlo[fb + j][lane] = to_bf16(w - from_bf16(h));
                }
            }
        }
    };
    auto multiply = [&]() {
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (i < my_tiles) {
                const int rowA = tP[i] * 32 + (lane & 31);
                const int rowB = tQ[i] * 32 + (lane & 31);
                if constexpr (PREC == 0) {
#pragma unroll 8
                    for (int ks = 0; ks < kChunk / 2; ++ks) {
                        const float av = xhi[rowA][2 * ks + (lane >> 5)];
                        const float bv = xhi[rowB][2 * ks + (lane >> 5)];
                        acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[i], 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int ks = 0; ks < kChunk / 16; ++ks) {
                        const int col = 16 * ks + 8 * (lane >> 5);
                        const bf8v ah = *reinterpret_cast<const bf8v*>(&xhi[rowA][col]);
                        const bf8v bh = *reinterpret_cast<const bf8v*>(&xhi[rowB][col]);
                        const bf8v al = *reinterpret_cast<const bf8v*>(&xlo[rowA][col]);
                        const bf8v bl = *reinterpret_cast<const bf8v*>(&xlo[rowB][col]);
                        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[i], 0, 0, 0);
                        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[i], 0, 0, 0);
                        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[i], 0, 0, 0);
                    }
                }
            }
        }
    };

    load(c0, buf);
    store(buf);
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
        const bool more = c + 1 < c1;
        if (more) load(c + 1, buf);  // in flight during the products
        multiply();
        __syncthreads();             // every wave is done with this chunk
        if (more) {
            store(buf);
            __syncthreads();
        }
    }

    // partial tiles of this segment: [system][seg][tile][r][lane]
    const int sys = a.per_channel ? k * (int)gridDim.y + sys_c : k;
    float* part = a.part + ((int64_t)sys * a.nseg + seg) * NT * 1024;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        if (i >= my_tiles) continue;
        const int t = wave + 4 * i;
#pragma unroll
        for (int r = 0; r < 16; ++r) part[t * 1024 + r * 64 + lane] = acc[i][r];
    }
}

// Sum the segment partials of each system in segment order (float64) and add them to the
// accumulators; the result does not depend on timing. (Letting the last segment of each system
// do this inside k_gram was measured 2.4x slower: every workgroup's device-scope release and
// acquire wrote back and invalidated its XCD's L2, which the sample gathers depend on.)
__global__ __launch_bounds__(256) void k_gram_reduce(GramArgs a, int T) {
    const int k = blockIdx.x, sys_c = blockIdx.y;
    const int sys = a.per_channel ? k * (int)gridDim.y + sys_c : k;
    const int chunks = (a.off[k + 1] - a.off[k] + kChunk - 1) / kChunk;
    const int per = seg_chunks(chunks, a.nseg);
    const int nseg = (chunks + per - 1) / per;                      // segments that ran
    if (nseg == 0) return;                                            // empty bucket: nothing to add
    add_partials(a, T, k, sys_c, sys, nseg);
}

// float32 YCbCr (or grey) planes of an RGB / grey image for the sample gathers, with a margin of
// kPad pixels on every side holding the clamped (replicated) border: padded element (y, x),
// -kPad <= y < h + kPad and -kPad <= x < w + kPad, is at out[(y + kPad) o_row + x + kPad].
__global__ void k_to_planes(ImageArg in, int32_t dtype, int32_t rgb_to_ycc, int32_t C, float* out, int64_t o_row,
                            int64_t o_plane) {
    const int xp = blockIdx.x * blockDim.x + threadIdx.x;
    const int yp = blockIdx.y;
    if (xp >= in.w + 2 * kPad || yp >= in.h + 2 * kPad) return;
    const int x = clampi(xp - kPad, 0, in.w - 1), y = clampi(yp - kPad, 0, in.h - 1);
    const int64_t off = (int64_t)y * in.row + x;
    float v[3] = {0, 0, 0};
    for (int c = 0; c < C; ++c) {
        v[c] = dtype == MDN_F16 ? __half2float(static_cast<const __half*>(in.data)[off + c * in.plane])
                                : static_cast<const float*>(in.data)[off + c * in.plane];
    }
    if (C == 3 && rgb_to_ycc) Ycc::from_rgb(v[0], v[1], v[2], v[0], v[1], v[2]);
    for (int c = 0; c < C; ++c) out[c * o_plane + (int64_t)yp * o_row + xp] = v[c];
}

__global__ void k_iota(int32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// off[k] = first position of a key >= k in the sorted keys, k = 0..K
template <typename TK>
__global__ void k_bucket_bounds(const TK* keys, int64_t n, int K, int32_t* off) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int)keys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    off[k] = (int32_t)lo;
}

__global__ void k_fill_zero(double* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_fill_zero_i64(int64_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Pooled statistics of one system-channel: sums over all buckets (fixed order).
__global__ void k_pool(const double* G, const double* b, int K, int sys_per_k, int D, int nrhs, double* Gp,
                       double* bp) {
    const int c = blockIdx.y;
    const int64_t nG = (int64_t)D * D, nb = (int64_t)nrhs * D;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nG + nb; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        if (i < nG) {
            for (int k = 0; k < K; ++k) s += G[((int64_t)k * sys_per_k + c) * nG + i];
            Gp[c * nG + i] = s;
        } else {
            const int64_t j = i - nG;
            for (int k = 0; k < K; ++k) s += b[((int64_t)k * sys_per_k + c) * nb + j];
            bp[c * nb + j] = s;
        }
    }
}

struct SolveArgs {
    const double* G;
    const double* b;
    const int64_t* n;
    const double* Gp;
    const double* bp;
    double* hp;           // pooled solutions [sys_per_k][nrhs][D]
    int32_t* ok;          // per bucket system: 1 solved, 0 needs the pooled solution
    const int64_t* n_all;
    int32_t K, sys_per_k, D, nrhs;
    double lam;
    int64_t min_count;
    void* out;            // [K][C][D] coefficients
    int32_t out_dtype, per_channel;
};

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Cholesky solve of (G/n + lam I) h = b/n for one system; L packed in LDS.
__global__ __launch_bounds__(256) void k_solve(SolveArgs a) {
    extern __shared__ double sm[];
    const int D = a.D, nrhs = a.nrhs;
    double* L = sm;                                  // D(D+1)/2
    double* rhs = sm + D * (D + 1) / 2;              // nrhs * D
    __shared__ int fail;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nsys = a.K * a.sys_per_k;
    const int id = blockIdx.x;
    const bool pooled = id >= nsys;
    const int c = pooled ? id - nsys : id % a.sys_per_k;
    const int k = pooled ? -1 : id / a.sys_per_k;
    const int64_t nk = pooled ? *a.n_all : a.n[k];
    if (!pooled && nk < a.min_count) {
        if (tid == 0) a.ok[id] = 0;
        return;
    }
    if (nk <= 0) {
        // empty level: the pooled solution is zero
        for (int i = tid; i < nrhs * D; i += 256) a.hp[(int64_t)c * nrhs * D + i] = 0.0;
        return;
    }
    const double* G = pooled ? a.Gp + (int64_t)c * D * D : a.G + (int64_t)id * D * D;
    const double* b = pooled ? a.bp + (int64_t)c * nrhs * D : a.b + (int64_t)id * nrhs * D;
    const double inv_n = 1.0 / (double)nk;
    for (int i = tid; i < D * (D + 1) / 2; i += 256) {
        // invert tri(r, col): r = floor((sqrt(8i+1)-1)/2)
        int r = (int)((sqrt(8.0 * i + 1.0) - 1.0) * 0.5);
        while (tri(r + 1, 0) <= i) ++r;
        while (tri(r, 0) > i) --r;
        const int col = i - tri(r, 0);
        L[i] = G[(int64_t)r * D + col] * inv_n + (r == col ? a.lam : 0.0);
    }
    for (int i = tid; i < nrhs * D; i += 256) rhs[i] = b[i] * inv_n;
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < D; ++j) {
        if (tid == 0) {
            const double d = L[tri(j, j)];
            if (!(d > 0.0)) fail = 1;
            L[tri(j, j)] = sqrt(d > 0.0 ? d : 1.0);
        }
        __syncthreads();
        const double piv = L[tri(j, j)];
        for (int i = j + 1 + tid; i < D; i += 256) L[tri(i, j)] /= piv;
        __syncthreads();
        for (int i = j + 1 + wave; i < D; i += 4) {
            const double lij = L[tri(i, j)];
            for (int kk = j + 1 + lane; kk <= i; kk += 64) L[tri(i, kk)] -= lij * L[tri(kk, j)];
        }
        __syncthreads();
    }
    // forward (L y = rhs) and backward (L^T h = y) substitution; every thread runs every step
    for (int r = 0; r < nrhs; ++r) {
        double* v = rhs + r * D;
        for (int j = 0; j < D; ++j) {
            if (tid == 0) v[j] /= L[tri(j, j)];
            __syncthreads();
            const double vj = v[j];
            for (int i = j + 1 + tid; i < D; i += 256) v[i] -= L[tri(i, j)] * vj;
            __syncthreads();
        }
        for (int j = D - 1; j >= 0; --j) {
            if (tid == 0) v[j] /= L[tri(j, j)];
            __syncthreads();
            const double vj = v[j];
            for (int i = tid; i < j; i += 256) v[i] -= L[tri(j, i)] * vj;
            __syncthreads();
        }
    }
    __syncthreads();
    if (pooled) {
        for (int i = tid; i < nrhs * D; i += 256) a.hp[(int64_t)c * nrhs * D + i] = fail ? 0.0 : rhs[i];
        return;
    }
    if (tid == 0) a.ok[id] = fail ? 0 : 1;
    if (fail) return;
    for (int i = tid; i < nrhs * D; i += 256) {
        const int r = i / D, t = i - r * D;
        const int ch = a.per_channel ? c : r;
        const int C = a.per_channel ? a.sys_per_k : nrhs;
        const int64_t off = ((int64_t)k * C + ch) * D + t;
        if (a.out_dtype == MDN_F16)
            store_d(static_cast<__half*>(a.out) + off, rhs[i]);
        else
            static_cast<float*>(a.out)[off] = (float)rhs[i];
    }
}

__global__ void k_fill_fallback(SolveArgs a, int32_t* n_fallback) {
    const int id = blockIdx.x;
    if (a.ok[id]) return;
    const int c = id % a.sys_per_k, k = id / a.sys_per_k;
    const int D = a.D, nrhs = a.nrhs;
    for (int i = threadIdx.x; i < nrhs * D; i += blockDim.x) {
        const int r = i / D, t = i - r * D;
        const int ch = a.per_channel ? c : r;
        const int C = a.per_channel ? a.sys_per_k : nrhs;
        const int64_t off = ((int64_t)k * C + ch) * D + t;
        const double v = a.hp[(int64_t)c * nrhs * D + i];
        if (a.out_dtype == MDN_F16)
            store_d(static_cast<__half*>(a.out) + off, v);
        else
            static_cast<float*>(a.out)[off] = (float)v;
    }
    if (threadIdx.x == 0 && n_fallback) atomicAdd(n_fallback, 1);
}

__global__ void k_count_all(const int64_t* n, int K, int64_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t s = 0;
        for (int k = 0; k < K; ++k) s += n[k];
        *out = s;
    }
}

}  // namespace

// ------------------------------------------------------------------------ host side

int gram_dims(const mdn_gram& g, int* D, int* nrhs, int* sys_per_k) {
    const int tf = g.radius_f >= 1 ? (2 * g.radius_f + 1) * (2 * g.radius_f + 1) : 0;
    const int tg = (2 * g.radius_g + 1) * (2 * g.radius_g + 1);
    if (g.layout == MDN_X_PER_CHANNEL) {
        *D = tf + tg;
        *nrhs = 1;
        *sys_per_k = g.channels;
    } else {
        *D = g.channels * tg;
        *nrhs = g.channels;
        *sys_per_k = 1;
    }
    return 0;
}

mdn_status gram_zero(const mdn_gram& g, hipStream_t st) {
    int D, nrhs, spk;
    gram_dims(g, &D, &nrhs, &spk);
    const int64_t nsys = (int64_t)g.K * spk;
    k_fill_zero<<<512, 256, 0, st>>>(g.G, nsys * D * D);
    k_fill_zero<<<64, 256, 0, st>>>(g.b, nsys * nrhs * D);
    k_fill_zero<<<1, 256, 0, st>>>(g.yy, nsys * nrhs);
    k_fill_zero_i64<<<1, 256, 0, st>>>(g.n, g.K);
    return check_launch("gram_zero");
}

static size_t sort_tmp_bytes(int64_t n, bool wide) {
    size_t tmp = 0;
    if (wide)
        (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint16_t*)nullptr, (uint16_t*)nullptr,
                                                 (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0, 16);
    else
        (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint8_t*)nullptr, (uint8_t*)nullptr,
                                                 (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0, 8);
    return tmp;
}

static int gram_tiles(const mdn_gram& g) {
    int D, nrhs, spk;
    gram_dims(g, &D, &nrhs, &spk);
    const int T = (D + nrhs + 31) / 32;
    return T * (T + 1) / 2;
}

// elements of one padded gather plane of a w x h image
static size_t padded_plane(int w, int h) { return (size_t)(w + 2 * kPad) * (size_t)(h + 2 * kPad); }

size_t train_ws_bytes(const mdn_gram& g, int w, int h) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    int D, nrhs, spk;
    gram_dims(g, &D, &nrhs, &spk);
    const int C = g.channels;
    const int wc = (w + 1) / 2, hc = (h + 1) / 2;
    const size_t n = (size_t)w * h;
    const size_t part = (size_t)g.K * spk * gram_segments((int64_t)n, g.K) * gram_tiles(g) * 1024 * 4;
    return al(padded_plane(w, h) * C * 4) * 2 + al(padded_plane(wc, hc) * C * 4) + al(n * 2) * 2 + al(n * 4) * 2 +
           al(((size_t)g.K + 1) * 4) + al(sort_tmp_bytes((int64_t)n, g.K > 256)) + al(part);
}

// padded float32 gather planes of im (row pitch and plane pitch of the padded planes)
mdn_status launch_to_planes(const mdn_image& im, float* out, int64_t row, int64_t plane, hipStream_t st) {
    ImageArg a{im.data, im.row_pitch, im.plane_pitch, im.width, im.height};
    dim3 grid((im.width + 2 * kPad + 255) / 256, im.height + 2 * kPad);
    k_to_planes<<<grid, 256, 0, st>>>(a, im.dtype, im.color == MDN_RGB, im.channels, out, row, plane);
    return check_launch("to_planes");
}

mdn_status train_accumulate(const mdn_gram& g, const mdn_image& z, const mdn_image* uc, const mdn_image& target,
                            const mdn_level& sel, int precision, void* ws, hipStream_t st) {
    int D, nrhs, spk;
    gram_dims(g, &D, &nrhs, &spk);
    const int W = z.width, H = z.height, C = z.channels;
    const int Wc = (W + 1) / 2, Hc = (H + 1) / 2;
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const int Wp = W + 2 * kPad, Hp = H + 2 * kPad, Wcp = Wc + 2 * kPad, Hcp = Hc + 2 * kPad;
    char* p = static_cast<char*>(ws);
    float* fine = reinterpret_cast<float*>(p);
    p += al(padded_plane(W, H) * C * 4);
    float* tgt = reinterpret_cast<float*>(p);
    p += al(padded_plane(W, H) * C * 4);
    float* coarse = reinterpret_cast<float*>(p);
    p += al(padded_plane(Wc, Hc) * C * 4);
    // selector map and sorted keys: uint8, or uint16 when K > 256
    const bool wide = g.K > 256;
    void* smap = p;
    p += al((size_t)W * H * 2);
    void* skeys = p;
    p += al((size_t)W * H * 2);
    int32_t* idx_in = reinterpret_cast<int32_t*>(p);
    p += al((size_t)W * H * 4);
    int32_t* idx = reinterpret_cast<int32_t*>(p);
    p += al((size_t)W * H * 4);
    int32_t* off = reinterpret_cast<int32_t*>(p);
    p += al(((size_t)g.K + 1) * 4);
    void* sort_tmp = p;
    p += al(sort_tmp_bytes((int64_t)W * H, wide));
    float* part = reinterpret_cast<float*>(p);
    mdn_status s;
    if ((s = launch_to_planes(z, fine, Wp, (int64_t)Wp * Hp, st))) return s;
    if ((s = launch_to_planes(target, tgt, Wp, (int64_t)Wp * Hp, st))) return s;
    if (uc && (s = launch_to_planes(*uc, coarse, Wcp, (int64_t)Wcp * Hcp, st))) return s;
    if ((s = launch_select_apply(z, uc, nullptr, W, smap, sel, nullptr, st))) return s;
    const int64_t npx = (int64_t)W * H;
    k_iota<<<256, 256, 0, st>>>(idx_in, npx);
    if ((s = check_launch("iota"))) return s;
    size_t tmp = sort_tmp_bytes(npx, wide);
    const hipError_t se =
        wide ? hipcub::DeviceRadixSort::SortPairs(sort_tmp, tmp, static_cast<const uint16_t*>(smap), static_cast<uint16_t*>(skeys),
                                                  idx_in, idx, (int)npx, 0, 16, st)
             : hipcub::DeviceRadixSort::SortPairs(sort_tmp, tmp, static_cast<const uint8_t*>(smap), static_cast<uint8_t*>(skeys),
                                                  idx_in, idx, (int)npx, 0, 8, st);
    if (se != hipSuccess) return fail(MDN_EDEVICE, "gram: bucket sort failed");
    if (wide) k_bucket_bounds<<<(g.K + 1 + 255) / 256, 256, 0, st>>>(static_cast<const uint16_t*>(skeys), npx, g.K, off);
    else k_bucket_bounds<<<(g.K + 1 + 255) / 256, 256, 0, st>>>(static_cast<const uint8_t*>(skeys), npx, g.K, off);
    if ((s = check_launch("bucket_bounds"))) return s;

    GramArgs a;
    memset(&a, 0, sizeof(a));
    a.planes = fine;
    a.target_off = (int32_t)(tgt - fine);
    a.coarse_off = (int32_t)(coarse - fine);
    a.f_row = Wp;
    a.f_plane = Wp * Hp;
    a.c_row = Wcp;
    a.c_plane = Wcp * Hcp;
    a.W = W;
    a.H = H;
    a.Wc = Wc;
    a.Hc = Hc;
    a.idx = idx;
    a.off = off;
    a.D = D;
    a.nrhs = nrhs;
    a.per_channel = g.layout == MDN_X_PER_CHANNEL;
    // tap rows in feature order: x = [coarse taps, row-major; fine taps, row-major] and the
    // target(s) last
    int f = 0, nr = 0;
    auto add_row = [&](int src, int plane, int dy, int r) {
        a.rows[nr++] = row_pack(src, plane, dy, -r, 2 * r + 1, f);
        f += 2 * r + 1;
    };
    if (a.per_channel) {
        if (g.radius_f >= 1)
            for (int dy = -g.radius_f; dy <= g.radius_f; ++dy) add_row(1, 0, dy, g.radius_f);
        for (int dy = -g.radius_g; dy <= g.radius_g; ++dy) add_row(0, 0, dy, g.radius_g);
        add_row(2, 0, 0, 0);
    } else {
        for (int c = 0; c < C; ++c)
            for (int dy = -g.radius_g; dy <= g.radius_g; ++dy) add_row(0, c, dy, g.radius_g);
        for (int c = 0; c < C; ++c) add_row(2, c, 0, 0);
    }
    a.nrows = nr;
    a.Daug = f;
    a.nseg = gram_segments((int64_t)W * H, g.K);
    a.part = part;
    a.G = g.G;
    a.b = g.b;
    a.n = g.n;
    a.yy = g.yy;
    const int T = (f + 31) / 32;
    dim3 grid(g.K, spk, a.nseg);
    bool launched = false;
    const int rpw = (nr + 3) / 4 <= 4 ? 4 : 6;
#define MDN_GRAM(P_, T_, R_)                                                              \
    if (!launched && precision == P_ && T == T_ && rpw == R_) {                            \
        k_gram<P_, T_, R_><<<grid, 256, 0, st>>>(a);                                       \
        launched = true;                                                                   \
    }
    MDN_GRAM(0, 1, 4) MDN_GRAM(0, 2, 4) MDN_GRAM(0, 3, 4) MDN_GRAM(0, 4, 4) MDN_GRAM(0, 5, 4)
    MDN_GRAM(1, 1, 4) MDN_GRAM(1, 2, 4) MDN_GRAM(1, 3, 4) MDN_GRAM(1, 4, 4) MDN_GRAM(1, 5, 4)
    MDN_GRAM(0, 2, 6) MDN_GRAM(0, 3, 6) MDN_GRAM(0, 4, 6) MDN_GRAM(0, 5, 6)
    MDN_GRAM(1, 2, 6) MDN_GRAM(1, 3, 6) MDN_GRAM(1, 4, 6) MDN_GRAM(1, 5, 6)
#undef MDN_GRAM
    if (!launched) return fail(MDN_ENOTSUP, "gram: %d features not supported", f);
    if ((s = check_launch("gram"))) return s;
    k_gram_reduce<<<dim3(g.K, spk), 256, 0, st>>>(a, T);
    return check_launch("gram_reduce");
}

size_t solve_ws_bytes(const mdn_gram& g) {
    int D, nrhs, spk;
    gram_dims(g, &D, &nrhs, &spk);
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    return al((size_t)spk * D * D * 8) + al((size_t)spk * nrhs * D * 8) * 2 + al((size_t)g.K * spk * 4) + al(8);
}

mdn_status train_solve(const mdn_gram& g, double lam, int64_t min_count, void* coeffs, int out_dtype,
                       int32_t* n_fallback, void* ws, hipStream_t st) {
    int D, nrhs, spk;
    gram_dims(g, &D, &nrhs, &spk);
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    char* p = static_cast<char*>(ws);
    double* Gp = reinterpret_cast<double*>(p);
    p += al((size_t)spk * D * D * 8);
    double* bp = reinterpret_cast<double*>(p);
    p += al((size_t)spk * nrhs * D * 8);
    double* hp = reinterpret_cast<double*>(p);
    p += al((size_t)spk * nrhs * D * 8);
    int32_t* ok = reinterpret_cast<int32_t*>(p);
    p += al((size_t)g.K * spk * 4);
    int64_t* n_all_dev = reinterpret_cast<int64_t*>(p);
    k_pool<<<dim3(64, spk), 256, 0, st>>>(g.G, g.b, g.K, spk, D, nrhs, Gp, bp);
    k_count_all<<<1, 64, 0, st>>>(g.n, g.K, n_all_dev);
    mdn_status s;
    if ((s = check_launch("pool"))) return s;
    SolveArgs a;
    memset(&a, 0, sizeof(a));
    a.G = g.G;
    a.b = g.b;
    a.n = g.n;
    a.Gp = Gp;
    a.bp = bp;
    a.hp = hp;
    a.ok = ok;
    a.n_all = n_all_dev;
    a.K = g.K;
    a.sys_per_k = spk;
    a.D = D;
    a.nrhs = nrhs;
    a.lam = lam;
    a.min_count = min_count;
    a.out = coeffs;
    a.out_dtype = out_dtype;
    a.per_channel = g.layout == MDN_X_PER_CHANNEL;
    const size_t lds = ((size_t)D * (D + 1) / 2 + (size_t)nrhs * D) * 8;
    const int nblocks = g.K * spk + spk;
    if (lds > 65536 && hipFuncSetAttribute((const void*)k_solve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(MDN_EDEVICE, "solve: cannot reserve %zu bytes of LDS", lds);
    k_solve<<<nblocks, 256, lds, st>>>(a);
    if ((s = check_launch("solve"))) return s;
    k_fill_fallback<<<g.K * spk, 256, 0, st>>>(a, n_fallback);
    return check_launch("fill_fallback");
}

}  // namespace mdn
