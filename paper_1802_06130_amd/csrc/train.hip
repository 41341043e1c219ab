// Per-bucket least-squares filter training (Eq. (7)-(8)).
//
// For every bucket k the filters minimise the squared error over the pixels with s(i) = k,
// which is one linear regression per bucket (and per YCbCr channel, footnote of Section 3).
// The normal equations are accumulated here and solved with a ridge term.
//
// Grouping: the pixel indices of the level are grouped by bucket with a stable counting sort of
// the selector map (see the bucket grouping below), so every bucket's pixels form one contiguous
// run in raster order.
//
// Accumulation (k_gram): one workgroup per (work item, system). A bucket's run is cut into items
// of S 64-sample chunks (the last one shorter), so that every workgroup has about the same work
// however the samples fall into buckets; S is chosen for about two items per resident workgroup
// (fewer, longer items write fewer partial sums; more, shorter ones balance better). The items
// are numbered bucket by bucket and a workgroup finds its bucket by binary search.
// A workgroup gathers 64 samples at a time into LDS as a feature-major matrix X^T (regression
// taps followed by the target value(s), zero padded to a multiple of 32; the gathers of the next
// chunk are in flight while the current one is multiplied). The planes are float32 copies with a
// replicated margin of kPad pixels, so every tap row of a sample is consecutive floats of one
// plane row: a wave takes whole tap rows, one sample per lane, each row one contiguous load. The
// upper-triangle 32x32 tiles of X^T X accumulate on MFMA with FP32 accumulators; the target value
// rides along as an extra feature, so the same tiles yield G = sum x x^T, b = sum x y and
// yy = sum y^2. Two products are offered:
//   MDN_GRAM_F32    : v_mfma_f32_32x32x2_f32 - exact FP32 products, FP32 accumulation;
//   MDN_GRAM_BF16X3 : v_mfma_f32_32x32x16_bf16 on a hi/lo split x = hi + lo (hi = bf16(x),
//                     lo = bf16(x - hi)); x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y.
// Each workgroup writes its FP32 tiles to a partial buffer; k_gram_reduce then adds the items of
// each system in item order into the FP64 accumulators (fixed order: bitwise reproducible).
//
// Solve (k_solve): one workgroup per system, (G/n + lambda I) h = b/n by Cholesky in float64,
// the lower triangle packed in LDS. Buckets with fewer than min_count samples (or a failed
// factorisation) take the pooled solution of the level (sums over all buckets).

#include "mdn_internal.h"
#include "walk_types.h"

#include <string.h>

#include <type_traits>

namespace mdn {

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kChunk = 64;                 // samples per MFMA chunk
constexpr int kPad = 3;                    // replicated margin of the gather planes (radius <= 3)
constexpr int kMaxRows = 24;               // tap rows per sample: 3 planes x 7 rows + 3 targets
constexpr int kMinItemChunks = 2;          // chunks per work item: at least
constexpr int kMaxItemChunks = 32;         // and at most
constexpr int kReduceBatch = 16;           // partials a reducing thread has in flight
// LDS row stride (elements) of X^T: 16-byte aligned rows for the 16-byte operand reads (four
// float32 or eight bf16 samples per lane), at 4 mod 64 dwords (float32) or 36 (bf16) so that
// the lanes of one read, 32 consecutive rows, fall in distinct banks.
template <int PREC> struct Ldw { static constexpr int v = PREC == 0 ? kChunk + 4 : kChunk + 8; };

// Upper bound on the work items of npx samples in K buckets at S chunks per item: the runs have
// sum ceil(n_k / 64) <= npx / 64 + K chunks, and ceil(c / S) <= c / S + 1.
int64_t max_work_items(int64_t npx, int K, int S) { return (npx / kChunk + K) / S + K + 1; }

// Chunks per work item for npx samples and spk systems per bucket on ncu compute units: about
// two items per workgroup slot, four slots per CU.
int item_chunks(int64_t npx, int spk, int ncu) {
    const int64_t chunks = spk * ((npx + kChunk - 1) / kChunk);
    const int64_t s = (chunks + 8LL * ncu - 1) / (8LL * ncu);
    return (int)(s < kMinItemChunks ? kMinItemChunks : (s > kMaxItemChunks ? kMaxItemChunks : s));
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
    const int32_t* items;   // [K+1] first work item of each bucket; items[K] = number of items
    int32_t K, D, Daug, nrhs, per_channel;
    int32_t item_chunks;    // chunks per work item
    int32_t nrows;          // tap rows per sample
    int32_t rows[kMaxRows];
    float* part;            // [work item][system of the bucket][tiles][1024] partial tiles
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

// The upper-triangle 32x32 tiles (P, Q) of each of the four waves, chosen so that a wave's tiles
// share 32-feature panels: a wave reads each panel it needs from LDS once per k-step, for all of
// its tiles. Tile (P, Q) is number P T - P (P - 1) / 2 + Q - P in row-major order (tile_pq).
struct WaveTiles {
    int n;
    int p[4], q[4];
};
__host__ __device__ constexpr WaveTiles wave_tiles(int T, int w) {
    switch (T) {
    case 1: return w == 0 ? WaveTiles{1, {0}, {0}} : WaveTiles{0, {}, {}};
    case 2:
        return w == 0 ? WaveTiles{1, {0}, {0}} : w == 1 ? WaveTiles{1, {0}, {1}} : w == 2 ? WaveTiles{1, {1}, {1}}
                                                                                         : WaveTiles{0, {}, {}};
    case 3:
        return w == 0 ? WaveTiles{2, {0, 0}, {0, 1}} : w == 1 ? WaveTiles{2, {1, 1}, {1, 2}}
                                                     : w == 2 ? WaveTiles{1, {0}, {2}} : WaveTiles{1, {2}, {2}};
    case 4:
        return w == 0 ? WaveTiles{3, {0, 0, 0}, {0, 1, 2}} : w == 1 ? WaveTiles{3, {1, 1, 1}, {1, 2, 3}}
                                                           : w == 2 ? WaveTiles{3, {2, 2, 0}, {2, 3, 3}}
                                                                    : WaveTiles{1, {3}, {3}};
    default:
        return w == 0 ? WaveTiles{4, {0, 0, 0, 0}, {0, 1, 2, 3}} : w == 1 ? WaveTiles{4, {1, 1, 1, 1}, {1, 2, 3, 4}}
                                                                 : w == 2 ? WaveTiles{4, {2, 2, 2, 0}, {2, 3, 4, 4}}
                                                                          : WaveTiles{3, {3, 3, 4}, {3, 4, 4}};
    }
}
__host__ __device__ constexpr int tile_number(int T, int P, int Q) { return P * T - P * (P - 1) / 2 + Q - P; }
__host__ __device__ constexpr unsigned wave_panels(int T, int w) {
    unsigned m = 0;
    for (int i = 0; i < wave_tiles(T, w).n; ++i) m |= (1u << wave_tiles(T, w).p[i]) | (1u << wave_tiles(T, w).q[i]);
    return m;
}
__host__ __device__ constexpr int most_wave_tiles(int T) {
    int m = 0;
    for (int w = 0; w < 4; ++w) m = wave_tiles(T, w).n > m ? wave_tiles(T, w).n : m;
    return m;
}
// every tile is owned by exactly one wave
__host__ __device__ constexpr bool wave_tiles_cover(int T) {
    int seen[15] = {};
    for (int w = 0; w < 4; ++w)
        for (int i = 0; i < wave_tiles(T, w).n; ++i) {
            const int P = wave_tiles(T, w).p[i], Q = wave_tiles(T, w).q[i];
            if (P > Q || Q >= T) return false;
            ++seen[tile_number(T, P, Q)];
        }
    for (int t = 0; t < T * (T + 1) / 2; ++t)
        if (seen[t] != 1) return false;
    return true;
}
static_assert(wave_tiles_cover(1) && wave_tiles_cover(2) && wave_tiles_cover(3) && wave_tiles_cover(4) &&
              wave_tiles_cover(5), "wave tile lists");

// Sum the partials of tile t of one system over the bucket's work items [i0, i1), in item order
// (float64), and add them to the accumulators (256 threads); the result does not depend on timing.
// An off-diagonal tile also goes, transposed through LDS, to the lower triangle, so that both
// halves of G are written along its rows.
// Columns of tile (P, Q) that hold features: 32, or fewer in the last column panel (the augmented
// features end at Daug). A tile with nq < 32 columns is stored compactly in its 1024-float slot:
// entry r of lane l (l mod 32 < nq) at r 2nq + (l / 32) nq + l mod 32, 32 nq floats in all.
__host__ __device__ inline int tile_cols(int T, int Q, int daug) { return Q == T - 1 ? daug - 32 * Q : 32; }

__device__ void add_partials(const GramArgs& a, int T, int t, int k, int sys_c, int sys, int i0, int i1, int spk) {
    __shared__ double tr[32][33];
    const int NT = T * (T + 1) / 2;
    if (t == 0 && sys_c == 0 && threadIdx.x == 0) a.n[k] += a.off[k + 1] - a.off[k];
    const int D = a.D;
    double* G = a.G + (int64_t)sys * D * D;
    double* bvec = a.b + (int64_t)sys * a.nrhs * D;
    double* yy = a.yy + (int64_t)sys * a.nrhs;
    int P, Q;
    tile_pq(T, t, &P, &Q);
    const int nq = tile_cols(T, Q, a.Daug);
    for (int e = threadIdx.x; e < 32 * nq; e += 256) {
        // kReduceBatch items' partials are loaded at once (past the last item, the last one is
        // re-read), then summed in item order
        double v = 0.0;
        for (int ib = i0; ib < i1; ib += kReduceBatch) {
            float pv[kReduceBatch];
#pragma unroll
            for (int j = 0; j < kReduceBatch; ++j) {
                const int it = min(ib + j, i1 - 1);
                pv[j] = a.part[(((int64_t)it * spk + sys_c) * NT + t) * 1024 + e];
            }
#pragma unroll
            for (int j = 0; j < kReduceBatch; ++j)
                if (ib + j < i1) v += (double)pv[j];
        }
        // accumulator layout of a 32x32 MFMA tile: entry r of lane (stored compactly when nq < 32)
        const int r = e / (2 * nq), kq = e - r * 2 * nq, half = kq >= nq ? 1 : 0, ql = kq - half * nq;
        const int pl = 8 * (r >> 2) + 4 * half + (r & 3);
        const int p = P * 32 + pl, q = Q * 32 + ql;
        tr[ql][pl] = v;
        if (p >= a.Daug || q >= a.Daug) continue;
        if (p < D && q < D) {
            G[(int64_t)p * D + q] += v;
        } else if (p < D && q >= D) {
            bvec[(int64_t)(q - D) * D + p] += v;
        } else if (p >= D && q >= D && p == q) {
            yy[p - D] += v;
        }
    }
    if (P != Q && Q * 32 < D) {
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * nq; e += 256) {
            const int ql = e >> 5, pl = e & 31;
            const int p = P * 32 + pl, q = Q * 32 + ql;
            if (p < D && q < D) G[(int64_t)q * D + p] += tr[ql][pl];
        }
    }
}

// RPW: tap rows per wave (the sample's rows are dealt to the four waves), at least ceil(nrows / 4).
template <int PREC, int T, int RPW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_gram(GramArgs a) {
    constexpr int DPAD = 32 * T;
    constexpr int NT = T * (T + 1) / 2;
    constexpr int TPW = most_wave_tiles(T);
    constexpr int LDW = Ldw<PREC>::v;
    using XT = typename std::conditional<PREC == 0, float, __bf16>::type;
    __shared__ XT xhi[DPAD][LDW];
    __shared__ XT xlo[PREC == 0 ? 1 : DPAD][PREC == 0 ? 1 : LDW];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: row decoding is scalar
    const int item = blockIdx.x;
    const int sys_c = blockIdx.y;                      // channel (per-channel systems) or 0
    const int plane_off = a.per_channel ? sys_c : 0;
    const int W = a.W;
    if (item >= a.items[a.K]) return;                  // the grid is sized for the most items
    // bucket of this item: items[k] <= item < items[k + 1] (empty buckets have no items)
    int lo = 0, hi = a.K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (__builtin_amdgcn_readfirstlane(a.items[mid]) <= item) lo = mid;
        else hi = mid - 1;
    }
    const int k = lo;

    // this item's chunks of the bucket's run
    const int beg = a.off[k], end = a.off[k + 1];
    const int chunks = (end - beg + kChunk - 1) / kChunk;
    const int S = a.item_chunks;
    const int c0 = (item - a.items[k]) * S, c1 = min(chunks, c0 + S);

    const float* planes = a.planes;
    const int nrows = __builtin_amdgcn_readfirstlane(a.nrows);
    const int daug = __builtin_amdgcn_readfirstlane(a.Daug);
    // feature rows past the last feature stay zero
    for (int e = tid; e < (DPAD - daug) * LDW; e += 256) {
        const int f = daug + e / LDW, col = e - (e / LDW) * LDW;
        xhi[f][col] = XT(0.0f);
        if constexpr (PREC != 0) xlo[f][col] = XT(0.0f);
    }

    // Gather: wave w takes tap rows w, w + 4, ... of every sample, one sample per lane; a row's
    // taps are consecutive floats of a padded plane row, loaded together. The next chunk's loads
    // are in flight while the current chunk is multiplied from LDS, and are consumed only when
    // that chunk is stored to LDS; the sample indices are read one chunk further ahead, so those
    // loads wait on no index load. (Loading each 5- or 7-tap row with two lanes, one 16-byte load
    // each, so that a load instruction touches half as many rows, measured slower.)
    struct Buf {
        float v[RPW][8];
        bool live;
    };
    Buf buf;
    // sample index of this lane in chunk `chunk` (-1 past the run's end)
    auto load_idx = [&](int chunk) __attribute__((always_inline)) {
        const int i = beg + chunk * kChunk + lane;
        return i < end ? a.idx[i] : -1;
    };
    auto load = [&](int pix, Buf& b) __attribute__((always_inline)) {
        b.live = pix >= 0;
        pix = max(pix, 0);
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
    auto store = [&](const Buf& b) __attribute__((always_inline)) {
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
    // The products of one chunk for the tiles of wave W: per k-step every panel the wave needs is
    // read once (float32: four samples per lane, used by four MFMAs; bf16: eight samples, hi and
    // lo) and every tile takes its MFMAs from those registers.
    auto multiply_wave = [&](auto wc, f16v (&acc)[TPW]) __attribute__((always_inline)) {
        constexpr int Wv = decltype(wc)::value;
        constexpr WaveTiles L = wave_tiles(T, Wv);
        constexpr unsigned need = wave_panels(T, Wv);
        const int row = lane & 31;
        if constexpr (PREC == 0) {
#pragma unroll 1
            for (int kq = 0; kq < kChunk / 8; ++kq) {
                const int col = 8 * kq + 4 * (lane >> 5);
                float4 x[T];
#pragma unroll
                for (int pn = 0; pn < T; ++pn)
                    if (need & (1u << pn)) x[pn] = *reinterpret_cast<const float4*>(&xhi[pn * 32 + row][col]);
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int i = 0; i < L.n; ++i)
                        acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[L.p[i]][m], x[L.q[i]][m], acc[i], 0, 0, 0);
            }
        } else {
            constexpr int U = T <= 4 ? 2 : 1;      // two k-steps of operands in flight where registers allow
#pragma unroll U
            for (int ks = 0; ks < kChunk / 16; ++ks) {
                const int col = 16 * ks + 8 * (lane >> 5);
                bf8v h[T], l[T];
#pragma unroll
                for (int pn = 0; pn < T; ++pn)
                    if (need & (1u << pn)) {
                        h[pn] = *reinterpret_cast<const bf8v*>(&xhi[pn * 32 + row][col]);
                        l[pn] = *reinterpret_cast<const bf8v*>(&xlo[pn * 32 + row][col]);
                    }
#pragma unroll
                for (int i = 0; i < L.n; ++i) {
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h[L.p[i]], h[L.q[i]], acc[i], 0, 0, 0);
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h[L.p[i]], l[L.q[i]], acc[i], 0, 0, 0);
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l[L.p[i]], h[L.q[i]], acc[i], 0, 0, 0);
                }
            }
        }
    };
    // partial tiles of this item and system: [item][system][tile][r][lane]
    float* part = a.part + ((int64_t)item * gridDim.y + sys_c) * NT * 1024;

    // the chunk loop, instantiated per wave so that each wave's accumulators are its own registers
    auto run = [&](auto wc) __attribute__((always_inline)) {
        constexpr WaveTiles L = wave_tiles(T, decltype(wc)::value);
        f16v acc[TPW];
#pragma unroll
        for (int i = 0; i < TPW; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][r] = 0.0f;
        load(load_idx(c0), buf);
        int pix = c0 + 1 < c1 ? load_idx(c0 + 1) : -1;
        store(buf);
        __syncthreads();
        for (int c = c0; c < c1; ++c) {
            const bool more = c + 1 < c1;
            if (more) {
                load(pix, buf);          // in flight during the products
                pix = c + 2 < c1 ? load_idx(c + 2) : -1;
            }
            multiply_wave(wc, acc);
            __syncthreads();             // every wave is done with this chunk
            if (more) {
                store(buf);
                __syncthreads();
            }
        }
#pragma unroll
        for (int i = 0; i < L.n; ++i) {
            const int t = tile_number(T, L.p[i], L.q[i]);
            const int nq = tile_cols(T, L.q[i], daug);
            if (nq == 32) {
#pragma unroll
                for (int r = 0; r < 16; ++r) part[t * 1024 + r * 64 + lane] = acc[i][r];
            } else if ((lane & 31) < nq) {
                // last column panel: only its feature columns, compactly
                const int o = t * 1024 + (lane >> 5) * nq + (lane & 31);
#pragma unroll
                for (int r = 0; r < 16; ++r) part[o + r * 2 * nq] = acc[i][r];
            }
        }
    };
    switch (wave) {
    case 0: run(std::integral_constant<int, 0>()); break;
    case 1: run(std::integral_constant<int, 1>()); break;
    case 2: run(std::integral_constant<int, 2>()); break;
    default: run(std::integral_constant<int, 3>()); break;
    }
}

// Sum the partials of each system in item order (float64) and add them to the accumulators, one
// workgroup per (bucket, system, tile); the result does not depend on timing. (Letting the last
// item of each system do this inside k_gram was measured 2.4x slower: every workgroup's
// device-scope release and acquire wrote back and invalidated its XCD's L2, which the sample
// gathers depend on.)
__global__ __launch_bounds__(256) void k_gram_reduce(GramArgs a, int T) {
    const int k = blockIdx.x, sys_c = blockIdx.y, t = blockIdx.z;
    const int sys = a.per_channel ? k * (int)gridDim.y + sys_c : k;
    const int i0 = a.items[k], i1 = a.items[k + 1];
    if (i0 == i1) return;                                             // empty bucket: nothing to add
    add_partials(a, T, t, k, sys_c, sys, i0, i1, gridDim.y);
}

// First work item of every bucket (exclusive scan of the item counts, one workgroup).
__global__ __launch_bounds__(1024) void k_work_items(const int32_t* off, int K, int S, int32_t* items) {
    __shared__ int32_t w[1024];
    const int t = threadIdx.x;
    const int per = (K + 1023) / 1024;
    const int k0 = t * per, k1 = min(K, k0 + per);
    int32_t s = 0;
    for (int k = k0; k < k1; ++k) {
        const int chunks = (off[k + 1] - off[k] + kChunk - 1) / kChunk;
        s += (chunks + S - 1) / S;
    }
    w[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t y = t >= o ? w[t - o] : 0;
        __syncthreads();
        w[t] += y;
        __syncthreads();
    }
    int32_t run = w[t] - s;
    for (int k = k0; k < k1; ++k) {
        items[k] = run;
        const int chunks = (off[k + 1] - off[k] + kChunk - 1) / kChunk;
        run += (chunks + S - 1) / S;
    }
    if (t == 1023) items[K] = w[1023];
}

// float32 YCbCr (or grey) planes of an RGB / grey image for the sample gathers, with a margin of
// kPad pixels on every side holding the clamped (replicated) border: padded element (y, x),
// -kPad <= y < h + kPad and -kPad <= x < w + kPad, is at out[(y + kPad) o_row + x + kPad].
struct PlaneJob {
    ImageArg in;
    int32_t dtype, rgb_to_ycc, C;
    float* out;
    int64_t o_row, o_plane;
};
struct PlaneJobs {
    PlaneJob job[3];
};

// blockIdx.z picks the image: z^l, u^l and (when given) u^{l+1} in one launch
__global__ void k_to_planes(PlaneJobs jobs) {
    const PlaneJob& j = jobs.job[blockIdx.z];
    const ImageArg& in = j.in;
    const int xp = blockIdx.x * blockDim.x + threadIdx.x;
    const int yp = blockIdx.y;
    if (xp >= in.w + 2 * kPad || yp >= in.h + 2 * kPad) return;
    const int x = clampi(xp - kPad, 0, in.w - 1), y = clampi(yp - kPad, 0, in.h - 1);
    const int64_t off = (int64_t)y * in.row + x;
    float v[3] = {0, 0, 0};
    for (int c = 0; c < j.C; ++c) {
        v[c] = j.dtype == MDN_F16 ? __half2float(static_cast<const __half*>(in.data)[off + c * in.plane])
                                  : static_cast<const float*>(in.data)[off + c * in.plane];
    }
    if (j.C == 3 && j.rgb_to_ycc) Ycc::from_rgb(v[0], v[1], v[2], v[0], v[1], v[2]);
    for (int c = 0; c < j.C; ++c) j.out[c * j.o_plane + (int64_t)yp * j.o_row + xp] = v[c];
}

// ---------------------------------------------------------------- bucket grouping
// A stable counting sort of the level's pixels by bucket. The pixels are split into B slices of P
// consecutive pixels (raster order), one wave per slice:
//  1. each slice counts its keys into cnt[k * B + b];
//  2. cnt is scanned (exclusive) in this bucket-major order, in blocks of kScanChunk entries whose
//     totals are scanned again where they are used, so every (bucket, slice) gets its first
//     position: each bucket's pixels form one run and, within it, the slices come in raster order;
//  3. each slice walks its pixels in order, 64 at a time: the lanes holding the same key find one
//     another with one ballot per key bit and take ranks in lane order, and the group's first lane
//     advances the slice's running position for that key; every lane writes its pixel index there.
// The result is the order a stable sort by key gives; off[k] is the first position of bucket k.

constexpr int kScanChunk = 1024;           // entries per block of the scan (at most 1024 blocks)
constexpr int kGroupBatch = 16;            // 64-pixel chunks whose keys a slice loads at once
constexpr int kGroupLdsK = 8192;           // largest K whose running positions stay in LDS

// Lanes (of the valid ones) whose key equals this lane's: one ballot per key bit.
__device__ __forceinline__ uint64_t same_key_lanes(int key, bool valid, int bits) {
    uint64_t m = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
        const bool bit = (key >> b) & 1;
        const uint64_t on = __ballot(bit);
        m &= bit ? on : ~on;
    }
    return m;
}

// keys of kGroupBatch chunks from pixel q0 on (-1 past the slice's end p1), all loads in flight
__device__ __forceinline__ void load_keys(const void* keys, int wide, int64_t q0, int64_t p1, int lane,
                                          int (&kb)[kGroupBatch]) {
#pragma unroll
    for (int j = 0; j < kGroupBatch; ++j) {
        const int64_t q = q0 + 64 * j + lane;
        kb[j] = q >= p1 ? -1
                        : (wide ? (int)static_cast<const uint16_t*>(keys)[q] : (int)static_cast<const uint8_t*>(keys)[q]);
    }
}

// Step 1: counts of slice blockIdx.x (one wave); LDS counters when K is small enough, else global
// atomics on a zeroed cnt.
template <bool LDS>
__global__ __launch_bounds__(64) void k_group_count(const void* keys, int wide, int64_t n, int K, int B, int P, int bits,
                                                    int32_t* cnt) {
    extern __shared__ int32_t h[];
    const int lane = threadIdx.x, b = blockIdx.x;
    if constexpr (LDS) {
        for (int k = lane; k < K; k += 64) h[k] = 0;
        __syncthreads();
    }
    const int64_t p0 = (int64_t)b * P, p1 = min(n, p0 + P);
    for (int64_t q0 = p0; q0 < p1; q0 += 64 * kGroupBatch) {
        int kb[kGroupBatch];
        load_keys(keys, wide, q0, p1, lane, kb);
#pragma unroll
        for (int j = 0; j < kGroupBatch; ++j) {
            if (q0 + 64 * j >= p1) break;                              // uniform
            const bool valid = kb[j] >= 0;
            const uint64_t m = same_key_lanes(kb[j], valid, bits);
            if (valid && (__ffsll((unsigned long long)m) - 1) == lane) {
                if constexpr (LDS) atomicAdd(&h[kb[j]], __popcll(m));
                else atomicAdd(&cnt[(int64_t)kb[j] * B + b], __popcll(m));
            }
        }
    }
    if constexpr (LDS) {
        __syncthreads();
        for (int k = lane; k < K; k += 64) cnt[(int64_t)k * B + b] = h[k];
    }
}

// Step 2: exclusive scan of cnt (M entries) within each block of kScanChunk; sums[block] = total.
__global__ __launch_bounds__(256) void k_scan_local(int32_t* v, int64_t M, int32_t* sums) {
    __shared__ int32_t w[256];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + 4 * t;
    int32_t x[4], s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        x[j] = base + j < M ? v[base + j] : 0;
        s += x[j];
    }
    w[t] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int32_t y = t >= o ? w[t - o] : 0;
        __syncthreads();
        w[t] += y;
        __syncthreads();
    }
    int32_t run = w[t] - s;                    // exclusive prefix of this thread's four
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < M) v[base + j] = run;
        run += x[j];
    }
    if (t == 255) sums[blockIdx.x] = w[255];
}

// Step 3: the stable scatter of slice blockIdx.x (one wave). The wave first scans the block totals
// (nb <= 1024) into LDS, so the start of entry e of cnt is cnt[e] + ss[e / kScanChunk]; slice 0
// also writes off.
template <bool LDS>
__global__ __launch_bounds__(64) void k_group_scatter(const void* keys, int wide, int64_t n, int K, int B, int P,
                                                      int bits, int32_t* cnt, const int32_t* sums, int nb,
                                                      int32_t* idx, int32_t* off) {
    extern __shared__ int32_t sh[];
    int32_t* ss = sh;                          // [kScanChunk] scanned block totals
    int32_t* pos = sh + kScanChunk;            // [K] running positions (LDS form)
    const int lane = threadIdx.x, b = blockIdx.x;
    {
        constexpr int per = kScanChunk / 64;
        int32_t x[per], t = 0;
#pragma unroll
        for (int j = 0; j < per; ++j) {
            const int i = lane * per + j;
            x[j] = i < nb ? sums[i] : 0;
            t += x[j];
        }
        int32_t incl = t;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        int32_t run = incl - t;
#pragma unroll
        for (int j = 0; j < per; ++j) {
            ss[lane * per + j] = run;
            run += x[j];
        }
    }
    __syncthreads();
    if constexpr (LDS) {
        for (int k = lane; k < K; k += 64) {
            const int64_t e = (int64_t)k * B + b;
            pos[k] = cnt[e] + ss[e / kScanChunk];
        }
    }
    if (b == 0) {
        for (int k = lane; k < K; k += 64) {
            const int64_t e = (int64_t)k * B;
            off[k] = cnt[e] + ss[e / kScanChunk];
        }
        if (lane == 0) off[K] = (int32_t)n;
    }
    __syncthreads();
    const int64_t p0 = (int64_t)b * P, p1 = min(n, p0 + P);
    const uint64_t below = (1ull << lane) - 1;                 // lanes before this one
    for (int64_t q0 = p0; q0 < p1; q0 += 64 * kGroupBatch) {
        int kb[kGroupBatch];
        load_keys(keys, wide, q0, p1, lane, kb);
#pragma unroll
        for (int j = 0; j < kGroupBatch; ++j) {
            if (q0 + 64 * j >= p1) break;                              // uniform
            const bool valid = kb[j] >= 0;
            const uint64_t m = same_key_lanes(kb[j], valid, bits);
            const int first = __ffsll((unsigned long long)m) - 1;
            int start = 0;
            if (valid && first == lane) {
                if constexpr (LDS) {
                    start = pos[kb[j]];
                    pos[kb[j]] = start + __popcll(m);
                } else {
                    const int64_t e = (int64_t)kb[j] * B + b;
                    start = atomicAdd(&cnt[e], __popcll(m)) + ss[e / kScanChunk];
                }
            }
            // every lane takes its group's start from the group's first lane
            start = __builtin_amdgcn_ds_bpermute((valid ? first : lane) << 2, start);
            if (valid) idx[start + __popcll(m & below)] = (int32_t)(q0 + 64 * j + lane);
        }
    }
}

__global__ void k_fill_zero(double* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_fill_zero_i32(int32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
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

// Slices of the bucket grouping: P pixels each (a power of two, at least 256), enough pixels per
// slice that the K x B counts stay within 2^20 entries (1024 scan blocks).
static void group_shape(int64_t n, int K, int* B, int* P) {
    int64_t p = 256;
    while ((int64_t)K * ((n + p - 1) / p) > (1 << 20)) p *= 2;
    *P = (int)p;
    *B = (int)((n + p - 1) / p);
}

static size_t group_ws_bytes(int64_t n, int K) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    int B, P;
    group_shape(n, K, &B, &P);
    const int64_t M = (int64_t)K * B;
    return al((size_t)M * 4) + al((size_t)((M + kScanChunk - 1) / kScanChunk) * 4);
}

// idx = the pixel indices of the selector map grouped by bucket (stable), off[k] = bucket k's start.
static mdn_status group_by_bucket(const void* smap, bool wide, int64_t n, int K, void* ws, int32_t* idx, int32_t* off,
                                  hipStream_t st) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    int B, P;
    group_shape(n, K, &B, &P);
    const int64_t M = (int64_t)K * B;
    const int nb = (int)((M + kScanChunk - 1) / kScanChunk);
    if (nb > kScanChunk) return fail(MDN_ENOTSUP, "gram: %d buckets over %lld pixels exceed the grouping's scan", K, (long long)n);
    int bits = 1;
    while ((1 << bits) < K) ++bits;
    int32_t* cnt = static_cast<int32_t*>(ws);
    int32_t* sums = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + al((size_t)M * 4));
    const bool lds = K <= kGroupLdsK;
    if (lds) {
        k_group_count<true><<<B, 64, (size_t)K * 4, st>>>(smap, wide, n, K, B, P, bits, cnt);
    } else {
        k_fill_zero_i32<<<256, 256, 0, st>>>(cnt, M);
        k_group_count<false><<<B, 64, 0, st>>>(smap, wide, n, K, B, P, bits, cnt);
    }
    k_scan_local<<<nb, 256, 0, st>>>(cnt, M, sums);
    if (lds)
        k_group_scatter<true><<<B, 64, (size_t)(kScanChunk + K) * 4, st>>>(smap, wide, n, K, B, P, bits, cnt, sums, nb,
                                                                            idx, off);
    else
        k_group_scatter<false><<<B, 64, (size_t)kScanChunk * 4, st>>>(smap, wide, n, K, B, P, bits, cnt, sums, nb, idx,
                                                                       off);
    return check_launch("bucket grouping");
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
    const size_t part = (size_t)max_work_items((int64_t)n, g.K, kMinItemChunks) * spk * gram_tiles(g) * 1024 * 4;
    return al(padded_plane(w, h) * C * 4) * 2 + al(padded_plane(wc, hc) * C * 4) + al(n * 2) + al(n * 4) +
           al(((size_t)g.K + 1) * 4) * 2 + al(group_ws_bytes((int64_t)n, g.K)) + al(part);
}

// padded float32 gather planes of im (row pitch and plane pitch of the padded planes)
// padded float32 gather planes of up to three images in one launch (row and plane pitches of the
// padded planes per image)
static mdn_status launch_to_planes(const mdn_image* const* ims, float* const* outs, const int64_t* rows, const int64_t* planes,
                            int n, hipStream_t st) {
    PlaneJobs jobs;
    memset(&jobs, 0, sizeof(jobs));
    int wmax = 0, hmax = 0;
    for (int i = 0; i < n; ++i) {
        const mdn_image& im = *ims[i];
        jobs.job[i] = PlaneJob{ImageArg{im.data, im.row_pitch, im.plane_pitch, im.width, im.height}, im.dtype,
                               im.color == MDN_RGB, im.channels, outs[i], rows[i], planes[i]};
        wmax = im.width > wmax ? im.width : wmax;
        hmax = im.height > hmax ? im.height : hmax;
    }
    dim3 grid((wmax + 2 * kPad + 255) / 256, hmax + 2 * kPad, n);
    k_to_planes<<<grid, 256, 0, st>>>(jobs);
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
    // selector map: uint8, or uint16 when K > 256
    const bool wide = g.K > 256;
    void* smap = p;
    p += al((size_t)W * H * 2);
    int32_t* idx = reinterpret_cast<int32_t*>(p);
    p += al((size_t)W * H * 4);
    int32_t* off = reinterpret_cast<int32_t*>(p);
    p += al(((size_t)g.K + 1) * 4);
    int32_t* items = reinterpret_cast<int32_t*>(p);
    p += al(((size_t)g.K + 1) * 4);
    void* gws = p;
    p += al(group_ws_bytes((int64_t)W * H, g.K));
    float* part = reinterpret_cast<float*>(p);
    mdn_status s;
    {
        const mdn_image* ims[3] = {&z, &target, uc};
        float* outs[3] = {fine, tgt, coarse};
        const int64_t rows[3] = {Wp, Wp, Wcp};
        const int64_t planes[3] = {(int64_t)Wp * Hp, (int64_t)Wp * Hp, (int64_t)Wcp * Hcp};
        if ((s = launch_to_planes(ims, outs, rows, planes, uc ? 3 : 2, st))) return s;
    }
    if ((s = launch_select_apply(z, uc, nullptr, W, smap, sel, nullptr, st))) return s;
    const int64_t npx = (int64_t)W * H;
    if ((s = group_by_bucket(smap, wide, npx, g.K, gws, idx, off, st))) return s;
    const int S = item_chunks(npx, spk, device_cus());
    k_work_items<<<1, 1024, 0, st>>>(off, g.K, S, items);

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
    a.items = items;
    a.K = g.K;
    a.item_chunks = S;
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
    a.part = part;
    a.G = g.G;
    a.b = g.b;
    a.n = g.n;
    a.yy = g.yy;
    const int T = (f + 31) / 32;
    const int64_t max_items = max_work_items(npx, g.K, S);
    if (max_items > 0x7fffffffLL) return fail(MDN_ENOTSUP, "gram: too many work items");
    dim3 grid((unsigned)max_items, spk);
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
    k_gram_reduce<<<dim3(g.K, spk, T * (T + 1) / 2), 256, 0, st>>>(a, T);
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
