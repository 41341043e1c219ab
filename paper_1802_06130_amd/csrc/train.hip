// Per-bucket least-squares filter training (Eq. (7)-(8)).
//
// For every bucket k the filters minimise the squared error over the pixels with s(i) = k,
// which is one linear regression per bucket (and per YCbCr channel, footnote of Section 3).
// The normal equations are accumulated here and solved with a ridge term.
//
// Accumulation (k_gram): one workgroup per (bucket, system). It walks the selector map in
// raster order, compacts the matching pixel indices with a block-wide scan (a fixed order, so
// the sums are bitwise reproducible), gathers 64 samples at a time into LDS as a feature-major
// matrix X^T (regression taps followed by the target value(s), zero padded to a multiple of 32),
// and accumulates the upper-triangle 32x32 tiles of X^T X on MFMA with FP32 accumulators. The
// target value rides along as an extra feature, so the same tiles yield G = sum x x^T,
// b = sum x y and yy = sum y^2. Two products are offered:
//   MDN_GRAM_F32    : v_mfma_f32_32x32x2_f32 - exact FP32 products, FP32 accumulation;
//   MDN_GRAM_BF16X3 : v_mfma_f32_32x32x16_bf16 on a hi/lo split x = hi + lo (hi = bf16(x),
//                     lo = bf16(x - hi)); x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y.
// Each workgroup adds its FP32 tiles once into the FP64 accumulators of its system.
//
// Solve (k_solve): one workgroup per system, (G/n + lambda I) h = b/n by Cholesky in float64,
// the lower triangle packed in LDS. Buckets with fewer than min_count samples (or a failed
// factorisation) take the pooled solution of the level (sums over all buckets).

#include "mdn_internal.h"

#include <string.h>

#include <type_traits>

namespace mdn {

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kChunk = 64;                 // samples per MFMA chunk
constexpr int kLdw = kChunk + 8;           // LDS row stride (elements) of X^T
constexpr int kScan = 1024;                // pixels examined per scan step (4 per thread)
constexpr int kListCap = kChunk + kScan;   // pending sample list capacity

// feature descriptor: source (0 fine, 1 coarse, 2 target), plane, dy, dx
__host__ __device__ inline int feat_pack(int src, int plane, int dy, int dx) {
    return (src << 24) | (plane << 16) | ((dy + 128) << 8) | (dx + 128);
}

struct GramArgs {
    const float* fine;      // YCbCr (or grey) planes of z^l, float32
    const float* coarse;    // planes of the coarser output u^{l+1}, float32 (may be null)
    const float* target;    // planes of the clean level u^l, float32
    int64_t f_row, f_plane, c_row, c_plane;
    int32_t W, H, Wc, Hc;
    const uint8_t* s;
    int64_t s_pitch;
    int32_t D, Daug, nrhs, per_channel;
    int32_t feat[kMaxFeat];
    double* G;
    double* b;
    int64_t* n;
    double* yy;
};

// float -> bfloat16, round to nearest even (inputs are finite).
__device__ __forceinline__ __bf16 to_bf16(float v) {
    const uint32_t u = __float_as_uint(v);
    const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    return __builtin_bit_cast(__bf16, (unsigned short)r);
}

__device__ __forceinline__ float from_bf16(__bf16 h) {
    return __uint_as_float((uint32_t)__builtin_bit_cast(unsigned short, h) << 16);
}

// Block-wide exclusive scan of one int per thread (256 threads). Returns the prefix; *total
// receives the block sum. Contains barriers: call from uniform control flow.
__device__ int block_scan(int v, int* buf, int* total) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = t >= off ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    const int incl = buf[t];
    *total = buf[255];
    __syncthreads();
    return incl - v;
}

template <int PREC, int T>
__global__ __launch_bounds__(256) void k_gram(GramArgs a) {
    constexpr int DPAD = 32 * T;
    constexpr int NT = T * (T + 1) / 2;
    constexpr int TPW = (NT + 3) / 4;
    using XT = typename std::conditional<PREC == 0, float, __bf16>::type;
    __shared__ XT xhi[DPAD][kLdw];
    __shared__ XT xlo[PREC == 0 ? 1 : DPAD][PREC == 0 ? 1 : kLdw];
    __shared__ int plist[kListCap];
    __shared__ int sbuf[256];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k = blockIdx.x;
    const int sys_c = blockIdx.y;                      // channel (per-channel systems) or 0
    const int plane_off = a.per_channel ? sys_c : 0;
    const int W = a.W, H = a.H;
    const int64_t N = (int64_t)W * H;

    // tiles owned by this wave
    int tP[TPW], tQ[TPW];
    {
        int t = 0;
        for (int P = 0; P < T; ++P)
            for (int Q = P; Q < T; ++Q) {
                if (t % 4 == wave && t / 4 < TPW) {
                    tP[t / 4] = P;
                    tQ[t / 4] = Q;
                }
                ++t;
            }
    }
    const int my_tiles = (NT - wave + 3) / 4;
    f16v acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][r] = 0.0f;

    auto process = [&](int count) {
        // gather X^T for `count` samples (the rest of the chunk is zero)
        for (int i = tid; i < DPAD * kChunk; i += 256) {
            const int f = i / kChunk, p = i - f * kChunk;
            float v = 0.0f;
            if (p < count && f < a.Daug) {
                const int pix = plist[p];
                const int y = pix / W, x = pix - y * W;
                const int e = a.feat[f];
                const int src = e >> 24, pl = ((e >> 16) & 0xff) + plane_off;
                const int dy = ((e >> 8) & 0xff) - 128, dx = (e & 0xff) - 128;
                if (src == 0) {
                    v = a.fine[pl * a.f_plane + (int64_t)clampi(y + dy, 0, H - 1) * a.f_row + clampi(x + dx, 0, W - 1)];
                } else if (src == 1) {
                    v = a.coarse[pl * a.c_plane + (int64_t)clampi(y / 2 + dy, 0, a.Hc - 1) * a.c_row +
                                 clampi(x / 2 + dx, 0, a.Wc - 1)];
                } else {
                    v = a.target[pl * a.f_plane + (int64_t)y * a.f_row + x];
                }
            }
            if constexpr (PREC == 0) {
                xhi[f][p] = v;
            } else {
                const __bf16 h = to_bf16(v);
                xhi[f][p] = h;
                xlo[f][p] = to_bf16(v - from_bf16(h));
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (i < my_tiles) {
                const int rowA = tP[i] * 32 + (lane & 31);
                const int rowB = tQ[i] * 32 + (lane & 31);
                if constexpr (PREC == 0) {
#pragma unroll 4
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
        __syncthreads();
    };

    int pending = 0;
    int64_t n_total = 0;
    for (int64_t base = 0; base < N; base += kScan) {
        int flags = 0, cnt = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t p = base + 4 * tid + j;
            if (p < N) {
                const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
                if (a.s[(int64_t)y * a.s_pitch + x] == k) {
                    flags |= 1 << j;
                    ++cnt;
                }
            }
        }
        int total;
        const int pos = block_scan(cnt, sbuf, &total);
        int w = pending + pos;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (flags & (1 << j)) plist[w++] = (int)(base + 4 * tid + j);
        __syncthreads();
        pending += total;
        n_total += total;
        while (pending >= kChunk) {
            process(kChunk);
            const int rest = pending - kChunk;
            int moved[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const int i = tid + 256 * j;
                moved[j] = i < rest ? plist[kChunk + i] : 0;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const int i = tid + 256 * j;
                if (i < rest) plist[i] = moved[j];
            }
            __syncthreads();
            pending = rest;
        }
    }
    if (pending > 0) process(pending);

    // add the tiles to the float64 accumulators of this system
    const int sys = a.per_channel ? k * (int)gridDim.y + sys_c : k;
    const int D = a.D;
    double* G = a.G + (int64_t)sys * D * D;
    double* bvec = a.b + (int64_t)sys * a.nrhs * D;
    double* yy = a.yy + (int64_t)sys * a.nrhs;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        if (i >= my_tiles) continue;
        const int P = tP[i], Q = tQ[i];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int p = P * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int q = Q * 32 + (lane & 31);
            const double v = (double)acc[i][r];
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
    if (sys_c == 0 && tid == 0) a.n[k] += n_total;
}

// float32 YCbCr (or grey) planes of an RGB / grey image, for the sample gathers.
__global__ void k_to_planes(ImageArg in, int32_t dtype, int32_t rgb_to_ycc, int32_t C, float* out, int64_t o_row,
                            int64_t o_plane) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= in.w || y >= in.h) return;
    const int64_t off = (int64_t)y * in.row + x;
    float v[3] = {0, 0, 0};
    for (int c = 0; c < C; ++c) {
        v[c] = dtype == MDN_F16 ? __half2float(static_cast<const __half*>(in.data)[off + c * in.plane])
                                : static_cast<const float*>(in.data)[off + c * in.plane];
    }
    if (C == 3 && rgb_to_ycc) Ycc::from_rgb(v[0], v[1], v[2], v[0], v[1], v[2]);
    for (int c = 0; c < C; ++c) out[c * o_plane + (int64_t)y * o_row + x] = v[c];
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

size_t train_ws_bytes(int w, int h, int C) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const int wc = (w + 1) / 2, hc = (h + 1) / 2;
    return al((size_t)w * h * C * 4) * 2 + al((size_t)wc * hc * C * 4) + al((size_t)w * h);
}

mdn_status launch_to_planes(const mdn_image& im, float* out, int64_t row, int64_t plane, hipStream_t st) {
    ImageArg a{im.data, im.row_pitch, im.plane_pitch, im.width, im.height};
    dim3 grid((im.width + 255) / 256, im.height);
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
    char* p = static_cast<char*>(ws);
    float* fine = reinterpret_cast<float*>(p);
    p += al((size_t)W * H * C * 4);
    float* tgt = reinterpret_cast<float*>(p);
    p += al((size_t)W * H * C * 4);
    float* coarse = reinterpret_cast<float*>(p);
    p += al((size_t)Wc * Hc * C * 4);
    uint8_t* smap = reinterpret_cast<uint8_t*>(p);
    mdn_status s;
    if ((s = launch_to_planes(z, fine, W, (int64_t)W * H, st))) return s;
    if ((s = launch_to_planes(target, tgt, W, (int64_t)W * H, st))) return s;
    if (uc && (s = launch_to_planes(*uc, coarse, Wc, (int64_t)Wc * Hc, st))) return s;
    if ((s = launch_select_apply(z, nullptr, nullptr, W, smap, sel, nullptr, st))) return s;

    GramArgs a;
    memset(&a, 0, sizeof(a));
    a.fine = fine;
    a.coarse = coarse;
    a.target = tgt;
    a.f_row = W;
    a.f_plane = (int64_t)W * H;
    a.c_row = Wc;
    a.c_plane = (int64_t)Wc * Hc;
    a.W = W;
    a.H = H;
    a.Wc = Wc;
    a.Hc = Hc;
    a.s = smap;
    a.s_pitch = W;
    a.D = D;
    a.nrhs = nrhs;
    a.per_channel = g.layout == MDN_X_PER_CHANNEL;
    int f = 0;
    if (a.per_channel) {
        if (g.radius_f >= 1)
            for (int dy = -g.radius_f; dy <= g.radius_f; ++dy)
                for (int dx = -g.radius_f; dx <= g.radius_f; ++dx) a.feat[f++] = feat_pack(1, 0, dy, dx);
        for (int dy = -g.radius_g; dy <= g.radius_g; ++dy)
            for (int dx = -g.radius_g; dx <= g.radius_g; ++dx) a.feat[f++] = feat_pack(0, 0, dy, dx);
        a.feat[f++] = feat_pack(2, 0, 0, 0);
    } else {
        for (int c = 0; c < C; ++c)
            for (int dy = -g.radius_g; dy <= g.radius_g; ++dy)
                for (int dx = -g.radius_g; dx <= g.radius_g; ++dx) a.feat[f++] = feat_pack(0, c, dy, dx);
        for (int c = 0; c < C; ++c) a.feat[f++] = feat_pack(2, c, 0, 0);
    }
    a.Daug = f;
    a.G = g.G;
    a.b = g.b;
    a.n = g.n;
    a.yy = g.yy;
    const int T = (f + 31) / 32;
    dim3 grid(g.K, spk);
#define MDN_GRAM(P_, T_) \
    if (precision == P_ && T == T_) { k_gram<P_, T_><<<grid, 256, 0, st>>>(a); return check_launch("gram"); }
    MDN_GRAM(0, 1) MDN_GRAM(0, 2) MDN_GRAM(0, 3) MDN_GRAM(0, 4) MDN_GRAM(0, 5)
    MDN_GRAM(1, 1) MDN_GRAM(1, 2) MDN_GRAM(1, 3) MDN_GRAM(1, 4) MDN_GRAM(1, 5)
#undef MDN_GRAM
    return fail(MDN_ENOTSUP, "gram: %d features not supported", f);
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
