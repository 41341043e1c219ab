// Column-walk selection pass (Section 3, Eq. (3)-(6)): bucket index s(i) of every pixel of an RGB
// level, written as a uint8 map for the filtering pass. The work of one strip, shared by the
// selection launch and the launch that runs it beside a pyramid step.
//
// A wavefront owns 58 output columns (64 lanes with a 3-column halo each side) and walks down a
// strip of rows. For each new row r = y+2 it forms, per lane and in float64, the differences
// dx = z(r, x+1) - z(r, x-1) (neighbouring columns from DPP wave shifts) and dy = z(r+1, x) -
// z(r-1, x), accumulates A = sum_c dx^2, B = sum_c dx dy, C = sum_c dy^2 (four times the products
// of the central-difference gradients: the factor is exact), replaces positions outside the image
// by the value at the clamped position (readlane), and sums 5 neighbouring lanes (their values
// exchanged through a per-wave LDS row). A 5-row ring then gives the 5 x 5 box sums of row y, 100
// times the box mean (a, b, c). The bucket needs no square root or division:
//   strength:  sqrt(lambda1) >= t  <=>  lambda1 >= t^2  <=>  mu >= 2 t^2 - tr      (mu^2 = (a-c)^2 + 4b^2)
//   coherence: (sqrt(l1)-sqrt(l2))/(sqrt(l1)+sqrt(l2)) >= t  <=>  mu >= (2t / (1 + t^2)) tr   (tr > 0)
//   orientation: the doubled-angle vector of the minor eigenvector, (c - a, -2b), against the bin
//   boundary directions by cross products.
// LDS holds a small table of bin boundary directions and, per wave, the three rows of products
// that the lanes exchange for the horizontal sums.

#pragma once

#include "walk_types.h"

#include <type_traits>
#include <utility>

namespace mdn {
namespace sw {

constexpr int kLanesOut = kSelLanesOut;
constexpr int kHboxW = 68;          // 64 lanes + 2 pads each side

__device__ __forceinline__ uint32_t shl1(uint32_t v) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ uint32_t shr1(uint32_t v) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ float shl1f(float v) { return __uint_as_float(shl1(__float_as_uint(v))); }
__device__ __forceinline__ float shr1f(float v) { return __uint_as_float(shr1(__float_as_uint(v))); }
__device__ __forceinline__ double shl1d(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return __longlong_as_double((long long)(((uint64_t)shl1((uint32_t)(u >> 32)) << 32) | shl1((uint32_t)u)));
}
__device__ __forceinline__ double shr1d(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return __longlong_as_double((long long)(((uint64_t)shr1((uint32_t)(u >> 32)) << 32) | shr1((uint32_t)u)));
}
// Orders this wave's LDS accesses across lanes: memory operations are not moved across it (the
// LDS itself serves one wave's requests in order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ float shl1x(float v) { return shl1f(v); }
__device__ __forceinline__ float shr1x(float v) { return shr1f(v); }
__device__ __forceinline__ double shl1x(double v) { return shl1d(v); }
__device__ __forceinline__ double shr1x(double v) { return shr1d(v); }
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

#define MDN_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ float ldo(const T* base, uint32_t elem) {
    const MDN_GLOBAL char* b = (const MDN_GLOBAL char*)(base);
    return (float)*(const MDN_GLOBAL T*)(b + elem * (uint32_t)sizeof(T));
}

struct P3 {
    double A, B, C;
};

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

// Boundary directions of the orientation bins within the upper half plane, in LDS so that each
// lane can index them (binary search).
struct BoundaryTable {
    double cs[kMaxTheta / 2], sn[kMaxTheta / 2];
};

// QS, QC: strength and coherence bin counts when fixed at compile time (0: read from the arguments).
// Orientation: with MQ > 0 (q_theta = 4 (MQ + 1)) the boundaries of the upper half plane are
// symmetric about the vertical one, so the vector is folded into the first quadrant and tested
// against the MQ boundaries below 90 degrees only (constants from the kernel arguments, no LDS, no
// branches); with MQ = 0 the q_theta/2 - 1 boundaries are searched in NSTEP binary steps over the
// LDS table (2^NSTEP > count).
template <int QS, int QC, int MQ, int NSTEP>
__device__ __forceinline__ int bucket(double a, double b, double c, const SelWalkArgs& sp, const BoundaryTable& bt) {
    const int q_s = QS ? QS : sp.q_s, q_c = QC ? QC : sp.q_c;
    const double tr = a + c;
    const double dd = a - c;
    const double m2 = dd * dd + 4.0 * b * b;
    int qs = 0;
#pragma unroll
    for (int j = 0; j < (QS ? QS : kMaxThr + 1) - 1; ++j) {
        if (!QS && j >= q_s - 1) break;
        // d <= 0 or m2 >= d^2, in one test: d |d| is -d^2 <= 0 <= m2 when d <= 0 (exact)
        const double d = 2.0 * sp.s_lim[j] - tr;
        qs += (m2 >= d * fabs(d)) ? 1 : 0;
    }
    int qc = 0;
    const double tr2 = tr * tr;
#pragma unroll
    for (int j = 0; j < (QC ? QC : kMaxThr + 1) - 1; ++j) {
        if (!QC && j >= q_c - 1) break;
        const double k2 = sp.c_k2[j];
        qc += (k2 < 0.0 || (tr > 0.0 && m2 >= k2 * tr2)) ? 1 : 0;
    }
    const double X = c - a, Y = -2.0 * b;
    // a zero vector (a = c, b = 0) has no orientation: it takes bin q_theta/2 (the oracle's theta = pi/2)
    const bool flat = X == 0.0 && Y == 0.0;
    const bool upper = (Y > 0.0) || (Y == 0.0 && X > 0.0);
    const double px = upper ? X : -X, py = upper ? Y : -Y;
    // boundary j (angle 2 pi (j+1) / q_theta) is passed iff its cross product with (px, py)
    // is >= 0; the count of passed boundaries is the bin within the half plane. The two products
    // are rounded alone (no fused multiply-add), so that an exact tie compares equal.
    int k = 0;
    if constexpr (MQ > 0) {
        // The boundary table is exactly mirror-symmetric (the mirror of (c_j, s_j) is (-c_j, s_j) and
        // the vertical one is (0, 1)), so this equals the test against every boundary:
        // px >= 0: boundaries 0..MQ-1 are passed iff c_j py - s_j px >= 0, the vertical one iff
        // px = 0, the mirrored ones never. px < 0: boundaries 0..MQ-1 and the vertical one always,
        // mirrored boundary q_theta/2 - 2 - j iff -c_j py - s_j px >= 0.
        const bool right = px >= 0.0;
        const double spy = right ? py : -py;
#pragma unroll
        for (int j = 0; j < MQ; ++j) k += (__dmul_rn(sp.bcos[j], spy) >= __dmul_rn(sp.bsin[j], px)) ? 1 : 0;
        k += right ? (px == 0.0 ? 1 : 0) : MQ + 1;
    } else {
        const int nb = sp.half - 1;
#pragma unroll
        for (int step = 1 << (NSTEP - 1); step >= 1; step >>= 1) {
            const int j = k + step - 1;
            const int jj = j < nb ? j : 0;
            k += ((j < nb) & (__dmul_rn(bt.cs[jj], py) >= __dmul_rn(bt.sn[jj], px))) ? step : 0;
        }
    }
    const int qt = flat ? sp.half : k + (upper ? 0 : sp.half);
    return (qt * q_s + qs) * q_c + qc;
}

// Fill the boundary table and clear the waves' rows (n doubles), by every thread of the workgroup;
// the caller synchronises the workgroup afterwards.
__device__ __forceinline__ void prologue(const SelWalkArgs& a, BoundaryTable& bt, double* hbox, int n, int nthreads) {
    for (int j = threadIdx.x; j < kMaxTheta / 2; j += nthreads) {
        bt.cs[j] = a.bcos[j];
        bt.sn[j] = a.bsin[j];
    }
    for (int j = threadIdx.x; j < n; j += nthreads) hbox[j] = 0.0;
}

// One strip of the selection pass, walked by the calling wave (lane = its lane number; hb = the
// wave's three LDS rows of kHboxW doubles).
template <typename TZ, typename TS, int C, bool LUMA, int QS, int QC, int MQ, int NSTEP>
__device__ __forceinline__ void strip(const SelWalkArgs& a, int strip, int lane, const BoundaryTable& bt, double* hb) {
    static_assert(!LUMA || C == 3, "the luma selector reads RGB");
    constexpr int NC = LUMA ? 1 : C;                             // channels of the selector image
    using RowT = double;                     // rows converted to float64 once, at load
    SelImage im;
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
    const int W = im.W, H = im.H;
    const int xs = sx * kLanesOut, ys = sy * im.rows;
    const int ye = min(ys + im.rows, H);
    const int x = xs - 3 + lane;
    const int xc = clampi(x, 0, W - 1);
    const bool out_lane = lane >= 3 && lane < 3 + kLanesOut && x < W;
    const int lane_x0 = 3 - xs, lane_xw = W - 1 - xs + 3;
    const bool fix_left = lane_x0 >= 0, fix_right = lane_xw <= 63;
    // image planes and selector map: wave-uniform, kept in scalar registers
    const TZ* zb = uniform_ptr(static_cast<const TZ*>(im.z));
    TS* sout = uniform_ptr(static_cast<TS*>(im.s));
    const uint32_t zrow = (uint32_t)im.z_row, zpl = (uint32_t)im.z_plane;

    // a row of the selector image: the channels as loaded, or the float64 luma of RGB
    auto load = [&](int row, RowT v[NC]) {
        const uint32_t o = (uint32_t)clampi(row, 0, H - 1) * zrow + (uint32_t)xc;
        if constexpr (LUMA) {
            v[0] = luma_d(ldo(zb, o), ldo(zb, o + zpl), ldo(zb, o + 2 * zpl));
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = ldo(zb, o + c * zpl);
        }
    };
    // horizontally summed products at an in-image row from its rows (above, centre, below)
    auto hrow = [&](const RowT zu[NC], const RowT zm[NC], const RowT zd[NC]) {
        P3 p{0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double dx = (double)shl1x(zm[c]) - (double)shr1x(zm[c]);
            const double dy = (double)zd[c] - (double)zu[c];
            p.A += dx * dx;
            p.B += dx * dy;
            p.C += dy * dy;
        }
        if (fix_left) {
            const double A0 = readlane_d(p.A, lane_x0), B0 = readlane_d(p.B, lane_x0), C0 = readlane_d(p.C, lane_x0);
            if (x < 0) {
                p.A = A0;
                p.B = B0;
                p.C = C0;
            }
        }
        if (fix_right) {
            const double A1 = readlane_d(p.A, lane_xw), B1 = readlane_d(p.B, lane_xw), C1 = readlane_d(p.C, lane_xw);
            if (x > W - 1) {
                p.A = A1;
                p.B = B1;
                p.C = C1;
            }
        }
        // the compiler must neither move this row's writes above the previous row's reads nor
        // the reads above the writes: other lanes' addresses alias them
        wave_sync();
        hb[lane + 2] = p.A;
        hb[kHboxW + lane + 2] = p.B;
        hb[2 * kHboxW + lane + 2] = p.C;
        wave_sync();
        const double Am2 = hb[lane], Am1 = hb[lane + 1], A1 = hb[lane + 3], A2 = hb[lane + 4];
        const double Bm2 = hb[kHboxW + lane], Bm1 = hb[kHboxW + lane + 1], B1 = hb[kHboxW + lane + 3],
                     B2 = hb[kHboxW + lane + 4];
        const double Cm2 = hb[2 * kHboxW + lane], Cm1 = hb[2 * kHboxW + lane + 1], C1 = hb[2 * kHboxW + lane + 3],
                     C2 = hb[2 * kHboxW + lane + 4];
        return P3{((Am2 + Am1) + p.A) + (A1 + A2), ((Bm2 + Bm1) + p.B) + (B1 + B2), ((Cm2 + Cm1) + p.C) + (C1 + C2)};
    };
    auto hrow_at = [&](int r) {      // row cl(r), loading its three input rows
        const int c = clampi(r, 0, H - 1);
        RowT zu[NC], zm[NC], zd[NC];
        load(c - 1, zu);
        load(c, zm);
        load(c + 1, zd);
        return hrow(zu, zm, zd);
    };

    // ring: h(r) in hr[(r - ys) mod 5]; rows ys-2 .. ys+1 first. Input rows r = ys+1 .. ys+5 sit
    // in zr[(r - ys) mod 5] (fixed slots over the 10-row step body).
    P3 hr[5];
    RowT zr[5][NC];
    // one row at a time (a rolled loop keeps the start-up within the register budget)
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        const P3 h = hrow_at(ys - 2 + k);
        hr[0] = hr[1];
        hr[1] = hr[2];
        hr[2] = hr[3];
        hr[3] = hr[4];
        hr[4] = h;
    }
    {
        const P3 h0 = hr[1], h1 = hr[2], h2 = hr[3], h3 = hr[4];   // rows ys-2 .. ys+1
        hr[3] = h0;
        hr[4] = h1;
        hr[0] = h2;
        hr[1] = h3;
    }
    load(ys + 1, zr[1]);
    load(ys + 2, zr[2]);
    load(ys + 3, zr[3]);
    load(ys + 4, zr[4]);
    for (int y0 = ys; y0 < ye; y0 += 10) {
        unroll([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            const int y = y0 + I;
            // rows are loaded two steps before their use; row y+5 replaces row y
            load(y + 5, zr[I % 5]);
            // h(y+2): rows y+1, y+2, y+3; below the last image row it repeats h(H-1)
            constexpr int slot = (I + 2) % 5;
            constexpr int prev = (I + 1) % 5;
            hr[slot] = (y + 2 <= H - 1) ? hrow(zr[(I + 1) % 5], zr[(I + 2) % 5], zr[(I + 3) % 5]) : hr[prev];
            const double sa = (((hr[0].A + hr[1].A) + hr[2].A) + hr[3].A) + hr[4].A;
            const double sb = (((hr[0].B + hr[1].B) + hr[2].B) + hr[3].B) + hr[4].B;
            const double sc = (((hr[0].C + hr[1].C) + hr[2].C) + hr[3].C) + hr[4].C;
            int s = bucket<QS, QC, MQ, NSTEP>(sa, sb, sc, a, bt);
            if (a.phases == 4) s = 4 * s + ((y & 1) << 1) + (x & 1);
            if (out_lane && y < ye) *((MDN_GLOBAL TS*)sout + (uint32_t)y * (uint32_t)im.s_pitch + (uint32_t)x) = (TS)s;
        }, std::make_integer_sequence<int, 10>{});
    }
}

}  // namespace sw
}  // namespace mdn
