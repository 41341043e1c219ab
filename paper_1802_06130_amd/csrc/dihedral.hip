// Training-set augmentation (Section 5: axial flips and 90-degree rotations of every training
// pair): symmetry t (0..7) of the square applied to a planar image, bit 2 = transpose (first),
// bit 0 = mirror the columns, bit 1 = mirror the rows. A pure permutation of the elements, so it
// moves raw 16- or 32-bit words and is exact for any dtype.
//
// Each 256-thread workgroup owns a 32 x 32 tile of the output plane. The tile's source is a
// 32 x 32 block of the input (mirrors map contiguous ranges to contiguous ranges); it is read row
// by row (coalesced), staged in LDS (stride 33 words: column reads of a transpose hit distinct
// banks) and written row by row.

#include "mdn_internal.h"

namespace mdn {

namespace {

constexpr int kTile = 32;

template <typename W>
__global__ __launch_bounds__(256) void k_dihedral(const W* in, W* out, int64_t i_row, int64_t i_plane, int64_t o_row,
                                                  int64_t o_plane, int Hi, int Wi, int Ho, int Wo, int t) {
    __shared__ W tile[kTile][kTile + 1];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;    // 32 x 8 threads
    const int oy0 = blockIdx.y * kTile, ox0 = blockIdx.x * kTile;
    const int oy1 = min(oy0 + kTile, Ho), ox1 = min(ox0 + kTile, Wo);
    // output rows [oy0, oy1) and columns [ox0, ox1) before the mirrors
    const int iy_lo = (t & 2) ? Ho - oy1 : oy0, ix_lo = (t & 1) ? Wo - ox1 : ox0;
    // source block: rows and columns of the input (swapped by the transpose)
    const int sy0 = (t & 4) ? ix_lo : iy_lo, sx0 = (t & 4) ? iy_lo : ix_lo;
    const int sh = (t & 4) ? ox1 - ox0 : oy1 - oy0, sw = (t & 4) ? oy1 - oy0 : ox1 - ox0;
    const W* src = in + (int64_t)blockIdx.z * i_plane;
    W* dst = out + (int64_t)blockIdx.z * o_plane;
    for (int a = ty; a < sh; a += 8)
        if (tx < sw) tile[a][tx] = src[(int64_t)(sy0 + a) * i_row + sx0 + tx];
    __syncthreads();
    for (int i = oy0 + ty; i < oy1; i += 8) {
        const int j = ox0 + tx;
        if (j >= ox1) continue;
        const int i1 = (t & 2) ? Ho - 1 - i : i, j1 = (t & 1) ? Wo - 1 - j : j;
        const int sy = (t & 4) ? j1 : i1, sx = (t & 4) ? i1 : j1;
        dst[(int64_t)i * o_row + j] = tile[sy - sy0][sx - sx0];
    }
}

}  // namespace

mdn_status launch_dihedral(const mdn_image& in, const mdn_image& out, int t, hipStream_t st) {
    if (out.width == 0 || out.height == 0) return MDN_OK;
    const dim3 grid((out.width + kTile - 1) / kTile, (out.height + kTile - 1) / kTile, in.channels);
    if (in.dtype == MDN_F16)
        k_dihedral<uint16_t><<<grid, 256, 0, st>>>(static_cast<const uint16_t*>(in.data), static_cast<uint16_t*>(out.data),
                                                   in.row_pitch, in.plane_pitch, out.row_pitch, out.plane_pitch,
                                                   in.height, in.width, out.height, out.width, t);
    else
        k_dihedral<uint32_t><<<grid, 256, 0, st>>>(static_cast<const uint32_t*>(in.data), static_cast<uint32_t*>(out.data),
                                                   in.row_pitch, in.plane_pitch, out.row_pitch, out.plane_pitch,
                                                   in.height, in.width, out.height, out.width, t);
    return check_launch("dihedral");
}

}  // namespace mdn
