// A pyramid step (level l -> l + 1) and the selection pass of level l in one launch. Both read the
// level-l image and neither needs the other's output. On its own the pyramid keeps the vector ALU
// about half busy (the rest is waiting on memory) while the selection's float64 arithmetic keeps
// it about 90% busy, so the workgroups here take the strips of both lists, interleaved in
// proportion to their counts: the SIMDs then hold waves of both kinds and the selection's
// arithmetic fills the pyramid's waits. Each strip is computed by the same code as in its own
// launch, so the outputs are bit for bit those of the two separate launches.

#include "down2_walk.h"
#include "select_walk.h"

namespace mdn {

namespace {

constexpr int kWaves = 4;

// T: the level's storage (pyramid input and selection input), TO: the next level's storage.
template <typename T, typename TO, int QS, int QC, int MQ, int NSTEP>
__global__ __launch_bounds__(64 * kWaves, 4) void k_pyr_sel(D2Args d, SelWalkArgs s) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    __shared__ sw::BoundaryTable bt;
    __shared__ double hbox[kWaves][3][sw::kHboxW];
    sw::prologue(s, bt, &hbox[0][0][0], kWaves * 3 * sw::kHboxW, 64 * kWaves);
    __syncthreads();
    // The strips go in groups of four consecutive ones of the same list, one per wave of a workgroup
    // (neighbouring strips share their edge lines in the caches, as in the separate launches). Group
    // j is pyramid group floor(j gp / g) when that count steps at j, else selection group
    // j - floor(j gp / g): each list keeps its own order and the two are spread evenly.
    const int64_t gp = (d.n_strips + kWaves - 1) / kWaves, g = gp + (s.n_strips + kWaves - 1) / kWaves;
    for (int64_t j = blockIdx.x; j < g; j += gridDim.x) {
        const int64_t p0 = j * gp / g, p1 = (j + 1) * gp / g;
        if (p1 > p0) {
            const int64_t k = p0 * kWaves + wave;
            if (k < d.n_strips) d2w::strip<T, TO, 3>(d, (int)k, lane);
        } else {
            const int64_t k = (j - p0) * kWaves + wave;
            if (k < s.n_strips)
                sw::strip<T, uint8_t, 3, false, QS, QC, MQ, NSTEP>(s, (int)k, lane, bt, &hbox[wave][0][0]);
        }
    }
}

}  // namespace

bool pyr_sel_fusable(const SelWalkArgs& s) {
    return !s.luma && s.q_theta * s.q_s * s.q_c * s.phases <= 256;
}

mdn_status launch_pyr_sel_args(const D2Args& d, const SelWalkArgs& s, int level_dtype, int next_dtype,
                               hipStream_t st) {
    if (!pyr_sel_fusable(s)) return fail(MDN_EINVAL, "pyramid and selection: bank not supported");
    const int64_t n = (int64_t)d.n_strips + s.n_strips;
    if (n <= 0) return MDN_OK;
    const int ncu = device_cus();
    const int64_t blocks = (n + kWaves - 1) / kWaves;
    // more workgroups than are resident at once (4 per CU): the dispatcher hands out the rest as
    // workgroups finish, which evens out the two kinds of work
    const int grid = (int)(blocks < 32 * ncu ? blocks : 32 * ncu);
    const int spec = (s.q_s == 3 && s.q_c == 3) ? (s.q_theta == 24 ? 1 : s.q_theta == 16 ? 2 : 0) : 0;
#define MDN_PS(T_, TO_)                                                                          \
    do {                                                                                         \
        if (spec == 1) k_pyr_sel<T_, TO_, 3, 3, 5, 0><<<grid, 64 * kWaves, 0, st>>>(d, s);        \
        else if (spec == 2) k_pyr_sel<T_, TO_, 3, 3, 3, 0><<<grid, 64 * kWaves, 0, st>>>(d, s);   \
        else k_pyr_sel<T_, TO_, 0, 0, 0, 5><<<grid, 64 * kWaves, 0, st>>>(d, s);                  \
    } while (0)
    if (level_dtype == MDN_F16 && next_dtype == MDN_F16) MDN_PS(_Float16, _Float16);
    else if (level_dtype == MDN_F32 && next_dtype == MDN_F16) MDN_PS(float, _Float16);
    else if (level_dtype == MDN_F32 && next_dtype == MDN_F32) MDN_PS(float, float);
    else if (level_dtype == MDN_F16 && next_dtype == MDN_F32) MDN_PS(_Float16, float);
    else return fail(MDN_EINVAL, "pyramid and selection: unsupported dtype pair");
#undef MDN_PS
    return check_launch("pyr_sel");
}

bool pyr_sel_fits(const mdn_level& lvl, int channels) {
    return channels == 3 && lvl.selector == MDN_SELECT_RGB && lvl.phases == 1 && level_buckets(lvl) <= 256;
}

mdn_status launch_pyr_sel(const mdn_image& z, const mdn_image& next, const mdn_level& lvl, void* s, int64_t s_pitch,
                          hipStream_t st) {
    if (!pyr_sel_fits(lvl, z.channels)) return fail(MDN_EINVAL, "pyramid and selection: level not supported");
    if (z.width == 0 || z.height == 0) return MDN_OK;
    D2Args d;
    SelWalkArgs a;
    fill_down2_single(z, next, d);
    fill_select_single(z, lvl, s, s_pitch, a);
    return launch_pyr_sel_args(d, a, z.dtype, next.dtype, st);
}

}  // namespace mdn
