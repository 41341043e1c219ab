/*
 * mdn.h -- C ABI of the MI355X (gfx950) multiscale adaptive-filter denoiser.
 *
 * Method: "Fast, Trainable, Multiscale Denoising" (Choi, Isidoro, Getreuer, Milanfar,
 * arXiv 1802.06130). A per-pixel filter index s(i) is chosen from features of the
 * colour structure tensor (Section 3, Eq. (3)-(6)); the selected FIR filter is applied
 * (Eq. (1)); over a factor-two bicubic pyramid each level upscales the coarser output
 * and denoises and blends the current level (Section 4, Eq. (9)-(10)); the filters are
 * fitted per bucket by least squares (Eq. (7)-(8)).
 *
 * Conventions shared by every entry point
 *  - Pixel, index and accumulator pointers are DEVICE pointers owned by the caller.
 *    The library never frees or retains them past the call's stream work.
 *  - Threshold arrays in mdn_level are HOST pointers, read during the call.
 *  - Every call validates its arguments synchronously, then enqueues its work on
 *    `stream` (a hipStream_t passed as void*; NULL = the null stream) and returns
 *    without waiting. A non-OK status means nothing was enqueued; the reason is in
 *    mdn_last_error() (thread-local). Launch failures return MDN_EDEVICE.
 *  - Images are planar: element (c, y, x) is at data + c*plane_pitch + y*row_pitch + x
 *    (pitches in elements). Width or height 0 is an empty image: calls on it do nothing
 *    and return MDN_OK.
 *  - Borders: every stencil reads clamp-to-edge (replicated) pixels.
 */
#ifndef MDN_H
#define MDN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MDN_OK = 0,
    MDN_EINVAL = 1,   /* bad argument: null pointer, size mismatch, unknown enum */
    MDN_ENOMEM = 2,   /* workspace too small */
    MDN_EDEVICE = 3,  /* HIP launch or runtime error */
    MDN_ENOTSUP = 4,  /* valid but unsupported configuration (filter radius, K > 65536, ...) */
    MDN_ETIMEOUT = 5, /* serving: the request waited longer than the queue time-out */
    MDN_ECANCELED = 6 /* serving: the request was cancelled */
} mdn_status;

typedef enum { MDN_F32 = 0, MDN_F16 = 1 } mdn_dtype;

/* Colour space of an image's channels. Colour images are filtered in full-range
 * ITU-R BT.601 YCbCr (footnote of Section 3): Y = .299R + .587G + .114B,
 * Cb = (B - Y)/1.772 + 1/2, Cr = (R - Y)/1.402 + 1/2. The structure tensor is
 * always taken on RGB. */
typedef enum { MDN_GRAY = 0, MDN_RGB = 1, MDN_YCC = 2 } mdn_color;

/* Image the structure tensor of the filter selector is taken on (Section 3): the colour image,
 * its channels summed as in Eq. (6) (the paper's choice), or its luma alone. Grey images are
 * their own luma. */
typedef enum { MDN_SELECT_RGB = 0, MDN_SELECT_LUMA = 1, MDN_SELECT_COARSE = 2 } mdn_selector;

typedef struct {
    void*   data;         /* device pointer */
    int32_t width;
    int32_t height;
    int32_t channels;     /* 1 (MDN_GRAY) or 3 (MDN_RGB / MDN_YCC) */
    int32_t dtype;        /* mdn_dtype of the stored elements */
    int32_t color;        /* mdn_color */
    int32_t reserved;     /* must be 0 */
    int64_t row_pitch;    /* elements between rows, >= width */
    int64_t plane_pitch;  /* elements between channel planes, >= height*row_pitch */
} mdn_image;

/* Filters and selector of one trained level (Eq. (9)-(10); Eq. (1) when radius_f < 0).
 * K = q_theta*q_s*q_c buckets, bucket index s = (q_theta_bin*q_s + q_s_bin)*q_c + q_c_bin:
 *   q_theta_bin: angle of the structure tensor's minor eigenvector (edge direction,
 *                from +x towards +y, rows downward) in q_theta uniform bins over [0, pi);
 *   q_s_bin:     number of t_s thresholds that sqrt(lambda1) reaches (>=);
 *   q_c_bin:     number of t_c thresholds that (sqrt(l1)-sqrt(l2))/(sqrt(l1)+sqrt(l2)) reaches.
 * The structure tensor sums, over the RGB (or grey) channels, products of central-difference
 * gradients averaged over a 5x5 box (Eq. (6)); it is evaluated in float64. With
 * selector = MDN_SELECT_LUMA it is taken on the BT.601 luma Y = 0.299 R + 0.587 G + 0.114 B of a
 * colour level instead (float64; the luma-only analysis Section 3 compares against, Fig. 2).
 * With selector = MDN_SELECT_COARSE (multiscale levels only) it is taken on the coarser level's
 * output u^{l+1} instead of the noisy z^l: u^{l+1} is upsampled onto this level's grid by linear
 * interpolation on the pyramid's alignment (coarse sample m lies between fine pixels 2m and 2m+1,
 * so fine 2m takes 3/4 of m and 1/4 of m-1, fine 2m+1 takes 3/4 of m and 1/4 of m+1, indices
 * clamped; rows, then columns) and taken back to RGB (float64). This is the alternative to the
 * noisy input that Eq. (9) leaves open: less noise, half the resolution.
 * coeffs[k][c] holds taps_f = (2*radius_f+1)^2 upscale taps applied to the coarser output at
 * floor(i/2) + j, then taps_g = (2*radius_g+1)^2 taps applied to this level's input at i + j,
 * both row-major over (dy, dx).
 * phases = 4 makes the buckets phase-aware (a reading of the non-integer i/2 of Eq. (9) for odd
 * i): the parity of the pixel on the coarser grid, p = 2 (y mod 2) + (x mod 2), joins the index as
 * s' = 4 s + p, so that every bucket has one filter pair per phase; all sizes and maps then count
 * 4K buckets. */
typedef struct {
    int32_t q_theta;      /* 2..64, even */
    int32_t q_s;          /* 1..16 */
    int32_t q_c;          /* 1..16 */
    int32_t radius_f;     /* -1 (single-scale filter), 1, 2 or 3 */
    int32_t radius_g;     /* 1, 2 or 3 */
    int32_t channels;     /* 1 or 3, must match the images */
    int32_t coeff_dtype;  /* mdn_dtype of coeffs */
    int32_t selector;     /* mdn_selector: MDN_SELECT_RGB (0), MDN_SELECT_LUMA (1) or MDN_SELECT_COARSE (2) */
    int32_t phases;       /* 1, or 4: phase-aware buckets (see above); coeffs then has 4K rows */
    int32_t reserved;     /* must be 0 */
    const double* t_s;    /* HOST, q_s-1 ascending strength thresholds */
    const double* t_c;    /* HOST, q_c-1 ascending coherence thresholds */
    const void*   coeffs; /* DEVICE, [K][channels][taps_f + taps_g] */
} mdn_level;

/* A multiscale bank: level[l] filters trained level l, l = 0 (finest) .. levels-1.
 * The pyramid then has levels+1 levels and the coarsest one passes through unfiltered
 * (Section 4). A single-scale bank has levels = 1 and radius_f < 0. */
typedef struct {
    int32_t levels;
    int32_t reserved;
    const mdn_level* level;   /* HOST array of `levels` entries */
} mdn_bank;

/* Factor-two bicubic pyramid (Section 4, "Multiscale filtering").
 * out[i] receives level i+1: out[i] = down2(level i), where level 0 is *level0.
 * down2: Keys cubic (a = -1/2) stretched by two and centred at 2m+1/2, i.e. the separable
 * 8-tap kernel [-12,-36,116,444,444,116,-36,-12]/1024 over input samples 2m-3..2m+4, rows
 * then columns; evaluated in float64 and rounded once to the output dtype. Each out[i] must
 * have width ceil(w_i/2), height ceil(h_i/2), the same channels and colour. */
mdn_status mdn_pyramid_build(const mdn_image* level0, int32_t n_out, const mdn_image* out,
                             void* stream);

/* Training-set augmentation (Section 5: the axial flips and 90-degree rotations of every
 * training pair are added so that the filters learn the symmetries).
 * out = symmetry `transform` (0..7) of the square applied to every plane of in: bit 2 transposes
 * (first), then bit 0 mirrors the columns (x -> w-1-x) and bit 1 mirrors the rows. out must be
 * h x w when bit 2 is set (w x h otherwise), with the channels, dtype and colour of in, and must
 * not alias it. Elements are moved bit for bit. */
mdn_status mdn_dihedral(const mdn_image* in, int32_t transform, const mdn_image* out, void* stream);

/* Filter selector s(i) (Section 3, "Filter selection"; Eq. (6); features as in mdn_level).
 * z: RGB or grey image of the level. s_out: device [height][s_pitch] selector map, uint8 when
 * K <= 256 and uint16 when K > 256 (the paper's 16 x 16 x 16 buckets, Section 5). */
mdn_status mdn_select_filters(const mdn_image* z, const mdn_level* lvl, void* s_out,
                              int64_t s_pitch, void* stream);

/* Filter selector of a level that selects on the coarser output (MDN_SELECT_COARSE, see mdn_level),
 * for a width x height level: u_coarse is the coarser output u^{l+1} (YCbCr, or RGB at the coarsest
 * pyramid level, or grey), ceil(width/2) x ceil(height/2). s_out as for mdn_select_filters. Levels
 * with another selector return MDN_EINVAL (and mdn_select_filters refuses coarse-selector levels). */
mdn_status mdn_select_filters_coarse(const mdn_image* u_coarse, int32_t width, int32_t height,
                                     const mdn_level* lvl, void* s_out, int64_t s_pitch, void* stream);

/* One filtering step (Eq. (1) or Eq. (9)).
 * z:        this level's noisy input, RGB or grey (colour images are converted to YCbCr for
 *           filtering, the selector reads RGB).
 * u_coarse: the coarser level's output (YCbCr, or RGB for the coarsest pyramid level, which
 *           is converted), size ceil(w/2) x ceil(h/2); NULL iff lvl->radius_f < 0.
 * s:        precomputed selector (device [height][s_pitch], uint8 or uint16 as for
 *           mdn_select_filters) or NULL to select inline.
 * u_out:    output, YCbCr (intermediate levels) or RGB (converted back), or grey.
 * s_out:    NULL, or a device map like s that receives the selector used (inline mode).
 * Float16 coefficients of 7x7/7x7 colour levels run the column-walk kernel in float16 arithmetic
 * with float32 accumulation; float32 coefficients keep float32 arithmetic throughout. */
mdn_status mdn_apply_level(const mdn_image* z, const mdn_image* u_coarse, const void* s,
                           int64_t s_pitch, const mdn_level* lvl, const mdn_image* u_out,
                           void* s_out, void* stream);

/* Bytes of device workspace mdn_denoise needs for a width x height image with `channels`
 * channels, a bank of `levels` trained levels and pyramid storage dtype `storage`. */
mdn_status mdn_denoise_workspace_size(int32_t width, int32_t height, int32_t channels,
                                      int32_t levels, int32_t storage, size_t* bytes);

/* Whole cascade (Section 4): pyramid of `in`, u^L = z^L, then Eq. (9) for l = L-1..0, the
 * last level written to `out` (RGB or grey, same size as `in`). `storage` is the dtype of the
 * intermediate pyramid and outputs kept in `ws` (caller-owned device memory of at least
 * mdn_denoise_workspace_size bytes, 256-byte aligned). A single-scale bank applies Eq. (1). */
mdn_status mdn_denoise(const mdn_image* in, const mdn_bank* bank, int32_t storage, void* ws,
                       size_t ws_bytes, const mdn_image* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mdn_denoise with its workspace taken from a static
 * device array of MDN_NOALLOC_SCRATCH_BYTES, which the library holds on every device it runs on
 * until the process ends. The call allocates nothing; the caller still owns `in` and `out`.
 * Arguments, results and errors are those of mdn_denoise, plus MDN_ENOMEM when the image needs
 * more workspace than the array holds (mdn_denoise_workspace_size; a 4032 x 3024 RGB frame fits
 * at either storage) and MDN_EDEVICE when the array's address cannot be obtained. The current
 * device must be the one `stream` belongs to. Every call on one device uses the same array:
 * calls that overlap in time on one device (several streams, several host threads) race and
 * must be serialised by the caller; calls in order on one stream are safe. */
#define MDN_NOALLOC_SCRATCH_BYTES (128ull << 20)
mdn_status mdn_denoise_noalloc(const mdn_image* in, const mdn_bank* bank, int32_t storage,
                               const mdn_image* out, void* stream);

/* ---------------------------------------------------------------------------------------
 * Training (Eq. (7)-(8)): one least-squares regression per bucket (and per YCbCr channel,
 * footnote of Section 3), level by level from the second-coarsest level down (Section 4).
 * --------------------------------------------------------------------------------------- */

/* Regression vector layouts.
 * MDN_X_PER_CHANNEL:   x_i = [R_{i/2} u^{l+1}_c ; R_i z^l_c] per channel c (Eq. (10)), target u^l_{i,c};
 *                      K*channels systems of D = taps_f + taps_g unknowns and one right-hand side.
 * MDN_X_CROSS_CHANNEL: x_i = [R_i z_Y ; R_i z_Cb ; R_i z_Cr] (g taps of all channels, no upscale
 *                      block), targets u_Y, u_Cb, u_Cr; K systems of D = 3 taps_g unknowns and 3
 *                      right-hand sides. Used for the precision study only. */
typedef enum { MDN_X_PER_CHANNEL = 0, MDN_X_CROSS_CHANNEL = 1 } mdn_x_layout;

/* Products used for the normal-equation accumulation (FP32 accumulators on MFMA; each call's
 * per-bucket sums are then added into float64 accumulators).
 * MDN_GRAM_F32:    FP32 products (v_mfma_f32_32x32x2_f32).
 * MDN_GRAM_BF16X3: BF16 products on a hi/lo split, x*y ~ hi hi + hi lo + lo hi (v_mfma_f32_32x32x16_bf16). */
typedef enum { MDN_GRAM_F32 = 0, MDN_GRAM_BF16X3 = 1 } mdn_gram_precision;

/* Normal equations of one level, caller-owned device memory (float64 / int64):
 * G [systems][D][D], b [systems][nrhs][D], yy [systems][nrhs], n [K] (samples per bucket).
 * System index: k*channels + c (per channel) or k (cross channel). Sizes: mdn_gram_dims. */
typedef struct {
    int32_t  K;          /* buckets (<= 65536) */
    int32_t  channels;   /* 1 or 3 */
    int32_t  layout;     /* mdn_x_layout */
    int32_t  radius_f;   /* -1 (single scale) or 1..3; must be -1 for the cross layout */
    int32_t  radius_g;   /* 1..3 */
    int32_t  reserved;   /* must be 0 */
    double*  G;
    double*  b;
    int64_t* n;
    double*  yy;
} mdn_gram;

/* D (unknowns per system), nrhs and number of systems of a gram configuration. */
mdn_status mdn_gram_dims(const mdn_gram* g, int32_t* D, int32_t* nrhs, int32_t* systems);

/* Zero the accumulators (enqueued on stream). */
mdn_status mdn_gram_zero(const mdn_gram* g, void* stream);

/* Bytes of workspace mdn_train_accumulate needs for this gram and a width x height level
 * (float32 planes, the selector map, the bucket grouping and the per-work-item partial tiles). */
mdn_status mdn_train_workspace_size(const mdn_gram* g, int32_t width, int32_t height, size_t* bytes);

/* Add one training pair's samples at one level to the normal equations (Eq. (8)):
 * z:        noisy level z^l (RGB or grey); selects s(i) with `sel` (thresholds; coefficients unused);
 * u_coarse: coarser output u^{l+1} (YCbCr, or RGB for the coarsest pyramid level), NULL for the
 *           single-scale or cross-channel layouts;
 * target:   clean level u^l (RGB or grey), same size as z.
 * Samples are grouped by bucket in raster order and summed in a fixed order, so repeated calls on
 * one device are bitwise reproducible (the work split follows the device's compute-unit count). */
mdn_status mdn_train_accumulate(const mdn_gram* g, const mdn_image* z, const mdn_image* u_coarse,
                                const mdn_image* target, const mdn_level* sel, int32_t precision,
                                void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace mdn_train_solve needs. */
mdn_status mdn_train_solve_workspace_size(const mdn_gram* g, size_t* bytes);

/* Solve every system: h = (G/n + lambda I)^{-1} b/n by Cholesky in float64 (ridge reading of the
 * regression; the paper defers its details to BLADE). Buckets with n < min_count, or whose
 * factorisation fails, take the pooled solution of the level (sums of G, b, n over all buckets);
 * *n_fallback (device int32, accumulated with atomics, zero it first) counts those systems.
 * coeffs: device [K][channels][D], written in coeff_dtype (MDN_F32 or MDN_F16, rounded once).
 * Enqueued on stream. */
mdn_status mdn_train_solve(const mdn_gram* g, double lambda, int64_t min_count, void* coeffs,
                           int32_t coeff_dtype, int32_t* n_fallback, void* ws, size_t ws_bytes,
                           void* stream);

/* Per-pixel strength sqrt(lambda1) and coherence of z's structure tensor (as used by the
 * selector: `selector` is an mdn_selector), float64, dense [height][width] device arrays. */
mdn_status mdn_level_features(const mdn_image* z, int32_t selector, double* strength, double* coherence,
                              void* stream);

/* The same features for the coarse selector: the structure tensor of u_coarse (ceil(width/2) x
 * ceil(height/2); YCbCr, RGB or grey) upsampled onto the width x height grid as for
 * MDN_SELECT_COARSE. Dense [height][width] device arrays. */
mdn_status mdn_level_features_coarse(const mdn_image* u_coarse, int32_t width, int32_t height, double* strength,
                                     double* coherence, void* stream);

/* Equal-population thresholds: the k/q quantiles (k = 1..q-1, linear interpolation between order
 * statistics) of n device doubles, written to out_host[q-1]. Synchronises `stream`. */
mdn_status mdn_quantiles_workspace_size(int64_t n, size_t* bytes);
mdn_status mdn_quantiles(const double* values, int64_t n, int32_t q, double* out_host, void* ws,
                         size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * Batched form: many RGB images of any sizes, level by level, one persistent launch per kernel
 * and level over all images (pyramid, selection, filtering), optionally as a replayed hipGraph.
 * --------------------------------------------------------------------------------------- */
typedef struct mdn_plan mdn_plan;

/* Create a plan for a multiscale colour bank. Each level runs in the batched form on the kernel
 * mdn_denoise uses for it, so batched outputs equal per-image ones bit for bit:
 *  - float16 7x7/7x7 levels of up to 243 buckets: a selection pass and the filtering column walk
 *    (strip heights autotuned);
 *  - levels that mdn_denoise filters with the tiled select-and-filter kernel (among them the
 *    paper's own configuration of Section 5: 16 x 16 x 16 buckets with 7x7 / 5x5 or 5x5 / 3x3
 *    filters, phase-aware banks, float16 or float32 coefficients): one launch per level over the
 *    64 x 16 tiles of every image, selection inline, coefficients read through the caches.
 * MDN_ENOTSUP for single-scale banks, float32 banks that fit in LDS one channel at a time, and
 * float16 7x7/7x7 levels that select on the coarser output. The plan copies the
 * level descriptors and thresholds (the coefficient buffers must stay valid while it is used),
 * creates its own stream, and allocates its device workspace and tables on first use: creation
 * and the first batch of a new size are the only calls that allocate. storage: pyramid dtype. */
mdn_status mdn_plan_create(const mdn_bank* bank, int32_t storage, int32_t max_images, mdn_plan** plan);
/* A plan over n_banks (1..8) banks, each accepted as by mdn_plan_create; they may differ in depth
 * (the paper's configuration deepens the pyramid with the noise level, Section 5). Every image of a
 * batch names its bank; the pyramid steps run over all images deep enough, and each level's
 * selection and filtering run one launch per bank over that bank's images. */
mdn_status mdn_plan_create_banks(const mdn_bank* banks, int32_t n_banks, int32_t storage, int32_t max_images,
                                 mdn_plan** plan);
mdn_status mdn_plan_destroy(mdn_plan* plan);

/* The batch calls below take, beside in[] and out[], bank: host int32[n], bank[i] the index of
 * image i's bank in the plan (0..n_banks-1), or NULL for bank 0 throughout. */

/* Time candidate strip heights of every kernel and level on this batch and keep the fastest
 * (rows_out, optional host int32[3*levels], levels = the deepest bank's: pyramid, selection,
 * filtering rows per level, shared by the banks). Runs the batch once; ordered after prior work
 * on `stream` and before later work. */
mdn_status mdn_plan_autotune(mdn_plan* plan, const mdn_image* in, const mdn_image* out, const int32_t* bank,
                             int32_t n, int32_t* rows_out, void* stream);

/* Device time of every launch of this batch: the launches of mdn_denoise_batch, in the same order
 * and with the same strip heights but without a graph, each kind of each level started on the idle
 * plan stream between two HIP events, `reps` times (1..1000); us_out (host float[3*levels]) receives
 * the mean microseconds of the pyramid, selection and filtering launches of each level (index
 * 3 l + k, all banks together; a level on the tiled kernel reports its launches as filtering and
 * about nothing for selection). Where a level's selection pass runs in the launch of its pyramid
 * step (a level with a single column-walk bank), that launch's time is the pyramid entry and the
 * selection entry is 0. The outputs are written as by mdn_denoise_batch. Synchronises the plan's
 * stream. */
mdn_status mdn_plan_kernel_times(mdn_plan* plan, const mdn_image* in, const mdn_image* out, const int32_t* bank,
                                 int32_t n, int32_t reps, float* us_out, void* stream);

/* Denoise n images (in[i] -> out[i] with bank[i], RGB, equal sizes per pair, one dtype per side).
 * With use_graph != 0 the launches are captured once per batch (same images, sizes, banks and
 * buffers) and replayed afterwards. Ordered after prior work on `stream` and before later work. */
mdn_status mdn_denoise_batch(mdn_plan* plan, const mdn_image* in, const mdn_image* out, const int32_t* bank,
                             int32_t n, int32_t use_graph, void* stream);

/* ---------------------------------------------------------------------------------------
 * Serving loop (host code above the calls of this header): requests of any sizes arrive over
 * time, each naming one of several device-resident banks (one per noise level, which is taken
 * as known, Section 5). A request is admitted when a slot is free and its device footprint
 * (input, output, pyramid levels, selector maps) fits the memory budget, first come first served
 * with no overtaking. Its input is copied to the device on a copy stream; it then joins the next
 * scheduling tick. A tick advances every active request by up to stages_per_tick cascade stages
 * (pyramid levels 0..L-1, then selection and filtering of levels L-1..0, Section 4) with one
 * persistent launch per kernel, level, bank and dtype over all requests at that point, so a
 * request that arrives while others are mid-cascade shares their next launches. Ticks queue on
 * one compute stream, at most max_ticks_in_flight ahead of the device; each result is copied back
 * on a second copy stream once the tick holding its last stage is done. A request's output is
 * bitwise the same whatever it was batched with, and the same as mdn_denoise's.
 *
 * Threads: mdn_server_submit, mdn_server_cancel and mdn_server_stats may be called from any
 * thread; mdn_server_poll, mdn_server_replay and mdn_server_destroy from one thread at a time.
 * --------------------------------------------------------------------------------------- */
typedef struct mdn_server mdn_server;

typedef enum { MDN_EXEC_HIP = 0, MDN_EXEC_FAKE = 1 } mdn_executor_kind;

typedef struct mdn_server_config {
    const mdn_bank* banks;        /* n_banks multiscale colour banks, each level accepted as by
                                     mdn_plan_create (float16 7x7/7x7 levels on the column walk,
                                     the levels of the tiled kernel with one launch per level and
                                     tick, among them the paper's 4096-bucket configuration); the
                                     descriptors and thresholds are copied, the coefficient buffers
                                     must stay valid while the server lives */
    int32_t n_banks;              /* 1..16 */
    int32_t storage;              /* pyramid dtype (float16 requests need MDN_F16) */
    int32_t max_slots;            /* requests admitted at once, 1..256 */
    int32_t stages_per_tick;      /* >= 1 */
    int32_t max_ticks_in_flight;  /* 1..8 */
    int32_t executor;             /* mdn_executor_kind */
    int32_t reserved[2];          /* must be zero */
    uint64_t hbm_budget;          /* device bytes for admitted requests, allocated once at creation */
    uint64_t staging_bytes;       /* pinned host bytes per slot for requests without host_out (0: none) */
    double queue_timeout;         /* seconds a request may wait for admission; <= 0: no limit */
    /* MDN_EXEC_FAKE only: virtual-clock cost model (0 or negative: defaults 25, 25, 20, 5) */
    double fake_h2d_gbps, fake_d2h_gbps, fake_gpx_per_s, fake_launch_us;
} mdn_server_config;

typedef struct mdn_request {
    const void* host_in;   /* planar RGB [3][height][width] in dtype, [0,1] scale; read until the
                              request's upload is done (pinned memory gives asynchronous copies) */
    void* host_out;        /* same layout and dtype, or NULL: the slot's staging buffer */
    int32_t width, height;
    int32_t dtype;         /* MDN_F16 or MDN_F32 */
    int32_t bank;          /* index into the server's banks */
    uint64_t tag;          /* caller's, returned in the completion (replay: ignored) */
} mdn_request;

typedef struct mdn_completion {
    uint64_t id, tag;
    int32_t status;        /* MDN_OK, MDN_EDEVICE, MDN_ETIMEOUT, MDN_ECANCELED, or the rejection */
    int32_t slot;          /* slot held while admitted (-1 if never admitted) */
    int32_t tick_first, tick_last;   /* ticks that ran its first and last stages (-1: none) */
    /* seconds on the server clock (negative: did not happen); device_done is when the host saw
       the tick with the last stage finish, host_done when it saw the copy back finish */
    double t_arrival, t_admit, t_device_done, t_host_done;
    void* host_out;        /* where the result is, NULL unless status is MDN_OK; a slot's staging
                              buffer stays valid until the next mdn_server_poll call (replay
                              reuses staging buffers at once: give host_out to keep results) */
} mdn_completion;

typedef struct mdn_server_stats {
    uint64_t submitted, admitted, completed, failed, rejected;
    uint64_t ticks, launches, tick_items;    /* tick_items: stages issued over all ticks */
    uint64_t arena_bytes, arena_used, arena_peak;
    int32_t queued, active;
} mdn_server_counters;

/* Create a server; with MDN_EXEC_HIP it allocates the budget, the tables, the staging buffers and
 * three streams (default priority) on the current device. */
mdn_status mdn_server_create(const mdn_server_config* cfg, mdn_server** server);
/* Wait for enqueued device work, then free everything; requests still queued or running are
 * dropped without completions. */
mdn_status mdn_server_destroy(mdn_server* server);

/* Queue a request (arrival time = now). Rejected at once, with nothing queued, when invalid
 * (MDN_EINVAL / MDN_ENOTSUP) or when its footprint exceeds the whole budget (MDN_ENOMEM). */
mdn_status mdn_server_submit(mdn_server* server, const mdn_request* req, uint64_t* id);
/* Cancel by id: a waiting request completes with MDN_ECANCELED at the next poll; a running one
 * stops being scheduled and completes with MDN_ECANCELED once its work in flight is done; one
 * whose last stage is already issued completes normally. */
mdn_status mdn_server_cancel(mdn_server* server, uint64_t id);
/* Advance the schedule for up to max_wait seconds (virtual seconds with MDN_EXEC_FAKE) or until a
 * completion is ready or nothing is left, then return up to max_out completions. */
mdn_status mdn_server_poll(mdn_server* server, double max_wait, mdn_completion* out, int32_t max_out,
                           int32_t* n_out);
/* Open-loop trace: request i is submitted at arrival[i] seconds after the call (non-decreasing)
 * by an arrival thread while the calling thread runs the schedule; returns when all n are
 * complete, out[i] being request i's completion (rejections included). Needs an idle server. */
mdn_status mdn_server_replay(mdn_server* server, const mdn_request* reqs, const double* arrival, int32_t n,
                             mdn_completion* out);
mdn_status mdn_server_stats(mdn_server* server, mdn_server_counters* out);
mdn_status mdn_server_now(mdn_server* server, double* seconds);
/* Device bytes the request would hold while admitted: input and output (each rounded up to 256
 * bytes) plus its pyramid levels (rows padded to 64 elements) and one selector map per level. */
mdn_status mdn_server_footprint(mdn_server* server, const mdn_request* req, uint64_t* bytes);

/* MDN_EXEC_FAKE only: move the virtual clock forward to t, and force failures or delays on the
 * request with the given tag (upload, launch, asynchronous tick failure, copy back, or a stall of
 * `value` seconds added to the tick that holds its next stage). */
typedef enum {
    MDN_FAKE_FAIL_UPLOAD = 0,
    MDN_FAKE_FAIL_LAUNCH = 1,
    MDN_FAKE_FAIL_TICK = 2,
    MDN_FAKE_FAIL_DOWNLOAD = 3,
    MDN_FAKE_STALL = 4
} mdn_fake_injection;
mdn_status mdn_server_fake_advance(mdn_server* server, double t);
mdn_status mdn_server_fake_inject(mdn_server* server, int32_t what, uint64_t tag, double value);

/* Thread-local description of the last non-OK status (empty string if none). */
const char* mdn_last_error(void);

/* Library version string. */
const char* mdn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MDN_H */
