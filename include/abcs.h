/*
 * abcs.h - C ABI of the MI355X (gfx950) adaptive block compressive sensing
 * library: AL-DCT-BBV / AL-DCT-DD / L-DCT-ZZ sensing with per-block DCT
 * coefficient budgets, the masked inverse 2D-DCT decoder, and IDA
 * post-processing.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers named d_* are device pointers (HIP global memory on the device
 *    the plan was created on); pointers named h_* are host pointers.  The
 *    caller owns and allocates every buffer; the library never frees caller
 *    memory.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *    that takes a stream only enqueues work on it and returns without waiting
 *    for the device (abcs_time_splits, the launch tuner's measurement, is the
 *    one exception).
 *  - Every call returns an abcs_status.  Arguments are checked on the host
 *    before anything is enqueued; on an error return no device memory has
 *    been written and abcs_last_error() describes the problem.  A failed HIP
 *    launch returns ABCS_EHIP.  Nothing throws or aborts across this ABI.
 *  - Thread safety: plans are immutable after creation and may be used from
 *    several host threads; calls that overlap on the device must not share
 *    output buffers.  One exception: a plan whose largest image has more
 *    than 8192 and at most 131,072 blocks owns device memory that
 *    abcs_budget and abcs_encode write (the apportionment's per-image tables
 *    for its images of more than 8192 blocks), so those calls on one such
 *    plan must not overlap on the device.  The launch table
 *    (abcs_set_launch_table) is one per process.
 *
 * Geometry (eq 20; Alg 1 and Alg 2 step 1): an H x W image is cropped to
 * H' = B floor(H/B) rows and W' = B floor(W/B) columns and cut into
 * n_B = (H'/B)(W'/B) blocks numbered in raster order.  The cropped image
 * holds N = H' W' pixels and the image's measurement budget is
 * M = floor(C_R N) with C_R the subrate and C_F = N / M the compression factor.
 *
 * Batch layout: per-block arrays (k, offsets, stat) hold the blocks of image
 * 0, then image 1, ...; y holds every block's DCT coefficients in zigzag order,
 * block after block and image after image; decoded images are H' x W' float32
 * arrays with row pitch W', stored one after the other.  abcs_plan_create
 * computes these offsets.
 */
#ifndef ABCS_H
#define ABCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Budget rule for an image. */
typedef enum abcs_method {
  ABCS_ZZ = 0,  /* L-DCT-ZZ: floor(B^2 C_R) lowest zigzag coefficients per
                   block (Section IV; eq 26).                                */
  ABCS_BBV = 1, /* AL-DCT-BBV (Algorithm 1; eqs 16-19, 21, 22).  Needs
                   C_R <= 0.5 (L = floor(C_F) >= 2); with n_S = floor(B/L) = 0
                   it reverts to L-DCT-ZZ.                                   */
  ABCS_DD = 2   /* AL-DCT-DD (Algorithm 2; eq 23; Table 1).                  */
} abcs_method;

typedef enum abcs_status {
  ABCS_OK = 0,
  ABCS_EINVAL = -1,      /* bad argument: null pointer, size, alignment     */
  ABCS_EDOMAIN = -2,     /* parameters outside the method's domain          */
  ABCS_EUNSUPPORTED = -3,/* valid but not supported by this build (e.g. B)  */
  ABCS_ENOSPACE = -4,    /* a caller buffer or workspace is too small       */
  ABCS_EHIP = -5         /* a HIP runtime call or kernel launch failed      */
} abcs_status;

/* IDA denoisers (Section VI-4). */
typedef enum abcs_denoiser {
  ABCS_DENOISE_IDENTITY = 0, /* D(v) = v: the loop without a denoiser        */
  ABCS_DENOISE_BM3D = 1,     /* plain BM3D (Dabov et al., ref [22])          */
  ABCS_DENOISE_CNN = 2,      /* learned 8-layer 3x3 CNN; parameters: the
                                weight blob (abcs_cnn_param_count floats)
                                followed by the accepted noise range
                                [lo, hi] (2 floats, hi may be +inf)         */
  ABCS_DENOISE_DNCNN = 3     /* DnCNN-17 with batch normalisation (Section
                                VI-4); parameters: the blob, the running
                                statistics (abcs_dncnn_*_count), then the
                                accepted noise range [lo, hi]               */
} abcs_denoiser;

/* Sensing transform of an image (Section IV): the 2-D DCT-II, or the 2-D
 * Walsh-Hadamard transform the paper names as the simpler alternative
 * ({+1, -1} / sqrt(B) entries, rows in sequency order, so that the zigzag scan
 * runs from low to high sequency).  DD's phase-1 coefficients are those of
 * the image's transform. */
typedef enum abcs_transform {
  ABCS_DCT = 0,
  ABCS_WHT = 1
} abcs_transform;

/* Arithmetic of the DCT transforms (B = 8, 16 and 32) in abcs_sense,
 * abcs_reconstruct, abcs_sense_decode and abcs_encode (Walsh-Hadamard images
 * always use the float32 matrix cores: their forward transform is exact
 * there).  The 16-bit modes run on the matrix cores with float32 sums; the
 * "x3" modes split each operand that is not exact in 16 bits into a high and a
 * low part and keep every product but low x low (about float32 accuracy); the
 * single-pass modes round the operands once.  Budgets (abcs_budget) never
 * depend on the mode.                                                        */
typedef enum abcs_precision {
  ABCS_FP32 = 0,
  ABCS_BF16X3 = 1,
  ABCS_FP16X3 = 2,
  ABCS_BF16 = 3,
  ABCS_FP16 = 4
} abcs_precision;

/* One image of a batch.  The caller fills the first block of fields;
 * abcs_plan_create fills the layout fields of its own copy, which
 * abcs_plan_image returns. */
typedef struct abcs_image {
  int32_t height;        /* H, rows of the uncropped image                   */
  int32_t width;         /* W, columns of the uncropped image                */
  int32_t row_pitch;     /* bytes between rows of the uint8 pixels; >= W,
                            multiple of 4                                    */
  int32_t block;         /* B: 8, 16 or 32                                   */
  double subrate;        /* C_R in (0, 1]                                    */
  int32_t method;        /* abcs_method                                      */
  int32_t transform;     /* abcs_transform (0: DCT)                          */
  int64_t pixel_offset;  /* byte offset of pixel (0,0) in the pixel buffer;
                            multiple of 4.  Several descriptors may name the
                            same pixels (e.g. one image at several C_R).      */
  /* ---- filled by abcs_plan_create ---- */
  int64_t block_offset;  /* first block of this image in per-block arrays    */
  int64_t meas_offset;   /* first coefficient of this image in y             */
  int64_t out_offset;    /* first pixel of this image in decoded buffers     */
  int64_t n_meas;        /* DCT coefficients this image puts in y:
                            ZZ: n_B floor(B^2 C_R); BBV: M - M_BBV; DD: M    */
  int32_t cropped_height;/* H'                                               */
  int32_t cropped_width; /* W'                                               */
  int64_t bbv_offset;    /* first BBV sample of this image (abcs_bbv_samples) */
  int64_t n_bbv;         /* BBV samples: 2 n_S n_B + n_S (n_bx + n_by) for an
                            adaptive BBV image, else 0                       */
} abcs_image;

typedef struct abcs_plan abcs_plan; /* opaque */

/* Validate a batch, compute its layout and upload every device table any call
 * on the plan needs (descriptors, tile lists, the denoisers' reference grids
 * and tiles, the bounds' tables) to the current HIP device in one allocation
 * and one copy.  Plan creation and destruction are the only calls that
 * allocate device memory or wait for the device (the first plan on a device
 * also uploads the library's constant tables); every other call only
 * enqueues kernels.
 * h_imgs: n descriptors (n >= 0), read only.  On success *out receives a plan
 * that must be released with abcs_plan_destroy.
 * Errors: EINVAL (null pointer, n < 0, pitch/offset/alignment), EDOMAIN
 * (C_R outside (0,1], no whole block, M = 0, BBV with C_R > 0.5, BBV samples
 * exceeding M), EINVAL (unknown transform), EUNSUPPORTED (B not 8, 16 or
 * 32), EHIP.  Sensing and the inverse transform run on the matrix cores for
 * every B; the DD statistics and the IDA transform step of B = 8 and 32 run
 * on the vector ALUs (same results and error bars for every B: budgets and
 * index sets exact, DD statistics evaluated in float64). */
int abcs_plan_create(const abcs_image* h_imgs, int n, abcs_plan** out);
/* abcs_plan_create with a choice of tables: the tables of the encoder and the
 * decoder (budget, sense, reconstruct, encode, the identity-denoiser IDA
 * loop, BBV samples, correlation) are always built; ABCS_PLAN_DENOISE adds
 * those of the denoisers (BM3D reference grids, CNN tiles, the per-64-pixel
 * image map: needed by every non-identity denoiser, amp_refine and the
 * training steps) and ABCS_PLAN_BOUNDS those of abcs_threshold.  A call that
 * needs a table the plan lacks returns EINVAL.  abcs_plan_create builds all
 * of them; a stream of encode-only batches saves their host work and device
 * memory (about 1 + 12 / B^2 bytes per pixel for the bounds' tables, and
 * most of the plan's creation time for large batches). */
typedef enum abcs_plan_feature { ABCS_PLAN_DENOISE = 1, ABCS_PLAN_BOUNDS = 2 } abcs_plan_feature;
int abcs_plan_create_ex(const abcs_image* h_imgs, int n, unsigned features, abcs_plan** out);
void abcs_plan_destroy(abcs_plan* plan);

/* Totals of a plan: number of blocks (length of k, offsets, stat), number of
 * DCT coefficients (length of y) and decoded pixels (length of an image
 * buffer).  Any pointer may be NULL. */
int abcs_plan_totals(const abcs_plan* plan, int64_t* h_blocks, int64_t* h_meas,
                     int64_t* h_pixels);
/* The totals one descriptor would add to a plan (blocks, coefficients in y,
 * decoded pixels), with the same validation and errors as abcs_plan_create
 * and nothing else: host only, no device, no allocation.  For admission
 * control: a request's device bytes follow from these before any plan is
 * made. */
int abcs_image_totals(const abcs_image* h_img, int64_t* h_blocks, int64_t* h_meas, int64_t* h_pixels);
/* Copy descriptor i, with its layout fields filled, into *h_out. */
int abcs_plan_image(const abcs_plan* plan, int i, abcs_image* h_out);

/* Phase 1 and budget estimation (Alg 1 steps 2-3; Alg 2 steps 2-4).
 * d_px:      uint8 pixels, px_bytes long; every image's cropped region must
 *            lie inside it (checked against px_bytes).
 * d_k:       out, int32[blocks]: DCT coefficients to sense from each block, the
 *            length of its zigzag prefix.  BBV: m_i^2 of eq 22; DD: m^1 + m_i^2
 *            (eq 23); ZZ: floor(B^2 C_R).
 * d_offsets: out, int64[blocks]: block i's coefficients are
 *            y[offsets[i] .. offsets[i] + k[i]) (exclusive prefix sum of k
 *            within each image, plus the image's meas_offset).
 * d_stat:    out, int32[blocks]: BBV_i (eq 19) or n_i (count of the first m^1
 *            zigzag coefficients with |c| > T); 0 for ZZ.
 * Budgets are exact integers: shares are floor(P w_i / S) of the pool P; a
 * block whose share reaches its cap (B^2 - m^1) is fixed at the cap and the
 * rest is re-split; the final leftover goes to the largest remainders
 * (P w_i mod S), ties to the lower block index; all-zero weights split
 * uniformly.  DD's |c| > T decisions are those of the float64 DCT computed in
 * the fixed order T = X D^T then D T, sums ascending, no fused multiply-add. */
int abcs_budget(const abcs_plan* plan, const uint8_t* d_px, int64_t px_bytes,
                int32_t* d_k, int64_t* d_offsets, int32_t* d_stat, void* stream);

/* Phase 2 sensing (Alg 1 step 4; Alg 2 step 5): y[offsets[i] + z] =
 * C_i[zigzag[z]] for z < k[i], where C_i = D X_i D^T is block i's orthonormal
 * 2D DCT-II of the raw [0, 255] pixels, computed in `precision`
 * (abcs_precision; EINVAL for other values).
 * d_y: out, float[meas]. */
int abcs_sense(const abcs_plan* plan, const uint8_t* d_px, int64_t px_bytes,
               const int32_t* d_k, const int64_t* d_offsets, float* d_y, int precision, void* stream);

/* Real-time decoder (Fig 1, I_o): zero-fill each block's unmeasured
 * coefficients and apply the inverse 2D DCT X = D^T C D, computed in
 * `precision` (abcs_precision).
 * Needs only y, k and offsets (the side information), never pixels.
 * d_out: out, float[pixels], each image H' x W' with row pitch W'. */
int abcs_reconstruct(const abcs_plan* plan, const float* d_y, const int32_t* d_k,
                     const int64_t* d_offsets, float* d_out, int precision, void* stream);

/* The whole encoder of Algorithms 1 and 2 in one call, with the decoder's
 * image alongside: abcs_budget (phase-1 statistics, apportionment, offsets),
 * then abcs_sense, then, when d_out is not NULL, the image abcs_reconstruct
 * would decode from the same y (an encoder's local decoder, as in the
 * real-time system of Fig 1).  The decoder takes the coefficients from the
 * forward transform instead of reading y back, with the same arithmetic as
 * abcs_reconstruct, so d_out equals abcs_reconstruct's output bit for bit.
 * When every image of the plan is a 16 x 16 DCT image of at most 1024
 * blocks, precision is float32, d_out is not NULL and d_ws holds
 * abcs_encode_workspace_bytes(plan) bytes (0 for other plans; its contents on
 * entry do not matter), everything runs in one launch (after a fill of the
 * workspace): statistics, each image's apportionment as soon as its
 * statistics are complete, then sensing and decoding of its tiles, one work
 * item per workgroup in one ticket order that always makes progress (word 1
 * of the workspace is set if a tile ever gave up waiting for its budgets; it
 * never should).  Otherwise (d_ws NULL included) the budget runs as its own
 * launches and sensing with decoding as one more, and d_ws is not used.
 * Both give the same bits.  The one launch is the slower of the two on a
 * batch that fills the chip (0.44 ms against 0.29 ms for 640 encodings of
 * 512 x 512): each image's statistics must be published across the chip's
 * XCDs, whose L2 caches are not coherent, and the fences that do this write
 * back or invalidate a whole L2; between two launches this happens once.
 * Arguments and errors as the three calls; d_out nullable, float[pixels],
 * 16-byte aligned; d_ws nullable, 4-byte aligned. */
size_t abcs_encode_workspace_bytes(const abcs_plan* plan);
int abcs_encode(const abcs_plan* plan, const uint8_t* d_px, int64_t px_bytes, int32_t* d_k,
                int64_t* d_offsets, int32_t* d_stat, float* d_y, float* d_out, int precision, void* d_ws,
                size_t ws_bytes, void* stream);
/* The second half of abcs_encode on its own (budgets already in d_k and
 * d_offsets): abcs_sense and the decoder's image in d_out (not NULL).  Each
 * tile is sensed and decoded in one pass (the coefficients stay in registers
 * between the forward and the masked inverse transform) for B = 8 and 32 in
 * every precision and B = 16 in ABCS_FP32; B = 16 in a 16-bit mode runs the
 * two kernels of abcs_sense and abcs_reconstruct.  Results equal those two
 * calls' bit for bit. */
int abcs_sense_decode(const abcs_plan* plan, const uint8_t* d_px, int64_t px_bytes, const int32_t* d_k,
                      const int64_t* d_offsets, float* d_y, float* d_out, int precision, void* stream);

/* Launch tuning (not part of the method: how its sensing and decoding
 * kernels are spread over the chip).  Those kernels give each tile (up to 16
 * horizontally adjacent blocks of one image) to one wavefront; a split s in
 * {0, 1, 2} gives it to 2^s wavefronts of 16 / 2^s blocks each, which fills
 * the chip's 1024 SIMDs better when a batch has few tiles and costs a little
 * per-wave set-up on large ones.  Results never depend on the split.  The
 * library keeps one split per (block size, transform, precision, size class),
 * the size class of a launch being that of its tile count: 0 below 256
 * tiles, 1 below 2048, 2 below 16384, 3 above (Walsh-Hadamard launches are
 * float32 and use the ABCS_FP32 entry).  All splits are 0 until a table is
 * set (the Python binding sets the table measured for this build, if one is
 * stored); the table is global to the process and read by every launch of
 * abcs_sense, abcs_reconstruct, abcs_sense_decode and abcs_encode. */
typedef struct abcs_launch_entry {
  int32_t block;       /* 8, 16 or 32 */
  int32_t transform;   /* abcs_transform */
  int32_t precision;   /* abcs_precision */
  int32_t size_class;  /* 0 .. 3 */
  int32_t split;       /* 0 .. 2 */
} abcs_launch_entry;
/* Replace the table: every split not named in entries[0..n) becomes 0 (n = 0
 * resets).  EINVAL on an entry out of range (the table is then unchanged). */
int abcs_set_launch_table(const abcs_launch_entry* entries, int n);
/* The split in force for a launch kind (>= 0), or EINVAL. */
int abcs_launch_split(int block, int transform, int precision, int size_class);
/* Size class of the plan's tiles of one kind, -1 if the plan has none, or
 * EINVAL. */
int abcs_plan_size_class(const abcs_plan* plan, int block, int transform);
/* The tuner's measurement: abcs_sense_decode on the plan (arguments as
 * there; budgets already in d_k and d_offsets) with every launch forced to
 * split s, for s = 0, 1, 2: one warm-up call, then reps timed calls between
 * two events on `stream`; h_ms[s] receives the mean milliseconds per call.
 * Waits for the device; no other call may use the library while it runs
 * (the forced split is process-wide). */
int abcs_time_splits(const abcs_plan* plan, const uint8_t* d_px, int64_t px_bytes, const int32_t* d_k,
                     const int64_t* d_offsets, float* d_y, float* d_out, int precision, int reps, float* h_ms,
                     void* stream);
/* Identity of this build: a hash of the library's sources (their code,
 * comments left out) and compiler flags, under which tuning results are
 * stored. */
const char* abcs_build_id(void);

/* IDA post-processing (Section VI; eqs 13, 15, 25, 28; Fig 6).
 * Starting from x^0 = 0 and z^{-1} = 0, iteration t = 0 .. iters-1 computes
 *   z^t       = y - A x^t + z^{t-1} / D_F
 *   sigma^t   = ||z^t||_2 / sqrt(m)            (per image, m = its n_meas)
 *   x^{t+1}   = D_{sigma^t}(x^t + A* z^t)
 * where A is the block-diagonal zigzag-DCT sensing operator of eq 26 (the
 * first k_i DCT basis functions of block i in zigzag order) and D the chosen
 * denoiser.  Decoder side: needs only y, k, offsets and the plan's geometry.
 * d_x:           out, float[pixels]: x^iters, each image H' x W' (row pitch W'),
 *                16-byte aligned.  Nothing is clipped.
 * d_sigma_trace: out, nullable, float[iters * n]: sigma^t of image i at
 *                t * n + i.
 * damping:       D_F >= 1 (D_F = 1 is undamped; +inf gives z^{t-1} weight 0).
 * denoiser:      abcs_denoiser; d_params its parameters (NULL unless CNN).
 * d_ws:          workspace of at least ida_workspace_bytes(plan, denoiser)
 *                bytes, 256-byte aligned; overwritten.
 * Errors: EINVAL, EDOMAIN (D_F < 1 or NaN), EUNSUPPORTED (denoiser not
 * built, or the CNN on a plan with an image whose W' is not a multiple of 16
 * or H' of 8 (possible with B = 8) or that has 2^24 pixels or more),
 * ENOSPACE (workspace too small), EHIP. */
size_t ida_workspace_bytes(const abcs_plan* plan, int denoiser);
/* Resumable form: runs iterations t = t_begin .. t_end-1 of the same loop.
 * t_begin = 0 starts from x^0 = 0 and z^{-1} = 0; t_begin > 0 continues from
 * the x^{t_begin} in d_x and the residual state left in d_ws by the call that
 * ran iteration t_begin - 1 (same plan, y, k, offsets, damping, denoiser).
 * d_sigma_trace (nullable) receives (t_end - t_begin) * n values; d_v_last
 * (nullable, float[pixels]) receives v^{t_end-1} = x + A* z, the denoiser's
 * input of the last iteration.  ida_refine(iters) = ida_iterate(0, iters). */
int ida_iterate(const abcs_plan* plan, const float* d_y, const int32_t* d_k, const int64_t* d_offsets,
                int t_begin, int t_end, double damping, int denoiser, const void* d_params, float* d_x,
                float* d_sigma_trace, float* d_v_last, void* d_ws, size_t ws_bytes, void* stream);
int ida_refine(const abcs_plan* plan, const float* d_y, const int32_t* d_k, const int64_t* d_offsets,
               int iters, double damping, int denoiser, const void* d_params, float* d_x,
               float* d_sigma_trace, void* d_ws, size_t ws_bytes, void* stream);

/* ida_refine for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same loop and results, with its workspace taken from a fixed scratch array
 * that the library holds on each device it runs on (ida_noalloc_scratch_bytes()
 * = 64 MiB per device, held until the process ends) instead of d_ws.  The
 * call allocates nothing and copies nothing from the host; the caller still
 * owns y, k, offsets, x and the trace.  Every call on a device shares that
 * device's scratch, which keeps the last call's contents (the loop
 * initialises everything it reads), so calls that overlap on one device race:
 * serialise them (one stream, or events).
 * Errors: those of ida_refine, and ENOSPACE when ida_workspace_bytes(plan,
 * denoiser) exceeds the scratch (the CNN needs about 260 bytes per pixel,
 * BM3D about 44, the identity about 8 plus 12 per coefficient). */
size_t ida_noalloc_scratch_bytes(void);
int ida_refine_noalloc(const abcs_plan* plan, const float* d_y, const int32_t* d_k, const int64_t* d_offsets,
                       int iters, double damping, int denoiser, const void* d_params, float* d_x,
                       float* d_sigma_trace, void* stream);

/* The signed BBV samples (Section V-A: the encoder measures them for eq 19
 * and may send them as extra reconstruction measurements): each is
 * d = I[a] - I[b] for two adjacent pixels on a block border, a the later one
 * along the border.  Per BBV image, at its bbv_offset: for each block in
 * raster order its n_S top-row then n_S left-column samples; then the n_S
 * bottom-row samples of each block of the last block row; then the n_S
 * right-column samples of each block of the last block column.
 * d_samples: out, float[sum of n_bbv] (exact integers).  Errors as
 * abcs_budget. */
int abcs_bbv_samples(const abcs_plan* plan, const uint8_t* d_px, int64_t px_bytes, float* d_samples,
                     void* stream);

/* ida_refine with the BBV samples as extra rows of A: every sample adds the
 * row (e_a - e_b) / sqrt 2 with measurement d / sqrt 2, so its residual joins
 * z^t (eqs 25, 28), A* adds it back to the two pixels (eq 13) and m of eq 15
 * counts the samples.  Images that are not adaptive BBV images run as in
 * ida_refine.  d_bbv: float[sum of n_bbv] as written by abcs_bbv_samples.
 * Other arguments, workspace and errors as ida_refine. */
int ida_refine_bbv(const abcs_plan* plan, const float* d_y, const int32_t* d_k, const int64_t* d_offsets,
                   const float* d_bbv, int iters, double damping, int denoiser, const void* d_params, float* d_x,
                   float* d_sigma_trace, void* d_ws, size_t ws_bytes, void* stream);

/* D-AMP and DAMP-D (eqs 13-15 with the Onsager coefficient of eq 24, or its
 * damped form eq 27), the algorithms IDA is derived from.  Same loop as
 * ida_refine, but the weight of z^{t-1} is, per image,
 *   alpha^t = div D_{sigma^{t-1}}(v^{t-1}) / m          (ABCS_ALGO_DAMP)
 *   alpha^t = div D_{sigma^{t-1}}(v^{t-1}) / (m D_F)    (ABCS_ALGO_DAMP_D)
 * with alpha^0 = 0.  (Eq 14 prints both 1/delta and /m; the AMP correction it
 * generalises, (1/delta) times the mean derivative over the N pixels, is
 * div / m.)  The divergence is estimated as in ref [13]:
 * b . (D(v + eps b) - D(v)) / eps with eps = max|v| / 1000 per image (1e-3
 * when v is 0): one more denoiser call per iteration.
 * d_probe:       in, float[pixels] (plan layout): the probe b, normally
 *                standard normal values; the caller draws it; it is reused at
 *                every iteration.
 * d_alpha_trace: out, nullable, float[iters * n]: alpha^t of image i at
 *                t * n + i.
 * damping:       D_F >= 1 (DAMP-D only; +inf gives alpha = 0).
 * d_ws:          amp_workspace_bytes(plan, denoiser) bytes, 256-byte aligned.
 * Other arguments and errors as ida_refine. */
typedef enum abcs_algorithm { ABCS_ALGO_DAMP = 1, ABCS_ALGO_DAMP_D = 2 } abcs_algorithm;
size_t amp_workspace_bytes(const abcs_plan* plan, int denoiser);
int amp_refine(const abcs_plan* plan, const float* d_y, const int32_t* d_k, const int64_t* d_offsets, int iters,
               double damping, int algorithm, int denoiser, const void* d_params, const float* d_probe,
               float* d_x, float* d_sigma_trace, float* d_alpha_trace, void* d_ws, size_t ws_bytes,
               void* stream);

/* The IDA loop as a replayable HIP graph: ida_graph_create records the
 * launches of ida_refine(plan, d_y, d_k, d_offsets, iters, damping, denoiser,
 * d_params, d_x, d_sigma_trace, d_ws, ws_bytes) into one instantiated graph
 * (stream capture; every node is a kernel), and each ida_graph_launch replays
 * the whole T-iteration loop on `stream` with one call.  The buffers named at
 * creation are the ones every replay reads and writes; the caller keeps them
 * (and the plan) alive and unchanged in size until ida_graph_destroy.  A replay
 * gives the same result as ida_refine with the same arguments.
 * Errors: as ida_refine, plus EHIP when capture or instantiation fails (no
 * graph is returned then). */
typedef struct abcs_ida_graph abcs_ida_graph;
int ida_graph_create(const abcs_plan* plan, const float* d_y, const int32_t* d_k, const int64_t* d_offsets,
                     int iters, double damping, int denoiser, const void* d_params, float* d_x,
                     float* d_sigma_trace, void* d_ws, size_t ws_bytes, abcs_ida_graph** out);
int ida_graph_launch(abcs_ida_graph* graph, void* stream);
void ida_graph_destroy(abcs_ida_graph* graph);

/* Apply an IDA denoiser D_sigma to every image of a plan (the step
 * x^{t+1} = D_sigma(v^t) of ida_refine, exposed on its own).
 * d_in, d_out: float[pixels], each image H' x W' with row pitch W', 16-byte
 *              aligned; must not alias except for the identity.
 * d_sigma:     float[n], the noise level of each image (sigma <= 0 returns the
 *              image unchanged).
 * BM3D follows Dabov et al. (ref [22]) with 8x8 patches, step 3, 39x39
 * search, groups of at most 16 / 32 (thresholds 2500 / 400 on ||P-Q||^2/64),
 * 8x8 DCT + Haar 3D transform, hard threshold 2.7 sigma, Wiener second stage,
 * Kaiser (beta 2) aggregation; results are bit-identical from run to run.
 * The learned denoisers (parameters in d_params: the weights, then the range
 * [lo, hi] of sigma whose network input the training covered: the sigma
 * channel is min(sigma, 255) / 255, so a network trained on noise up to 255
 * or more accepts every larger sigma, hi = +inf) fall back to BM3D for every
 * image whose sigma lies outside [lo, hi] (NaN included) or whose network
 * output holds a non-finite value; the decision is taken on the device, and
 * BM3D's kernels skip the other images.  A NaN sigma gives a NaN image.
 * d_ws: workspace of abcs_denoise_workspace_bytes(plan, denoiser) bytes,
 * 256-byte aligned (NULL allowed when that is 0). */
size_t abcs_denoise_workspace_bytes(const abcs_plan* plan, int denoiser);
/* Number of float32 values in the CNN parameter blob (223361).  The blob
 * holds, layer after layer (2->64, six 64->64, 64->1 channels, 3x3 kernels),
 * the weights [C_out][3][3][C_in] followed by the biases [C_out].  The
 * network maps an image v and its noise level sigma to
 * v - 255 f([v/255, min(sigma,255)/255]); ReLU after layers 1..7, zero
 * padding; weights and activations are rounded to bfloat16, sums are float32.
 * A stand-in for the paper's DnCNN (Section VI-4), whose weights are not
 * available; trained with abcs_cnn_train_step. */
size_t abcs_cnn_param_count(void);

/* One training step of the CNN on a batch described by a plan (its images'
 * geometry only: method, subrate and pixel fields are not used).
 * d_input, d_target: float[pixels] (plan layout) network input v and the
 *                    clean image; d_sigma: float[n] noise level per image.
 * Loss: mean over all pixels of ((D(v) - target) / 255)^2, written to
 * d_loss[0].  Gradients of the loss w.r.t. every parameter (bfloat16
 * activations, float32 sums, fixed summation order) are written to d_grad
 * (float[param_count], nullable).  When lr > 0, Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias correction for `step` >= 1) updates d_params (float32 master
 * weights) with moments d_adam_m, d_adam_v (float[param_count], zero before
 * the first step).  d_ws: abcs_cnn_train_workspace_bytes(plan) bytes. */
size_t abcs_cnn_train_workspace_bytes(const abcs_plan* plan);
int abcs_cnn_train_step(const abcs_plan* plan, float* d_params, float* d_adam_m, float* d_adam_v, int64_t step,
                        float lr, const float* d_input, const float* d_sigma, const float* d_target,
                        float* d_loss, float* d_grad, void* d_ws, size_t ws_bytes, void* stream);
int abcs_denoise(const abcs_plan* plan, int denoiser, const void* d_params, const float* d_in,
                 const float* d_sigma, float* d_out, void* d_ws, size_t ws_bytes, void* stream);

/* Full-sensing bounds (Section IV; Section V-C).  Every DCT coefficient of
 * every block is measured and M = floor(C_R N) of them (N = H'W', C_R the
 * image's subrate) are kept; the image's method field is not used.
 *   ABCS_THI: the M coefficients of largest magnitude over the whole image
 *             (one threshold per image), the best any adaptive 2-D DCT
 *             scheme with M coefficients can do in error energy;
 *   ABCS_THB: the floor(M / n_B) largest of every block (one threshold per
 *             block, the same count in each).
 * Magnitudes are compared on float64 coefficients computed in the fixed
 * order T[r][v] = sum_j X[r][j] D[v][j], C[u][v] = sum_r D[u][r] T[r][v]
 * (ascending indices, no fused multiply-add), so the kept set is exactly that
 * definition's.  Ties in magnitude go to the lower block index (raster
 * order), then the lower zigzag rank.
 * d_px:  pixels as for abcs_budget (px_bytes >= the plan's extent).
 * d_m:   out, int32[blocks] (plan block order): coefficients kept per block.
 * d_out: out, nullable, float[pixels] (plan layout, 16-byte aligned): inverse
 *        DCT of the kept coefficients, the others zero (float32 transform).
 * d_ws:  abcs_threshold_workspace_bytes(plan) bytes (12 per pixel, 4 per
 *        block and about 16 KiB per image), 256-byte aligned; its contents on
 *        entry do not matter.
 * Errors: EINVAL (unknown rule, null or misaligned buffer), ENOSPACE (pixel
 * buffer or workspace too small), EUNSUPPORTED (an image of 2^29 pixels or
 * more, or a Walsh-Hadamard image: the bounds are the DCT's), EHIP. */
typedef enum abcs_threshold_rule { ABCS_THI = 1, ABCS_THB = 2 } abcs_threshold_rule;
size_t abcs_threshold_workspace_bytes(const abcs_plan* plan);
int abcs_threshold(const abcs_plan* plan, const uint8_t* d_px, int64_t px_bytes, int rule, int32_t* d_m,
                   float* d_out, void* d_ws, size_t ws_bytes, void* stream);

/* Pearson's correlation rho between two per-block counts over the blocks of
 * each image (Table 2 correlates THI's m_i with the budgets an adaptive rule
 * estimates), and the probability p of the null hypothesis rho = 0 that
 * Section V-C reports: two-sided Student t test, t = rho sqrt(nu / (1 -
 * rho^2)), nu = n_B - 2, p = I_{1-rho^2}(nu/2, 1/2) (regularised incomplete
 * beta function, continued fraction; relative error ~1e-13).
 * d_m, d_m_hat: int32[blocks]; d_rho: out, double[n], NaN for an image where
 * either count is constant; d_p: out, nullable, double[n] (NaN where rho is
 * or n_B < 3).  rho is computed from exact integer moments.
 * Errors: EINVAL (null or misaligned buffer), EHIP. */
int abcs_budget_correlation(const abcs_plan* plan, const int32_t* d_m, const int32_t* d_m_hat, double* d_rho,
                            double* d_p, void* stream);

/* DnCNN-17 (Section VI-4): layer 1 3x3 conv 2 -> 64 + bias + ReLU; layers
 * 2..16 3x3 conv 64 -> 64 (no bias) + batch normalisation (gamma, beta) +
 * ReLU; layer 17 3x3 conv 64 -> 1 + bias; the same input [v/255, sigma map]
 * and residual output v - 255 f as the 8-layer network, bfloat16 weights and
 * activations, float32 sums.  The parameter blob holds W1 [64][3][3][2], b1
 * [64], then per middle layer W [64][3][3][64], gamma [64], beta [64], then
 * W17 [1][3][3][64], b17 (abcs_dncnn_param_count floats).  The running
 * statistics hold per middle layer mean [64] then variance [64]
 * (abcs_dncnn_running_count floats).  As a denoiser (ABCS_DENOISE_DNCNN) the
 * parameter pointer addresses the blob immediately followed by the running
 * statistics and the accepted noise range [lo, hi]; normalisation is folded
 * into the convolutions (inference). */
size_t abcs_dncnn_param_count(void);
size_t abcs_dncnn_running_count(void);

/* One DnCNN training step: forward with batch statistics (mean and biased
 * variance over all pixels of the batch, eps 1e-5, sums in float64), MSE loss
 * as abcs_cnn_train_step, gradients of every parameter (d_grad, nullable,
 * float[param_count]), and, when lr > 0, Adam as abcs_cnn_train_step.
 * d_running (nullable): the running statistics, moved by 0.1 towards the
 * batch statistics.  d_ws: abcs_dncnn_train_workspace_bytes(plan) bytes.
 * Errors as abcs_cnn_train_step. */
size_t abcs_dncnn_train_workspace_bytes(const abcs_plan* plan);
int abcs_dncnn_train_step(const abcs_plan* plan, float* d_params, float* d_adam_m, float* d_adam_v,
                          float* d_running, int64_t step, float lr, const float* d_input, const float* d_sigma,
                          const float* d_target, float* d_loss, float* d_grad, void* d_ws, size_t ws_bytes,
                          void* stream);

/* Where a workspace keeps the values a call leaves behind, for callers that
 * inspect them (the parity tests check each layer of a training step, and
 * BM3D's groups, from these values).  Byte offset and size within the
 * workspace of the given kind for this plan:
 *   ABCS_WS_CNN_TRAIN / ABCS_WS_DNCNN_TRAIN (abcs_cnn_train_step /
 *   abcs_dncnn_train_step):
 *     ACTIVATIONS: bfloat16, the output of every hidden layer after its ReLU
 *                  (7 layers / 16 layers), layer after layer, each
 *                  [pixel][64 channels] with pixels in plan order;
 *     PRENORM:     (DnCNN only) bfloat16, the 15 middle layers' convolution
 *                  outputs before normalisation, same layout;
 *     OUTPUT:      float[pixels], the network output D(v).
 *   ABCS_WS_DENOISE_BM3D (abcs_denoise with ABCS_DENOISE_BM3D):
 *     GROUPS: int32, per reference patch (images in plan order, each image's
 *             references in raster order of the 3-pixel grid) 33 entries: the
 *             member count, then the members' positions y W' + x in group
 *             order; after a call it holds the second (Wiener) stage's groups;
 *     BASIC:  float[pixels], the first stage's estimate.
 * The contents are those of the last call that used the workspace.
 * Errors: EINVAL (null argument, unknown kind or part). */
typedef enum abcs_workspace_kind {
  ABCS_WS_CNN_TRAIN = 1,
  ABCS_WS_DNCNN_TRAIN = 2,
  ABCS_WS_DENOISE_BM3D = 3
} abcs_workspace_kind;
typedef enum abcs_workspace_part_id {
  ABCS_PART_ACTIVATIONS = 1,
  ABCS_PART_PRENORM = 2,
  ABCS_PART_OUTPUT = 3,
  ABCS_PART_GROUPS = 4,
  ABCS_PART_BASIC = 5
} abcs_workspace_part_id;
int abcs_workspace_part(const abcs_plan* plan, int kind, int part, size_t* h_offset, size_t* h_bytes);

/* Host copy of the float64 orthonormal DCT-II basis the library uses,
 * D[u*B + j] = s_u cos((2j+1) u pi / (2B)), for checking.  B in {8, 16, 32}. */
int abcs_dct_basis(int block, double* h_out);

/* Message describing the last error returned on the calling thread. */
const char* abcs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ABCS_H */
