/*
 * libhog355 — HOG sliding-window face detection on AMD Instinct MI355X
 * (gfx950), as a C ABI.
 *
 * The method is the HOG face detector of arXiv 2006.00816, Sec. IV-A
 * ("Algorithm breakdown"): an image pyramid in 5/6 steps down to the
 * 80x80 window, central-difference gradients discretised into 18 signed
 * orientations, 18-bin histograms of 8x8-pixel cells with bilinear votes,
 * normalisation by the energy of neighbouring 2x2-cell blocks into 31
 * features per cell, a linear 10x10x31 filter per face rotation scored at
 * every window, a threshold, and non-maximum suppression.  Sec. V-A
 * describes the paper's GPU kernels for the same steps.
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless the comment says "host".
 *  - The caller owns every buffer, including the workspace `ws`; the
 *    library allocates no device memory in these calls.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and the call returns without waiting for it, except where noted.
 *  - Return value: HOG_OK (0) when the work was enqueued, a negative
 *    HOG_E_* code when the host-side checks rejected the arguments (then
 *    nothing was enqueued).  HOG_E_HIP means a launch failed.  No
 *    exception crosses the ABI.
 *  - Frames are 8-bit grayscale, row-major, `pitch` bytes per row
 *    (w <= pitch <= 65536).  Sides are limited to 80 <= h, w <= 4096; smaller
 *    frames have no pyramid level and yield no detections.
 *  - Filters are float32 [nf][10][10][31] (row, column, channel of the
 *    window), bias float32 [nf].  1 <= nf <= 32.
 *  - Distinct workspaces may be used concurrently from several host
 *    threads and streams; one workspace must not be used by two calls in
 *    flight at the same time.
 */
#ifndef LIBHOG355_H
#define LIBHOG355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOG_OK            0
#define HOG_E_INVAL      -1   /* bad argument (null pointer, bad size, bad option) */
#define HOG_E_TOO_LARGE  -2   /* frame side above 4096 px, or too many filters */
#define HOG_E_WORKSPACE  -3   /* ws_bytes below hog_workspace_bytes() */
#define HOG_E_CAP        -4   /* an output capacity argument is out of range */
#define HOG_E_HIP        -5   /* a HIP launch or runtime call failed */
#define HOG_E_NOTIMPL    -6
#define HOG_E_DEVICE     -7   /* written to n_dets: a bounded device-side wait of the fused kernel
                                 gave up; that frame's detections are not valid */
#define HOG_E_SCRATCH    -8   /* hog_detect_batch_static: the call needs more workspace than
                                 HOG_STATIC_SCRATCH_BYTES */

#define HOG_MAX_SIDE     4096
#define HOG_MAX_FILTERS  32
#define HOG_MAX_LEVELS   28
#define HOG_MAX_DETS     4096 /* largest per-frame detection capacity */
#define HOG_STATIC_SCRATCH_BYTES (64u << 20)  /* fixed workspace of hog_detect_batch_static */

/* Or-ed into an `upsample` argument (or hog_params.upsample): the recursive
 * pyramid of the paper's image-scaling kernel (Sec. V-A: each scaled image
 * is computed from the image one scale higher) instead of resampling every
 * level from the frame.  Level 0 is the frame (upsample 1) or its 2x
 * enlargement rounded to grey levels (upsample 2); level k is the bilinear
 * 5/6 reduction of level k-1 (output pixel i at (12 i + 1) / 10 of the
 * input, weights rounded to 1/256) rounded half up to 8-bit grey levels,
 * of size floor(5 h_{k-1} / 6) x floor(5 w_{k-1} / 6).  Windows map back to
 * the frame with the nominal scale u (5/6)^k as before.  The level images
 * are built in the workspace.  Forward calls only: hog_filter_backward
 * returns HOG_E_NOTIMPL for it. */
#define HOG_PYRAMID_CASCADE 0x100

/* Search region of one frame: only windows of pyramid levels
 * k_lo <= k <= k_hi whose frame-pixel box lies inside the half-open
 * rectangle [x0, x1) x [y0, y1) are candidates.  Sec. VII proposes
 * restricting the scales and locations analysed per frame, as faces move
 * little between consecutive video frames; hog_track_regions derives the
 * next frame's region from this frame's detections.  The whole frame at
 * every level is {0, 0, w, h, 0, HOG_ALL_LEVELS}. */
typedef struct hog_region {
    int32_t x0, y0, x1, y1, k_lo, k_hi;
} hog_region;
#define HOG_ALL_LEVELS (1 << 30)

/* Detection parameters (Sec. IV-A, classification and NMS; Sec. V-A,
 * image sequence with constant size). */
typedef struct hog_params {
    int32_t upsample;  /* 1, or 2 to start the pyramid at twice the frame size
                          (Sec. III-B evaluates on 2x upscaled images) */
    float   thresh;    /* a window is a candidate iff score > thresh (strict) */
    float   iou;       /* greedy NMS drops a box whose IoU with a kept,
                          better-ranked box exceeds iou, 0.5 <= iou < 1
                          (tested exactly on integer areas as
                          inter > iou * union, iou taken as its float32
                          value) */
    int32_t min_face;  /* 0, or the smallest face side in frame pixels: the
                          levels whose 80x80 window spans fewer frame pixels,
                          80 / s_k < min_face, are not analysed at all
                          (Sec. V-A skips the largest scale of 640x480 frames
                          whose faces are at least 20 % of the image:
                          min_face 96).  0 <= min_face <= 65536. */
    const hog_region* regions;  /* NULL, or (device) one search region per
                          frame of the call: windows outside it are not
                          candidates, and histogram tiles and window rows
                          that no window inside it needs are skipped.  Read
                          when the work runs, so a captured graph sees the
                          values current at each replay. */
    int32_t score_arith;  /* HOG_ARITH_F32 (the default): window scores from
                          FP32 products on the matrix cores.
                          HOG_ARITH_F16X3: each product of the window
                          scores (Sec. IV-A linear classification) from
                          three fp16 matrix products of split operands,
                          v = fp16(v) + 2^-11 fp16((v - fp16(v)) 2^11),
                          summed in FP32 (Ootomo and Yokota 2022): about
                          FP32 accuracy (operands kept to 2^-23 |v| +
                          2^-36) at a fraction of the FP32 matrix time.
                          Filter weights must lie below 2^15 in magnitude
                          (larger ones give non-finite scores).  Applies
                          to full filters in hog_detect, hog_detect_batch*,
                          their graphs and hog_autotune (which then run
                          the per-stage schedule); separable filter banks
                          use FP32; hog_detect_topk returns HOG_E_INVAL
                          for it.  Any other value: HOG_E_INVAL. */
} hog_params;

#define HOG_ARITH_F32 0
#define HOG_ARITH_F16X3 1

/* One pyramid level.  Level k has scale s_k = upsample * (5/6)^k and size
 * floor(h * s_k) x floor(w * s_k); levels continue while both sides are at
 * least 80 px (Sec. IV-A).  Cells are 8x8 px: cy = h/8, cx = w/8.  A window
 * is 10x10 cells anchored at its top-left cell: rows = cy-9, cols = cx-9
 * anchors.  `sig` is the inverse scale 1/s_k in fixed point with 40
 * fractional bits, rounded half-up; it defines the resampling taps and the
 * mapping of window boxes back to frame pixels. */
typedef struct hog_level {
    int32_t k, h, w, cy, cx, rows, cols;
    int32_t reserved;
    int64_t sig;
    int64_t feat_offset;   /* float offset of this level in hog_features() output */
    int64_t score_offset;  /* float offset of this level in hog_scores() output */
} hog_level;

/* One detection: filter f of level k at window (row, col); the half-open
 * box [x0, x1) x [y0, y1) is in frame pixels. */
typedef struct hog_det {
    int32_t frame, filter, level, row, col;
    int32_t x0, y0, x1, y1;
    float   score;
} hog_det;

/* A window: filter f of pyramid level k anchored at cell (row, col) of
 * frame `frame` of a batch. */
typedef struct hog_window {
    int32_t frame, filter, level, row, col;
} hog_window;

/* The defaults of the detection parameters: upsample 1, thresh 0 (a window
 * is a face when its score is positive), iou 0.5.  The other constants of
 * the method are fixed at compile time, because the kernels' tiles are
 * shaped by them: 8x8-pixel cells and 18 signed orientation bins
 * (Sec. IV-A, gradient computation and histogramisation), 31 features per
 * cell and 10x10-cell windows (Sec. IV-A, feature computation and linear
 * classification), the 5/6 pyramid step down to an 80-px side (Sec. IV-A),
 * truncation at 0.2 and 1e-4 added to block energies; hog_constants_get
 * reports them.  Host only; HOG_E_INVAL if p is NULL. */
int hog_params_default(hog_params* p);

/* The compile-time constants of the method (see hog_params_default). */
typedef struct hog_constants {
    int32_t cell_px, bins, features, window_cells, min_side, scale_num, scale_den;
    float clip, eps;
} hog_constants;
int hog_constants_get(hog_constants* c);

/* Version of the library, as major*10000 + minor*100 + patch.  Host only. */
int hog_version(void);

/* Static string naming a status code.  Host only. */
const char* hog_strerror(int status);

/* The float64 direction table of the orientation decision, cos(o*pi/9) and
 * sin(o*pi/9) for o = 0..8, each the double nearest to the exact value
 * (host arrays of 9).  Sec. IV-A discretises the gradient into 18 signed
 * directions; the decision picks the direction of largest |projection|.
 * Host only. */
int hog_orientation_table(double* cos9, double* sin9);

/* The pyramid of an h x w frame (host output array `levels` of capacity
 * max_levels; *n_levels receives the count, 0 for frames below 80 px).
 * feat_offset/score_offset are filled for nf filters.  Host only. */
int hog_pyramid(int h, int w, int upsample, int nf,
                hog_level* levels, int max_levels, int* n_levels);

/* Bytes of workspace needed by the calls below for n_frames frames of
 * h x w and nf filters.  0 on invalid arguments.  Host only. */
size_t hog_workspace_bytes(int h, int w, int upsample, int n_frames, int nf);

/* 31-d features of every cell of every level (Sec. IV-A, gradient
 * computation through feature computation; Sec. V-A, gradient-histogram,
 * energy and feature kernels).  Output `feat` (float32, capacity feat_cap
 * floats) holds level k at levels[k].feat_offset as [cy][cx][31]:
 * 18 signed + 9 unsigned + 4 block-energy features. */
int hog_features(const uint8_t* frame, int h, int w, int pitch, int upsample,
                 float* feat, int64_t feat_cap,
                 void* ws, size_t ws_bytes, void* stream);

/* Window scores S_f(k, r, c) = bias_f + <filter_f, features of the 10x10
 * window at (r, c) of level k> for every filter, level and window
 * (Sec. IV-A, linear classification; Sec. V-A, classifier kernels).
 * Output `scores` (float32, capacity scores_cap floats) holds level k at
 * levels[k].score_offset as [nf][rows][cols]. */
int hog_scores(const uint8_t* frame, int h, int w, int pitch, int upsample,
               const float* filters, const float* bias, int nf,
               float* scores, int64_t scores_cap,
               void* ws, size_t ws_bytes, void* stream);

/* A set of nf linear filters with their biases.  rank = 0: full filters
 * W float32 [nf][10][10][31] (row, column, channel of the window).
 * rank = 1..4: separable filters.  The paper's classifier kernels
 * (Sec. V-A) filter each feature channel along the 10 horizontal
 * neighbours of a cell (row filter, into a scratch image) and then along
 * the 10 vertical neighbours (column filter), and add the channels: a
 * filter of that form, or a sum of `rank` of them per channel, is
 *   W_f[dr][dc][ch] = sum_i col[f][i][dr][ch] * row[f][i][dc][ch],
 * given as row and col, float32 [nf][rank][10][31].  Scores of a
 * separable filter equal those of its full W up to float32 rounding (the
 * sums run in another order); the scoring kernel does 20 rank instead of
 * 100 multiply-adds per window, channel and filter.  bias float32 [nf].
 * 1 <= nf <= 32.  Unused pointers may be NULL. */
typedef struct hog_filterbank {
    int32_t nf;
    int32_t rank;
    const float* W;
    const float* row;
    const float* col;
    const float* bias;
} hog_filterbank;

/* hog_scores with a choice of the scoring arithmetic, score_arith as in
 * hog_params (HOG_ARITH_F32: the same as hog_scores; HOG_ARITH_F16X3:
 * products from split fp16 operands, weights below 2^15 in magnitude).
 * HOG_E_INVAL for any other value, else as hog_scores. */
int hog_scores_arith(const uint8_t* frame, int h, int w, int pitch, int upsample,
                     const float* filters, const float* bias, int nf, int score_arith,
                     float* scores, int64_t scores_cap,
                     void* ws, size_t ws_bytes, void* stream);

/* hog_scores for a filter bank (full or separable). */
int hog_scores_bank(const uint8_t* frame, int h, int w, int pitch, int upsample,
                    const hog_filterbank* fb, float* scores, int64_t scores_cap,
                    void* ws, size_t ws_bytes, void* stream);

/* Detect faces in one frame: features, scores, threshold, box mapping and
 * NMS pooled over filters and levels (Sec. IV-A; Sec. V-A detection kernel
 * and non-maximum suppression).  Writes up to `cap` detections (1 <= cap
 * <= HOG_MAX_DETS) to `dets`, best first: score descending, then filter,
 * level, row, column ascending.  `n_dets` (device int) receives the number
 * of kept detections, which may exceed cap (extra rows are dropped). */
int hog_detect(const hog_params* prm, const uint8_t* frame, int h, int w, int pitch,
               const float* filters, const float* bias, int nf,
               hog_det* dets, int cap, int* n_dets,
               void* ws, size_t ws_bytes, void* stream);

/* hog_detect for n frames of one size in one set of launches covering
 * every frame and pyramid level (Sec. V-A, image combinations: an extra
 * grid dimension selects the image).  Frame i starts at
 * frames + i * frame_stride.  dets is [n][cap], n_dets is [n].
 * The schedule is the one hog_tuning_get reports for this shape: either
 * one kernel per stage, or one persistent kernel that runs the histogram,
 * feature and scoring work of all frames and levels from a work list.
 * Both give bit-identical detections. */
int hog_detect_batch(const hog_params* prm, const uint8_t* frames, int n,
                     int h, int w, int pitch, int64_t frame_stride,
                     const float* filters, const float* bias, int nf,
                     hog_det* dets, int cap, int* n_dets,
                     void* ws, size_t ws_bytes, void* stream);

/* hog_detect_batch without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The workspace is a fixed array
 * of HOG_STATIC_SCRATCH_BYTES (64 MiB) inside the library, one per GPU,
 * held from the first call (or hog_init) on that GPU until the process
 * ends.  Shapes whose hog_workspace_bytes(h, w, upsample, n, nf) exceeds it
 * return HOG_E_SCRATCH with nothing enqueued (64 MiB holds 8 frames of
 * 640x480 with 5 filters, or 3 of 1280x720).  The call allocates nothing:
 * no hipMalloc, no hipFree, no allocating library routine.  Every call on
 * one GPU uses the same array and leaves its contents behind; each call
 * clears what must start at zero.  Calls that overlap in time on one GPU
 * (two streams, two host threads) race on the array and give wrong
 * detections: serialise them.  Arguments, outputs, schedule and detections
 * are those of hog_detect_batch. */
int hog_detect_batch_static(const hog_params* prm, const uint8_t* frames, int n,
                            int h, int w, int pitch, int64_t frame_stride,
                            const float* filters, const float* bias, int nf,
                            hog_det* dets, int cap, int* n_dets, void* stream);

/* hog_detect_batch for a filter bank (full or separable; separable banks
 * run the per-stage schedule, with the shape's frame split and NMS rounds). */
int hog_detect_batch_bank(const hog_params* prm, const uint8_t* frames, int n,
                          int h, int w, int pitch, int64_t frame_stride,
                          const hog_filterbank* fb, hog_det* dets, int cap, int* n_dets,
                          void* ws, size_t ws_bytes, void* stream);

/* The next frame's search regions from this frame's detections, one per
 * frame of a batch (for example, one per video stream): the box of the
 * frame's best detection (dets[i * cap], the first in rank order) grown by
 * `margin` frame pixels on every side and clipped to the h x w frame, with
 * levels [level - span, level + span] (k_lo clipped at 0); where a frame has
 * no valid detection (n_dets[i] <= 0), the whole frame at every level.
 * Sec. VII proposes restricting the scales and locations analysed per
 * frame, since faces move little between consecutive frames.  Runs on the
 * device, so a detect -> track -> detect sequence needs no host round trip.
 * dets [n][cap], n_dets [n], regions [n] (device).  0 <= margin <= 65536,
 * 0 <= span <= HOG_MAX_LEVELS. */
int hog_track_regions(const hog_det* dets, const int* n_dets, int n, int cap, int h, int w,
                      int margin, int span, hog_region* regions, void* stream);

/* A hipGraph holding the launches of one hog_detect_batch call with fixed
 * buffers, for replay.  The caller refreshes the frame buffer between
 * replays.  Creation captures on `stream` and returns after instantiation;
 * it enqueues no work.  Launch enqueues one replay on `stream`. */
typedef struct hog_graph hog_graph;
int hog_graph_create(hog_graph** out, const hog_params* prm, const uint8_t* frames, int n,
                     int h, int w, int pitch, int64_t frame_stride,
                     const float* filters, const float* bias, int nf,
                     hog_det* dets, int cap, int* n_dets,
                     void* ws, size_t ws_bytes, void* stream);
int hog_graph_create_bank(hog_graph** out, const hog_params* prm, const uint8_t* frames, int n,
                          int h, int w, int pitch, int64_t frame_stride, const hog_filterbank* fb,
                          hog_det* dets, int cap, int* n_dets, void* ws, size_t ws_bytes, void* stream);
int hog_graph_launch(hog_graph* g, void* stream);
int hog_graph_destroy(hog_graph* g);

/* Set-up of the calling host thread on the current device: the helper
 * streams and events (default priority) that split schedules fork onto,
 * and the device address of the fixed array of hog_detect_batch_static.
 * hog_tuning_set (for a split schedule) and hog_autotune call it; a detect
 * call never creates them.  A split schedule run on a thread without them
 * runs its frame groups one after another on the caller's stream, with
 * the same detections.  Idempotent.  Host only. */
int hog_init(void);

/* Schedule of hog_detect_batch for one shape (h, w, upsample, n, nf).
 * fused = 0: one kernel per stage (histograms, features, scores, NMS);
 *   with split = 2..4 the frames run as that many groups on forked
 *   streams (joined before the call's work ends), so that one group's NMS
 *   overlaps another group's histograms and scores.
 * fused = 1: one persistent kernel for histograms, features and scores.
 *   Its work list splits the frames over `queues` (1..8) atomic ticket
 *   queues, each served by `wg_per_queue` workgroups; in a queue, the
 *   feature items of a frame come lag_f slots and its scoring items lag_s
 *   slots after its histogram items (1 <= lag_f < lag_s), so every item
 *   waits only on earlier tickets.  split must be 1.
 * nms_rounds (0..16): NMS decision rounds run over all window positions of
 *   all frames of a group before the per-frame NMS kernel decides the rest
 *   (any value gives the same detections).
 * score_rows (per-stage schedule): window rows per scoring workgroup, 4 or
 *   16; 0 picks 4 when the batch has fewer 16-row items than compute units. */
typedef struct hog_tuning {
    int32_t fused;
    int32_t queues;
    int32_t wg_per_queue;
    int32_t lag_f;
    int32_t lag_s;
    int32_t split;
    int32_t nms_rounds;
    int32_t score_rows;
    int32_t stagger;   /* split schedules: 0 the groups start together; 1 group j starts once
                          group j - 1 has its histograms, 2 once it has its scores, so that one
                          group's NMS runs beside the next group's histograms and scores */
} hog_tuning;

/* The schedule in effect for a shape: the one set by hog_tuning_set or
 * hog_autotune, else the default.  Returns 1 if set, 0 for the default,
 * or an error code.  Host only; thread-safe. */
int hog_tuning_get(int h, int w, int upsample, int n, int nf, hog_tuning* out);

/* Sets (t non-NULL) or clears (t NULL) the schedule of a shape for this
 * process.  HOG_E_INVAL if t is out of range.  Host only; thread-safe. */
int hog_tuning_set(int h, int w, int upsample, int n, int nf, const hog_tuning* t);

/* Autotuner: times hog_detect_batch on the given frames under each
 * candidate schedule (one untimed run, then `reps` timed runs each, with
 * HIP events on `stream`), keeps the fastest for this shape as with
 * hog_tuning_set and returns it in `best` with its mean time per call in
 * `best_ms`.  Arguments as hog_detect_batch; blocks the host until done.
 * The candidates: the per-stage schedule with split 1, 2 and 4 (staggered
 * 0, 1 or 2 when split), 2, 3, 4, 6, 8 or 12 NMS rounds and scoring items
 * of 4 or 16 rows, and the fused
 * kernel with 8 or 1 queues, one workgroup per compute unit, and
 * lags (1,2), (1,3), (2,3), (2,4); a candidate that reports an error in
 * any n_dets entry is skipped. */
int hog_autotune(const hog_params* prm, const uint8_t* frames, int n,
                 int h, int w, int pitch, int64_t frame_stride,
                 const float* filters, const float* bias, int nf,
                 hog_det* dets, int cap, int* n_dets,
                 void* ws, size_t ws_bytes, int reps,
                 hog_tuning* best, float* best_ms, void* stream);

/* Inspection of one pyramid level of one frame (test entry point).
 * `level_px` (float32 [h_k][w_k]) receives the resampled level, `bins`
 * (uint8 [h_k][w_k]) the orientation bin of every pixel (0 where the
 * gradient is zero), `hist` (float32 [cy][cx][18]) the cell histograms.
 * Any output may be NULL. */
int hog_level_maps(const uint8_t* frame, int h, int w, int pitch, int upsample, int level,
                   float* level_px, uint8_t* bins, float* hist,
                   void* ws, size_t ws_bytes, void* stream);

/* The windows of `level` (of an h x w frame's pyramid) that a search region
 * lets through, as the kernels compute them (test entry point): range4 =
 * {r_lo, r_hi, c_lo, c_hi}, the anchor rows and columns whose boxes lie
 * inside the region's rectangle; empty when r_lo > r_hi or c_lo > c_hi, or
 * when the level is outside [k_lo, k_hi].  Host only. */
int hog_region_windows(int h, int w, int upsample, int level, const hog_region* region, int32_t* range4);

/* The orientation decision alone (test entry point): bins[i] for the
 * integer gradient (gx[i], gy[i]) in units of 2^-16 (|gx|, |gy| < 2^24),
 * n <= 2^31 - 1.  Sec. IV-A: one of eighteen signed directions. */
int hog_orient_bins(const int32_t* gx, const int32_t* gy, int64_t n,
                    uint8_t* bins, void* stream);

/* Bytes of workspace needed by hog_window_scores, hog_topk_windows and
 * hog_filter_backward for n_frames frames of h x w, nf filters and up to
 * n_windows windows.  0 on invalid arguments.  Host only. */
size_t hog_grad_workspace_bytes(int h, int w, int upsample, int n_frames, int nf, int n_windows);

/* Host check of listed windows (host array `windows` of n_windows): every
 * window must address a frame of the batch (0 <= frame < n), a filter
 * (0 <= filter < nf), a pyramid level of an h x w frame and an anchor
 * inside that level (0 <= row < rows, 0 <= col < cols).  Returns HOG_OK, or
 * HOG_E_INVAL with *first_bad (may be NULL) the index of the first window
 * that fails.  The kernels below apply the same test to every window they
 * read.  Host only. */
int hog_windows_check(int h, int w, int upsample, int n, int nf, const hog_window* windows, int n_windows,
                      int* first_bad);

/* Scores of listed windows (Sec. IV-A, linear classification filter: the
 * 3100 features of a 10x10-cell window times the filter weights, summed):
 * scores[i] = bias[f_i] + <filter f_i, 10x10x31 features of window i>.
 * `windows` (device, n_windows) index frames of the batch as in
 * hog_detect_batch; the features are computed from the frames in this
 * call.  Used as the forward pass of filter training.  A window that
 * fails the test of hog_windows_check is not read and scores NaN. */
int hog_window_scores(const uint8_t* frames, int n, int h, int w, int pitch, int64_t frame_stride, int upsample,
                      const float* filters, const float* bias, int nf,
                      const hog_window* windows, int n_windows, float* scores,
                      void* ws, size_t ws_bytes, void* stream);

/* The k (1..16) best windows of every frame over all filters, levels and
 * positions, in rank order (score descending, then filter, level, row,
 * column ascending).  Sec. IV-A scores every 10x10-cell window of every
 * level with each of the five filters; the selection here reads "the top
 * window scores" as the k highest of all those scores, taken before the
 * threshold and before non-maximum suppression, so a frame always has k
 * windows even when none passes the threshold.  Outputs (device):
 * windows [n][k], scores [n][k]. */
int hog_topk_windows(const uint8_t* frames, int n, int h, int w, int pitch, int64_t frame_stride, int upsample,
                     const float* filters, const float* bias, int nf, int k,
                     hog_window* windows, float* scores,
                     void* ws, size_t ws_bytes, void* stream);

/* hog_detect_batch and hog_topk_windows of the same frames from one
 * forward pass: the scoring launch writes the dense scores the top k are
 * taken from and the candidate keys the detection starts from.  Outputs as
 * the two calls give them, bit for bit.  The top k range over every window
 * of every level, so prm->min_face must be 0 and prm->regions NULL.  The
 * workspace is hog_grad_workspace_bytes(h, w, upsample, n, nf, 1) bytes. */
int hog_detect_topk(const hog_params* prm, const uint8_t* frames, int n, int h, int w, int pitch,
                    int64_t frame_stride, const float* filters, const float* bias, int nf,
                    hog_det* dets, int cap, int* n_dets, int k, hog_window* windows, float* scores,
                    void* ws, size_t ws_bytes, void* stream);

/* Backward pass of window scores: every forward step of Sec. IV-A
 * differentiated in reverse order (linear classification, feature
 * computation and normalisation, histogramisation, gradient computation,
 * pyramid resampling).  With upstream gradients dscore[i] for windows[i]
 * (device arrays of n_windows):
 *   dfilters[f] += sum_i [f_i = f] dscore[i] * features(window i)   (float32 [nf][10][10][31])
 *   dbias[f]    += sum_i [f_i = f] dscore[i]                         (float32 [nf], may be NULL)
 *   dpixels     += sum_i dscore[i] * d score_i / d frame pixels      (float32 [n][h][w], may be NULL)
 * The features of each window's support (its 10x10 cells and the ring of
 * cells whose energies normalise them) are recomputed from the frames;
 * nothing is kept from a forward call.  The pixel gradient runs through
 * the clip at 0.2, the block normalisation and energies, the bilinear cell
 * votes, the gradient magnitude (d mag / d g = g / mag, 0 at mag = 0), the
 * central differences and the pyramid resampling.  The orientation bin
 * and the clip are step functions; their derivative is taken as zero, so
 * the bins and clip decisions stay at their forward values (exact away
 * from the switching points).  dfilters and dbias are summed in a fixed
 * order (deterministic); dpixels with atomic adds.  A window that fails
 * the test of hog_windows_check is skipped without a read and makes
 * dfilters[0] NaN. */
int hog_filter_backward(const uint8_t* frames, int n, int h, int w, int pitch, int64_t frame_stride, int upsample,
                        const float* filters, int nf,
                        const hog_window* windows, const float* dscore, int n_windows,
                        float* dfilters, float* dbias, float* dpixels,
                        void* ws, size_t ws_bytes, void* stream);

/* Training objective of the linear filter (Sec. IV-A trains one linear
 * filter per face rotation; the loss is not given there, and this library
 * takes a linear SVM's): the mean hinge loss of scores with labels +-1
 * plus l2 * ||filters||^2, the bias not regularised:
 *   loss (device float[1]) = mean_i max(0, 1 - y_i s_i) + l2 ||W||^2,
 *   dscore[i] = -y_i / n where y_i s_i < 1, else 0 (at the kink y_i s_i = 1
 *   the zero subgradient), and dfilters += 2 l2 filters.  n <= 2^30. */
int hog_hinge_loss(const float* scores, const float* labels, int n, const float* filters, int nf, float l2,
                   float* loss, float* dscore, float* dfilters, void* stream);

/* Host pipeline (Sec. V-C, pipelining: while the GPU detects faces in one
 * batch of frames, CPU threads process the detections of the previous
 * batch; Sec. V-A, data transfers between host and device).  A pipeline
 * owns `depth` stages, each a stream with its own device frame buffer,
 * workspace and detection buffers, and page-locked host buffers.
 * hog_pipeline_submit() takes a free stage (waiting for one if all are in
 * flight), puts the host frames on the device, enqueues hog_detect_batch
 * and the copy of the detections back to page-locked memory, and returns;
 * consumer threads wait for each batch, call `consumer` with its
 * detections and free the stage.  Frames are copied to the device either
 * through the stage's page-locked staging buffer (staging = 1: a host copy,
 * then an asynchronous transfer that overlaps the GPU work of other
 * stages) or straight from the caller's memory (staging = 0; from pageable
 * memory the runtime blocks the caller for the transfer).
 *
 * Unlike the calls above, a pipeline allocates its buffers (device and
 * page-locked host memory) at creation and frees them in destroy.  The
 * filters and bias (device) must outlive it; prm->regions must be NULL. */
typedef void (*hog_consumer_fn)(void* user, int64_t first_frame, int n, const hog_det* dets /* host [n][cap] */,
                                const int* n_dets /* host [n] */, int cap);
typedef struct hog_pipeline_config {
    int32_t h, w;              /* frame size (frames are packed: pitch w, stride h * w) */
    int32_t batch;             /* frames per submit, 1..1024 */
    int32_t depth;             /* stages, 1..16 */
    int32_t cap;               /* detections kept per frame, 1..HOG_MAX_DETS */
    int32_t consumer_threads;  /* 1..64 */
    int32_t staging;           /* 1: through page-locked staging, 0: straight from the caller's memory */
    int32_t reserved;
    hog_consumer_fn consumer;  /* called on a consumer thread per batch; may be NULL.  The
                                  pointers are valid during the call only; it must not call
                                  hog_pipeline_* on the same pipeline. */
    void* user;
} hog_pipeline_config;
typedef struct hog_pipeline hog_pipeline;
int hog_pipeline_create(hog_pipeline** out, const hog_params* prm, const hog_pipeline_config* cfg,
                        const float* filters, const float* bias, int nf);
/* frames: host [n][h][w], 1 <= n <= batch; first_frame is passed to the
 * consumer.  Returns once the work is enqueued (the frames have been read
 * when it returns). */
int hog_pipeline_submit(hog_pipeline* p, const uint8_t* frames, int n, int64_t first_frame);
/* Waits until every submitted batch has been consumed; returns the first
 * error of a batch since the last drain (HOG_OK if none). */
int hog_pipeline_drain(hog_pipeline* p);
int hog_pipeline_destroy(hog_pipeline* p);

/* Kernel timing with HIP events, for benchmarks.  While enabled, each
 * launch of the library's kernels outside graph capture is bracketed by
 * two events on its stream.  hog_profile_read synchronises on the recorded
 * events and returns the summed milliseconds and the launch count of the
 * kernel named `kernel` ("geom", "hist", "feat", "score", "nms_edges", "nms").  Not
 * thread-safe.  Host only. */
int hog_profile_enable(int on);
int hog_profile_reset(void);
int hog_profile_read(const char* kernel, double* total_ms, int64_t* count);

#ifdef __cplusplus
}
#endif
#endif /* LIBHOG355_H */
