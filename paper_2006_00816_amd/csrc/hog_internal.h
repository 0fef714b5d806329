// Internal definitions shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "libhog355.h"

namespace hog {

constexpr int CELL = 8;        // 8x8-pixel cells
constexpr int NBINS = 18;      // signed orientation bins
constexpr int NORIENT = 9;     // unsigned orientations
constexpr int WIN = 10;        // window side in cells
constexpr int NFEAT = 31;      // features per cell
constexpr int FPAD = 32;       // features per cell in the internal layout (31 + zero)
// Internal feature maps: per level row, two half-planes of 16 floats per
// cell (channels 0..15 of every cell of the padded row, then channels
// 16..31), so that a wave reading one half of 16 consecutive cells reads
// 1 KB of consecutive bytes.  Element (row r, cell x, channel ch) is at
// r * FPAD * (cx + 2) + (ch / 16) * 16 * (cx + 2) + 16 x + ch % 16.
constexpr int FHALF = FPAD / 2;
// Internal histogram record of a cell: 18 bins, energy, zero (20 floats).
// A level's records are stored part-major: plane q (q = 0..4) holds part q
// (floats 4q .. 4q + 3) of every cell as one float4, cells in row-major
// order, so that a wave reading part q of consecutive cells reads
// consecutive bytes.
constexpr int HSTRIDE = 20;
constexpr int MIN_SIDE = 80;
constexpr int SCALE_NUM = 5, SCALE_DEN = 6;   // pyramid step 5/6
constexpr int SIG_BITS = 40;   // fractional bits of the fixed-point inverse scale
constexpr int MAX_LEVELS = 28;
constexpr int MAX_SIDE = 4096;
constexpr int MAX_PITCH = 1 << 16;  // bytes per frame row (frame offsets stay 32-bit)
constexpr int MAX_FILTERS = 32;
constexpr int MAX_DETS = 4096;

// Histogram kernel tile: TCY x TCX complete cells per workgroup, from
// (TCY+1) x (TCX+1) "quad blocks" of 8x8 pixels.  A quad block spans the
// pixels between four neighbouring cell centres, so all its pixels vote
// into the same four cells with weights that depend only on the pixel's
// offset inside the block.
constexpr int TCY = 7, TCX = 15;
constexpr int QBY = TCY + 1, QBX = TCX + 1;     // 8 x 16 quad blocks
constexpr int TPY = 8 * QBY + 2, TPX = 8 * QBX + 2;  // 66 x 130 level pixels incl. 1-px halo
constexpr int HIST_THREADS = 512;

constexpr int FEAT_THREADS = 256;

// Window scoring (see stage_score.h): one wave scores one window row as a
// matrix product on v_mfma_f32_16x16x4_f32 with M = 16 cell positions,
// N = (filter f of a group of 5, window column dc) = 50 columns, of which
// 48 (three N tiles) go to the matrix cores and the last 2 (f = 4,
// dc = 8, 9) to the vector ALUs, and K = (window row dr, channel) = 320.
constexpr int FGROUP = 5;
constexpr int SC_K = WIN * FPAD;                 // 320
constexpr int SC_KC = SC_K / 16;                 // 20 chunks of 16 K values
constexpr int SC_NT = 3;                         // N tiles of 16 on the matrix cores
constexpr int SC_RSTR = 20;                      // floats per column of a wave's partial-product tile (16 cells + pad)
constexpr int SC_RING = 50 * SC_RSTR;             // floats of that tile: 50 columns (f, dc)
constexpr int SCORE_THREADS = 1024;
constexpr int ROWS_PER_ITEM = SCORE_THREADS / 64;   // window rows per scoring workgroup item
constexpr int SCORE_SMALL_ROWS = 4;                 // rows per item for batches too small to fill the GPU
constexpr int SCORE_ORDER_MAX = 128;                // slots per frame with a host-chosen dispatch order
constexpr int SCORE_ORDER_SEARCH = 48;              // slots per frame up to which that order is searched
constexpr int BPACK_MFMA = SC_KC * SC_NT * 64;      // float4 B operands of the matrix-core columns
constexpr int BPACK_XTRA = SC_KC * 4 * 2;           // float4 weights of the two vector-ALU columns
constexpr int BPACK_PER_GROUP = BPACK_MFMA + BPACK_XTRA;   // 64,000 bytes per filter group
// Split fp16 operands (HOG_ARITH_F16X3, see stage_score.h): per filter
// group, window row dr, N tile (4, all 50 columns) and part (hi, lo), one
// 8-half B operand per lane.
constexpr int B16_NT = 4;
constexpr int B16_PER_GROUP = WIN * B16_NT * 2 * 64;       // uint4, 81,920 bytes per filter group
constexpr size_t BPACK_GROUP_BYTES =
    (size_t)BPACK_PER_GROUP * 16 > (size_t)B16_PER_GROUP * 16 ? (size_t)BPACK_PER_GROUP * 16 : (size_t)B16_PER_GROUP * 16;

// Fused persistent kernel (k_fused.hip): counters in the workspace, as
// u32 words: queue tickets [0, 8), error flag [8], then per frame the
// finished-wave counts of its histogram, feature and scoring items.
constexpr int FUSED_MAX_QUEUES = 8;
constexpr int FUSED_SYNC_ERR = 8;
constexpr int FUSED_SYNC_HEAD = 16;
constexpr unsigned FUSED_SPIN_LIMIT = 1u << 20;   // polls (about a second) before a wait gives up

struct FusedCfg {
    int queues;          // 1..8; 8 keeps each queue on one XCD
    int wg_per_queue;    // persistent workgroups per queue
    int lag_f, lag_s;    // slot lags of the feature and scoring items, 1 <= lag_f < lag_s
};

constexpr int NMS_THREADS = 1024;
constexpr int SORT_CAP = 4096;
constexpr int NMS_LIST = 128;       // neighbour-list record per window position: count + 127 entries

struct DevLevel {
    int h, w, cy, cx;
    int rows, cols, k;
    int src;                      // 0: sampled from the frame through the taps; 1: an 8-bit level image
                                  // of the recursive pyramid at src_off (pitch w, identity taps)
    long long sig;                // inverse scale, 40 fractional bits
    int tap_y, tap_x;             // offsets (int4 units) of the row / column taps
    int box_r, box_c;             // offsets (int2 units) of the row / column box edges
    int hist_off;                 // cell offset inside one frame's histogram block
    int feat_off;                 // float offset inside one frame's feature block
    int pos_off;                  // window-position offset inside one frame
    int pk_off;                   // float offset of the packed [cy][cx][31] features (one frame)
    int sc_off;                   // float offset of the dense scores [nf][rows][cols] (one frame)
    int th_off, tf_off;           // first workgroup of this level in the hist / feat grids
    int row_off;                  // first window row of this level in the frame's list of window rows
    int nms_klo, nms_khi;         // levels whose boxes can overlap this level's boxes with IoU > 1/2
    int wmin, wmax, hmin, hmax;   // bounds of this level's box widths / heights (frame px)
    int src_off;                  // byte offset of the level image in a frame's block (src = 1)
    int ident;                    // the taps are the identity (a copy of the source, zero weights)
};

struct LevelTable {
    int n;                        // number of levels
    int th_total, tf_total;       // histogram tiles / feature blocks per frame
    int rows_total;               // window rows per frame, over all levels
    int ts_total;                 // scoring items per frame and filter group: ceil(rows_total / ROWS_PER_ITEM)
    int hist_frame;               // cells per frame
    int feat_frame;               // floats per frame (padded layout)
    int pos_frame;                // window positions per frame
    int taps_total, boxes_total;  // geometry table entries
    int h, w, upsample;
    int dense_frame;              // floats of dense scores per frame: sum over levels of nf * rows * cols
    int k_base;                   // pyramid level of table entry 0 (levels below it are not analysed)
    long long casc_frame;         // bytes of 8-bit level images per frame (recursive pyramid), else 0
    DevLevel L[MAX_LEVELS];
};

static_assert(sizeof(LevelTable) <= 3600, "kernel argument block too large");

// Device-side lookup of the level owning workgroup index `b` for a prefix
// field (th_off / tf_off / ts_off).
#define HOG_FIND_LEVEL(T, b, field)                                      \
    ({ int _k = 0;                                                       \
       while (_k + 1 < (T).n && (T).L[_k + 1].field <= (b)) ++_k;        \
       _k; })

// Candidate key: higher value = higher rank.  High word: the score mapped
// to an unsigned integer with the same order; low word: the bitwise NOT of
// (filter, level, row, column) so that smaller indices rank higher.
__host__ __device__ inline unsigned int score_order(float s) {
    unsigned int u = __builtin_bit_cast(unsigned int, s);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float score_from_order(unsigned int o) {
    unsigned int u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __builtin_bit_cast(float, u);
}
// A listed window addresses frame `frame` of a batch of n, filter `filter`
// of nf, and an anchor (row, col) of a window of pyramid level `level`.
__host__ __device__ inline bool window_in_range(const LevelTable& T, int n, int nf, const hog_window& w) {
    if (w.frame < 0 || w.frame >= n || w.filter < 0 || w.filter >= nf || w.level < 0 || w.level >= T.n)
        return false;
    const DevLevel& L = T.L[w.level];
    return w.row >= 0 && w.row < L.rows && w.col >= 0 && w.col < L.cols;
}

__host__ __device__ inline unsigned int pack_window(int f, int k, int r, int c) {
    return ((unsigned)f << 27) | ((unsigned)k << 22) | ((unsigned)r << 11) | (unsigned)c;
}

// The per-call set-up (stage_setup.h): segment 0 the taps and box edges,
// 1 the filter operands (split fp16 ones with f16x3), 2 cleared keys and
// fused-kernel counters; m elements per segment.
struct SetupArgs {
    int4* taps;
    int2* boxes;
    const float* W;
    int nf;
    float4* bpack;
    unsigned long long* keys;
    long long nkeys;
    unsigned* sync;
    int nsync;
    int f16x3;
    long long m;
    int segs;
};
SetupArgs setup_args(const LevelTable& T, int4* taps, int2* boxes, const float* filters, int nf, float4* bpack,
                     unsigned long long* poskey_zero, long long poskey_count, unsigned* sync_zero, int sync_count,
                     bool f16x3);

// Launchers (host functions defined next to their kernels).
hipError_t launch_setup(const LevelTable& T, int4* taps, int2* boxes,
                        const float* filters, int nf, float4* bpack,
                        unsigned long long* poskey_zero, long long poskey_count, unsigned* sync_zero,
                        int sync_count, hipStream_t s, bool f16x3 = false);
// setup (optional): the set-up's work runs in extra workgroups of the
// same launch (nothing the histograms read comes from it)
hipError_t launch_hist(const LevelTable& T, const uint8_t* frames, long long fstride, int pitch,
                       int n, float* hist, const hog_region* regions, const uint8_t* casc, hipStream_t s,
                       const SetupArgs* setup = nullptr);
// One level of the recursive pyramid for n frames: the 8-bit image
// [h_out][w_out] at dst_off of each frame's block of `casc`, scaled down by
// 5/6 from the level image [h_in][w_in] at src_off (src_off < 0: the frame
// itself), or (sig > 0) the level sampled from the frame at inverse scale
// sig (the 2x level 0), rounded to grey levels.
hipError_t launch_cascade(const uint8_t* frames, long long fstride, int pitch, int n, uint8_t* casc,
                          long long casc_frame, int h_out, int w_out, int dst_off, int h_in, int w_in, int src_off,
                          long long sig, hipStream_t s);
// f16x3: the maps hold split fp16 operands for the scorer (HOG_ARITH_F16X3)
hipError_t launch_feat(const LevelTable& T, int n, const float* hist, float* feat,
                       float* packed, hipStream_t s, bool f16x3 = false);
int fused_sync_words(int n);
struct FusedNeed {
    unsigned hist, feat, score;   // finished-wave counts of a complete frame
};
FusedNeed fused_need(const LevelTable& T, int nf);
hipError_t launch_fused(const LevelTable& T, int n, const FusedCfg& cfg, const uint8_t* frames, long long fstride,
                        int pitch, float* hist, float* feat, const float4* bpack, const float* bias, int nf,
                        float thresh, unsigned long long* poskey, bool atomic_key, unsigned* sync, hipStream_t s);
int score_rows_auto(const LevelTable& T, int n, int nf, int cus);
int sep_rows_auto(const LevelTable& T, int n, int nf, int cus);
// f16x3: B was packed by launch_setup with f16x3 set, and the products are
// formed from split fp16 operands (HOG_ARITH_F16X3).
hipError_t launch_score(const LevelTable& T, int n, const float* feat, const float4* bpack,
                        const float* bias, int nf, float thresh, float* dense,
                        unsigned long long* poskey, bool atomic_key, int rows, const hog_region* regions,
                        hipStream_t s, bool f16x3 = false);
constexpr int SEP_MAX_RANK = 4;   // row / column filter pairs per channel of a separable filter
constexpr int SEP_ROWS = 8;       // window rows per separable scoring item (256 VGPRs per lane at 512 threads)
hipError_t launch_score_sep(const LevelTable& T, int n, const float* feat, const float* row, const float* col,
                            int rank, const float* bias, int nf, float thresh, float* dense,
                            unsigned long long* poskey, bool atomic_key, int rows, const hog_region* regions,
                            hipStream_t s);
// Search regions of the next frames from the detections of these (one per
// frame): the best detection's box grown by margin px and its levels
// +- span, or the whole frame where a frame has no detection.
hipError_t launch_track(const hog_det* dets, const int* n_dets, int n, int cap, int h, int w, int margin, int span,
                        hog_region* regions, hipStream_t s);
// NMS records hold 32-bit position indices when a frame has 65536 window
// positions or more, else 16-bit ones.
inline bool nms_wide_lists(long long positions) { return positions > 65535; }
hipError_t launch_nms_edges(const LevelTable& T, int n, const unsigned long long* poskey, const int2* boxes,
                            long long iou_num, long long iou_den, void* lists, unsigned char* state8, int rounds,
                            hipStream_t s);
hipError_t launch_nms(const LevelTable& T, int n, const unsigned long long* poskey, const void* lists,
                      const int2* boxes, long long iou_num, long long iou_den, void* dets, int cap, int* n_dets,
                      unsigned* gstate, int* work, const unsigned char* state8, const unsigned* upstream,
                      FusedNeed need, int frame_base, hipStream_t s);
hipError_t launch_level_maps(const LevelTable& T, int level, const uint8_t* frame, int pitch,
                             const int4* taps, float* level_px, uint8_t* bins, const uint8_t* casc, hipStream_t s);
hipError_t launch_orient(const int32_t* gx, const int32_t* gy, long long n, uint8_t* bins,
                         hipStream_t s);
hipError_t launch_fill(int* p, int n, int v, hipStream_t s);
void orientation_table_host(double* c, double* s);
hipError_t launch_window_scores(const LevelTable& T, int n, int nf, const float* feat, const hog_window* win,
                                int n_win, const float* W, const float* bias, float* scores, hipStream_t s);
hipError_t launch_topk(const LevelTable& T, int n, const float* dense, long long dense_frame, int nf, int K,
                       hog_window* out, float* out_scores, hipStream_t s);
hipError_t launch_hinge(const float* S, const float* y, int n, const float* W, int nw, float lam, float* loss,
                        float* dscore, float* dW, hipStream_t s);
int backward_groups(int n_win);
size_t backward_lds_bytes();
hipError_t launch_backward(const LevelTable& T, int n, const uint8_t* frames, long long fstride, int pitch,
                           const int4* taps, const float* W, const hog_window* win, const float* dscore, int n_win,
                           int nf, float* partial, float* dW, float* db, float* dpixels, hipStream_t s);

}  // namespace hog
