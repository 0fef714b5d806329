// C ABI of libhog355: argument checks, pyramid planning, workspace layout,
// launch sequences, hipGraph capture and kernel timing.
#include <string.h>

#include <algorithm>
#include <array>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hog_device.h"

using namespace hog;

namespace {

// One image of the recursive pyramid: level k of the full pyramid (also
// when the level is not analysed, since later levels are computed from
// it), at byte offset `off` of a frame's block; off < 0: the frame itself.
struct ChainLevel {
    int h = 0, w = 0, off = -1;
    long long sig = 0;
};

struct Plan {
    LevelTable T;
    int n = 0, nf = 0, groups = 0;
    bool cascade = false;            // recursive pyramid (HOG_PYRAMID_CASCADE)
    int chain_n = 0;
    ChainLevel chain[MAX_LEVELS];
    // workspace offsets (bytes)
    size_t o_taps = 0, o_boxes = 0, o_bpack = 0, o_hist = 0, o_feat = 0, o_key = 0, o_state = 0, o_list = 0,
           o_work = 0, o_state8 = 0, o_sync = 0, o_casc = 0, o_dense = 0, o_partial = 0, total = 0;
    long long packed_floats = 0, dense_floats = 0;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int MAX_MIN_FACE = 1 << 16;

typedef __int128 i128;

// Levels of an h x w frame: scale s_k = u 5^k / 6^k, size floor(h s_k) x
// floor(w s_k), kept while both sides are >= 80 px (Sec. IV-A).
// With `cascade` the sizes are those of the recursive pyramid instead:
// u h x u w, then floor(5 x / 6) of the previous level (Sec. V-A,
// image-scaling kernel); the scales s_k, and so the inverse scales, are
// the same.
int pyramid_levels(int h, int w, int u, int* hk, int* wk, long long* sig, int maxl, bool cascade = false) {
    int n = 0;
    i128 p = u, q = 1;
    long long ch = (long long)u * h, cw = (long long)u * w;
    for (int k = 0; k < 64; ++k) {
        const i128 hh = cascade ? (i128)ch : (i128)h * p / q, ww = cascade ? (i128)cw : (i128)w * p / q;
        ch = ch * SCALE_NUM / SCALE_DEN;
        cw = cw * SCALE_NUM / SCALE_DEN;
        if (hh < MIN_SIDE || ww < MIN_SIDE) break;
        if (n >= maxl) return -1;
        hk[n] = (int)hh;
        wk[n] = (int)ww;
        // inverse scale q/p with 40 fractional bits, rounded half-up
        sig[n] = (long long)((q * ((i128)1 << (SIG_BITS + 1)) + p) / (2 * p));
        ++n;
        p *= 5;
        q *= 6;
    }
    return n;
}

int check_frame(int h, int w, int upsample) {
    const int u = upsample & ~HOG_PYRAMID_CASCADE;
    if (h <= 0 || w <= 0 || (u != 1 && u != 2)) return HOG_E_INVAL;
    if (h > MAX_SIDE || w > MAX_SIDE) return HOG_E_TOO_LARGE;
    return HOG_OK;
}

// Box side bounds of a level: an edge is floor(v sig / 2^40 + 1/2), so a
// side of 80 level px spans floor(80 sig / 2^40) or one more frame px.
void box_bounds(long long sig, int* lo, int* hi) {
    const i128 num = (i128)80 * sig;
    const long long fl = (long long)(num >> SIG_BITS);
    *lo = (int)fl;
    *hi = (int)fl + 1;
}

// n_windows > 0 adds the regions of the gradient calls: dense scores of
// every frame and the per-workgroup partial filter gradients.
// min_face > 0 leaves out the leading levels whose 80-px window spans
// fewer than min_face frame px (80 q_k < min_face p_k, exact): the table
// then starts at pyramid level k_base.
int make_plan(int h, int w, int upsample, int n, int nf, Plan* P, int n_windows = 0, int min_face = 0) {
    int st = check_frame(h, w, upsample);
    if (st) return st;
    if (n < 1 || nf < 0 || min_face < 0 || min_face > MAX_MIN_FACE) return HOG_E_INVAL;
    if (nf > MAX_FILTERS) return HOG_E_TOO_LARGE;
    const bool cascade = (upsample & HOG_PYRAMID_CASCADE) != 0;
    const int u = upsample & ~HOG_PYRAMID_CASCADE;
    int hk[MAX_LEVELS], wk[MAX_LEVELS];
    long long sig[MAX_LEVELS];
    int nl = pyramid_levels(h, w, u, hk, wk, sig, MAX_LEVELS, cascade);
    if (nl < 0) return HOG_E_TOO_LARGE;
    // images of the recursive pyramid, one per level of the full pyramid
    // (level 0 at upsample 1 is the frame itself)
    P->cascade = cascade;
    P->chain_n = cascade ? nl : 0;
    long long casc_bytes = 0;
    for (int k = 0; k < P->chain_n; ++k) {
        ChainLevel& c = P->chain[k];
        c.h = hk[k];
        c.w = wk[k];
        c.sig = sig[k];
        c.off = -1;
        if (k > 0 || u != 1) {
            c.off = (int)casc_bytes;
            casc_bytes += ((long long)hk[k] * wk[k] + 255) & ~255LL;
        }
    }
    if (casc_bytes > 0x7fffffffLL) return HOG_E_TOO_LARGE;
    int k_base = 0;
    {
        i128 p = u, q = 1;
        while (k_base < nl && (i128)MIN_SIDE * q < (i128)min_face * p) {
            ++k_base;
            p *= 5;
            q *= 6;
        }
    }
    nl -= k_base;
    for (int i = 0; i < nl; ++i) {
        hk[i] = hk[i + k_base];
        wk[i] = wk[i + k_base];
        sig[i] = sig[i + k_base];
    }
    LevelTable& T = P->T;
    memset(&T, 0, sizeof(T));
    T.n = nl;
    T.k_base = k_base;
    T.h = h;
    T.w = w;
    T.upsample = upsample;
    T.casc_frame = casc_bytes;
    int taps = 0, boxes = 0, th = 0, tf = 0, ts = 0;
    long long hist = 0, feat = 0, pos = 0, pk = 0, sc = 0;
    for (int k = 0; k < nl; ++k) {
        DevLevel& L = T.L[k];
        L.k = k + k_base;
        L.src = cascade && P->chain[k + k_base].off >= 0 ? 1 : 0;
        L.src_off = L.src ? P->chain[k + k_base].off : 0;
        L.ident = L.src || sig[k] == (1LL << SIG_BITS);
        L.h = hk[k];
        L.w = wk[k];
        L.cy = hk[k] / CELL;
        L.cx = wk[k] / CELL;
        L.rows = L.cy - WIN + 1;
        L.cols = L.cx - WIN + 1;
        L.sig = sig[k];
        L.tap_y = taps;
        taps += L.h;
        L.tap_x = taps;
        taps += L.w;
        L.box_r = boxes;
        boxes += L.rows;
        L.box_c = boxes;
        boxes += L.cols;
        L.hist_off = (int)hist;
        hist += (long long)L.cy * L.cx;
        L.feat_off = (int)feat;
        feat += (long long)L.cy * (L.cx + 2) * FPAD;
        L.pos_off = (int)pos;
        pos += (long long)L.rows * L.cols;
        L.pk_off = (int)pk;
        pk += (long long)L.cy * L.cx * NFEAT;
        L.sc_off = (int)sc;
        sc += (long long)(nf > 0 ? nf : 1) * L.rows * L.cols;
        L.th_off = th;
        th += ((L.cy + TCY - 1) / TCY) * ((L.cx + TCX - 1) / TCX);
        L.tf_off = tf;
        tf += (L.cy * (L.cx + 2) + FEAT_THREADS - 1) / FEAT_THREADS;
        L.row_off = ts;
        ts += L.rows;
        box_bounds(L.sig, &L.wmin, &L.wmax);
        L.hmin = L.wmin;
        L.hmax = L.wmax;
    }
    if (feat > 0x7fffffffLL || hist > 0x7fffffffLL / HSTRIDE || pk > 0x7fffffffLL || sc > 0x7fffffffLL)
        return HOG_E_TOO_LARGE;
    // levels whose boxes can reach IoU > 1/2 with this level's boxes: the
    // IoU of two boxes is at most (smaller area) / (larger area)
    for (int k = 0; k < nl; ++k) {
        DevLevel& L = T.L[k];
        L.nms_klo = k;
        L.nms_khi = k;
        for (int k2 = 0; k2 < nl; ++k2) {
            const DevLevel& M = T.L[k2];
            const long long amax_s = (long long)std::min(L.wmax, M.wmax) * std::min(L.hmax, M.hmax);
            const long long amin_b = (long long)std::max(L.wmin, M.wmin) * std::max(L.hmin, M.hmin);
            if (2 * amax_s > amin_b) {
                L.nms_klo = std::min(L.nms_klo, k2);
                L.nms_khi = std::max(L.nms_khi, k2);
            }
        }
    }
    T.th_total = th;
    T.tf_total = tf;
    T.rows_total = ts;
    T.ts_total = (ts + ROWS_PER_ITEM - 1) / ROWS_PER_ITEM;
    T.hist_frame = (int)hist;
    T.feat_frame = (int)feat;
    T.pos_frame = (int)pos;
    T.taps_total = taps;
    T.boxes_total = boxes;
    P->n = n;
    P->nf = nf;
    P->groups = nf > 0 ? (nf + FGROUP - 1) / FGROUP : 0;
    P->packed_floats = pk;
    P->dense_floats = sc;
    size_t o = 0;
    P->o_taps = o;
    o = align256(o + sizeof(int4) * (size_t)std::max(taps, 1));
    P->o_boxes = o;
    o = align256(o + sizeof(int2) * (size_t)std::max(boxes, 1));
    P->o_bpack = o;
    o = align256(o + BPACK_GROUP_BYTES * (size_t)std::max(P->groups, 1));
    P->o_hist = o;
    o = align256(o + sizeof(float) * (size_t)n * std::max(hist, 1LL) * HSTRIDE);
    P->o_feat = o;
    o = align256(o + sizeof(float) * (size_t)n * std::max(feat, 1LL));
    P->o_key = o;
    o = align256(o + sizeof(unsigned long long) * (size_t)n * std::max(pos, 1LL));
    P->o_state = o;
    o = align256(o + sizeof(unsigned) * (size_t)n * ((std::max(pos, 1LL) + 15) / 16));
    P->o_list = o;
    o = align256(o + (nms_wide_lists(pos) ? 4 : 2) * (size_t)NMS_LIST * (size_t)n * std::max(pos, 1LL));
    P->o_work = o;
    o = align256(o + sizeof(int) * 2 * (size_t)n * std::max(pos, 1LL));
    P->o_state8 = o;
    o = align256(o + (size_t)n * std::max(pos, 1LL));
    P->o_sync = o;
    o = align256(o + sizeof(unsigned) * (size_t)fused_sync_words(n));
    P->o_casc = o;
    o = align256(o + (size_t)n * casc_bytes);
    T.dense_frame = (int)sc;
    P->o_dense = o;
    P->o_partial = o;
    if (n_windows > 0) {
        o = align256(o + sizeof(float) * (size_t)n * std::max(sc, 1LL));
        P->o_partial = o;
        o = align256(o + sizeof(float) * (size_t)backward_groups(n_windows) *
                             ((size_t)std::max(nf, 1) * WIN * WIN * NFEAT + std::max(nf, 1)));
    }
    P->total = o;
    return HOG_OK;
}

template <class T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ------------------------------------------------------------ profiling
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

template <class F>
int timed(const char* name, hipStream_t s, F&& launch) {
    const bool prof = g_prof_on && !capturing(s);
    ProfRec rec;
    if (prof) {
        rec.name = name;
        if (hipEventCreate(&rec.a) != hipSuccess || hipEventCreate(&rec.b) != hipSuccess) return HOG_E_HIP;
        if (hipEventRecord(rec.a, s) != hipSuccess) return HOG_E_HIP;
    }
    if (launch() != hipSuccess) return HOG_E_HIP;
    if (prof) {
        if (hipEventRecord(rec.b, s) != hipSuccess) return HOG_E_HIP;
        std::lock_guard<std::mutex> g(g_prof_mu);
        g_prof.push_back(rec);
    }
    return HOG_OK;
}

#define HOG_TRY(x)                 \
    do {                           \
        const int _st = (x);       \
        if (_st != HOG_OK) return _st; \
    } while (0)

int check_ws(const Plan& P, void* ws, size_t ws_bytes) {
    if (!ws) return HOG_E_INVAL;
    if (ws_bytes < P.total) return HOG_E_WORKSPACE;
    return HOG_OK;
}

// The level images of the recursive pyramid for m frames (casc: the block
// of the first), level by level, each from the one before.  Nothing for
// the direct pyramid.
int run_cascade(const Plan& P, int m, const uint8_t* frames, long long fstride, int pitch, uint8_t* casc,
                hipStream_t s) {
    for (int k = 0; k < P.chain_n; ++k) {
        const ChainLevel& c = P.chain[k];
        if (c.off < 0) continue;   // level 0 at upsample 1: the frame itself
        HOG_TRY(timed("cascade", s, [&] {
            if (k == 0)
                return launch_cascade(frames, fstride, pitch, m, casc, P.T.casc_frame, c.h, c.w, c.off, P.T.h, P.T.w,
                                      -1, c.sig, s);
            const ChainLevel& q = P.chain[k - 1];
            return launch_cascade(frames, fstride, pitch, m, casc, P.T.casc_frame, c.h, c.w, c.off, q.h, q.w, q.off,
                                  0, s);
        }));
    }
    return HOG_OK;
}

int run_pixels(const Plan& P, const uint8_t* frames, long long fstride, int pitch, void* ws, float* packed,
               const float* filters, hipStream_t s, bool zero_keys, bool f16x3 = false) {
    const LevelTable& T = P.T;
    HOG_TRY(timed("geom", s, [&] {
        return launch_setup(T, at<int4>(ws, P.o_taps), at<int2>(ws, P.o_boxes), filters, P.nf,
                            at<float4>(ws, P.o_bpack), zero_keys ? at<unsigned long long>(ws, P.o_key) : nullptr,
                            (long long)P.n * T.pos_frame, nullptr, 0, s, f16x3);
    }));
    HOG_TRY(run_cascade(P, P.n, frames, fstride, pitch, at<uint8_t>(ws, P.o_casc), s));
    HOG_TRY(timed("hist", s, [&] {
        return launch_hist(T, frames, fstride, pitch, P.n, at<float>(ws, P.o_hist), nullptr, at<uint8_t>(ws, P.o_casc),
                           s);
    }));
    HOG_TRY(timed("feat", s, [&] {
        return launch_feat(T, P.n, at<float>(ws, P.o_hist), at<float>(ws, P.o_feat), packed, s, f16x3);
    }));
    return HOG_OK;
}

// ------------------------------------------------------------- schedules
using ShapeKey = std::array<int, 5>;
std::mutex g_tune_mu;
std::map<ShapeKey, hog_tuning> g_tune;

int compute_units() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

constexpr int MAX_SPLIT = 4;

constexpr int MAX_NMS_ROUNDS = 16;

bool tuning_valid(const hog_tuning& t) {
    if (t.split < 1 || t.split > MAX_SPLIT) return false;
    if (t.nms_rounds < 0 || t.nms_rounds > MAX_NMS_ROUNDS) return false;
    if (t.score_rows != 0 && t.score_rows != SCORE_SMALL_ROWS && t.score_rows != ROWS_PER_ITEM) return false;
    if (t.stagger < 0 || t.stagger > 2 || (t.stagger && t.fused)) return false;
    if (t.fused == 0) return true;
    return t.fused == 1 && t.split == 1 && t.queues >= 1 && t.queues <= FUSED_MAX_QUEUES && t.wg_per_queue >= 1 &&
           t.wg_per_queue <= 65536 && t.lag_f >= 1 && t.lag_s > t.lag_f && t.lag_s <= 64;
}

hog_tuning default_tuning(int, int, int, int n, int) {
    hog_tuning t{};
    // parallel NMS rounds: small batches leave most of the GPU to them
    t.nms_rounds = n <= 2 ? 8 : n <= 8 ? 5 : 3;
    t.score_rows = 0;   // by batch size: small items when the batch does not fill the GPU
    t.fused = 0;
    t.queues = 8;
    t.wg_per_queue = 32;
    t.lag_f = 1;
    t.lag_s = 2;
    t.split = 1;
    t.stagger = 0;
    return t;
}

hog_tuning lookup_tuning(int h, int w, int u, int n, int nf, bool* found = nullptr) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(ShapeKey{h, w, u, n, nf});
    if (found) *found = it != g_tune.end();
    return it != g_tune.end() ? it->second : default_tuning(h, w, u, n, nf);
}

// Pointers of the per-frame workspace regions, starting at frame `lo` of
// the batch.
struct FrameBufs {
    int lo;   // batch index of the group's first frame
    const uint8_t* frames;
    float* hist;
    float* feat;
    unsigned long long* keys;
    unsigned* gstate;
    void* lists;
    int* work;
    unsigned char* state8;
    hog_det* dets;
    int* n_dets;
    const hog_region* regions;   // search regions of the group's frames, or nullptr
    uint8_t* casc;               // the group's level images of the recursive pyramid
};

FrameBufs frame_bufs(const Plan& P, void* ws, const uint8_t* frames, long long fstride, hog_det* dets, int cap,
                     int* n_dets, int lo, const hog_region* regions = nullptr) {
    const LevelTable& T = P.T;
    const long long pos = T.pos_frame;
    FrameBufs b;
    b.lo = lo;
    b.frames = frames + (long long)lo * fstride;
    b.hist = at<float>(ws, P.o_hist) + (long long)lo * T.hist_frame * HSTRIDE;
    b.feat = at<float>(ws, P.o_feat) + (long long)lo * T.feat_frame;
    b.keys = at<unsigned long long>(ws, P.o_key) + lo * pos;
    b.gstate = at<unsigned>(ws, P.o_state) + lo * ((pos + 15) / 16);
    b.lists = at<char>(ws, P.o_list) + lo * pos * NMS_LIST * (nms_wide_lists(pos) ? 4 : 2);
    b.work = at<int>(ws, P.o_work) + lo * 2 * pos;
    b.state8 = at<unsigned char>(ws, P.o_state8) + lo * pos;
    b.dets = dets + (long long)lo * cap;
    b.n_dets = n_dets + lo;
    b.regions = regions ? regions + lo : nullptr;
    b.casc = at<uint8_t>(ws, P.o_casc) + (long long)lo * T.casc_frame;
    return b;
}

// Helper streams and events of a host thread for split schedules (default
// priority), per device.  hog_init creates them; a detect call only looks
// them up.
constexpr int MAX_DEVICES = 64;
struct SplitRes {
    bool ready = false;
    hipStream_t st[MAX_SPLIT - 1] = {};
    hipEvent_t ev[MAX_SPLIT] = {};
    hipEvent_t stage[MAX_SPLIT] = {};   // a group's histograms (or scores) done: the next group may start
};
thread_local SplitRes g_split[MAX_DEVICES];

int init_split_resources() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HOG_E_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return HOG_E_INVAL;
    SplitRes& r = g_split[dev];
    if (r.ready) return HOG_OK;
    for (int j = 0; j < MAX_SPLIT - 1; ++j)
        if (hipStreamCreateWithFlags(&r.st[j], hipStreamNonBlocking) != hipSuccess) return HOG_E_HIP;
    for (int j = 0; j < MAX_SPLIT; ++j)
        if (hipEventCreateWithFlags(&r.ev[j], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&r.stage[j], hipEventDisableTiming) != hipSuccess)
            return HOG_E_HIP;
    r.ready = true;
    return HOG_OK;
}

// The calling thread's helper streams on the current device, or nullptr
// if hog_init has not created them.
SplitRes* split_resources() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    return g_split[dev].ready ? &g_split[dev] : nullptr;
}

int nms_chain(const Plan& P, int m, const FrameBufs& b, const hog_params* prm, int cap, const unsigned* upstream,
              int rounds, void* ws, hipStream_t s) {
    const LevelTable& T = P.T;
    // iou (a float32 in [1/2, 1)) as the exact binary fraction num / 2^e,
    // e <= 24, so that inter * 2^e stays below 2^63
    double v = prm->iou;
    int e = 0;
    while (v != (double)(long long)v) {
        v *= 2.0;
        ++e;
    }
    const long long num = (long long)v, den = 1LL << e;
    HOG_TRY(timed("nms_edges", s, [&] {
        return launch_nms_edges(T, m, b.keys, at<int2>(ws, P.o_boxes), num, den, b.lists, b.state8, rounds, s);
    }));
    return timed("nms", s, [&] {
        return launch_nms(T, m, b.keys, b.lists, at<int2>(ws, P.o_boxes), num, den, b.dets, cap, b.n_dets, b.gstate,
                          b.work, b.state8, upstream, fused_need(T, P.nf), b.lo, s);
    });
}

// The filters of a call: full [nf][10][10][31] (rank 0), or separable
// row and column factors [nf][rank][10][31] (rank 1..4).
struct Bank {
    const float* W = nullptr;
    const float* row = nullptr;
    const float* col = nullptr;
    int rank = 0;
    const float* bias = nullptr;
    bool f16x3 = false;   // full filters scored from split fp16 operands (HOG_ARITH_F16X3)
};

// Window scores of m frames into dense maps and / or keys.
int score_stage(const Plan& P, int m, const float* feat, const Bank& bank, float thresh, float* dense,
                unsigned long long* keys, int score_rows, void* ws, hipStream_t s,
                const hog_region* regions = nullptr) {
    const LevelTable& T = P.T;
    const bool multi = P.groups > 1;
    return timed("score", s, [&] {
        if (bank.rank == 0) {
            const int rows = score_rows ? score_rows : score_rows_auto(T, m, P.nf, compute_units());
            return launch_score(T, m, feat, at<float4>(ws, P.o_bpack), bank.bias, P.nf, thresh, dense, keys,
                                keys && multi, rows, regions, s, bank.f16x3);
        }
        const int rows = score_rows == SCORE_SMALL_ROWS ? SCORE_SMALL_ROWS
                         : score_rows ? SEP_ROWS
                                      : sep_rows_auto(T, m, P.nf, compute_units());
        return launch_score_sep(T, m, feat, bank.row, bank.col, bank.rank, bank.bias, P.nf, thresh, dense, keys,
                                keys && multi, rows, regions, s);
    });
}

// histograms -> features -> scores -> NMS for frames lo .. lo + m - 1.
// `mark` (if any) is recorded after the histograms (stagger 1) or after
// the scores (stagger 2), for the next group of a staggered split.
// `setup` (if any): the call's set-up, run by extra workgroups of the
// histogram launch.
int staged_chain(const Plan& P, int m, const FrameBufs& b, long long fstride, int pitch, const hog_params* prm,
                 const Bank& bank, int cap, int rounds, int score_rows, void* ws, hipStream_t s,
                 hipEvent_t mark = nullptr, int stagger = 0, const SetupArgs* setup = nullptr) {
    const LevelTable& T = P.T;
    HOG_TRY(run_cascade(P, m, b.frames, fstride, pitch, b.casc, s));
    HOG_TRY(timed("hist", s, [&] {
        return launch_hist(T, b.frames, fstride, pitch, m, b.hist, b.regions, b.casc, s, setup);
    }));
    if (mark && stagger == 1 && hipEventRecord(mark, s) != hipSuccess) return HOG_E_HIP;
    HOG_TRY(timed("feat", s, [&] { return launch_feat(T, m, b.hist, b.feat, nullptr, s, bank.f16x3); }));
    HOG_TRY(score_stage(P, m, b.feat, bank, prm->thresh, nullptr, b.keys, score_rows, ws, s, b.regions));
    if (mark && stagger == 2 && hipEventRecord(mark, s) != hipSuccess) return HOG_E_HIP;
    return nms_chain(P, m, b, prm, cap, nullptr, rounds, ws, s);
}

int detect_sequence(const Plan& P, const hog_params* prm, const uint8_t* frames, long long fstride, int pitch,
                    const Bank& bank_in, hog_det* dets, int cap, int* n_dets, void* ws, const hog_tuning& tune_in,
                    hipStream_t s) {
    Bank bank = bank_in;
    bank.f16x3 = bank.rank == 0 && prm->score_arith == HOG_ARITH_F16X3;
    // separable filters, search regions, the recursive pyramid and split
    // fp16 scoring run the per-stage schedule
    hog_tuning tune = tune_in;
    if ((bank.rank != 0 || prm->regions || P.cascade || bank.f16x3) && tune.fused) {
        tune.fused = 0;
        tune.split = 1;
    }
    const hog_region* regions = prm->regions;
    const float* filters = bank.W;
    const float* bias = bank.bias;
    const LevelTable& T = P.T;
    if (T.n == 0) {
        // no pyramid level: zero detections for every frame
        return timed("fill", s, [&] { return launch_fill(n_dets, P.n, 0, s); });
    }
    const bool multi = P.groups > 1;
    unsigned* sync = at<unsigned>(ws, P.o_sync);
    const int parts = std::min(std::max(tune.split, 1), P.n);
    if (!tune.fused && parts == 1) {
        // one group: the set-up's work (first read by the scorer) runs in
        // extra workgroups of the histogram launch, one launch fewer
        const SetupArgs sa = setup_args(T, at<int4>(ws, P.o_taps), at<int2>(ws, P.o_boxes), filters, P.nf,
                                        at<float4>(ws, P.o_bpack),
                                        multi ? at<unsigned long long>(ws, P.o_key) : nullptr,
                                        (long long)P.n * T.pos_frame, nullptr, 0, bank.f16x3);
        return staged_chain(P, P.n, frame_bufs(P, ws, frames, fstride, dets, cap, n_dets, 0, regions), fstride,
                            pitch, prm, bank, cap, tune.nms_rounds, tune.score_rows, ws, s, nullptr, 0, &sa);
    }
    HOG_TRY(timed("geom", s, [&] {
        return launch_setup(T, at<int4>(ws, P.o_taps), at<int2>(ws, P.o_boxes), filters, P.nf,
                            at<float4>(ws, P.o_bpack), multi ? at<unsigned long long>(ws, P.o_key) : nullptr,
                            (long long)P.n * T.pos_frame, tune.fused ? sync : nullptr,
                            tune.fused ? fused_sync_words(P.n) : 0, s, bank.f16x3);
    }));
    if (tune.fused) {
        FusedCfg cfg;
        cfg.queues = tune.queues;
        cfg.wg_per_queue = tune.wg_per_queue;
        cfg.lag_f = tune.lag_f;
        cfg.lag_s = tune.lag_s;
        HOG_TRY(timed("fused", s, [&] {
            return launch_fused(T, P.n, cfg, frames, fstride, pitch, at<float>(ws, P.o_hist), at<float>(ws, P.o_feat),
                                at<float4>(ws, P.o_bpack), bias, P.nf, prm->thresh,
                                at<unsigned long long>(ws, P.o_key), multi, sync, s);
        }));
        return nms_chain(P, P.n, frame_bufs(P, ws, frames, fstride, dets, cap, n_dets, 0), prm, cap, sync,
                         tune.nms_rounds, ws, s);
    }
    // the frames in `parts` groups on forked streams: one group's NMS
    // overlaps another's histograms and scores.  Without the calling
    // thread's helper streams (hog_init) the groups run one after another
    // on the caller's stream, with the same detections.
    SplitRes* r = split_resources();
    if (!r) {
        for (int j = 0; j < parts; ++j) {
            const int lo = (int)((long long)j * P.n / parts), hi = (int)((long long)(j + 1) * P.n / parts);
            HOG_TRY(staged_chain(P, hi - lo, frame_bufs(P, ws, frames, fstride, dets, cap, n_dets, lo, regions),
                                 fstride, pitch, prm, bank, cap, tune.nms_rounds, tune.score_rows, ws, s));
        }
        return HOG_OK;
    }
    if (hipEventRecord(r->ev[0], s) != hipSuccess) return HOG_E_HIP;
    for (int j = 1; j < parts; ++j)
        if (hipStreamWaitEvent(r->st[j - 1], r->ev[0], 0) != hipSuccess) return HOG_E_HIP;
    // staggered: group j starts once group j - 1 has its histograms (or
    // scores), so that the groups are in different stages at a time and a
    // group's latency-bound NMS runs beside the next group's compute
    const int stagger = tune.stagger;
    int st = HOG_OK;
    for (int j = 0; j < parts && st == HOG_OK; ++j) {
        const int lo = (int)((long long)j * P.n / parts), hi = (int)((long long)(j + 1) * P.n / parts);
        hipStream_t sj = j == 0 ? s : r->st[j - 1];
        if (stagger && j > 0 && hipStreamWaitEvent(sj, r->stage[j - 1], 0) != hipSuccess) st = HOG_E_HIP;
        if (st == HOG_OK)
            st = staged_chain(P, hi - lo, frame_bufs(P, ws, frames, fstride, dets, cap, n_dets, lo, regions), fstride,
                              pitch, prm, bank, cap, tune.nms_rounds, tune.score_rows, ws, sj,
                              stagger && j + 1 < parts ? r->stage[j] : nullptr, stagger);
    }
    // join (also after an error, so that no forked stream is left behind a capture)
    for (int j = 1; j < parts; ++j) {
        if (hipEventRecord(r->ev[j], r->st[j - 1]) != hipSuccess) return HOG_E_HIP;
        if (hipStreamWaitEvent(s, r->ev[j], 0) != hipSuccess) return HOG_E_HIP;
    }
    return st;
}

// ------------------------------------------ fixed scratch (no allocation)
// The workspace of hog_detect_batch_static: one fixed array per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (its host-side name is not a device address); it uses the address
// that hipGetSymbolAddress reports for the current device.
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[HOG_STATIC_SCRATCH_BYTES];

namespace {

// Device address of the current device's scratch array, looked up once per
// device (hog_init, else the first hog_detect_batch_static on the device).
int static_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HOG_E_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return HOG_E_INVAL;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HOG_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HOG_OK;
}

int check_bank(const hog_filterbank* fb) {
    if (!fb || !fb->bias || fb->nf < 1) return HOG_E_INVAL;
    if (fb->nf > MAX_FILTERS) return HOG_E_TOO_LARGE;
    if (fb->rank == 0) return fb->W ? HOG_OK : HOG_E_INVAL;
    if (fb->rank < 1 || fb->rank > SEP_MAX_RANK || !fb->row || !fb->col) return HOG_E_INVAL;
    return HOG_OK;
}

Bank bank_of(const hog_filterbank* fb) {
    Bank b;
    b.W = fb->rank == 0 ? fb->W : nullptr;
    b.row = fb->row;
    b.col = fb->col;
    b.rank = fb->rank;
    b.bias = fb->bias;
    return b;
}

hog_filterbank full_bank(const float* filters, const float* bias, int nf) {
    hog_filterbank fb{};
    fb.nf = nf;
    fb.rank = 0;
    fb.W = filters;
    fb.bias = bias;
    return fb;
}

int check_detect_args(const hog_params* prm, const void* frames, int pitch, int w, const float* filters,
                      const float* bias, int nf, const hog_det* dets, int cap, const int* n_dets) {
    if (!prm || !frames || !filters || !bias || !dets || !n_dets) return HOG_E_INVAL;
    if (pitch < w || pitch > MAX_PITCH) return HOG_E_INVAL;
    if (nf < 1) return HOG_E_INVAL;
    if (nf > MAX_FILTERS) return HOG_E_TOO_LARGE;
    if (cap < 1 || cap > MAX_DETS) return HOG_E_CAP;
    if (!(prm->iou >= 0.5f && prm->iou < 1.f)) return HOG_E_INVAL;
    if (prm->thresh != prm->thresh) return HOG_E_INVAL;
    if (prm->min_face < 0 || prm->min_face > MAX_MIN_FACE) return HOG_E_INVAL;
    if (prm->score_arith != HOG_ARITH_F32 && prm->score_arith != HOG_ARITH_F16X3) return HOG_E_INVAL;
    return HOG_OK;
}

}  // namespace

struct hog_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int hog_version(void) { return 200; }

int hog_params_default(hog_params* p) {
    if (!p) return HOG_E_INVAL;
    p->upsample = 1;
    p->thresh = 0.f;
    p->iou = 0.5f;
    p->min_face = 0;
    p->regions = nullptr;
    p->score_arith = HOG_ARITH_F32;
    return HOG_OK;
}

int hog_constants_get(hog_constants* c) {
    if (!c) return HOG_E_INVAL;
    c->cell_px = CELL;
    c->bins = NBINS;
    c->features = NFEAT;
    c->window_cells = WIN;
    c->min_side = MIN_SIDE;
    c->scale_num = 5;
    c->scale_den = 6;
    c->clip = 0.2f;
    c->eps = 1e-4f;
    return HOG_OK;
}

const char* hog_strerror(int st) {
    switch (st) {
        case HOG_OK: return "ok";
        case HOG_E_INVAL: return "invalid argument";
        case HOG_E_TOO_LARGE: return "frame or filter count above the supported maximum";
        case HOG_E_WORKSPACE: return "workspace smaller than hog_workspace_bytes()";
        case HOG_E_CAP: return "output capacity out of range";
        case HOG_E_HIP: return "HIP launch or runtime failure";
        case HOG_E_NOTIMPL: return "not implemented";
        case HOG_E_DEVICE: return "a bounded device-side wait gave up (detections not valid)";
        case HOG_E_SCRATCH: return "the call needs more workspace than the library's fixed scratch array";
        default: return "unknown status";
    }
}

int hog_orientation_table(double* c, double* s) {
    if (!c || !s) return HOG_E_INVAL;
    orientation_table_host(c, s);
    return HOG_OK;
}

int hog_pyramid(int h, int w, int upsample, int nf, hog_level* levels, int max_levels, int* n_levels) {
    if (!n_levels || (max_levels > 0 && !levels)) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, 1, nf < 0 ? 0 : nf, &P));
    *n_levels = P.T.n;
    for (int k = 0; k < P.T.n && k < max_levels; ++k) {
        const DevLevel& L = P.T.L[k];
        hog_level& o = levels[k];
        o.k = k;
        o.h = L.h;
        o.w = L.w;
        o.cy = L.cy;
        o.cx = L.cx;
        o.rows = L.rows;
        o.cols = L.cols;
        o.reserved = 0;
        o.sig = L.sig;
        o.feat_offset = L.pk_off;
        o.score_offset = L.sc_off;
    }
    return P.T.n > max_levels ? HOG_E_CAP : HOG_OK;
}

size_t hog_workspace_bytes(int h, int w, int upsample, int n_frames, int nf) {
    Plan P;
    if (make_plan(h, w, upsample, n_frames, nf, &P) != HOG_OK) return 0;
    return P.total;
}

int hog_features(const uint8_t* frame, int h, int w, int pitch, int upsample, float* feat, int64_t feat_cap,
                 void* ws, size_t ws_bytes, void* stream) {
    if (!frame || !feat || pitch < w || pitch > MAX_PITCH) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, 1, 0, &P));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    if (feat_cap < P.packed_floats) return HOG_E_CAP;
    if (P.T.n == 0) return HOG_OK;
    return run_pixels(P, frame, 0, pitch, ws, feat, nullptr, (hipStream_t)stream, false);
}

int hog_scores_bank(const uint8_t* frame, int h, int w, int pitch, int upsample, const hog_filterbank* fb,
                    float* scores, int64_t scores_cap, void* ws, size_t ws_bytes, void* stream) {
    if (!frame || !scores || pitch < w || pitch > MAX_PITCH) return HOG_E_INVAL;
    HOG_TRY(check_bank(fb));
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, 1, fb->nf, &P));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    if (scores_cap < P.dense_floats) return HOG_E_CAP;
    if (P.T.n == 0) return HOG_OK;
    hipStream_t s = (hipStream_t)stream;
    const Bank bank = bank_of(fb);
    HOG_TRY(run_pixels(P, frame, 0, pitch, ws, nullptr, bank.W, s, false));
    return score_stage(P, 1, at<float>(ws, P.o_feat), bank, 0.f, scores, nullptr, 0, ws, s);
}

int hog_scores(const uint8_t* frame, int h, int w, int pitch, int upsample, const float* filters,
               const float* bias, int nf, float* scores, int64_t scores_cap, void* ws, size_t ws_bytes,
               void* stream) {
    if (!filters || !bias || nf < 1) return HOG_E_INVAL;
    const hog_filterbank fb = full_bank(filters, bias, nf);
    return hog_scores_bank(frame, h, w, pitch, upsample, &fb, scores, scores_cap, ws, ws_bytes, stream);
}

int hog_scores_arith(const uint8_t* frame, int h, int w, int pitch, int upsample, const float* filters,
                     const float* bias, int nf, int score_arith, float* scores, int64_t scores_cap, void* ws,
                     size_t ws_bytes, void* stream) {
    if (score_arith != HOG_ARITH_F32 && score_arith != HOG_ARITH_F16X3) return HOG_E_INVAL;
    if (score_arith == HOG_ARITH_F32)
        return hog_scores(frame, h, w, pitch, upsample, filters, bias, nf, scores, scores_cap, ws, ws_bytes, stream);
    if (!frame || !scores || !filters || !bias || pitch < w || pitch > MAX_PITCH) return HOG_E_INVAL;
    if (nf < 1) return HOG_E_INVAL;
    if (nf > MAX_FILTERS) return HOG_E_TOO_LARGE;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, 1, nf, &P));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    if (scores_cap < P.dense_floats) return HOG_E_CAP;
    if (P.T.n == 0) return HOG_OK;
    hipStream_t s = (hipStream_t)stream;
    const hog_filterbank fb = full_bank(filters, bias, nf);
    Bank bank = bank_of(&fb);
    bank.f16x3 = true;
    HOG_TRY(run_pixels(P, frame, 0, pitch, ws, nullptr, bank.W, s, false, true));
    return score_stage(P, 1, at<float>(ws, P.o_feat), bank, 0.f, scores, nullptr, 0, ws, s);
}

int hog_detect_batch_bank(const hog_params* prm, const uint8_t* frames, int n, int h, int w, int pitch,
                          int64_t frame_stride, const hog_filterbank* fb, hog_det* dets, int cap, int* n_dets,
                          void* ws, size_t ws_bytes, void* stream) {
    HOG_TRY(check_bank(fb));
    HOG_TRY(check_detect_args(prm, frames, pitch, w, fb->rank ? fb->row : fb->W, fb->bias, fb->nf, dets, cap,
                              n_dets));
    if (n < 1 || (n > 1 && frame_stride < (int64_t)pitch * h)) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, prm->upsample, n, fb->nf, &P, 0, prm->min_face));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    const hog_tuning tune = lookup_tuning(h, w, prm->upsample, n, fb->nf);
    return detect_sequence(P, prm, frames, frame_stride, pitch, bank_of(fb), dets, cap, n_dets, ws, tune,
                           (hipStream_t)stream);
}

int hog_detect_batch(const hog_params* prm, const uint8_t* frames, int n, int h, int w, int pitch,
                     int64_t frame_stride, const float* filters, const float* bias, int nf, hog_det* dets, int cap,
                     int* n_dets, void* ws, size_t ws_bytes, void* stream) {
    HOG_TRY(check_detect_args(prm, frames, pitch, w, filters, bias, nf, dets, cap, n_dets));
    const hog_filterbank fb = full_bank(filters, bias, nf);
    return hog_detect_batch_bank(prm, frames, n, h, w, pitch, frame_stride, &fb, dets, cap, n_dets, ws, ws_bytes,
                                 stream);
}

int hog_detect_batch_static(const hog_params* prm, const uint8_t* frames, int n, int h, int w, int pitch,
                            int64_t frame_stride, const float* filters, const float* bias, int nf, hog_det* dets,
                            int cap, int* n_dets, void* stream) {
    HOG_TRY(check_detect_args(prm, frames, pitch, w, filters, bias, nf, dets, cap, n_dets));
    if (n < 1 || (n > 1 && frame_stride < (int64_t)pitch * h)) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, prm->upsample, n, nf, &P, 0, prm->min_face));
    if (P.total > (size_t)HOG_STATIC_SCRATCH_BYTES) return HOG_E_SCRATCH;
    void* ws = nullptr;
    HOG_TRY(static_scratch(&ws));
    const hog_filterbank fb = full_bank(filters, bias, nf);
    const hog_tuning tune = lookup_tuning(h, w, prm->upsample, n, nf);
    return detect_sequence(P, prm, frames, frame_stride, pitch, bank_of(&fb), dets, cap, n_dets, ws, tune,
                           (hipStream_t)stream);
}

int hog_detect(const hog_params* prm, const uint8_t* frame, int h, int w, int pitch, const float* filters,
               const float* bias, int nf, hog_det* dets, int cap, int* n_dets, void* ws, size_t ws_bytes,
               void* stream) {
    return hog_detect_batch(prm, frame, 1, h, w, pitch, 0, filters, bias, nf, dets, cap, n_dets, ws, ws_bytes,
                            stream);
}

int hog_graph_create_bank(hog_graph** out, const hog_params* prm, const uint8_t* frames, int n, int h, int w,
                          int pitch, int64_t frame_stride, const hog_filterbank* fb, hog_det* dets, int cap,
                          int* n_dets, void* ws, size_t ws_bytes, void* stream) {
    if (!out) return HOG_E_INVAL;
    *out = nullptr;
    HOG_TRY(check_bank(fb));
    HOG_TRY(check_detect_args(prm, frames, pitch, w, fb->rank ? fb->row : fb->W, fb->bias, fb->nf, dets, cap,
                              n_dets));
    if (n < 1 || (n > 1 && frame_stride < (int64_t)pitch * h)) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, prm->upsample, n, fb->nf, &P, 0, prm->min_face));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    hipStream_t cs = (hipStream_t)stream;
    bool own = false;
    if (!cs) {
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return HOG_E_HIP;
        own = true;
    }
    hog_graph* g = new hog_graph();
    int st = HOG_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = HOG_E_HIP;
    } else {
        const hog_tuning tune = lookup_tuning(h, w, prm->upsample, n, fb->nf);
        st = detect_sequence(P, prm, frames, frame_stride, pitch, bank_of(fb), dets, cap, n_dets, ws, tune, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (st == HOG_OK && e != hipSuccess) st = HOG_E_HIP;
        g->graph = graph;
        if (st == HOG_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
            st = HOG_E_HIP;
    }
    if (own) (void)hipStreamDestroy(cs);
    if (st != HOG_OK) {
        hog_graph_destroy(g);
        return st;
    }
    *out = g;
    return HOG_OK;
}

int hog_graph_create(hog_graph** out, const hog_params* prm, const uint8_t* frames, int n, int h, int w,
                     int pitch, int64_t frame_stride, const float* filters, const float* bias, int nf,
                     hog_det* dets, int cap, int* n_dets, void* ws, size_t ws_bytes, void* stream) {
    if (!out) return HOG_E_INVAL;
    *out = nullptr;
    HOG_TRY(check_detect_args(prm, frames, pitch, w, filters, bias, nf, dets, cap, n_dets));
    const hog_filterbank fb = full_bank(filters, bias, nf);
    return hog_graph_create_bank(out, prm, frames, n, h, w, pitch, frame_stride, &fb, dets, cap, n_dets, ws,
                                 ws_bytes, stream);
}

int hog_graph_launch(hog_graph* g, void* stream) {
    if (!g || !g->exec) return HOG_E_INVAL;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? HOG_OK : HOG_E_HIP;
}

int hog_graph_destroy(hog_graph* g) {
    if (!g) return HOG_E_INVAL;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return HOG_OK;
}

int hog_tuning_get(int h, int w, int upsample, int n, int nf, hog_tuning* out) {
    if (!out) return HOG_E_INVAL;
    bool found = false;
    *out = lookup_tuning(h, w, upsample, n, nf, &found);
    return found ? 1 : 0;
}

int hog_track_regions(const hog_det* dets, const int* n_dets, int n, int cap, int h, int w, int margin, int span,
                      hog_region* regions, void* stream) {
    if (!dets || !n_dets || !regions || n < 1 || cap < 1 || cap > MAX_DETS) return HOG_E_INVAL;
    if (h < 1 || w < 1 || h > MAX_SIDE || w > MAX_SIDE) return HOG_E_INVAL;
    if (margin < 0 || margin > MAX_MIN_FACE || span < 0 || span > MAX_LEVELS) return HOG_E_INVAL;
    return timed("track", (hipStream_t)stream, [&] {
        return launch_track(dets, n_dets, n, cap, h, w, margin, span, regions, (hipStream_t)stream);
    });
}

int hog_region_windows(int h, int w, int upsample, int level, const hog_region* region, int32_t* range4) {
    if (!region || !range4) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, 1, 0, &P));
    if (level < 0 || level >= P.T.n) return HOG_E_INVAL;
    const RegionRange R = region_range(P.T.L[level], level, *region);
    range4[0] = R.r_lo;
    range4[1] = R.r_hi;
    range4[2] = R.c_lo;
    range4[3] = R.c_hi;
    return HOG_OK;
}

int hog_init(void) {
    HOG_TRY(init_split_resources());
    void* p = nullptr;
    return static_scratch(&p);
}

int hog_tuning_set(int h, int w, int upsample, int n, int nf, const hog_tuning* t) {
    if (t && tuning_valid(*t) && t->split > 1) HOG_TRY(init_split_resources());
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (!t) {
        g_tune.erase(ShapeKey{h, w, upsample, n, nf});
        return HOG_OK;
    }
    if (!tuning_valid(*t)) return HOG_E_INVAL;
    g_tune[ShapeKey{h, w, upsample, n, nf}] = *t;
    return HOG_OK;
}

int hog_autotune(const hog_params* prm, const uint8_t* frames, int n, int h, int w, int pitch, int64_t frame_stride,
                 const float* filters, const float* bias, int nf, hog_det* dets, int cap, int* n_dets, void* ws,
                 size_t ws_bytes, int reps, hog_tuning* best, float* best_ms, void* stream) {
    HOG_TRY(check_detect_args(prm, frames, pitch, w, filters, bias, nf, dets, cap, n_dets));
    if (!best || !best_ms || reps < 1 || reps > 1000) return HOG_E_INVAL;
    if (n < 1 || (n > 1 && frame_stride < (int64_t)pitch * h)) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, prm->upsample, n, nf, &P, 0, prm->min_face));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    const int cus = compute_units();
    if (cus < 1) return HOG_E_HIP;
    HOG_TRY(init_split_resources());
    std::vector<hog_tuning> cand;
    for (int sp : {1, 2, 4}) {
        if (sp > n) break;
        for (int sg = 0; sg <= (sp > 1 ? 2 : 0); ++sg) {
            for (int nr : {2, 3, 4, 6, 8, 12}) {
                for (int rows : {SCORE_SMALL_ROWS, ROWS_PER_ITEM}) {
                    cand.push_back(default_tuning(h, w, prm->upsample, n, nf));
                    cand.back().split = sp;
                    cand.back().stagger = sg;
                    cand.back().nms_rounds = nr;
                    cand.back().score_rows = rows;
                }
            }
        }
    }
    const int lags[4][2] = {{1, 2}, {1, 3}, {2, 3}, {2, 4}};
    for (int q : {8, 1}) {
        for (const auto& lg : lags) {
            hog_tuning t{};
            t.fused = 1;
            t.queues = q;
            t.wg_per_queue = std::max(1, cus / q);
            t.lag_f = lg[0];
            t.lag_s = lg[1];
            t.split = 1;
            t.nms_rounds = default_tuning(h, w, prm->upsample, n, nf).nms_rounds;
            cand.push_back(t);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const hog_filterbank fbk = full_bank(filters, bias, nf);
    const Bank bank = bank_of(&fbk);
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return HOG_E_HIP;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return HOG_E_HIP;
    }
    int st = HOG_OK;
    float best_t = -1.f;
    hog_tuning pick = cand[0];
    for (const hog_tuning& t : cand) {
        st = detect_sequence(P, prm, frames, frame_stride, pitch, bank, dets, cap, n_dets, ws, t, s);
        if (st != HOG_OK) break;
        if (hipEventRecord(a, s) != hipSuccess) { st = HOG_E_HIP; break; }
        for (int i = 0; i < reps && st == HOG_OK; ++i)
            st = detect_sequence(P, prm, frames, frame_stride, pitch, bank, dets, cap, n_dets, ws, t, s);
        if (st != HOG_OK) break;
        float ms = 0.f;
        if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
            st = HOG_E_HIP;
            break;
        }
        ms /= (float)reps;
        // a schedule that reports an error for any frame is not a candidate
        std::vector<int> counts((size_t)n);
        if (hipMemcpy(counts.data(), n_dets, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) {
            st = HOG_E_HIP;
            break;
        }
        if (std::any_of(counts.begin(), counts.end(), [](int c) { return c < 0; })) continue;
        if (best_t < 0.f || ms < best_t) {
            best_t = ms;
            pick = t;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != HOG_OK) return st;
    HOG_TRY(hog_tuning_set(h, w, prm->upsample, n, nf, &pick));
    *best = pick;
    *best_ms = best_t;
    return HOG_OK;
}

int hog_level_maps(const uint8_t* frame, int h, int w, int pitch, int upsample, int level, float* level_px,
                   uint8_t* bins, float* hist, void* ws, size_t ws_bytes, void* stream) {
    if (!frame || pitch < w || pitch > MAX_PITCH) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, 1, 0, &P));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    if (level < 0 || level >= P.T.n) return HOG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const LevelTable& T = P.T;
    HOG_TRY(timed("geom", s, [&] {
        return launch_setup(T, at<int4>(ws, P.o_taps), at<int2>(ws, P.o_boxes), nullptr, 0, nullptr, nullptr, 0, nullptr, 0, s);
    }));
    uint8_t* casc = at<uint8_t>(ws, P.o_casc);
    HOG_TRY(run_cascade(P, 1, frame, 0, pitch, casc, s));
    if (level_px || bins) {
        HOG_TRY(timed("maps", s, [&] {
            return launch_level_maps(T, level, frame, pitch, at<int4>(ws, P.o_taps), level_px, bins, casc, s);
        }));
    }
    if (hist) {
        HOG_TRY(timed("hist", s, [&] {
            return launch_hist(T, frame, 0, pitch, 1, at<float>(ws, P.o_hist), nullptr, casc, s);
        }));
        const DevLevel& L = T.L[level];
        // part-major records: bins 4q .. 4q + 3 of every cell from plane q
        const size_t ncell = (size_t)L.cy * L.cx;
        const float* src = at<float>(ws, P.o_hist) + (size_t)L.hist_off * HSTRIDE;
        for (int q = 0; q < 5; ++q) {
            const int nb = std::min(4, NBINS - 4 * q);
            if (hipMemcpy2DAsync(hist + 4 * q, NBINS * sizeof(float), src + 4 * q * ncell, 4 * sizeof(float),
                                 nb * sizeof(float), ncell, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return HOG_E_HIP;
        }
    }
    return HOG_OK;
}

size_t hog_grad_workspace_bytes(int h, int w, int upsample, int n_frames, int nf, int n_windows) {
    Plan P;
    if (nf < 1 || make_plan(h, w, upsample, n_frames, nf, &P, std::max(n_windows, 1)) != HOG_OK) return 0;
    return P.total;
}

int hog_window_scores(const uint8_t* frames, int n, int h, int w, int pitch, int64_t frame_stride, int upsample,
                      const float* filters, const float* bias, int nf, const hog_window* windows, int n_windows,
                      float* scores, void* ws, size_t ws_bytes, void* stream) {
    if (!frames || !filters || !bias || !windows || !scores || pitch < w || pitch > MAX_PITCH) return HOG_E_INVAL;
    if (n < 1 || nf < 1 || n_windows < 0 || (n > 1 && frame_stride < (int64_t)pitch * h)) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, n, nf, &P, std::max(n_windows, 1)));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    if (P.T.n == 0 || n_windows == 0) return n_windows == 0 ? HOG_OK : HOG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    HOG_TRY(run_pixels(P, frames, frame_stride, pitch, ws, nullptr, nullptr, s, false));
    return timed("window_scores", s, [&] {
        return launch_window_scores(P.T, n, nf, at<float>(ws, P.o_feat), windows, n_windows, filters, bias, scores,
                                    s);
    });
}

int hog_topk_windows(const uint8_t* frames, int n, int h, int w, int pitch, int64_t frame_stride, int upsample,
                     const float* filters, const float* bias, int nf, int k, hog_window* windows, float* scores,
                     void* ws, size_t ws_bytes, void* stream) {
    if (!frames || !filters || !bias || !windows || !scores || pitch < w || pitch > MAX_PITCH) return HOG_E_INVAL;
    if (n < 1 || nf < 1 || k < 1 || k > 16 || (n > 1 && frame_stride < (int64_t)pitch * h)) return HOG_E_INVAL;
    if (nf > MAX_FILTERS) return HOG_E_TOO_LARGE;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, n, nf, &P, 1));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    if (P.T.n == 0) return HOG_E_INVAL;
    long long total = 0;
    for (int l = 0; l < P.T.n; ++l) total += (long long)P.T.L[l].rows * P.T.L[l].cols * nf;
    if (total < k) return HOG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    HOG_TRY(run_pixels(P, frames, frame_stride, pitch, ws, nullptr, filters, s, false));
    HOG_TRY(timed("score", s, [&] {
        return launch_score(P.T, n, at<float>(ws, P.o_feat), at<float4>(ws, P.o_bpack), bias, nf, 0.f,
                            at<float>(ws, P.o_dense), nullptr, false, score_rows_auto(P.T, n, nf, compute_units()),
                            nullptr, s);
    }));
    return timed("topk", s, [&] {
        return launch_topk(P.T, n, at<float>(ws, P.o_dense), P.T.dense_frame, nf, k, windows, scores, s);
    });
}

int hog_detect_topk(const hog_params* prm, const uint8_t* frames, int n, int h, int w, int pitch, int64_t frame_stride,
                    const float* filters, const float* bias, int nf, hog_det* dets, int cap, int* n_dets, int k,
                    hog_window* windows, float* scores, void* ws, size_t ws_bytes, void* stream) {
    HOG_TRY(check_detect_args(prm, frames, pitch, w, filters, bias, nf, dets, cap, n_dets));
    if (!windows || !scores || k < 1 || k > 16) return HOG_E_INVAL;
    // the top k are taken over every window of every level, in FP32
    if (prm->regions || prm->min_face || prm->score_arith != HOG_ARITH_F32) return HOG_E_INVAL;
    if (n < 1 || (n > 1 && frame_stride < (int64_t)pitch * h)) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, prm->upsample, n, nf, &P, 1));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    if (P.T.n == 0) return HOG_E_INVAL;
    long long total = 0;
    for (int l = 0; l < P.T.n; ++l) total += (long long)P.T.L[l].rows * P.T.L[l].cols * nf;
    if (total < k) return HOG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const bool multi = P.groups > 1;
    const hog_tuning tune = lookup_tuning(h, w, prm->upsample, n, nf);
    // one forward pass: dense scores for the top k and candidate keys for
    // the detection from the same scoring launch
    HOG_TRY(run_pixels(P, frames, frame_stride, pitch, ws, nullptr, filters, s, multi));
    const hog_filterbank fb = full_bank(filters, bias, nf);
    HOG_TRY(score_stage(P, n, at<float>(ws, P.o_feat), bank_of(&fb), prm->thresh, at<float>(ws, P.o_dense),
                        at<unsigned long long>(ws, P.o_key), tune.score_rows, ws, s));
    HOG_TRY(nms_chain(P, n, frame_bufs(P, ws, frames, frame_stride, dets, cap, n_dets, 0), prm, cap, nullptr,
                      tune.nms_rounds, ws, s));
    return timed("topk", s, [&] {
        return launch_topk(P.T, n, at<float>(ws, P.o_dense), P.T.dense_frame, nf, k, windows, scores, s);
    });
}

int hog_filter_backward(const uint8_t* frames, int n, int h, int w, int pitch, int64_t frame_stride, int upsample,
                        const float* filters, int nf, const hog_window* windows, const float* dscore, int n_windows,
                        float* dfilters, float* dbias, float* dpixels, void* ws, size_t ws_bytes, void* stream) {
    if (!frames || !filters || !windows || !dscore || !dfilters || pitch < w || pitch > MAX_PITCH) return HOG_E_INVAL;
    if (n < 1 || nf < 1 || n_windows < 0 || (n > 1 && frame_stride < (int64_t)pitch * h)) return HOG_E_INVAL;
    if (nf > MAX_FILTERS) return HOG_E_TOO_LARGE;
    // the recursive pyramid rounds every level to grey levels: no pixel
    // gradient; the backward recomputes levels from the frame directly
    if (upsample & HOG_PYRAMID_CASCADE) return HOG_E_NOTIMPL;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, n, nf, &P, std::max(n_windows, 1)));
    HOG_TRY(check_ws(P, ws, ws_bytes));
    if (n_windows == 0) return HOG_OK;
    if (P.T.n == 0) return HOG_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const LevelTable& T = P.T;
    HOG_TRY(timed("geom", s, [&] {
        return launch_setup(T, at<int4>(ws, P.o_taps), at<int2>(ws, P.o_boxes), nullptr, 0, nullptr, nullptr, 0, nullptr, 0, s);
    }));
    return timed("backward", s, [&] {
        return launch_backward(T, n, frames, frame_stride, pitch, at<int4>(ws, P.o_taps), filters, windows, dscore,
                               n_windows, nf, at<float>(ws, P.o_partial), dfilters, dbias, dpixels, s);
    });
}

int hog_windows_check(int h, int w, int upsample, int n, int nf, const hog_window* windows, int n_windows,
                      int* first_bad) {
    if (first_bad) *first_bad = -1;
    if (n_windows < 0 || (n_windows > 0 && !windows) || nf < 1) return HOG_E_INVAL;
    Plan P;
    HOG_TRY(make_plan(h, w, upsample, n, nf, &P));
    for (int i = 0; i < n_windows; ++i) {
        if (!window_in_range(P.T, n, nf, windows[i])) {
            if (first_bad) *first_bad = i;
            return HOG_E_INVAL;
        }
    }
    return HOG_OK;
}

int hog_hinge_loss(const float* scores, const float* labels, int n, const float* filters, int nf, float l2,
                   float* loss, float* dscore, float* dfilters, void* stream) {
    if (!scores || !labels || !filters || !loss || !dscore || !dfilters || n < 1 || n > (1 << 30) || nf < 1)
        return HOG_E_INVAL;
    if (nf > MAX_FILTERS) return HOG_E_TOO_LARGE;
    hipStream_t s = (hipStream_t)stream;
    return timed("hinge", s, [&] {
        return launch_hinge(scores, labels, n, filters, nf * WIN * WIN * NFEAT, l2, loss, dscore, dfilters, s);
    });
}

int hog_orient_bins(const int32_t* gx, const int32_t* gy, int64_t n, uint8_t* bins, void* stream) {
    if (n < 0 || n > 0x7fffffffLL) return HOG_E_INVAL;
    if (n > 0 && (!gx || !gy || !bins)) return HOG_E_INVAL;
    return launch_orient(gx, gy, n, bins, (hipStream_t)stream) == hipSuccess ? HOG_OK : HOG_E_HIP;
}

int hog_profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    return HOG_OK;
}

int hog_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto& r : g_prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    return HOG_OK;
}

int hog_profile_read(const char* kernel, double* total_ms, int64_t* count) {
    if (!kernel || !total_ms || !count) return HOG_E_INVAL;
    std::lock_guard<std::mutex> g(g_prof_mu);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto& r : g_prof) {
        if (r.name != kernel) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return HOG_E_HIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return HOG_E_HIP;
        tot += ms;
        ++cnt;
    }
    *total_ms = tot;
    *count = cnt;
    return HOG_OK;
}

}  // extern "C"
