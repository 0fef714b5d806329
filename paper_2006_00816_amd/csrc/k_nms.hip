// Non-maximum suppression on the GPU (Sec. IV-A: detections of one face
// are reduced to the best-scoring one; the paper runs this step on the
// CPU, Sec. V-A).
//
// Every window position holds its best candidate key over the filters (a
// window's other filters have the same box and a lower rank, so they are
// suppressed by it or by whatever suppresses it).  Greedy NMS in rank order
// keeps a candidate iff no kept, better-ranked candidate overlaps it with
// IoU > iou.  Two kernels compute exactly that:
//  - hog_nms_edges: for every candidate, in parallel over all frames, the
//    list of better-ranked candidates that overlap it with IoU > iou
//    (exact integer areas), as a record of position indices (16-bit when
//    a frame has fewer than 65536 window positions, else 32-bit);
//  - hog_nms_round: a few decision rounds in parallel over all frames;
//  - hog_nms_resolve: one workgroup per frame decides the rest in rounds
//    over a shrinking worklist (DROPPED if a listed neighbour is kept, KEPT
//    if all are dropped); the best undecided candidate always decides, so
//    the rounds end, with the result of the sequential greedy pass.  Then
//    the kept keys are sorted (the top min(cap, 4096) when there are more)
//    and written out.
#include <algorithm>

#include "hog_device.h"

namespace hog {

enum : unsigned { UNDECIDED = 0, KEPT = 1, DROPPED = 2 };


struct Box {
    int x0, y0, x1, y1;
};

__device__ __forceinline__ Box window_box(const DevLevel& L, const int2* boxes, int r, int c) {
    const int2 ry = boxes[L.box_r + r], cx = boxes[L.box_c + c];
    return Box{cx.x, ry.x, cx.y, ry.y};
}

__device__ __forceinline__ long long floordiv(long long a, long long b) {
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

struct Range {
    int r_lo, r_hi, c_lo, c_hi;
};

// Windows of level M that can overlap box X with IoU > 1/2 (so also with
// IoU above any larger threshold).  IoU > 1/2 needs 3 I > A + A', and
// I <= ov_x * min(h, h'), so the horizontal overlap must exceed
// t_x = (A + A'_min) / (3 min(h, h'_max)): the window's left edge x0' lies
// in (X.x0 + t_x - w'_max, X.x1 - t_x), and x0' is within 1/2 px of
// 8 c' s'^-1.  Bounds in float, widened by 1e-2 window to cover rounding;
// every window inside is then tested exactly.
__device__ __forceinline__ Range neighbour_range(const DevLevel& M, const Box& X, int AX) {
    const float wX = (float)(X.x1 - X.x0), hX = (float)(X.y1 - X.y0);
    const float amin = (float)M.wmin * (float)M.hmin;
    const float tx = ((float)AX + amin) / (3.f * fminf(hX, (float)M.hmax));
    const float ty = ((float)AX + amin) / (3.f * fminf(wX, (float)M.wmax));
    const float inv8 = 137438953472.0f / (float)M.sig;   // 2^40 / (8 sig): level cells per frame px
    Range R;
    R.c_lo = max((int)floorf(((float)X.x0 + tx - (float)M.wmax - 0.5f) * inv8 - 1e-2f) + 1, 0);
    R.c_hi = min((int)ceilf(((float)X.x1 - tx + 0.5f) * inv8 + 1e-2f) - 1, M.cols - 1);
    R.r_lo = max((int)floorf(((float)X.y0 + ty - (float)M.hmax - 0.5f) * inv8 - 1e-2f) + 1, 0);
    R.r_hi = min((int)ceilf(((float)X.y1 - ty + 0.5f) * inv8 + 1e-2f) - 1, M.rows - 1);
    return R;
}

__device__ __forceinline__ int range_bits(const Range& R) {
    return (R.r_hi >= R.r_lo && R.c_hi >= R.c_lo) ? (R.r_hi - R.r_lo + 1) * (R.c_hi - R.c_lo + 1) : 0;
}

// Exact IoU test on integer areas (areas < 2^27): inter / union > num / den.
__device__ __forceinline__ bool conflicts(const Box& X, int AX, const int2& ry, const int2& cx, long long inum,
                                          long long iden) {
    const int iw = min(X.x1, cx.y) - max(X.x0, cx.x);
    const int ih = min(X.y1, ry.y) - max(X.y0, ry.x);
    if (iw <= 0 || ih <= 0) return false;
    const int I = iw * ih;
    const int U = AX + (cx.y - cx.x) * (ry.y - ry.x) - I;
    if (inum == 1 && iden == 2) return 2 * I > U;
    return (long long)I * iden > inum * (long long)U;
}

__device__ __forceinline__ void decode(unsigned long long key, int& f, int& k, int& r, int& c) {
    const unsigned int pk = ~(unsigned int)(key & 0xffffffffu);
    f = pk >> 27;
    k = (pk >> 22) & 31;
    r = (pk >> 11) & 2047;
    c = pk & 2047;
}

// ------------------------------------------------------------ records
// The record of window position p of a frame: NMS_LIST entries of type E,
// entry 0 the count, entries 1.. the conflicting better-ranked positions.
// A count above NMS_LIST - 1 means the list was cut short and the
// candidate is decided by a direct scan instead.  Records are read and
// written in 64-byte chunks of CH entries, stored chunk-major per frame:
// chunk c of position p at lists + frame P NMS_LIST + (c P + p) CH, so the
// first chunks of neighbouring positions (which every pass reads) are
// contiguous.
template <typename E>
struct Rec {
    static constexpr int CH = 64 / (int)sizeof(E);   // entries per chunk
    uint4 c[4];
    // the 64-byte chunk at `chunk`
    __device__ __forceinline__ void load(const E* chunk) {
        const uint4* r4 = reinterpret_cast<const uint4*>(chunk);
        c[0] = r4[0];
        c[1] = r4[1];
        c[2] = r4[2];
        c[3] = r4[3];
    }
    // entry j of the loaded chunk (j a compile-time constant after unrolling)
    __device__ __forceinline__ unsigned at(int j) const {
        if (sizeof(E) == 2) {
            const int w = j >> 1;
            const uint4 q = c[w >> 2];
            const unsigned x = (w & 3) == 0 ? q.x : (w & 3) == 1 ? q.y : (w & 3) == 2 ? q.z : q.w;
            return (j & 1) ? x >> 16 : x & 0xffffu;
        } else {
            const uint4 q = c[j >> 2];
            return (j & 3) == 0 ? q.x : (j & 3) == 1 ? q.y : (j & 3) == 2 ? q.z : q.w;
        }
    }
};

// Per-thread staging of one 64-byte chunk in LDS, as 16 words; word w of
// thread t at stage[w][t], so a wave's accesses fall in different banks.
template <typename E, int BS>
__device__ __forceinline__ void stage_put(unsigned (*stage)[BS], int t, int slot, unsigned v) {
    if (sizeof(E) == 2) {
        unsigned& wd = stage[slot >> 1][t];
        wd = (slot & 1) ? (wd & 0xffffu) | (v << 16) : (wd & 0xffff0000u) | (v & 0xffffu);
    } else {
        stage[slot][t] = v;
    }
}

template <int BS>
__device__ __forceinline__ void stage_flush(unsigned (*stage)[BS], int t, void* dst) {
    uint4* d = reinterpret_cast<uint4*>(dst);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        d[q] = make_uint4(stage[4 * q][t], stage[4 * q + 1][t], stage[4 * q + 2][t], stage[4 * q + 3][t]);
}

// ------------------------------------------------------------ edges
// Exact conflict test from hoisted terms: I = iw+ ih+ (the clamped
// intersection sides), A' the neighbour's area.  IoU > num/den is
// I den > num (AX + A' - I); for 1/2 (HALF) that is 3 I > AX + A'.  A
// box with no overlap has I = 0 and never conflicts (num >= 1, areas > 0).
template <bool HALF>
__device__ __forceinline__ bool conflict_terms(int I, int AX, int A2, long long inum, long long iden) {
    if (HALF) return 3 * I > AX + A2;
    return (long long)I * iden > inum * (long long)(AX + A2 - I);
}

// The better-ranked windows of level M that conflict with candidate X
// (key kx, box X of area AX), in order of column block, row, column;
// `hit` receives each position index.  8 columns at a time: their clamped
// horizontal overlaps and widths once (a column past the range gets
// overlap 0 and re-reads the last key), then each row's 8 keys in flight
// together and a branch-free mask of the conflicting, better-ranked ones.
template <bool HALF, typename F>
__device__ __forceinline__ void scan_level(const DevLevel& M, const Box& X, int AX, unsigned long long kx,
                                           const unsigned long long* __restrict__ keys,
                                           const int2* __restrict__ boxes, long long inum, long long iden, F&& hit) {
    const Range R = neighbour_range(M, X, AX);
    for (int c0 = R.c_lo; c0 <= R.c_hi; c0 += 8) {
        int iw[8], wq[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int2 cb = boxes[M.box_c + min(c0 + q, R.c_hi)];
            iw[q] = c0 + q <= R.c_hi ? max(min(X.x1, cb.y) - max(X.x0, cb.x), 0) : 0;
            wq[q] = cb.y - cb.x;
        }
        for (int r2 = R.r_lo; r2 <= R.r_hi; ++r2) {
            const int2 ry = boxes[M.box_r + r2];
            const int ih = max(min(X.y1, ry.y) - max(X.y0, ry.x), 0);
            const int hr = ry.y - ry.x;
            const unsigned base = (unsigned)(M.pos_off + r2 * M.cols);
            unsigned long long kk[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) kk[q] = keys[base + (unsigned)min(c0 + q, R.c_hi)];
            unsigned hits = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const unsigned better = kk[q] > kx ? 1u : 0u;
                const unsigned h = conflict_terms<HALF>(iw[q] * ih, AX, wq[q] * hr, inum, iden) ? 1u : 0u;
                hits |= (better & h) << q;
            }
            while (hits) {
                const int c2 = c0 + __builtin_ctz(hits);
                hits &= hits - 1;
                hit(base + (unsigned)c2);
            }
        }
    }
}

// One thread per window position of every frame: the record of the
// position, and its first-round state (a candidate with no better-ranked
// conflict is kept).  Workgroups of BS threads (64 for a few frames, so
// that they spread over more compute units).
template <typename E, bool HALF, int BS>
__global__ __launch_bounds__(BS) void hog_nms_edges_kernel(
    LevelTable T, const unsigned long long* __restrict__ poskey, const int2* __restrict__ boxes, long long inum,
    long long iden, E* __restrict__ lists, unsigned char* __restrict__ state8) {
    constexpr int CH = Rec<E>::CH;
    __shared__ unsigned st0[16][BS], st1[16][BS];   // chunk 0 (holds the count) and the current chunk
    const int frame = blockIdx.y;
    const int t = threadIdx.x;
    const int p = blockIdx.x * BS + t;
    if (p >= T.pos_frame) return;
    const unsigned long long* keys = poskey + (long long)frame * T.pos_frame;
    const int P = T.pos_frame;
    E* fl = lists + (long long)frame * P * NMS_LIST;   // the frame's records
    const unsigned long long kx = keys[p];
    int cnt = 0;
    if (kx) {
        int f, k, r, c;
        decode(kx, f, k, r, c);
        const DevLevel& L = T.L[k];
        const Box X = window_box(L, boxes, r, c);
        const int AX = (X.x1 - X.x0) * (X.y1 - X.y0);
        for (int k2 = L.nms_klo; k2 <= L.nms_khi; ++k2)
            scan_level<HALF>(T.L[k2], X, AX, kx, keys, boxes, inum, iden, [&](unsigned y) {
                const int e = 1 + cnt;
                if (e < CH) {
                    stage_put<E, BS>(st0, t, e, y);
                } else if (e < NMS_LIST) {
                    stage_put<E, BS>(st1, t, e % CH, y);
                    if (e % CH == CH - 1) stage_flush(st1, t, fl + ((long long)(e / CH) * P + p) * CH);
                }
                ++cnt;
            });
    }
    stage_put<E, BS>(st0, t, 0, (unsigned)min(cnt, 65535));
    stage_flush(st0, t, fl + (long long)p * CH);
    const int last = min(cnt, NMS_LIST - 1);
    if (last >= CH && last % CH != CH - 1) stage_flush(st1, t, fl + ((long long)(last / CH) * P + p) * CH);
    state8[(long long)frame * T.pos_frame + p] = (unsigned char)(kx == 0ull ? DROPPED : cnt == 0 ? KEPT : UNDECIDED);
}

// The same records for a few frames, where one frame has too few positions
// to fill the GPU: 64 positions per workgroup, and wave s scans level
// nms_klo + s of each (up to 4 levels) into an LDS list; then wave 0
// concatenates the lists in level order, which gives the entries in the
// order of the kernel above.  A level list longer than EDGE_SUB entries
// marks the record as cut short (the per-frame kernel then scans the
// neighbourhood directly, exactly as for any record over NMS_LIST - 1).
constexpr int EDGE_SUB = 64;

template <typename E, bool HALF>
__global__ __launch_bounds__(256) void hog_nms_edges_split_kernel(
    LevelTable T, const unsigned long long* __restrict__ poskey, const int2* __restrict__ boxes, long long inum,
    long long iden, E* __restrict__ lists, unsigned char* __restrict__ state8) {
    constexpr int CH = Rec<E>::CH;
    __shared__ E sub[4][EDGE_SUB][64];
    __shared__ int sub_n[4][64];
    __shared__ unsigned st0[16][64], st1[16][64];
    const int frame = blockIdx.y;
    const int t = threadIdx.x & 63, s = threadIdx.x >> 6;
    const int P = T.pos_frame;
    const int p = blockIdx.x * 64 + t;
    const unsigned long long* keys = poskey + (long long)frame * P;
    const unsigned long long kx = p < P ? keys[p] : 0ull;
    int n = 0;
    if (kx) {
        int f, k, r, c;
        decode(kx, f, k, r, c);
        const DevLevel& L = T.L[k];
        const int k2 = L.nms_klo + s;
        if (k2 <= L.nms_khi) {
            const Box X = window_box(L, boxes, r, c);
            const int AX = (X.x1 - X.x0) * (X.y1 - X.y0);
            scan_level<HALF>(T.L[k2], X, AX, kx, keys, boxes, inum, iden, [&](unsigned y) {
                if (n < EDGE_SUB) sub[s][n][t] = (E)y;
                ++n;
            });
        }
    }
    sub_n[s][t] = n;
    __syncthreads();
    if (s != 0 || p >= P) return;
    E* fl = lists + (long long)frame * P * NMS_LIST;
    int cnt = 0;
    bool cut = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        cnt += sub_n[q][t];
        cut |= sub_n[q][t] > EDGE_SUB;
    }
    if (!cut && cnt < NMS_LIST) {
        int e = 1;
        for (int q = 0; q < 4; ++q) {
            const int nq = sub_n[q][t];
            for (int i = 0; i < nq; ++i, ++e) {
                const unsigned y = sub[q][i][t];
                if (e < CH) {
                    stage_put<E, 64>(st0, t, e, y);
                } else {
                    stage_put<E, 64>(st1, t, e % CH, y);
                    if (e % CH == CH - 1) stage_flush(st1, t, fl + ((long long)(e / CH) * P + p) * CH);
                }
            }
        }
        const int last = cnt;
        if (last >= CH && last % CH != CH - 1) stage_flush(st1, t, fl + ((long long)(last / CH) * P + p) * CH);
    } else {
        cnt = max(cnt, NMS_LIST);
    }
    stage_put<E, 64>(st0, t, 0, (unsigned)min(cnt, 65535));
    stage_flush(st0, t, fl + (long long)p * CH);
    state8[(long long)frame * P + p] = (unsigned char)(kx == 0ull ? DROPPED : cnt == 0 ? KEPT : UNDECIDED);
}

// One parallel round over every window position of every frame: an
// undecided candidate is dropped if a listed neighbour is kept and kept if
// all are dropped.  Neighbour states read while other threads update them
// can only be stale towards UNDECIDED, which delays a decision but never
// changes it.  So the neighbour reads are workgroup-scope atomic loads,
// which may be served by the compute unit's L1 cache: a state that another
// workgroup writes during this round may be seen late, and every state
// written before this launch is seen as written (the L1 is invalidated at
// launch).  A frame's states are a few KB, so the gathers mostly hit L1.
// Candidates whose list overflowed are left to the per-frame kernel.
template <typename E>
__global__ __launch_bounds__(256) void hog_nms_round_kernel(
    LevelTable T, const E* __restrict__ lists, unsigned char* __restrict__ state8) {
    // workgroups of 64 or 256 threads
    constexpr int CH = Rec<E>::CH;
    const int frame = blockIdx.y;
    const int P = T.pos_frame;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    unsigned char* st = state8 + (long long)frame * P;
    if (st[p] != UNDECIDED) return;
    const E* rec = lists + (long long)frame * P * NMS_LIST + (long long)p * CH;
    Rec<E> R;
    R.load(rec);
    const int cnt = (int)R.at(0);
    if (cnt >= NMS_LIST) return;
    bool blocked = false;
    for (int ch = 0; ch * CH <= cnt; ++ch) {
        if (ch) R.load(rec + (long long)ch * P * CH);
        unsigned char sy[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int e = ch * CH + j;
            const bool in = e >= 1 && e <= cnt;
            const unsigned char w =
                __hip_atomic_load(st + (in ? R.at(j) : (unsigned)p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            sy[j] = in ? w : (unsigned char)DROPPED;
        }
        bool kept = false, und = false;
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            kept |= sy[j] == KEPT;
            und |= sy[j] == UNDECIDED;
        }
        if (kept) {
            __hip_atomic_store(st + p, (unsigned char)DROPPED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        blocked |= und;
    }
    if (!blocked) __hip_atomic_store(st + p, (unsigned char)KEPT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------------- resolve
// Decision states live in LDS, 2 bits per window position (16 per word);
// a state only ever changes from UNDECIDED to KEPT or DROPPED, by atomic OR.
// (Frames with too many positions for LDS keep them in global memory,
// accessed with device-scope atomics.)
template <bool G>
__device__ __forceinline__ unsigned state_word(const unsigned* S, int w) {
    if (G) return __hip_atomic_load(S + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return S[w];
}

template <bool G>
__device__ __forceinline__ unsigned state_of(const unsigned* S, int y) {
    return (state_word<G>(S, y >> 4) >> ((y & 15) * 2)) & 3u;
}

// The KEPT positions of a state word, as one bit (the low one) per 2-bit state.
__device__ __forceinline__ unsigned kept_bits(unsigned w) {
    return w & ~(w >> 1) & 0x55555555u;
}

// Direct scan of the neighbourhood (lists that did not fit).
template <bool G>
__device__ unsigned decide_scan(const LevelTable& T, const unsigned long long* keys, const unsigned* S,
                                const int2* boxes, unsigned long long kx, long long inum, long long iden) {
    int f, k, r, c;
    decode(kx, f, k, r, c);
    const DevLevel& L = T.L[k];
    const Box X = window_box(L, boxes, r, c);
    const int AX = (X.x1 - X.x0) * (X.y1 - X.y0);
    bool blocked = false;
    for (int k2 = L.nms_klo; k2 <= L.nms_khi; ++k2) {
        const DevLevel& M = T.L[k2];
        const Range R = neighbour_range(M, X, AX);
        for (int r2 = R.r_lo; r2 <= R.r_hi; ++r2) {
            const int2 ry = boxes[M.box_r + r2];
            const int base = M.pos_off + r2 * M.cols;
            for (int c2 = R.c_lo; c2 <= R.c_hi; ++c2) {
                if (keys[base + c2] <= kx) continue;
                const unsigned sy = state_of<G>(S, base + c2);
                if (sy == DROPPED) continue;
                if (!conflicts(X, AX, ry, boxes[M.box_c + c2], inum, iden)) continue;
                if (sy == KEPT) return DROPPED;
                blocked = true;
            }
        }
    }
    return blocked ? UNDECIDED : KEPT;
}

// Decision from a position's record whose first chunk (at rec) is loaded
// in R; chunk c is at rec + c * cstride.
template <typename E, bool G>
__device__ __forceinline__ unsigned decide_rec(const unsigned* S, const E* rec, long long cstride, Rec<E>& R,
                                               int cnt) {
    constexpr int CH = Rec<E>::CH;
    bool blocked = false;
    for (int ch = 0; ch * CH <= cnt; ++ch) {
        if (ch) R.load(rec + ch * cstride);
        // all state reads of the chunk in flight together, then the checks
        // (16 at a time; unconditional reads, entries past the count
        // redirected to position 0, so that the compiler does not
        // serialise them)
#pragma unroll
        for (int h = 0; h < CH; h += 16) {
            unsigned sy[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int e = ch * CH + h + j;
                const bool in = e >= 1 && e <= cnt;
                const unsigned w = state_of<G>(S, in ? (int)R.at(h + j) : 0);
                sy[j] = in ? w : (unsigned)DROPPED;
            }
            // branch-free over the 16 entries, one branch per block
            bool kept = false, und = false;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                kept |= sy[j] == KEPT;
                und |= sy[j] == UNDECIDED;
            }
            if (kept) return DROPPED;
            blocked |= und;
        }
    }
    return blocked ? UNDECIDED : KEPT;
}

// Appends p to a worklist when `take`; one LDS atomic per wave.
template <typename W>
__device__ __forceinline__ void wave_append(bool take, int p, W* list, int* counter) {
    const unsigned long long m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == __builtin_ctzll(m)) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, __builtin_ctzll(m), 64);
    if (take) list[base + __popcll(m & ((1ull << lane) - 1ull))] = (W)p;
}

constexpr int RESOLVE_BATCH = 2;   // worklist items per thread whose records are loaded together

// Record cache of the per-frame kernel: once the worklist is short enough,
// the records of its candidates are copied into LDS and the rest is
// decided from LDS.  Layout of the dynamic LDS after the states:
// RC_CHUNKS 64-byte chunks (also the sort buffer afterwards), then per
// cached candidate its position and first chunk, then two worklists of
// cached-candidate indices (the first also the rank order), then the
// cached candidates' keys.
constexpr int RC_MAXI = 2048;
// Cached candidates decided in rank order by one wave.  Up to this many
// the single-wave pass is the shorter chain; above it (many undecided
// after few parallel rounds) its 64-lane blocks run one after another and
// parallel passes over the cache are faster (one 64-frame clip after 3
// rounds: 221 us with 2048 here, 108 us with 256).
constexpr int RANK_DECIDE_MAX = 256;
constexpr int RC_CHUNKS = 1536;
constexpr int RC_BYTES = RC_CHUNKS * 64 + RC_MAXI * (4 + 2 + 2 + 2 + 8);
static_assert(RC_CHUNKS * 64 >= SORT_CAP * 8, "sort buffer aliases the chunk cache");
static_assert(SORT_CAP % NMS_THREADS == 0, "kept keys per thread in the gather");

template <typename E, bool G>
__global__ __launch_bounds__(NMS_THREADS) void hog_nms_resolve_kernel(
    LevelTable T, const unsigned long long* __restrict__ poskey, const E* __restrict__ lists,
    const int2* __restrict__ boxes, long long inum, long long iden, hog_det* __restrict__ dets, int cap,
    int* __restrict__ n_dets, unsigned* __restrict__ gstate, int* __restrict__ work,
    const unsigned char* __restrict__ state8, const unsigned* __restrict__ upstream, FusedNeed need, int n,
    int frame_base) {
    extern __shared__ __align__(16) unsigned dyn[];   // [2-bit states (LDS variant)] + record cache
    __shared__ unsigned int hist[256];
    __shared__ int s_count, s_next;
    __shared__ unsigned long long s_prefix, s_mask;
    __shared__ int s_remaining;

    const int tid = threadIdx.x;
    const int frame = blockIdx.x;
    // after the fused kernel: if one of its bounded waits gave up, or this
    // frame's items did not all finish, the candidates are not
    // trustworthy; report the error in place of a count
    if (upstream) {
        const unsigned* cnt = upstream + FUSED_SYNC_HEAD;
        if (upstream[FUSED_SYNC_ERR] || cnt[frame] != need.hist || cnt[n + frame] != need.feat ||
            cnt[2 * n + frame] != need.score) {
            if (tid == 0) n_dets[frame] = HOG_E_DEVICE;
            return;
        }
    }
    const int P = T.pos_frame;
    const int nw = (P + 15) >> 4;
    const int sw = G ? 0 : (nw + 3) & ~3;          // state words in LDS, 16-byte multiple
    unsigned* S = G ? gstate + (long long)frame * nw : dyn;
    uint4* rc_chunks = reinterpret_cast<uint4*>(dyn + sw);
    unsigned long long* sk = reinterpret_cast<unsigned long long*>(rc_chunks);
    int* rc_pos = reinterpret_cast<int*>(rc_chunks + 4 * RC_CHUNKS);
    unsigned short* rc_first = reinterpret_cast<unsigned short*>(rc_pos + RC_MAXI);
    // the two worklists of each kind are addressed by offset, not through an
    // array of pointers, so that the compiler keeps their address spaces
    // (LDS / global) instead of generic flat accesses
    unsigned short* const rc_wl = rc_first + RC_MAXI;   // rc_wl + b * RC_MAXI, b = 0, 1
    unsigned long long* const rc_key = reinterpret_cast<unsigned long long*>(rc_wl + 2 * RC_MAXI);
    __shared__ int s_chunks;
    const unsigned long long* keys = poskey + (long long)frame * P;
    const E* lst = lists + (long long)frame * P * NMS_LIST;
    int* const wl = work + (long long)frame * 2 * P;   // wl + b * P, b = 0, 1

    // states left by the parallel rounds, and the worklist of the undecided
    const unsigned char* st8 = state8 + (long long)frame * P;
    if (tid == 0) s_count = 0;
    __syncthreads();
    for (int w0 = 0; w0 < nw; w0 += NMS_THREADS) {
        const int w = w0 + tid;
        if (w < nw) {
            unsigned v = 0;
            for (int j = 0; j < 16; ++j) {
                const int p = 16 * w + j;
                v |= (p < P ? (unsigned)st8[p] : (unsigned)DROPPED) << (2 * j);
            }
            if (G) __hip_atomic_store(S + w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else S[w] = v;
        }
    }
    __syncthreads();
    for (int p0 = 0; p0 < P; p0 += NMS_THREADS) {
        const int p = p0 + tid;
        wave_append(p < P && state_of<G>(S, p) == UNDECIDED, p, wl, &s_count);
    }
    __syncthreads();

    constexpr int CH = Rec<E>::CH;
    int cur = 0;
    bool cached = false;
    for (int round = 0; round <= P; ++round) {
        const int n_in = s_count;
        if (n_in == 0) break;
        if (!cached && n_in <= RC_MAXI) {
            // try to cache the records of the worklist: count their chunks
            if (tid == 0) s_chunks = 0;
            __syncthreads();
            const int* in = wl + (long long)cur * P;
            for (int i = tid; i < n_in; i += NMS_THREADS) {
                const int p = in[i];
                const int cnt = (int)lst[(long long)p * CH];
                rc_pos[i] = p;
                // overflowed lists (decided by a scan) take no chunks: 0xffff
                rc_first[i] = cnt < NMS_LIST ? (unsigned short)min(atomicAdd(&s_chunks, cnt / CH + 1), 65534)
                                             : (unsigned short)0xffff;
            }
            __syncthreads();
            if (s_chunks <= RC_CHUNKS) {
                for (int i = tid; i < n_in; i += NMS_THREADS) {
                    rc_wl[i] = (unsigned short)i;
                    if (rc_first[i] == 0xffff) continue;
                    const E* rec = lst + (long long)rc_pos[i] * CH;
                    const int cnt = (int)rec[0];
                    uint4* dst = rc_chunks + 4 * (int)rc_first[i];
                    for (int c = 0; c <= cnt / CH; ++c) {
                        const uint4* src = reinterpret_cast<const uint4*>(rec + (long long)c * P * CH);
#pragma unroll
                        for (int q = 0; q < 4; ++q) dst[4 * c + q] = src[q];
                    }
                }
                cached = true;
                cur = 0;
                __syncthreads();
                // Up to RANK_DECIDE_MAX cached candidates: in rank order (a
                // candidate's place is the number of larger keys; keys are
                // distinct), then decided in that order by the first wave,
                // 64 at a time.  More: parallel passes over the cache.
                // Every listed neighbour of a candidate ranks better, so it
                // is decided in an earlier block or is an earlier lane of
                // this block; the earliest undecided lane can therefore
                // always decide, and each step of a block decides at least
                // one lane.  The result is the sequential greedy pass.
                if (n_in > RANK_DECIDE_MAX) continue;
                for (int i = tid; i < n_in; i += NMS_THREADS) rc_key[i] = keys[rc_pos[i]];
                __syncthreads();
                for (int i = tid; i < n_in; i += NMS_THREADS) {
                    const unsigned long long ki = rc_key[i];
                    int rank = 0;
                    for (int q = 0; q < n_in; ++q) rank += rc_key[q] > ki ? 1 : 0;
                    rc_wl[rank] = (unsigned short)i;
                }
                __syncthreads();
                if (tid < 64) {
                    for (int b0 = 0; b0 < n_in; b0 += 64) {
                        const int idx = b0 + tid;
                        bool und = idx < n_in;
                        const int it = und ? (int)rc_wl[idx] : 0;
                        const int p = rc_pos[it];
                        const int first = rc_first[it];
                        // at most 64 steps (each decides a lane); the bound
                        // also ends the loop if that did not hold
                        for (int step = 0; step < 64 && __ballot(und); ++step) {
                            if (und) {
                                unsigned v;
                                if (first != 0xffff) {
                                    const E* rec = reinterpret_cast<const E*>(rc_chunks + 4 * first);
                                    Rec<E> R;
                                    R.load(rec);
                                    v = decide_rec<E, G>(S, rec, CH, R, (int)R.at(0));
                                } else {
                                    v = decide_scan<G>(T, keys, S, boxes, keys[p], inum, iden);
                                }
                                if (v != UNDECIDED) {
                                    atomicOr(&S[p >> 4], v << ((p & 15) * 2));
                                    und = false;
                                }
                            }
                            // this step's decisions before the next step's reads
                            if (G) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                            wave_lds_order();
                        }
                    }
                }
                __syncthreads();
                break;
            }
        }
        if (tid == 0) s_next = 0;
        __syncthreads();
        if (cached) {
            const unsigned short* in = rc_wl + cur * RC_MAXI;
            for (int i0 = 0; i0 < n_in; i0 += NMS_THREADS) {
                const int i = i0 + tid;
                bool keep_working = false;
                int it = 0;
                if (i < n_in) {
                    it = in[i];
                    const int p = rc_pos[it];
                    const int first = rc_first[it];
                    unsigned v;
                    if (first != 0xffff) {
                        const E* rec = reinterpret_cast<const E*>(rc_chunks + 4 * first);
                        Rec<E> R;
                        R.load(rec);
                        v = decide_rec<E, G>(S, rec, CH, R, (int)R.at(0));
                    } else {
                        v = decide_scan<G>(T, keys, S, boxes, keys[p], inum, iden);
                    }
                    if (v != UNDECIDED) atomicOr(&S[p >> 4], v << ((p & 15) * 2));
                    else keep_working = true;
                }
                wave_append(keep_working, it, rc_wl + (cur ^ 1) * RC_MAXI, &s_next);
            }
        } else {
            const int* in = wl + (long long)cur * P;
            for (int i0 = 0; i0 < n_in; i0 += RESOLVE_BATCH * NMS_THREADS) {
                int pp[RESOLVE_BATCH];
                Rec<E> R[RESOLVE_BATCH];
#pragma unroll
                for (int b = 0; b < RESOLVE_BATCH; ++b) {
                    const int i = i0 + b * NMS_THREADS + tid;
                    pp[b] = i < n_in ? in[i] : -1;
                }
#pragma unroll
                for (int b = 0; b < RESOLVE_BATCH; ++b)
                    if (pp[b] >= 0) R[b].load(lst + (long long)pp[b] * CH);
#pragma unroll
                for (int b = 0; b < RESOLVE_BATCH; ++b) {
                    bool keep_working = false;
                    const int p = pp[b];
                    if (p >= 0) {
                        const int cnt = (int)R[b].at(0);
                        const unsigned v = cnt < NMS_LIST
                                               ? decide_rec<E, G>(S, lst + (long long)p * CH, (long long)P * CH, R[b], cnt)
                                               : decide_scan<G>(T, keys, S, boxes, keys[p], inum, iden);
                        if (v != UNDECIDED) atomicOr(&S[p >> 4], v << ((p & 15) * 2));
                        else keep_working = true;
                    }
                    wave_append(keep_working, p, wl + (long long)(cur ^ 1) * P, &s_next);
                }
            }
        }
        __syncthreads();
        if (tid == 0) s_count = s_next;
        cur ^= 1;
        __syncthreads();
    }

    // count the kept candidates
    if (tid == 0) s_count = 0;
    __syncthreads();
    // (positions past the end of the last word are DROPPED)
    int mine = 0;
    for (int w = tid; w < nw; w += NMS_THREADS) mine += __popc(kept_bits(state_word<G>(S, w)));
    if (mine) atomicAdd(&s_count, mine);
    __syncthreads();
    const int nkept = s_count;
    const int want = min(nkept, min(cap, SORT_CAP));

    // threshold key: the want-th largest kept key (keys are unique)
    unsigned long long thr = 0ull;
    if (nkept > SORT_CAP) {
        if (tid == 0) { s_prefix = 0ull; s_mask = 0ull; s_remaining = want; }
        __syncthreads();
        for (int shift = 56; shift >= 0; shift -= 8) {
            for (int b = tid; b < 256; b += NMS_THREADS) hist[b] = 0u;
            __syncthreads();
            const unsigned long long pre = s_prefix, msk = s_mask;
            for (int p = tid; p < P; p += NMS_THREADS) {
                if (state_of<G>(S, p) != KEPT) continue;
                const unsigned long long kk = keys[p];
                if ((kk & msk) == pre) atomicAdd(&hist[(kk >> shift) & 255], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                int rem = s_remaining, cum = 0, dsel = 0;
                for (int dgt = 255; dgt >= 0; --dgt) {
                    if (cum + (int)hist[dgt] >= rem) { dsel = dgt; break; }
                    cum += hist[dgt];
                }
                s_remaining = rem - cum;
                s_prefix = pre | ((unsigned long long)dsel << shift);
                s_mask = msk | (255ull << shift);
            }
            __syncthreads();
        }
        thr = s_prefix;
    }

    // gather kept keys >= thr
    if (tid == 0) s_count = 0;
    __syncthreads();
    if (nkept <= SORT_CAP) {
        // all kept: their positions first, then their keys, each thread's
        // loads in flight together
        for (int w = tid; w < nw; w += NMS_THREADS) {
            unsigned m = kept_bits(state_word<G>(S, w));
            if (!m) continue;
            int slot = atomicAdd(&s_count, __popc(m));
            while (m) {
                sk[slot++] = (unsigned long long)(16 * w + (__builtin_ctz(m) >> 1));
                m &= m - 1u;
            }
        }
        __syncthreads();
        constexpr int KU = SORT_CAP / NMS_THREADS;
        unsigned long long kk[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int e = tid + u * NMS_THREADS;
            kk[u] = e < nkept ? keys[(int)sk[e]] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int e = tid + u * NMS_THREADS;
            if (e < nkept) sk[e] = kk[u];
        }
    } else {
        for (int w = tid; w < nw; w += NMS_THREADS) {
            unsigned m = kept_bits(state_word<G>(S, w));
            while (m) {
                const int p = 16 * w + (__builtin_ctz(m) >> 1);
                m &= m - 1u;
                const unsigned long long kk = keys[p];
                if (kk < thr) continue;
                const int slot = atomicAdd(&s_count, 1);
                if (slot < SORT_CAP) sk[slot] = kk;
            }
        }
    }
    __syncthreads();
    const int ng = min(s_count, SORT_CAP);
    if (ng <= NMS_THREADS) {
        // the keys are distinct, so a key's place in descending order is
        // the number of larger keys (all threads of a wave read the same
        // two keys at a time: LDS broadcasts; waves without a key skip)
        const unsigned long long mykey = tid < ng ? sk[tid] : 0ull;
        int rank = 0;
        if ((tid & ~63) < ng) {
            const ulonglong2* __restrict__ sk2 = reinterpret_cast<const ulonglong2*>(sk);
            for (int i = 0; i < (ng >> 1); ++i) {
                const ulonglong2 q = sk2[i];
                rank += (q.x > mykey ? 1 : 0) + (q.y > mykey ? 1 : 0);
            }
            if (ng & 1) rank += sk[ng - 1] > mykey ? 1 : 0;
        }
        __syncthreads();
        if (tid < ng) sk[rank] = mykey;
        __syncthreads();
    } else {
        int npow = 1;
        while (npow < ng) npow <<= 1;
        for (int e = ng + tid; e < npow; e += NMS_THREADS) sk[e] = 0ull;
        __syncthreads();
        // bitonic sort, descending
        for (int size = 2; size <= npow; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int e = tid; e < npow; e += NMS_THREADS) {
                    const int partner = e ^ stride;
                    if (partner > e) {
                        const bool desc = (e & size) == 0;
                        const unsigned long long a = sk[e], b = sk[partner];
                        if ((a < b) == desc) { sk[e] = b; sk[partner] = a; }
                    }
                }
                __syncthreads();
            }
        }
    }

    const int nout = min(ng, cap);
    for (int e = tid; e < nout; e += NMS_THREADS) {
        const unsigned long long kk = sk[e];
        int f, k, r, c;
        decode(kk, f, k, r, c);
        const Box b = window_box(T.L[k], boxes, r, c);
        hog_det d;
        d.frame = frame_base + frame; d.filter = f; d.level = T.k_base + k; d.row = r; d.col = c;
        d.x0 = b.x0; d.y0 = b.y0; d.x1 = b.x1; d.y1 = b.y1;
        d.score = score_from_order((unsigned int)(kk >> 32));
        dets[(long long)frame * cap + e] = d;
    }
    if (tid == 0) n_dets[frame] = nkept;
}

// Positions whose states fit in LDS next to the sort buffer.
constexpr int NMS_LDS_STATE_WORDS = (160 * 1024 - RC_BYTES - 2048) / 4;

// Up to this many frames, the per-position kernels use 64-thread workgroups.
constexpr int NMS_SMALL_BATCH = 4;

template <typename E>
void edges_launch(bool half, int bs, dim3 grid, const LevelTable& T, const unsigned long long* poskey,
                  const int2* boxes, long long inum, long long iden, E* lists, unsigned char* state8, hipStream_t s) {
    int span = 0;
    for (int k = 0; k < T.n; ++k) span = std::max(span, T.L[k].nms_khi - T.L[k].nms_klo + 1);
    if (bs == 64 && span > 4) {
        if (half)
            hipLaunchKernelGGL((hog_nms_edges_kernel<E, true, 64>), grid, dim3(64), 0, s, T, poskey, boxes, inum,
                               iden, lists, state8);
        else
            hipLaunchKernelGGL((hog_nms_edges_kernel<E, false, 64>), grid, dim3(64), 0, s, T, poskey, boxes, inum,
                               iden, lists, state8);
    } else if (bs == 64) {
        // a few frames: the 4-wave kernel that scans the levels of a
        // position in parallel (each position's levels span at most 4)
        if (half)
            hipLaunchKernelGGL((hog_nms_edges_split_kernel<E, true>), grid, dim3(256), 0, s, T, poskey, boxes, inum,
                               iden, lists, state8);
        else
            hipLaunchKernelGGL((hog_nms_edges_split_kernel<E, false>), grid, dim3(256), 0, s, T, poskey, boxes, inum,
                               iden, lists, state8);
    } else if (half) {
        hipLaunchKernelGGL((hog_nms_edges_kernel<E, true, 256>), grid, dim3(256), 0, s, T, poskey, boxes, inum, iden,
                           lists, state8);
    } else {
        hipLaunchKernelGGL((hog_nms_edges_kernel<E, false, 256>), grid, dim3(256), 0, s, T, poskey, boxes, inum,
                           iden, lists, state8);
    }
}

hipError_t launch_nms_edges(const LevelTable& T, int n, const unsigned long long* poskey, const int2* boxes,
                            long long iou_num, long long iou_den, void* lists, unsigned char* state8, int rounds,
                            hipStream_t s) {
    // a few frames: workgroups of 64 threads, so that the positions of a
    // frame spread over four times as many compute units
    const int bs = n <= NMS_SMALL_BATCH ? 64 : 256;
    const dim3 grid((T.pos_frame + bs - 1) / bs, n);
    const bool half = iou_num == 1 && iou_den == 2;
    if (nms_wide_lists(T.pos_frame)) {
        edges_launch<unsigned>(half, bs, grid, T, poskey, boxes, iou_num, iou_den, (unsigned*)lists, state8, s);
        for (int r = 0; r < rounds; ++r)
            hipLaunchKernelGGL(hog_nms_round_kernel<unsigned>, grid, dim3(bs), 0, s, T, (const unsigned*)lists,
                               state8);
    } else {
        edges_launch<unsigned short>(half, bs, grid, T, poskey, boxes, iou_num, iou_den, (unsigned short*)lists,
                                     state8, s);
        for (int r = 0; r < rounds; ++r)
            hipLaunchKernelGGL(hog_nms_round_kernel<unsigned short>, grid, dim3(bs), 0, s, T,
                               (const unsigned short*)lists, state8);
    }
    return hipGetLastError();
}

template <typename E>
void launch_resolve(const LevelTable& T, int n, const unsigned long long* poskey, const void* lists,
                    const int2* boxes, long long iou_num, long long iou_den, void* dets, int cap, int* n_dets,
                    unsigned* gstate, int* work, const unsigned char* state8, const unsigned* upstream,
                    FusedNeed need, int frame_base, hipStream_t s) {
    const int nw = (T.pos_frame + 15) >> 4;
    if (nw <= NMS_LDS_STATE_WORDS) {
        const size_t lds = sizeof(unsigned) * (size_t)((nw + 3) & ~3) + RC_BYTES;
        (void)hipFuncSetAttribute((const void*)hog_nms_resolve_kernel<E, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((hog_nms_resolve_kernel<E, false>), dim3(n), dim3(NMS_THREADS), lds, s, T, poskey,
                           (const E*)lists, boxes, iou_num, iou_den, (hog_det*)dets, cap, n_dets, gstate, work,
                           state8, upstream, need, n, frame_base);
    } else {
        (void)hipFuncSetAttribute((const void*)hog_nms_resolve_kernel<E, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, RC_BYTES);
        hipLaunchKernelGGL((hog_nms_resolve_kernel<E, true>), dim3(n), dim3(NMS_THREADS), RC_BYTES, s, T, poskey,
                           (const E*)lists, boxes, iou_num, iou_den, (hog_det*)dets, cap, n_dets, gstate, work,
                           state8, upstream, need, n, frame_base);
    }
}

hipError_t launch_nms(const LevelTable& T, int n, const unsigned long long* poskey, const void* lists,
                      const int2* boxes, long long iou_num, long long iou_den, void* dets, int cap, int* n_dets,
                      unsigned* gstate, int* work, const unsigned char* state8, const unsigned* upstream,
                      FusedNeed need, int frame_base, hipStream_t s) {
    if (nms_wide_lists(T.pos_frame))
        launch_resolve<unsigned>(T, n, poskey, lists, boxes, iou_num, iou_den, dets, cap, n_dets, gstate, work,
                                 state8, upstream, need, frame_base, s);
    else
        launch_resolve<unsigned short>(T, n, poskey, lists, boxes, iou_num, iou_den, dets, cap, n_dets, gstate,
                                       work, state8, upstream, need, frame_base, s);
    return hipGetLastError();
}

}  // namespace hog
