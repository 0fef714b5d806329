// Linear window scoring on the matrix cores (Sec. IV-A linear
// classification; Sec. V-A classifier and detection kernels), one launch
// over all frames, filter groups and levels.
#include <algorithm>
#include <array>
#include <functional>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "stage_score.h"

namespace hog {

// Work item = (frame, filter group, ROWS window rows of the frame's list
// of rows; 16, or 4 for small batches, which then spread over more
// compute units).  Neighbouring rows read 9 of their 10 feature rows in
// common, so the items of a frame are placed on one XCD (one L2): the
// launch is 1-D and block b runs on XCD b mod 8 (blocks are dealt to the
// XCDs in turn, and each XCD starts its blocks in order).  With 8 or more
// (frame, group) units, XCD x takes units [x U / 8, (x + 1) U / 8) and
// runs them slot by slot: block 8 p + x runs slot ord[p / u] of unit
// p mod u (u units on the XCD), where ord is a dispatch order of the
// slots chosen on the host (score_order below).  With fewer units, XCD x
// takes items [x P, (x + 1) P) of the unit-major list (P = blocks / 8).
struct ScoreOrder {
    unsigned char s[SCORE_ORDER_MAX];
};

// The (unit, slot) of this block under the mapping above; false for a
// block past the end.
__device__ __forceinline__ bool score_slot(const ScoreOrder& ord, int per_frame, int units, int* unit_out,
                                           int* it_out) {
    const int x = (int)(blockIdx.x & 7), p = (int)(blockIdx.x >> 3);
    int unit, it;
    if (units >= 8) {
        const int u0 = (int)((long long)x * units / 8);
        const int nu = (int)((long long)(x + 1) * units / 8) - u0;
        it = p / nu;
        unit = u0 + (p - it * nu);
        if (it >= per_frame) return false;
        if (per_frame <= SCORE_ORDER_MAX) it = ord.s[it];
    } else {
        const int item = x * (int)(gridDim.x >> 3) + p;
        if (item >= units * per_frame) return false;
        it = item % per_frame;
        unit = item / per_frame;
    }
    *unit_out = unit;
    *it_out = it;
    return true;
}

// F16: products from split fp16 operands (HOG_ARITH_F16X3).
template <int ROWS, bool F16>
__global__ __launch_bounds__(ROWS * 64) void hog_score_kernel(
    LevelTable T, ScoreOrder ord, int groups, int per_frame, int units, int parts, const float* __restrict__ feat,
    const float4* __restrict__ bpack, const float* __restrict__ bias, int nf, float thresh,
    float* __restrict__ dense, unsigned long long* __restrict__ poskey, int atomic_key,
    const hog_region* __restrict__ regions) {
    using SM = typename std::conditional<F16, Score16SmemT<ROWS>, ScoreSmemT<ROWS>>::type;
    __shared__ SM sm;
    int unit, it;
    if (!score_slot(ord, per_frame, units, &unit, &it)) return;
    const int grp = unit % groups;
    const int frame = unit / groups;
    const int tid = threadIdx.x;
    load_bpack(sm, bpack, grp, tid);
    __syncthreads();
    // parts > 1: slot it runs part it % parts of the tiles of row block it / parts
    score_item<ROWS, F16>(T, frame, grp, parts > 1 ? it / parts : it, sm, sm.P[tid >> 6], feat, nf, bias, thresh,
                          dense, poskey, atomic_key, tid, parts > 1 ? it % parts : -1, regions, parts);
}

// The same work items and dispatch with separable filters (row and column
// factors, RANK pairs per channel; see score_row_sep).
template <int ROWS, int RANK>
__global__ __launch_bounds__(ROWS * 64) void hog_sep_score_kernel(
    LevelTable T, ScoreOrder ord, int groups, int per_frame, int units, int parts, const float* __restrict__ feat,
    const float* __restrict__ row, const float* __restrict__ col, const float* __restrict__ bias, int nf,
    float thresh, float* __restrict__ dense, unsigned long long* __restrict__ poskey, int atomic_key,
    const hog_region* __restrict__ regions) {
    __shared__ SepSmemT<ROWS, RANK> sm;
    int unit, it;
    if (!score_slot(ord, per_frame, units, &unit, &it)) return;
    const int grp = unit % groups;
    const int frame = unit / groups;
    const int tid = threadIdx.x;
    load_sep(sm, row, col, nf, grp, tid);
    __syncthreads();
    score_item_sep<ROWS, RANK>(T, frame, grp, parts > 1 ? it / parts : it, sm, sm.P[tid >> 6], feat, nf, bias,
                               thresh, dense, poskey, atomic_key, tid, parts > 1 ? it % parts : -1, regions, parts);
}

namespace {

// Estimated duration of each slot of ROWS rows, in wave-tiles of the
// busiest SIMD (waves w, w + 4, ... of a workgroup share a SIMD and its
// matrix core), plus the start-up of a workgroup (B to LDS, first loads).
std::vector<double> slot_costs(const LevelTable& T, int rows, int per_frame) {
    std::vector<double> c(per_frame, 0.0);
    for (int s = 0; s < per_frame; ++s) {
        double simd[4] = {0, 0, 0, 0};
        for (int w = 0; w < rows; ++w) {
            const int q = s * rows + w;
            if (q >= T.rows_total) break;
            int k = 0;
            while (k + 1 < T.n && T.L[k + 1].row_off <= q) ++k;
            simd[w & 3] += (T.L[k].cx + 15) / 16;
        }
        c[s] = std::max(std::max(simd[0], simd[1]), std::max(simd[2], simd[3])) + 0.5;
    }
    return c;
}

// Makespan of one XCD: `units` copies of every slot, dispatched slot by
// slot in the given order, each to the compute unit that frees first.
double xcd_makespan(const std::vector<double>& cost, const std::vector<int>& order, int units, int cus) {
    std::vector<double> free_at(cus, 0.0);
    std::make_heap(free_at.begin(), free_at.end(), std::greater<double>());
    double end = 0.0;
    for (int s : order)
        for (int u = 0; u < units; ++u) {
            std::pop_heap(free_at.begin(), free_at.end(), std::greater<double>());
            const double t = free_at.back() + cost[s];
            free_at.back() = t;
            std::push_heap(free_at.begin(), free_at.end(), std::greater<double>());
            end = std::max(end, t);
        }
    return end;
}

std::mutex g_order_mu;
std::map<std::array<int, 6>, ScoreOrder> g_order;

// Dispatch order of the slots for (level geometry, rows, units per XCD,
// compute units per XCD): longest first, then improved by moving single
// slots while the simulated makespan drops.
ScoreOrder score_order(const LevelTable& T, int rows, int per_frame, int units, int cus_xcd) {
    const std::array<int, 6> key{T.h, T.w, T.upsample, rows, units, cus_xcd};
    {
        std::lock_guard<std::mutex> g(g_order_mu);
        auto it = g_order.find(key);
        if (it != g_order.end()) return it->second;
    }
    const std::vector<double> cost = slot_costs(T, rows, per_frame);
    std::vector<int> order(per_frame);
    for (int i = 0; i < per_frame; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    if (per_frame <= SCORE_ORDER_SEARCH) {
        double best = xcd_makespan(cost, order, units, cus_xcd);
        for (int pass = 0; pass < 8; ++pass) {
            bool improved = false;
            for (int i = 0; i < per_frame; ++i)
                for (int j = 0; j < per_frame; ++j) {
                    if (i == j) continue;
                    std::vector<int> o = order;
                    const int v = o[i];
                    o.erase(o.begin() + i);
                    o.insert(o.begin() + j, v);
                    const double m = xcd_makespan(cost, o, units, cus_xcd);
                    if (m < best - 1e-9) {
                        best = m;
                        order = o;
                        improved = true;
                    }
                }
            if (!improved) break;
        }
    }
    ScoreOrder r{};
    for (int i = 0; i < per_frame; ++i) r.s[i] = (unsigned char)order[i];
    std::lock_guard<std::mutex> g(g_order_mu);
    g_order[key] = r;
    return r;
}

}  // namespace

// Grid and dispatch order of a scoring launch (shared by both scorers).
struct ScoreGrid {
    int groups, per_frame, units, parts, blocks;
    ScoreOrder ord;
};

bool score_grid(const LevelTable& T, int n, int nf, int rows, ScoreGrid* g) {
    const int groups = (nf + FGROUP - 1) / FGROUP;
    const long long units = (long long)n * groups;
    int cus = 0;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
    }
    // small items that still leave compute units idle: split the rows'
    // tiles over two slots (a level-0 row takes 3 tile times, not 5), or
    // four where even those fit the compute units (2 tile times)
    const int blocks_of_rows = (T.rows_total + rows - 1) / rows;
    const long long small = rows == SCORE_SMALL_ROWS ? (long long)blocks_of_rows * units : (long long)cus;
    const int parts = 4 * small <= cus ? 4 : small < cus ? 2 : 1;
    const int per_frame = blocks_of_rows * parts;
    const long long items = (long long)per_frame * units;
    if (items <= 0 || items > 0x7fffff00LL) return false;
    g->groups = groups;
    g->per_frame = per_frame;
    g->units = (int)units;
    g->parts = parts;
    g->blocks = units >= 8 ? (int)((units + 7) / 8 * per_frame * 8) : (int)((items + 7) / 8 * 8);
    for (int i = 0; i < SCORE_ORDER_MAX; ++i) g->ord.s[i] = (unsigned char)i;
    if (units >= 8 && per_frame <= SCORE_ORDER_MAX && rows > SCORE_SMALL_ROWS && cus >= 8)
        g->ord = score_order(T, rows, per_frame, (int)((units + 7) / 8), cus / 8);
    return true;
}

hipError_t launch_score_sep(const LevelTable& T, int n, const float* feat, const float* row, const float* col,
                            int rank, const float* bias, int nf, float thresh, float* dense,
                            unsigned long long* poskey, bool atomic_key, int rows, const hog_region* regions,
                            hipStream_t s) {
    ScoreGrid g;
    if (T.rows_total <= 0 || n <= 0) return hipSuccess;
    if (!score_grid(T, n, nf, rows, &g)) return hipErrorInvalidValue;
    const int ak = atomic_key ? 1 : 0;
#define HOG_SEP_LAUNCH(R, K)                                                                                      \
    hipLaunchKernelGGL((hog_sep_score_kernel<R, K>), dim3(g.blocks), dim3(R * 64), 0, s, T, g.ord, g.groups,      \
                       g.per_frame, g.units, g.parts, feat, row, col, bias, nf, thresh, dense, poskey, ak, regions)
    if (rows == SCORE_SMALL_ROWS) {
        switch (rank) {
            case 1: HOG_SEP_LAUNCH(SCORE_SMALL_ROWS, 1); break;
            case 2: HOG_SEP_LAUNCH(SCORE_SMALL_ROWS, 2); break;
            case 3: HOG_SEP_LAUNCH(SCORE_SMALL_ROWS, 3); break;
            case 4: HOG_SEP_LAUNCH(SCORE_SMALL_ROWS, 4); break;
            default: return hipErrorInvalidValue;
        }
    } else if (rows == SEP_ROWS) {
        switch (rank) {
            case 1: HOG_SEP_LAUNCH(SEP_ROWS, 1); break;
            case 2: HOG_SEP_LAUNCH(SEP_ROWS, 2); break;
            case 3: HOG_SEP_LAUNCH(SEP_ROWS, 3); break;
            case 4: HOG_SEP_LAUNCH(SEP_ROWS, 4); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef HOG_SEP_LAUNCH
    return hipGetLastError();
}

int sep_rows_auto(const LevelTable& T, int n, int nf, int cus) {
    const long long items = (long long)((T.rows_total + SEP_ROWS - 1) / SEP_ROWS) * n * ((nf + FGROUP - 1) / FGROUP);
    return items < cus ? SCORE_SMALL_ROWS : SEP_ROWS;
}

int score_rows_auto(const LevelTable& T, int n, int nf, int cus) {
    const long long items16 = (long long)T.ts_total * n * ((nf + FGROUP - 1) / FGROUP);
    return items16 < cus ? SCORE_SMALL_ROWS : ROWS_PER_ITEM;
}

hipError_t launch_score(const LevelTable& T, int n, const float* feat, const float4* bpack, const float* bias,
                        int nf, float thresh, float* dense, unsigned long long* poskey, bool atomic_key, int rows,
                        const hog_region* regions, hipStream_t s, bool f16x3) {
    ScoreGrid g;
    if (T.rows_total <= 0 || n <= 0) return hipSuccess;
    if (!score_grid(T, n, nf, rows, &g)) return hipErrorInvalidValue;
#define HOG_SCORE_LAUNCH(R, F)                                                                                   \
    hipLaunchKernelGGL((hog_score_kernel<R, F>), dim3(g.blocks), dim3(R * 64), 0, s, T, g.ord, g.groups,          \
                       g.per_frame, g.units, g.parts, feat, bpack, bias, nf, thresh, dense, poskey,             \
                       atomic_key ? 1 : 0, regions)
    if (rows == SCORE_SMALL_ROWS) {
        if (f16x3) HOG_SCORE_LAUNCH(SCORE_SMALL_ROWS, true);
        else HOG_SCORE_LAUNCH(SCORE_SMALL_ROWS, false);
    } else if (rows == ROWS_PER_ITEM) {
        if (f16x3) HOG_SCORE_LAUNCH(ROWS_PER_ITEM, true);
        else HOG_SCORE_LAUNCH(ROWS_PER_ITEM, false);
    } else {
        return hipErrorInvalidValue;
    }
#undef HOG_SCORE_LAUNCH
    return hipGetLastError();
}

}  // namespace hog
