// One persistent launch for resample -> gradients -> orientation -> cell
// histograms -> normalisation/31-d features -> window scores of every frame
// and every pyramid level of a batch (Sec. IV-A steps; Sec. V-A runs them
// as separate kernels per scale).
#include "stage_feat.h"
#include "stage_hist.h"
#include "stage_score.h"

namespace hog {

union FusedSmem {
    HistSmem hist[2];        // two histogram tiles side by side (512 threads each)
    ScoreSmem score;         // one scoring item (16 waves)
};

// Item completion is published through per-frame counters.  Two
// protocols:
//  - XCD-local (queues = 8): a workgroup serves the queue of the XCD it
//    runs on (hardware register XCC_ID), so the producers and consumers of
//    a frame share one L2.  A wave waits for its own stores to complete
//    (they are written through to L2) before a relaxed counter increment;
//    a consumer invalidates its CU's L1 after seeing the count.  This is
//    the workgroup-scope protocol of waves that share an L2 but not an L1.
//  - device-wide (queues != 8): release increment / acquire after the
//    count, at agent scope, which writes back and invalidates L2.
// Waits are bounded: past `limit` polls the error word is set and the item
// proceeds, so the kernel always drains.
template <bool LOCAL>
__device__ __forceinline__ void wait_count(const unsigned* c, unsigned need, unsigned* err, unsigned limit,
                                           int tid) {
    if (tid == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (++spins > limit) {
                atomicOr(err, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        if (LOCAL) asm volatile("buffer_inv sc0" ::: "memory");
        else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

template <bool LOCAL>
__device__ __forceinline__ void wave_done(unsigned* c, int tid) {
    if (LOCAL) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if ((tid & 63) == 0) __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        if ((tid & 63) == 0) __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ unsigned xcc_id() {
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & 15u;
}

// Work list.  Frames are split over Q queues (frame f in queue f mod Q).
// With Q = 8 a workgroup serves the queue of its XCD, so a frame's
// histograms, features and scores stay in one L2 (workgroups are
// dispatched to the 8 XCDs in turn, so each XCD gets wg_per_queue of
// them); otherwise workgroup b serves queue b mod Q.  A queue is a sequence
// of slots; slot s holds, in this order,
//   the scoring items of the queue's frame s - lag_s   (ts_total x groups),
//   the feature items of its frame s - lag_f           (4 blocks of 256 cells each),
//   the histogram items of its frame s                 (2 tiles each),
// and workgroups take items in ticket order from the queue's atomic
// counter.  A feature item waits until its frame's histogram items are
// done, a scoring item until its frame's feature items are done; with
// 1 <= lag_f < lag_s those have smaller tickets, so they were taken by
// running workgroups and every wait ends (no co-residency assumption).
// Every finished item also counts in its frame's counters; the NMS kernel
// that follows checks them, so a queue that no workgroup served shows up
// as an error instead of missing detections.
template <bool LOCAL>
__global__ __launch_bounds__(SCORE_THREADS) void hog_fused_kernel(
    LevelTable T, int n, int groups, int Q, int lag_f, int lag_s, const uint8_t* __restrict__ frames,
    long long fstride, int pitch, float* __restrict__ hist, float* __restrict__ feat,
    const float4* __restrict__ bpack, const float* __restrict__ bias, int nf, float thresh,
    unsigned long long* __restrict__ poskey, int atomic_key, unsigned* __restrict__ sync, unsigned spin_limit) {
    __shared__ FusedSmem sm;
    __shared__ int s_ticket;
    const int tid = threadIdx.x;
    const int q = LOCAL ? (int)(xcc_id() % (unsigned)Q) : (int)(blockIdx.x % (unsigned)Q);
    const int nq = (n - q + Q - 1) / Q;
    if (nq <= 0) return;
    const int nH = (T.th_total + 1) / 2, nF = (T.tf_total + 3) / 4, nS = T.ts_total * groups;
    const int Z = nS + nF + nH;
    const long long total = (long long)(nq + lag_s) * Z;
    unsigned* ticket = sync + q;
    unsigned* err = sync + FUSED_SYNC_ERR;
    unsigned* hdone = sync + FUSED_SYNC_HEAD;
    unsigned* fdone = hdone + n;
    unsigned* sdone = fdone + n;
    const unsigned waves = SCORE_THREADS / 64;

    // the two barriers around the ticket also separate one item's LDS use
    // from the next one's
    for (;;) {
        if (tid == 0) s_ticket = (int)atomicAdd(ticket, 1u);
        __syncthreads();
        const long long tk = s_ticket;
        __syncthreads();
        if (tk >= total) break;
        const int slot = (int)(tk / Z), o = (int)(tk % Z);
        if (o < nS) {
            const int jf = slot - lag_s;
            if (jf < 0 || jf >= nq) continue;
            const int frame = q + Q * jf;
            wait_count<LOCAL>(fdone + frame, waves * nF, err, spin_limit, tid);
            const int grp = o / T.ts_total, it = o % T.ts_total;
            load_bpack<ROWS_PER_ITEM>(sm.score, bpack, grp, tid);
            __syncthreads();
            score_item<ROWS_PER_ITEM>(T, frame, grp, it, sm.score, sm.score.P[tid >> 6], feat, nf, bias, thresh, nullptr, poskey,
                       atomic_key, tid);
            wave_done<LOCAL>(sdone + frame, tid);
        } else if (o < nS + nF) {
            const int jf = slot - lag_f;
            if (jf < 0 || jf >= nq) continue;
            const int frame = q + Q * jf;
            wait_count<LOCAL>(hdone + frame, waves * nH, err, spin_limit, tid);
            const int blk = 4 * (o - nS) + (tid >> 8);
            if (blk < T.tf_total) feat_cell(T, hist, feat, nullptr, frame, blk, tid & 255);
            wave_done<LOCAL>(fdone + frame, tid);
        } else {
            const int jf = slot;
            if (jf >= nq) continue;
            const int frame = q + Q * jf;
            int tile = 2 * (o - nS - nF) + (tid >> 9);
            if (tile >= T.th_total) tile = -1;
            hist_tile(T, frames, fstride, pitch, hist, frame, tile, tid & 511, sm.hist[tid >> 9]);
            wave_done<LOCAL>(hdone + frame, tid);
        }
    }
}

int fused_sync_words(int n) { return FUSED_SYNC_HEAD + 3 * n; }

FusedNeed fused_need(const LevelTable& T, int nf) {
    const unsigned waves = SCORE_THREADS / 64;
    FusedNeed nd;
    nd.hist = waves * (unsigned)((T.th_total + 1) / 2);
    nd.feat = waves * (unsigned)((T.tf_total + 3) / 4);
    nd.score = waves * (unsigned)(T.ts_total * ((nf + FGROUP - 1) / FGROUP));
    return nd;
}

hipError_t launch_fused(const LevelTable& T, int n, const FusedCfg& cfg, const uint8_t* frames, long long fstride,
                        int pitch, float* hist, float* feat, const float4* bpack, const float* bias, int nf,
                        float thresh, unsigned long long* poskey, bool atomic_key, unsigned* sync, hipStream_t s) {
    const int groups = (nf + FGROUP - 1) / FGROUP;
    if (cfg.queues < 1 || cfg.queues > FUSED_MAX_QUEUES || cfg.lag_f < 1 || cfg.lag_s <= cfg.lag_f ||
        cfg.wg_per_queue < 1)
        return hipErrorInvalidValue;
    const long long per_slot = (long long)T.ts_total * groups + (T.tf_total + 3) / 4 + (T.th_total + 1) / 2;
    if (per_slot * ((long long)n + cfg.lag_s) > 0x7fffffffLL) return hipErrorInvalidValue;
    const int blocks = cfg.queues * cfg.wg_per_queue;
    if (cfg.queues == FUSED_MAX_QUEUES)
        hipLaunchKernelGGL(hog_fused_kernel<true>, dim3(blocks), dim3(SCORE_THREADS), 0, s, T, n, groups, cfg.queues,
                           cfg.lag_f, cfg.lag_s, frames, fstride, pitch, hist, feat, bpack, bias, nf, thresh,
                           poskey, atomic_key ? 1 : 0, sync, (unsigned)FUSED_SPIN_LIMIT);
    else
        hipLaunchKernelGGL(hog_fused_kernel<false>, dim3(blocks), dim3(SCORE_THREADS), 0, s, T, n, groups,
                           cfg.queues, cfg.lag_f, cfg.lag_s, frames, fstride, pitch, hist, feat, bpack, bias, nf,
                           thresh, poskey, atomic_key ? 1 : 0, sync, (unsigned)FUSED_SPIN_LIMIT);
    return hipGetLastError();
}

}  // namespace hog
