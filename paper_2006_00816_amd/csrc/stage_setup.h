// Device stage: the per-call set-up (pyramid geometry tables, filter
// repacking for the scorers, clearing of the candidate-key map), run by
// the set-up kernel or by extra workgroups of the histogram kernel.
#pragma once
#include "hog_device.h"

namespace hog {

// Element e of segment 0: resampling taps of every level (rows, then
// columns; Sec. IV-A pyramid) and the frame-pixel edges of every window row
// and column (used for boxes and NMS).
// Segment 1: filters [nf][10][10][31] -> scorer operands, per group of 5
// filters.  Column n = 10 f + dc (filter f of the group, window column dc)
// and K index k = 32 dr + ch (window row dr, channel ch; ch = 31 is zero):
//  - matrix-core part, columns 0..47: entry [kc][nt][lane] holds the four
//    K values 16 kc + 4 (lane / 16) + s, s = 0..3, of column
//    16 nt + lane % 16, for four consecutive MFMAs;
//  - vector-ALU part, columns 48 and 49 (f = 4, dc = 8, 9): entry
//    [kc][g][col] holds the K values 16 kc + 4 g + s of that column.
// Segment 2: zero the per-position candidate keys (when several filter
// groups merge their keys with atomic max) and the counters of the fused
// persistent kernel.
__device__ __forceinline__ void setup_element(const LevelTable& T, const SetupArgs& a, int seg, long long e) {
    if (seg == 0) {
        if (e < T.taps_total) {
            for (int k = 0; k < T.n; ++k) {
                const DevLevel& L = T.L[k];
                // a level image of the recursive pyramid is read as is
                if (e >= L.tap_y && e < L.tap_y + L.h) {
                    const int i = (int)(e - L.tap_y);
                    a.taps[e] = level_tap(L, i, L.h, T.h);
                    return;
                }
                if (e >= L.tap_x && e < L.tap_x + L.w) {
                    const int i = (int)(e - L.tap_x);
                    a.taps[e] = level_tap(L, i, L.w, T.w);
                    return;
                }
            }
        } else if (e < (long long)T.taps_total + T.boxes_total) {
            const long long b = e - T.taps_total;
            for (int k = 0; k < T.n; ++k) {
                const DevLevel& L = T.L[k];
                long long i = -1;
                if (b >= L.box_r && b < L.box_r + L.rows) i = b - L.box_r;
                if (b >= L.box_c && b < L.box_c + L.cols) i = b - L.box_c;
                if (i >= 0) {
                    a.boxes[b] = make_int2(box_edge(8 * i, L.sig), box_edge(8 * i + 80, L.sig));
                    return;
                }
            }
        }
    } else if (seg == 1 && a.f16x3) {
        // split fp16 B operands: entry ((dr B16_NT + nt) 2 + part) 64 + lane
        // of group grp holds the hi (part 0) or lo (part 1) halves of the
        // weights of channels 8 (lane / 16) + i, column 16 nt + lane % 16
        const int ngroups = (a.nf + FGROUP - 1) / FGROUP;
        if (!a.W || e >= (long long)ngroups * B16_PER_GROUP) return;
        const int grp = (int)(e / B16_PER_GROUP);
        const int rem = (int)(e % B16_PER_GROUP);
        const int lane = rem & 63, part = (rem >> 6) & 1, nt = (rem >> 7) % B16_NT, dr = rem / (B16_NT * 128);
        const int n = 16 * nt + (lane & 15);
        const int f = grp * FGROUP + n / WIN, dc = n % WIN;
        _Float16 v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int ch = 8 * (lane >> 4) + i;
            const bool ok = n < FGROUP * WIN && f < a.nf && ch < NFEAT;
            const float w = ok ? a.W[((f * WIN + dr) * WIN + dc) * NFEAT + ch] : 0.f;
            const _Float16 h = (_Float16)w;
            v[i] = part ? (_Float16)((w - (float)h) * 2048.f) : h;
        }
        uint4 q;
        __builtin_memcpy(&q, v, sizeof q);
        reinterpret_cast<uint4*>(a.bpack)[e] = q;
    } else if (seg == 1) {
        const int ngroups = (a.nf + FGROUP - 1) / FGROUP;
        if (!a.W || e >= (long long)ngroups * BPACK_PER_GROUP) return;
        const int grp = (int)(e / BPACK_PER_GROUP);
        const int rem = (int)(e % BPACK_PER_GROUP);
        int n, k0;
        if (rem < BPACK_MFMA) {
            const int kc = rem / (SC_NT * 64);
            const int nt = (rem / 64) % SC_NT;
            const int lane = rem % 64;
            n = 16 * nt + (lane & 15);
            k0 = 16 * kc + 4 * (lane >> 4);
        } else {
            const int x = rem - BPACK_MFMA;
            n = 48 + (x & 1);
            k0 = 16 * (x >> 3) + 4 * ((x >> 1) & 3);
        }
        const int f = grp * FGROUP + n / WIN, dc = n % WIN;
        float v[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + s;
            const int dr = k / FPAD, ch = k % FPAD;
            const bool ok = f < a.nf && ch < NFEAT;
            v[s] = ok ? a.W[((f * WIN + dr) * WIN + dc) * NFEAT + ch] : 0.f;
        }
        a.bpack[e] = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        if (e < a.nkeys) a.keys[e] = 0ull;
        if (e < a.nsync) a.sync[e] = 0u;
    }
}

// Element g of the set-up's flattened (segment, element) space.
__device__ __forceinline__ void setup_flat(const LevelTable& T, const SetupArgs& a, long long g) {
    const int seg = (int)(g / a.m);
    if (seg < a.segs) setup_element(T, a, seg, g - (long long)seg * a.m);
}

}  // namespace hog
