// Window scores of listed windows, per-frame top-k windows, the hinge
// loss, and the backward pass of window scores to the filter weights and
// to the frame pixels.  The backward recomputes the features of each
// window's support from the frame; nothing is kept from a forward call.
#include "hog_device.h"

namespace hog {

// ------------------------------------------------------- window scores
// S = bias_f + <W_f, F[r:r+10, c:c+10, :]> for listed windows, one wave per
// window, from the padded feature maps; the 3100 products are summed per
// lane in a fixed order and reduced across the wave in a fixed tree.
// A window outside the batch (see window_in_range) reads nothing and
// scores NaN.
__global__ __launch_bounds__(256) void hog_window_score_kernel(LevelTable T, int n, int nf,
                                                               const float* __restrict__ feat,
                                                               const hog_window* __restrict__ win, int n_win,
                                                               const float* __restrict__ W,
                                                               const float* __restrict__ bias,
                                                               float* __restrict__ scores) {
    const int wi = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wi >= n_win) return;
    const hog_window w = win[wi];
    if (!window_in_range(T, n, nf, w)) {
        if (lane == 0) scores[wi] = __builtin_nanf("");
        return;
    }
    const DevLevel& L = T.L[w.level];
    const float* F = feat + (long long)w.frame * T.feat_frame + L.feat_off;
    const float* Wf = W + (long long)w.filter * WIN * WIN * NFEAT;
    const int pitch = (L.cx + 2) * FPAD, hp = (L.cx + 2) * FHALF;
    float acc = 0.f;
    for (int e = lane; e < WIN * WIN * NFEAT; e += 64) {
        const int ch = e % NFEAT, cell = e / NFEAT;
        const int dr = cell / WIN, dc = cell % WIN;
        // feature-map half-planes: channels 0..15, then 16..31 of the row
        acc = fmaf(Wf[e], F[(long long)(w.row + dr) * pitch + (ch >> 4) * hp + (w.col + dc) * FHALF + (ch & 15)], acc);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) scores[wi] = acc + bias[w.filter];
}

hipError_t launch_window_scores(const LevelTable& T, int n, int nf, const float* feat, const hog_window* win,
                                int n_win, const float* W, const float* bias, float* scores, hipStream_t s) {
    if (n_win <= 0) return hipSuccess;
    hipLaunchKernelGGL(hog_window_score_kernel, dim3((n_win + 3) / 4), dim3(256), 0, s, T, n, nf, feat, win, n_win, W,
                       bias, scores);
    return hipGetLastError();
}

// ---------------------------------------------------------------- top-k
// The k best windows of a frame over every filter, level and position, in
// the rank order of the detector (score descending, then filter, level,
// row, column ascending), from the dense score maps [level][nf][rows][cols].
constexpr int TOPK_MAX = 16;

__global__ __launch_bounds__(1024) void hog_topk_kernel(LevelTable T, const float* __restrict__ dense,
                                                        long long dense_frame, int nf, int K,
                                                        hog_window* __restrict__ out, float* __restrict__ out_scores) {
    __shared__ unsigned long long red[1024];
    const int frame = blockIdx.x;
    const int tid = threadIdx.x;
    const float* D = dense + (long long)frame * dense_frame;
    unsigned long long best[TOPK_MAX];
#pragma unroll
    for (int i = 0; i < TOPK_MAX; ++i) best[i] = 0ull;
    for (int k = 0; k < T.n; ++k) {
        const DevLevel& L = T.L[k];
        const int per = L.rows * L.cols, tot = nf * per;
        for (int e = tid; e < tot; e += 1024) {
            const int f = e / per, rc = e - f * per;
            const int r = rc / L.cols, c = rc - r * L.cols;
            const float s = D[L.sc_off + e];
            const unsigned long long key =
                ((unsigned long long)score_order(s) << 32) | (unsigned long long)(~pack_window(f, k, r, c));
            if (key > best[K - 1]) {
                // insertion into the sorted (descending) list
                int i = K - 1;
                while (i > 0 && best[i - 1] < key) {
                    best[i] = best[i - 1];
                    --i;
                }
                best[i] = key;
            }
        }
    }
    // K rounds of a block-wide maximum over the lists' heads
    int head = 0;
    for (int j = 0; j < K; ++j) {
        const unsigned long long mine = head < K ? best[head] : 0ull;
        red[tid] = mine;
        __syncthreads();
        for (int st = 512; st > 0; st >>= 1) {
            if (tid < st) red[tid] = max(red[tid], red[tid + st]);
            __syncthreads();
        }
        const unsigned long long top = red[0];
        __syncthreads();
        if (mine == top && top != 0ull) ++head;   // keys are unique: exactly one owner
        if (tid == 0) {
            const unsigned pk = ~(unsigned)(top & 0xffffffffu);
            hog_window w;
            w.frame = frame;
            w.filter = (int)(pk >> 27);
            w.level = (int)((pk >> 22) & 31);
            w.row = (int)((pk >> 11) & 2047);
            w.col = (int)(pk & 2047);
            out[(long long)frame * K + j] = w;
            out_scores[(long long)frame * K + j] = score_from_order((unsigned)(top >> 32));
        }
        __syncthreads();
    }
}

hipError_t launch_topk(const LevelTable& T, int n, const float* dense, long long dense_frame, int nf, int K,
                       hog_window* out, float* out_scores, hipStream_t s) {
    hipLaunchKernelGGL(hog_topk_kernel, dim3(n), dim3(1024), 0, s, T, dense, dense_frame, nf, K, out, out_scores);
    return hipGetLastError();
}

// ----------------------------------------------------------- hinge loss
// Mean hinge loss over n windows with labels +-1 and its score gradient
// dscore_i = -y_i / n where y_i S_i < 1, plus lam ||W||^2 and its gradient
// 2 lam W added to dW.  One workgroup; fixed-order reductions.
__global__ __launch_bounds__(1024) void hog_hinge_kernel(const float* __restrict__ S, const float* __restrict__ y,
                                                         int n, const float* __restrict__ W, int nw, float lam,
                                                         float* __restrict__ loss, float* __restrict__ dscore,
                                                         float* __restrict__ dW) {
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int i = tid; i < n; i += 1024) {
        const float m = y[i] * S[i];
        acc += m < 1.f ? (double)(1.f - m) : 0.0;
        dscore[i] = m < 1.f ? -y[i] / (float)n : 0.f;
    }
    double reg = 0.0;
    for (int e = tid; e < nw; e += 1024) {
        reg += (double)W[e] * W[e];
        dW[e] += 2.f * lam * W[e];
    }
    red[tid] = acc / n + (double)lam * reg;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) loss[0] = (float)red[0];
}

hipError_t launch_hinge(const float* S, const float* y, int n, const float* W, int nw, float lam, float* loss,
                        float* dscore, float* dW, hipStream_t s) {
    hipLaunchKernelGGL(hog_hinge_kernel, dim3(1), dim3(1024), 0, s, S, y, n, W, nw, lam, loss, dscore, dW);
    return hipGetLastError();
}

// ------------------------------------------------------------- backward
// Support of window (r, c): the 12 x 12 cells [r-1, r+11) x [c-1, c+11)
// (the window's cells and the ring whose energies normalise them), the
// 104 x 104 pixels that vote into those cells, and a one-pixel gradient
// halo: 106 x 106 level pixels.
constexpr int BC = WIN + 2;              // 12 cells
constexpr int BV = 8 * BC + 8;           // 104 voting pixels
constexpr int BP = BV + 2;               // 106 level pixels
constexpr int BWIN_PER_WG = 16;          // windows per workgroup (dW partial per workgroup)
constexpr int BTHREADS = 512;

struct BwdShared {
    int V[BP * BP];                                  // level pixels * 2^16
    unsigned char bin[BV * BV];                      // orientation bins of the voting pixels
    float dmag[BV * BV];                             // d / d magnitude of the voting pixels
    unsigned long long hq[BC * BC * NBINS];          // fixed-point histograms (then reused)
    float h[BC * BC * NBINS];                        // float histograms
    float dh[BC * BC * NBINS];                       // d / d histograms
    float E[BC * BC];                                // cell energies (0 outside the grid)
    float dB[BC * BC * 4];                           // d / d block energies of the window cells
    int4 ty[BP], tx[BP];                             // resampling taps of the region rows / columns
};

// A window outside the batch (see window_in_range) is skipped without a
// read and makes the workgroup's partial of dW[0] NaN, so that the filter
// gradient shows the error.
__global__ __launch_bounds__(BTHREADS) void hog_backward_kernel(
    LevelTable T, int n, const uint8_t* __restrict__ frames, long long fstride, int pitch,
    const int4* __restrict__ taps, const float* __restrict__ W, const hog_window* __restrict__ win,
    const float* __restrict__ dscore, int n_win, int nf, float* __restrict__ partial, float* __restrict__ dpixels) {
    __shared__ BwdShared sm;
    const int tid = threadIdx.x;
    const int w0 = blockIdx.x * BWIN_PER_WG;
    float* P = partial + (long long)blockIdx.x * (nf * WIN * WIN * NFEAT + nf);   // this workgroup's dW, db
    for (int e = tid; e < nf * WIN * WIN * NFEAT + nf; e += BTHREADS) P[e] = 0.f;

    for (int wi = w0; wi < min(w0 + BWIN_PER_WG, n_win); ++wi) {
        const hog_window w = win[wi];
        if (!window_in_range(T, n, nf, w)) {
            // every thread reads the same record, so the skip is uniform;
            // element 0 is owned by thread 0, which alone writes it
            if (tid == 0) P[0] = __builtin_nanf("");
            continue;
        }
        const float ds = dscore[wi];
        const DevLevel& L = T.L[w.level];
        const uint8_t* __restrict__ U = frames + (long long)w.frame * fstride;
        const int y0 = 8 * w.row - 13, x0 = 8 * w.col - 13;   // level coords of region pixel (0, 0)
        const int ylim = min(8 * L.cy - 1, L.h - 2), xlim = min(8 * L.cx - 1, L.w - 2);
        __syncthreads();   // previous window done with the shared arrays
        for (int e = tid; e < BP; e += BTHREADS) {
            const int y = y0 + e, x = x0 + e;
            sm.ty[e] = (y >= 0 && y < L.h) ? taps[L.tap_y + y] : make_int4(0, 0, 0, -1);
            sm.tx[e] = (x >= 0 && x < L.w) ? taps[L.tap_x + x] : make_int4(0, 0, 0, -1);
        }
        for (int e = tid; e < BC * BC * NBINS; e += BTHREADS) sm.hq[e] = 0ull;
        __syncthreads();
        // level pixels of the region, 8 per thread at a time with their
        // frame loads in flight together (taps are clamped to the frame;
        // a pixel outside the level discards its value)
        for (int e0 = tid; e0 < BP * BP; e0 += 8 * BTHREADS) {
            int u00[8], u01[8], u10[8], u11[8], az[8], bz[8], in[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int e = min(e0 + r * BTHREADS, BP * BP - 1);
                const int iy = e / BP, ix = e - iy * BP;
                const int4 a = sm.ty[iy], b = sm.tx[ix];
                in[r] = (a.w | b.w) == 0;
                az[r] = a.z;
                bz[r] = b.z;
                const uint8_t* r0 = U + (long long)a.x * pitch;
                const uint8_t* r1 = U + (long long)a.y * pitch;
                u00[r] = r0[b.x];
                u01[r] = r0[b.y];
                u10[r] = r1[b.x];
                u11[r] = r1[b.y];
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int top = (256 - bz[r]) * u00[r] + bz[r] * u01[r];
                const int bot = (256 - bz[r]) * u10[r] + bz[r] * u11[r];
                if (e0 + r * BTHREADS < BP * BP) sm.V[e0 + r * BTHREADS] = in[r] ? (256 - az[r]) * top + az[r] * bot : 0;
            }
        }
        __syncthreads();
        // gradients, bins and fixed-point votes into the 12 x 12 cells
        for (int e = tid; e < BV * BV; e += BTHREADS) {
            const int vy = e / BV, vx = e - vy * BV;
            const int yl = y0 + 1 + vy, xl = x0 + 1 + vx;        // level coords
            int bn = 0;
            if (yl >= 1 && yl <= ylim && xl >= 1 && xl <= xlim) {
                const int p = (vy + 1) * BP + vx + 1;
                const int gx = sm.V[p + 1] - sm.V[p - 1];
                const int gy = sm.V[p + BP] - sm.V[p - BP];
                if (gx | gy) {
                    bn = orient_bin(gx, gy);
                    const unsigned long long M = vote_magnitude(gx, gy);
                    // cell centres 8i + 3.5: lower cell of pixel yl is floor((yl - 3.5) / 8)
                    const int cyl = (yl + 4) / 8 - 1, cxl = (xl + 4) / 8 - 1;   // yl >= 1
                    const int oy = (yl + 4) & 7, ox = (xl + 4) & 7;               // offset inside the quad block
                    const unsigned wy[2] = {(unsigned)(15 - 2 * oy), (unsigned)(2 * oy + 1)};
                    const unsigned wx[2] = {(unsigned)(15 - 2 * ox), (unsigned)(2 * ox + 1)};
#pragma unroll
                    for (int dy = 0; dy < 2; ++dy) {
                        const int ci = cyl + dy - (w.row - 1);
                        if (ci < 0 || ci >= BC || cyl + dy >= L.cy) continue;
#pragma unroll
                        for (int dx = 0; dx < 2; ++dx) {
                            const int cj = cxl + dx - (w.col - 1);
                            if (cj < 0 || cj >= BC || cxl + dx >= L.cx || cxl + dx < 0 || cyl + dy < 0) continue;
                            atomicAdd(&sm.hq[(ci * BC + cj) * NBINS + bn], M * (wy[dy] * wx[dx]));
                        }
                    }
                }
            }
            sm.bin[e] = (unsigned char)bn;
        }
        __syncthreads();
        // float histograms and energies
        for (int e = tid; e < BC * BC * NBINS; e += BTHREADS) {
            sm.h[e] = (float)((double)sm.hq[e] * 0x1p-30);
            sm.dh[e] = 0.f;
        }
        __syncthreads();
        if (tid < BC * BC) {
            const int gi = w.row - 1 + tid / BC, gj = w.col - 1 + tid % BC;
            float E = 0.f;
            if (gi >= 0 && gi < L.cy && gj >= 0 && gj < L.cx) {
                const float* hh = &sm.h[tid * NBINS];
#pragma unroll
                for (int o = 0; o < NORIENT; ++o) {
                    const float u = hh[o] + hh[o + NORIENT];
                    E = fmaf(u, u, E);
                }
            }
            sm.E[tid] = E;
        }
        __syncthreads();
        // window cells: features, dW partial, direct d/dh and d/dB
        if (tid < WIN * WIN) {
            const int dr = tid / WIN, dc = tid % WIN;
            const int li = dr + 1, lj = dc + 1;
            const float* hh = &sm.h[(li * BC + lj) * NBINS];
            auto Eat = [&](int i, int j) { return sm.E[i * BC + j]; };
            const float e0 = Eat(li, lj);
            float B[4];
            B[0] = e0 + Eat(li - 1, lj) + Eat(li, lj - 1) + Eat(li - 1, lj - 1);
            B[1] = e0 + Eat(li - 1, lj) + Eat(li, lj + 1) + Eat(li - 1, lj + 1);
            B[2] = e0 + Eat(li + 1, lj) + Eat(li, lj - 1) + Eat(li + 1, lj - 1);
            B[3] = e0 + Eat(li + 1, lj) + Eat(li, lj + 1) + Eat(li + 1, lj + 1);
            float n[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) n[q] = 1.0f / sqrtf(B[q] + 1e-4f);
            const float* Wc = W + ((long long)(w.filter * WIN + dr) * WIN + dc) * NFEAT;
            float* Pc = P + ((w.filter * WIN + dr) * WIN + dc) * NFEAT;
            float F[NFEAT];
#pragma unroll
            for (int c = 0; c < NFEAT; ++c) F[c] = 0.f;
            float dn[4] = {0.f, 0.f, 0.f, 0.f};
            float dhl[NBINS];
#pragma unroll
            for (int b = 0; b < NBINS; ++b) dhl[b] = 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float tsum = 0.f;
                const float gt = 0.23570226039551584f * ds * Wc[27 + q];
#pragma unroll
                for (int b = 0; b < NBINS; ++b) {
                    const float v = hh[b] * n[q];
                    const float tv = fminf(v, 0.2f);
                    F[b] += 0.5f * tv;
                    tsum += tv;
                    if (v < 0.2f) {
                        const float g = 0.5f * ds * Wc[b] + gt;
                        dhl[b] += g * n[q];
                        dn[q] += g * hh[b];
                    }
                }
#pragma unroll
                for (int o = 0; o < NORIENT; ++o) {
                    const float u = hh[o] + hh[o + NORIENT];
                    const float v = u * n[q];
                    F[NBINS + o] += 0.5f * fminf(v, 0.2f);
                    if (v < 0.2f) {
                        const float g = 0.5f * ds * Wc[NBINS + o];
                        dhl[o] += g * n[q];
                        dhl[o + NORIENT] += g * n[q];
                        dn[q] += g * u;
                    }
                }
                F[27 + q] = 0.23570226039551584f * tsum;
            }
#pragma unroll
            for (int c = 0; c < NFEAT; ++c) Pc[c] += ds * F[c];
#pragma unroll
            for (int b = 0; b < NBINS; ++b) sm.dh[(li * BC + lj) * NBINS + b] = dhl[b];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float be = B[q] + 1e-4f;
                sm.dB[tid * 4 + q] = dn[q] * -0.5f / (be * sqrtf(be));
            }
        }
        if (tid == 0) P[nf * WIN * WIN * NFEAT + w.filter] += ds;
        __syncthreads();
        if (!dpixels) continue;
        // energies: every cell of the support gathers d/dE from the blocks of
        // the window cells that contain it, then d/dh += 2 (h_o + h_{o+9}) dE
        if (tid < BC * BC) {
            const int li = tid / BC, lj = tid % BC;
            const int gi = w.row - 1 + li, gj = w.col - 1 + lj;
            if (gi >= 0 && gi < L.cy && gj >= 0 && gj < L.cx) {
                float dE = 0.f;
                for (int a = -1; a <= 1; ++a) {
                    for (int bb = -1; bb <= 1; ++bb) {
                        const int oi = li + a, oj = lj + bb;          // a window cell (dr+1, dc+1)
                        if (oi < 1 || oi > WIN || oj < 1 || oj > WIN) continue;
                        const int wc = (oi - 1) * WIN + (oj - 1);
                        // block q of cell (oi, oj) spans rows {oi, oi+dy_q}, cols {oj, oj+dx_q}
                        const int dyq[4] = {-1, -1, 1, 1}, dxq[4] = {-1, 1, -1, 1};
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const bool rin = (-a == 0) || (-a == dyq[q]);
                            const bool cin = (-bb == 0) || (-bb == dxq[q]);
                            if (rin && cin) dE += sm.dB[wc * 4 + q];
                        }
                    }
                }
                float* dh = &sm.dh[tid * NBINS];
                const float* hh = &sm.h[tid * NBINS];
#pragma unroll
                for (int o = 0; o < NORIENT; ++o) {
                    const float g = 2.f * (hh[o] + hh[o + NORIENT]) * dE;
                    dh[o] += g;
                    dh[o + NORIENT] += g;
                }
            }
        }
        __syncthreads();
        // d / d magnitude of each voting pixel: its four bilinear votes
        for (int e = tid; e < BV * BV; e += BTHREADS) {
            const int vy = e / BV, vx = e - vy * BV;
            const int yl = y0 + 1 + vy, xl = x0 + 1 + vx;
            float dm = 0.f;
            if (yl >= 1 && yl <= ylim && xl >= 1 && xl <= xlim) {
                const int bn = sm.bin[e];
                const int cyl = (yl + 4) / 8 - 1, cxl = (xl + 4) / 8 - 1;
                const int oy = (yl + 4) & 7, ox = (xl + 4) & 7;
                const float wy[2] = {(15 - 2 * oy) * 0.0625f, (2 * oy + 1) * 0.0625f};
                const float wx[2] = {(15 - 2 * ox) * 0.0625f, (2 * ox + 1) * 0.0625f};
#pragma unroll
                for (int dy = 0; dy < 2; ++dy) {
                    const int ci = cyl + dy - (w.row - 1);
                    if (ci < 0 || ci >= BC) continue;
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx) {
                        const int cj = cxl + dx - (w.col - 1);
                        if (cj < 0 || cj >= BC) continue;
                        dm += wy[dy] * wx[dx] * sm.dh[(ci * BC + cj) * NBINS + bn];
                    }
                }
            }
            sm.dmag[e] = dm;
        }
        __syncthreads();
        // d / d level pixels (central-difference transpose), scattered onto
        // the frame through the resampling taps
        float* D = dpixels + (long long)w.frame * T.h * T.w;
        for (int e = tid; e < BP * BP; e += BTHREADS) {
            const int iy = e / BP, ix = e - iy * BP;
            const int4 a = sm.ty[iy], b = sm.tx[ix];
            if ((a.w | b.w) != 0) continue;
            // voting pixel q = (vy, vx) sits at region (vy + 1, vx + 1)
            auto dg = [&](int qy, int qx, bool xdir) -> float {
                if (qy < 0 || qy >= BV || qx < 0 || qx >= BV) return 0.f;
                const float dm = sm.dmag[qy * BV + qx];
                if (dm == 0.f) return 0.f;
                const int p = (qy + 1) * BP + qx + 1;
                const float gx = (float)(sm.V[p + 1] - sm.V[p - 1]);
                const float gy = (float)(sm.V[p + BP] - sm.V[p - BP]);
                const float mag = __builtin_sqrtf(fmaf(gx, gx, gy * gy));
                if (mag == 0.f) return 0.f;
                return dm * (xdir ? gx : gy) / mag;
            };
            const int qy = iy - 1, qx = ix - 1;
            const float dL = dg(qy, qx - 1, true) - dg(qy, qx + 1, true) + dg(qy - 1, qx, false) -
                             dg(qy + 1, qx, false);
            if (dL == 0.f) continue;
            const float wy0 = (256 - a.z) * 0.00390625f, wy1 = a.z * 0.00390625f;
            const float wx0 = (256 - b.z) * 0.00390625f, wx1 = b.z * 0.00390625f;
            atomicAdd(&D[(long long)a.x * T.w + b.x], wy0 * wx0 * dL);
            if (b.z) atomicAdd(&D[(long long)a.x * T.w + b.y], wy0 * wx1 * dL);
            if (a.z) {
                atomicAdd(&D[(long long)a.y * T.w + b.x], wy1 * wx0 * dL);
                if (b.z) atomicAdd(&D[(long long)a.y * T.w + b.y], wy1 * wx1 * dL);
            }
        }
    }
}

size_t backward_lds_bytes() { return sizeof(BwdShared); }

// Sum of the per-workgroup dW / db partials, in workgroup order.
__global__ __launch_bounds__(256) void hog_backward_reduce_kernel(const float* __restrict__ partial, int groups, int nf,
                                                                  float* __restrict__ dW, float* __restrict__ db) {
    const int n = nf * WIN * WIN * NFEAT + nf;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    float acc = 0.f;
    for (int g = 0; g < groups; ++g) acc += partial[(long long)g * n + e];
    if (e < nf * WIN * WIN * NFEAT) dW[e] += acc;
    else if (db) db[e - nf * WIN * WIN * NFEAT] += acc;
}

int backward_groups(int n_win) { return (n_win + BWIN_PER_WG - 1) / BWIN_PER_WG; }

hipError_t launch_backward(const LevelTable& T, int n, const uint8_t* frames, long long fstride, int pitch,
                           const int4* taps, const float* W, const hog_window* win, const float* dscore, int n_win,
                           int nf, float* partial, float* dW, float* db, float* dpixels, hipStream_t s) {
    if (n_win <= 0) return hipSuccess;
    const int groups = backward_groups(n_win);
    hipLaunchKernelGGL(hog_backward_kernel, dim3(groups), dim3(BTHREADS), 0, s, T, n, frames, fstride,
                       pitch, taps, W, win, dscore, n_win, nf, partial, dpixels);
    const int nw = nf * WIN * WIN * NFEAT + nf;
    hipLaunchKernelGGL(hog_backward_reduce_kernel, dim3((nw + 255) / 256), dim3(256), 0, s, partial, groups, nf, dW,
                       db);
    return hipGetLastError();
}

}  // namespace hog
