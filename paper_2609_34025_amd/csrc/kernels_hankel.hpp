// kernels_hankel.hpp -- the Hankel-GEMM evaluation of a table (the paper's
// attention-width appendix "Hankel-GEMM"): for a table with depths
// 0..H and backbone positions 0..X,
//     G_q[s] = sum_{r <= H} sum_{t <= X} f(q + r + |s - t|) A_r[t]
// splits at l = q + |s - t| into a depth correlation, a product with the
// Hankel matrix F[l][r] = f(l + r),
//     B[l][t] = sum_r f(l + r) A_r[t],      0 <= l <= H + X,
// and a walk along the backbone,
//     G_q[s] = sum_{t < s} B[q + s - t][t] + sum_{t >= s} B[q + t - s][t].
// The first sum runs along the antidiagonal l + t = q + s of B, the second
// along the diagonal l - t = q - s: one running sum per (anti)diagonal and
// channel gives every cell on it.
//
// B of a group of jobs is one buffer of rows (job, l, t) of cw channels
// (a chunk of at most 64 of the d channels); map[job][r][t] is the value
// row of the table cell at (r, t), or -1.
#pragma once

#include "kernels.hpp"

namespace tfi {

constexpr int kHankCh = 64;       // channels per chunk (one per lane)
constexpr int kHankHmax = 127;    // deepest table the LDS column holds (H + 1 <= 128)
constexpr int kHankRowsPerThread = 4;

// Per job of a group: jh[4 j .. 4 j + 3] = (H, X, map offset, B row offset).

// B rows of one (job, t) column per workgroup: the column A_r[t] (r <= H)
// of cw channels is staged in LDS, every thread then forms
// kHankRowsPerThread rows l of one channel. Items it[2 i], it[2 i + 1] =
// (job, t).
template <typename T>
__global__ void __launch_bounds__(256)
k_hankel_b(const int32_t* __restrict__ items, const int64_t* __restrict__ jh,
           const int32_t* __restrict__ map, const T* __restrict__ f,
           const T* __restrict__ val, int32_t d, int32_t c0, int32_t cw, T* __restrict__ B) {
    __shared__ T col[(kHankHmax + 1) * kHankCh];
    const int32_t job = items[2 * blockIdx.x], t = items[2 * blockIdx.x + 1];
    const int32_t H = (int32_t)jh[4 * job], X = (int32_t)jh[4 * job + 1];
    const int32_t* mp = map + jh[4 * job + 2];
    const int64_t boff = jh[4 * job + 3];
    for (int i = threadIdx.x; i < (H + 1) * kHankCh; i += blockDim.x) {
        const int r = i / kHankCh, c = i % kHankCh;
        const int32_t row = mp[r * (X + 1) + t];
        col[i] = (row >= 0 && c < cw) ? val[(int64_t)row * d + c0 + c] : (T)0;
    }
    __syncthreads();
    const int c = threadIdx.x % kHankCh;
    if (c >= cw) return;
    const int L = H + X + 1;  // rows l of B
    for (int l0 = (threadIdx.x / kHankCh) * kHankRowsPerThread; l0 < L;
         l0 += (blockDim.x / kHankCh) * kHankRowsPerThread) {
        T acc[kHankRowsPerThread] = {};
        // rows past the last are clamped to it (f is read up to 2 H + X only)
        int lu[kHankRowsPerThread];
#pragma unroll
        for (int u = 0; u < kHankRowsPerThread; ++u) lu[u] = min(l0 + u, L - 1);
        for (int r = 0; r <= H; ++r) {
            const T a = col[r * kHankCh + c];
#pragma unroll
            for (int u = 0; u < kHankRowsPerThread; ++u) acc[u] += f[lu[u] + r] * a;
        }
#pragma unroll
        for (int u = 0; u < kHankRowsPerThread; ++u)
            if (l0 + u < L) B[(boff + (int64_t)(l0 + u) * (X + 1) + t) * cw + c] = acc[u];
    }
}

// The walks along the backbone, one (job, line) item per 64 lanes (a lane
// per channel). ANTI: line = q + s, t = 0, 1, ...: the running sum before
// the step at t = s is sum_{t < s} B[q + s - t][t]; it is written to the
// cell (q, s) = (line - t, t). !ANTI: line = q - s + X, t = X, X - 1, ...:
// the running sum including t = s is sum_{t >= s} B[q + t - s][t]; it is
// added to the cell (q, s) = (line - X + t, t). Items it[2 i], it[2 i + 1].
template <typename T, bool ANTI>
__global__ void __launch_bounds__(256)
k_hankel_walk(int64_t nitems, const int32_t* __restrict__ items, const int64_t* __restrict__ jh,
              const int32_t* __restrict__ map, const T* __restrict__ B, int32_t d, int32_t c0,
              int32_t cw, T* __restrict__ g) {
    const int64_t item = (int64_t)blockIdx.x * (blockDim.x / kHankCh) + threadIdx.x / kHankCh;
    const int c = threadIdx.x % kHankCh;
    if (item >= nitems || c >= cw) return;
    const int32_t job = items[2 * item], line = items[2 * item + 1];
    const int32_t H = (int32_t)jh[4 * job], X = (int32_t)jh[4 * job + 1];
    const int32_t* mp = map + jh[4 * job + 2];
    const T* bj = B + jh[4 * job + 3] * cw + c;
    T run = 0;
    if (ANTI) {
        const int32_t te = min(line, X);
        for (int32_t t = 0; t <= te; ++t) {
            const int32_t q = line - t;  // l = q here
            const T b = bj[((int64_t)q * (X + 1) + t) * cw];
            if (q <= H) {
                const int32_t row = mp[q * (X + 1) + t];
                if (row >= 0) g[(int64_t)row * d + c0 + c] = run;
            }
            run += b;
        }
    } else {
        const int32_t delta = line - X;  // q - s = l - t
        for (int32_t t = X; t >= 0 && t + delta >= 0; --t) {
            const int32_t q = t + delta;
            run += bj[((int64_t)q * (X + 1) + t) * cw];
            if (q <= H) {
                const int32_t row = mp[q * (X + 1) + t];
                if (row >= 0) g[(int64_t)row * d + c0 + c] += run;
            }
        }
    }
}

}  // namespace tfi
