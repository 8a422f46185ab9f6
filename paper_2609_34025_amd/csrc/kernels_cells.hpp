// kernels_cells.hpp -- the cell sums of every call in one launch.
//
// Every recursive call S reads its field through cell sums (Section 2.2 and
// equation "stad-E"): a b-cell b_alpha[r] sums the field rows of the
// vertices of component alpha at depth r (backbone position x), and an
// A-cell A_r[x] sums the b-cells at (r, x). The table kernels then read only
// these rows.
//
// The incidences (vertex per (call, cell)) are cut into segments of at most
// kCallSeg consecutive incidences of one b-cell, and the segments of each
// call into pieces of at most kPieceSegs segments, one workgroup each. A
// piece sums its segments from the field rows into LDS rows (one round trip:
// all indices, then all rows), a b-cell row as the sum of its segment rows
// in order, an A-cell row as the sum of its b-cell rows in order. A cell
// whose segments all lie in the piece is written to the value matrix
// (A-cells at rows [0, NA), b-cells at NA + b); a cell that the piece's ends
// cut is written as a partial row, and k_cells_combine (the next launch, so
// no fence or atomic is needed between workgroups) adds each cut cell's
// partial rows in piece order. Every sum has a fixed order, so the results
// are bitwise reproducible.
// Channels go in chunks of cw = lanes x VEC (at most 64); lanes threads
// share one row.
#pragma once

#include "kernels.hpp"

namespace tfi {

constexpr int kCallThreads = 256;
constexpr int kCallSeg = 16;   // incidences per segment
constexpr int kCallRec = 8;    // ints per piece record
constexpr int kCallBEnt = 4;   // ints per b-cell entry
constexpr int kCallAEnt = 4;   // ints per A-cell entry

// Piece record (kCallRec ints):
//   [0] [1]  segments   (LDS segment row = segment - [0])
//   [2] [3]  b-cell entries (b, first and end segment row, out); LDS b row
//            = entry - [2]
//   [4] [5]  A-cell entries (a, first and end b entry, out); LDS A row =
//            entry - [4]
// out of an entry: -1 = the value-matrix row of the cell, else the partial
// row it is written to.

// Sum of rows F[inc_v[i]] over i in [beg, beg + len), len <= kCallSeg, VEC
// channels from c, in order: all indices, then all rows (one round trip).
template <typename T, int VEC>
__device__ __forceinline__ vec4<T> cell_seg_sum(const int32_t* __restrict__ inc_v,
                                                const T* __restrict__ F, int32_t d, int32_t c,
                                                int32_t beg, int32_t len) {
    int32_t rows[kCallSeg];
#pragma unroll
    for (int u = 0; u < kCallSeg; ++u) rows[u] = inc_v[beg + min(u, len - 1)];
    vec4<T> acc = {0, 0, 0, 0};
    if (VEC == 4) {
        vec4<T> v[kCallSeg];
#pragma unroll
        for (int u = 0; u < kCallSeg; ++u)
            v[u] = (u < len) ? ld4(F + (int64_t)rows[u] * d + c) : vec4<T>{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < kCallSeg; ++u)
            if (u < len) add4(acc, v[u]);
    } else {
        T v[kCallSeg];
#pragma unroll
        for (int u = 0; u < kCallSeg; ++u) v[u] = (u < len) ? F[(int64_t)rows[u] * d + c] : (T)0;
#pragma unroll
        for (int u = 0; u < kCallSeg; ++u)
            if (u < len) acc.x += v[u];
    }
    return acc;
}

template <typename T, int VEC>
__device__ __forceinline__ vec4<T> lds_ld(const T* p) {
    if (VEC == 4) return ld4(p);
    return {p[0], (T)0, (T)0, (T)0};
}

template <typename T, int VEC>
__device__ __forceinline__ void lds_st(T* p, vec4<T> v) {
    if (VEC == 4)
        st4(p, v);
    else
        p[0] = v.x;
}

// VEC channels of a global row at channel c (only channels below d).
template <typename T, int VEC>
__device__ __forceinline__ void row_st(T* p, int32_t c, int32_t d, vec4<T> v) {
    if (c >= d) return;
    if (VEC == 4)
        st4(p, v);
    else
        p[0] = v.x;
}

template <typename T, int VEC>
__device__ __forceinline__ vec4<T> row_ld(const T* p, int32_t c, int32_t d) {
    if (c >= d) return {0, 0, 0, 0};
    if (VEC == 4) return ld4(p);
    return {p[0], (T)0, (T)0, (T)0};
}

// One workgroup per piece; each XCD takes a contiguous range of the pieces
// (xcd_block), which are ordered by region of the forest. d: channels;
// lanes: threads per row (a power of two, at most 16); dynamic LDS:
// (segments + b entries) rows of cw elements for the largest piece.
template <typename T, int VEC>
__global__ void __launch_bounds__(kCallThreads)
k_cells(int32_t d, int32_t lanes, const int32_t* __restrict__ piece,
        const int32_t* __restrict__ seg, const int32_t* __restrict__ bent,
        const int32_t* __restrict__ aent, const int32_t* __restrict__ inc_v,
        const T* __restrict__ F, int64_t NA, T* __restrict__ part, T* __restrict__ val) {
    extern __shared__ __attribute__((aligned(16))) unsigned char cell_lds[];
    const int32_t* pc = piece + (int64_t)kCallRec * xcd_block();
    const int32_t s0 = pc[0], s1 = pc[1], e0 = pc[2], e1 = pc[3], q0 = pc[4], q1 = pc[5];
    const int32_t nseg = s1 - s0, nb = e1 - e0, na = q1 - q0;
    const int32_t cw = lanes * VEC;
    const int32_t lane = threadIdx.x & (lanes - 1);
    const int32_t unit0 = threadIdx.x / lanes, units = kCallThreads / lanes;
    T* srow = reinterpret_cast<T*>(cell_lds);  // segment rows
    T* brow = srow + nseg * cw;                // b-cell rows
    for (int32_t c0 = 0; c0 < d; c0 += cw) {
        const int32_t c = c0 + lane * VEC;
        const int32_t lc = lane * VEC;  // channel offset within an LDS row
        if (c0 > 0) __syncthreads();    // the previous chunk is done with the rows
        for (int32_t s = unit0; s < nseg; s += units) {
            const int32_t beg = seg[2 * (s0 + s)], len = seg[2 * (s0 + s) + 1];
            const vec4<T> v = c < d ? cell_seg_sum<T, VEC>(inc_v, F, d, c, beg, len)
                                    : vec4<T>{0, 0, 0, 0};
            lds_st<T, VEC>(srow + s * cw + lc, v);
        }
        __syncthreads();
        // b-cell rows: their segment rows in order
        for (int32_t k = unit0; k < nb; k += units) {
            const int32_t* be = bent + (int64_t)kCallBEnt * (e0 + k);
            const int32_t lo = be[1], hi = be[2], out = be[3];
            vec4<T> acc = lds_ld<T, VEC>(srow + lo * cw + lc);
            for (int32_t i = lo + 1; i < hi; ++i) add4(acc, lds_ld<T, VEC>(srow + i * cw + lc));
            lds_st<T, VEC>(brow + k * cw + lc, acc);
            T* dst = out < 0 ? val + (NA + be[0]) * d : part + (int64_t)out * d;
            row_st<T, VEC>(dst + c, c, d, acc);
        }
        __syncthreads();
        // A-cell rows: their b-cell rows in order
        for (int32_t k = unit0; k < na; k += units) {
            const int32_t* ae = aent + (int64_t)kCallAEnt * (q0 + k);
            const int32_t lo = ae[1], hi = ae[2], out = ae[3];
            vec4<T> acc = lds_ld<T, VEC>(brow + lo * cw + lc);
            for (int32_t i = lo + 1; i < hi; ++i) add4(acc, lds_ld<T, VEC>(brow + i * cw + lc));
            T* dst = out < 0 ? val + (int64_t)ae[0] * d : part + (int64_t)out * d;
            row_st<T, VEC>(dst + c, c, d, acc);
        }
    }
}

// Cut cells: the partial rows of a cell that pieces share, added in piece
// order into its value-matrix row (comb[4 m .. 4 m + 3] = (0: b-cell, 1:
// A-cell; its id; first partial row; count)). Runs after k_cells.
template <typename T, int VEC>
__global__ void __launch_bounds__(kCallThreads)
k_cells_combine(int32_t d, int32_t lanes, int32_t ncomb, const int32_t* __restrict__ comb,
                const T* __restrict__ part, T* __restrict__ val, int64_t NA) {
    const int32_t cw = lanes * VEC;
    const int32_t lane = threadIdx.x & (lanes - 1);
    const int64_t m = ((int64_t)blockIdx.x * kCallThreads + threadIdx.x) / lanes;
    if (m >= ncomb) return;
    const int32_t ck = comb[4 * m], id = comb[4 * m + 1], pf = comb[4 * m + 2], n = comb[4 * m + 3];
    T* dst = val + (ck ? (int64_t)id : NA + id) * d;
    for (int32_t c0 = 0; c0 < d; c0 += cw) {
        const int32_t c = c0 + lane * VEC;
        if (c >= d) break;
        vec4<T> acc = row_ld<T, VEC>(part + (int64_t)pf * d + c, c, d);
        for (int32_t i = 1; i < n; ++i)
            add4(acc, row_ld<T, VEC>(part + (int64_t)(pf + i) * d + c, c, d));
        row_st<T, VEC>(dst + c, c, d, acc);
    }
}

}  // namespace tfi
