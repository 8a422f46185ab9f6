// kernels_conv1d.hpp -- one-dimensional FFT convolutions too large for LDS.
//
// A table job with H = 0 (every cell on the backbone, e.g. a whole path
// tree taken as its own backbone) is a Toeplitz product along the backbone,
//     G(x) = sum_t f(|x - x_t|) v_t,
// a 1-D circular convolution on P = 2^lg >= 2X + 1 lattice points (lemma
// "stad-2d-fft" with one row; the paper keeps the FFT for pure paths in its
// attention-width appendix). Beyond LDS it runs as a four-step transform in
// three kernels over a channel-tiled buffer
//     buf[slot][i][c],  slot = job * ntiles + tile,  c < TC channel pairs,
// so that every access moves TC contiguous complex values. When the buffer
// of all tiles would exceed kConvGroupBytes, the three kernels run on groups
// of tiles in turn (the buffer then holds one group):
//   k_conv1d_hi<false>  gathers the job's cells (TC channel pairs each) at the
//                       points i = e 2^lgL + l of one low value l and runs the
//                       DIF stages of the high bits [lgL, lg);
//   k_conv1d_lo         runs, on 2^lgL consecutive points, the DIF stages of the
//                       low bits, multiplies by the kernel spectrum (the same
//                       bit-reversed layout) and runs the DIT stages of the
//                       low bits;
//   k_conv1d_hi<true>   runs the DIT stages of the high bits and writes the
//                       cells' table rows, scaled by 1/P.
// The butterflies and twiddles are those of the in-place radix-2 DIF/DIT
// transforms of the LDS and blocked global paths (span 2^s, twiddle
// exp(-+2 pi i j / 2^(s+1)), j = index mod 2^s).
//
// A workgroup transforms a block of 2^lgB points (lgB <= 10) x TC pairs in two
// register phases with one LDS exchange between them: the block index
// e = (a << RB) + b splits into RA = lgB - lgB/2 high bits a and RB = lgB/2
// low bits b. Phase A gives each thread one (b, pair) and the 2^RA points
// that differ in a; phase B one (a, pair) and the 2^RB points that differ
// in b. The twiddle of register bit u factors as
//     W_{2^(s+1)}^{(k mod 2^u) 2^shift + j0} = W_{2^(u+1)}^{k mod 2^u} W_{2^(s+1)}^{j0},
// a compile-time 32nd root of unity times one factor per stage (s = shift + u,
// j0 = the index bits below shift), loaded once per phase.
//
// The split of the point index is a template argument (LGB, LGL) for the
// block sizes of large transforms, so that the register loops and stages
// unroll into straight-line code; 0 takes it from the arguments.
//
// Cells reach the kernels through map[job * mstride + c] = row of the cell
// at coordinate c <= cmax, or -1 (unoccupied lattice point). A one-row table
// (H = 0) is indexed by the backbone coordinate x: source and output at
// point x. A one-column table (a single backbone position: G(q) =
// sum_r f(q + r) A_r, the Hankel product of a centroid call or of a
// correction) is indexed by the depth r: the source sits at point -r mod P
// (reflect), so that the circular convolution puts f(q + r) A_r at output
// point q. Two real channels ride in one complex value, as in the other FFT
// paths.
#pragma once

#include "kernels.hpp"

namespace tfi {

constexpr int kC1MaxR = 5;      // register bits per phase (32 points per thread)
constexpr int64_t kConvGroupBytes = (int64_t)2 << 30;  // buffer of one tile group
constexpr int kC1Pad = 8;       // complex values of padding per LDS row

// Per-stage factors fs[u] = W_{2^(shift+u+1)}^{j0} for u < R (j0 < 2^shift).
template <typename T>
__device__ __forceinline__ void stage_factors(cpx<T> (&fs)[kC1MaxR], int R, int shift, int64_t j0,
                                              const cpx<T>* __restrict__ tw, int lgtw) {
#pragma unroll
    for (int u = 0; u < kC1MaxR; ++u)
        fs[u] = (u < R) ? tw[j0 << (lgtw - shift - u - 1)] : cpx<T>{(T)1, (T)0};
}

// R radix-2 stages over the register index k of x (2^R <= 32 live values):
// DIF from register bit R-1 down to 0, or DIT (conjugate twiddles) from 0 up.
// The twiddle of the pair (k, k + 2^u) is W_{2^(u+1)}^{k mod 2^u} fs[u]
// (fs unused when FS is false).
template <typename T, bool INV, bool FS>
__device__ __forceinline__ void reg_fft(cpx<T> (&x)[1 << kC1MaxR], int R,
                                        const cpx<T> (&fs)[kC1MaxR]) {
#pragma unroll
    for (int uu = 0; uu < kC1MaxR; ++uu) {
        const int u = INV ? uu : kC1MaxR - 1 - uu;
        if (u >= R) continue;
        const int h = 1 << u;
#pragma unroll
        for (int k = 0; k < (1 << kC1MaxR); ++k) {
            if ((k & h) || k >= (1 << R)) continue;
            const int m = (k & (h - 1)) << (4 - u);  // W_{2^(u+1)}^{k mod 2^u} = W_32^m
            const cpx<T> p = x[k], q = x[k + h];
            if (!INV) {
                x[k] = cadd(p, q);
                x[k + h] = FS ? cmul(csub(p, q), mul_w32(fs[u], m)) : mul_w32(csub(p, q), m);
            } else {
                const cpx<T> qw = FS ? cmulc(q, mul_w32(fs[u], m)) : mul_w32c(q, m);
                x[k] = cadd(p, qw);
                x[k + h] = csub(p, qw);
            }
        }
    }
}

// LDS block layout: row a (2^RA rows) holds the 2^RB points b x TC pairs,
// padded by kC1Pad complex values so that phase B's lanes (different a, same
// b) spread over the banks.
template <int TC>
__device__ __forceinline__ int lds_at(int a, int b, int c, int RB) {
    return a * ((TC << RB) + kC1Pad) + b * TC + c;
}

// High-bit passes. Grid: (2^lgL low values l, tiles of the group, jobs of
// the chunk); block: 2^RB x TC threads, RB = lgB/2, lgB = lg - lgL. The
// group's tiles start at tile0 (channel pairs from tile0 TC); its slots in
// buf are job x (tiles of the group) + tile.
// INV = false: gather the cells' channel pairs [tile TC, tile TC + TC) from
// src (rows of d channels) at the points of low value l, DIF stages of bits
// [lgL, lg), store to buf.
// INV = true: load from buf, DIT stages of bits [lgL, lg), write the rows of
// the occupied points to dst, scaled by 1/P.
template <typename T, int TC, bool INV, int LGB = 0>
__global__ void __launch_bounds__(512)
k_conv1d_hi(int lg, int lgL, int32_t cmax, int reflect, const int32_t* __restrict__ map,
            int64_t mstride, int32_t d, const T* __restrict__ src, T* __restrict__ dst,
            cpx<T>* __restrict__ buf, const cpx<T>* __restrict__ tw, int lgtw, int32_t tile0) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_raw);
    const int lgB = LGB ? LGB : lg - lgL, RB = lgB / 2, RA = lgB - RB;
    if (LGB) lgL = lg - LGB;
    const int64_t l = blockIdx.x;
    const int64_t slot = (int64_t)blockIdx.z * gridDim.y + blockIdx.y;
    const int32_t* mp = map + (int64_t)blockIdx.z * mstride;
    cpx<T>* sb = buf + (slot << lg) * TC;
    const int c = threadIdx.x % TC;
    const int b = threadIdx.x / TC;  // phase A: low bits; phase B: first high value
    const int32_t ch = 2 * ((tile0 + (int32_t)blockIdx.y) * TC + c);
    const bool has0 = ch < d, has1 = ch + 1 < d;
    // rows of even length in an aligned buffer: one access per channel pair
    const T* io = INV ? dst : src;
    const bool pairs = (d & 1) == 0 && ((uintptr_t)io & (2 * sizeof(T) - 1)) == 0;
    // unreflected, points beyond cmax are zero: e <= emax; reflected (the
    // sources of a one-column table) every e is looked at
    const bool refl = !INV && reflect != 0;
    const int64_t emax64 = (int64_t)cmax >= l ? (((int64_t)cmax - l) >> lgL) : -1;
    const int emax = refl ? (1 << lgB) - 1
                          : (int)(emax64 < (1 << lgB) - 1 ? emax64 : (1 << lgB) - 1);
    const int64_t pmask = ((int64_t)1 << lg) - 1;
    cpx<T> x[1 << kC1MaxR];
    // every global load that does not depend on the data is issued first:
    // the stage factors of both phases and the map rows of phase A's points
    cpx<T> fsA[kC1MaxR], fsB[kC1MaxR];
    stage_factors(fsA, RA, RB + lgL, ((int64_t)b << lgL) + l, tw, lgtw);
    stage_factors(fsB, RB, lgL, l, tw, lgtw);
    int32_t row[1 << kC1MaxR];
#pragma unroll
    for (int k = 0; k < (1 << kC1MaxR); ++k) {
        const int e = (k << RB) + b;
        const int64_t i = ((int64_t)e << lgL) + l;
        const int64_t pos = refl ? ((pmask + 1 - i) & pmask) : i;
        row[k] = (k < (1 << RA) && e <= emax && pos <= cmax) ? mp[pos] : -1;
    }
    if (!INV) {
        // phase A: points e = (k << RB) + b, gathered through the map
        if (pairs) {
#pragma unroll
            for (int k = 0; k < (1 << kC1MaxR); ++k) {
                x[k] = {(T)0, (T)0};
                if (row[k] >= 0 && has0) x[k] = ld_pair(src + (int64_t)row[k] * d + ch);
            }
        } else {
#pragma unroll
            for (int k = 0; k < (1 << kC1MaxR); ++k) {
                x[k] = {(T)0, (T)0};
                if (row[k] >= 0 && has0) {
                    const T* p = src + (int64_t)row[k] * d + ch;
                    x[k].x = p[0];
                    if (has1) x[k].y = p[1];
                }
            }
        }
        reg_fft<T, false, true>(x, RA, fsA);
#pragma unroll
        for (int k = 0; k < (1 << kC1MaxR); ++k)
            if (k < (1 << RA)) z[lds_at<TC>(k, b, c, RB)] = x[k];
        __syncthreads();
        // phase B: points e = (a << RB) + k, a = b + j 2^RB
        for (int a = b; a < (1 << RA); a += (1 << RB)) {
#pragma unroll
            for (int k = 0; k < (1 << kC1MaxR); ++k)
                if (k < (1 << RB)) x[k] = z[lds_at<TC>(a, k, c, RB)];
            reg_fft<T, false, true>(x, RB, fsB);
#pragma unroll
            for (int k = 0; k < (1 << kC1MaxR); ++k)
                if (k < (1 << RB)) sb[((((int64_t)a << RB) + k) << lgL | l) * TC + c] = x[k];
        }
    } else {
        // phase B first (DIT goes from the low bits up). RA - RB <= 1: a thread
        // has one or two values of a, and the points of both (at most 32, slot
        // j 16 + k) are loaded before either is transformed
        cpx<T> y[1 << kC1MaxR];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 16 * (2 - j); ++k) {
                const int a = b + (j << RB);
                if (k < (1 << RB) && a < (1 << RA))
                    y[j * 16 + k] = sb[((((int64_t)a << RB) + k) << lgL | l) * TC + c];
            }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int a = b + (j << RB);
            if (a >= (1 << RA)) continue;
#pragma unroll
            for (int k = 0; k < (1 << kC1MaxR); ++k)
                if (k < (1 << RB) && j * 16 + k < (1 << kC1MaxR)) x[k] = y[j * 16 + k];
            reg_fft<T, true, true>(x, RB, fsB);
#pragma unroll
            for (int k = 0; k < (1 << kC1MaxR); ++k)
                if (k < (1 << RB)) z[lds_at<TC>(a, k, c, RB)] = x[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < (1 << kC1MaxR); ++k)
            if (k < (1 << RA)) x[k] = z[lds_at<TC>(k, b, c, RB)];
        reg_fft<T, true, true>(x, RA, fsA);
        const T scale = (T)1 / (T)((int64_t)1 << lg);
        if (pairs) {
#pragma unroll
            for (int k = 0; k < (1 << kC1MaxR); ++k)
                if (row[k] >= 0 && has0)
                    st_pair(dst + (int64_t)row[k] * d + ch,
                            cpx<T>{x[k].x * scale, x[k].y * scale});
        } else {
#pragma unroll
            for (int k = 0; k < (1 << kC1MaxR); ++k) {
                if (row[k] >= 0 && has0) {
                    T* p = dst + (int64_t)row[k] * d + ch;
                    p[0] = x[k].x * scale;
                    if (has1) p[1] = x[k].y * scale;
                }
            }
        }
    }
}

// Low-bit pass. Grid: (2^(lg - lgL) high values h x TC / CW channel parts,
// tiles, jobs of the chunk); block: 2^(lgL/2) x CW threads. The 2^lgL
// consecutive points x TC pairs of one h are contiguous in buf: DIF stages of
// bits [0, lgL), product with the kernel spectrum, DIT stages, store back.
// With CW < TC a workgroup takes CW of the TC pairs (a smaller LDS block, so
// that two workgroups share a CU); the parts of one h are dispatched 8
// workgroups apart, which places them on the same XCD (workgroups go to the
// XCDs in turn), so each 128-byte row is fetched into one L2 only.
template <typename T, int TC, int LGL = 0, int CW = TC>
__global__ void __launch_bounds__(512)
k_conv1d_lo(int lg, int lgL, cpx<T>* __restrict__ buf, const cpx<T>* __restrict__ spec,
            const cpx<T>* __restrict__ tw, int lgtw) {
    static_assert(CW <= TC && TC % CW == 0, "channel parts divide the tile");
    constexpr int NS = TC / CW;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_raw);
    if (LGL) lgL = LGL;
    const int RB = lgL / 2, RA = lgL - RB;
    int64_t h = blockIdx.x;
    int c0 = 0;
    if (NS > 1) {
        if (gridDim.x >= 8 * NS) {
            const int w = (int)(blockIdx.x % (8 * NS));
            h = (int64_t)(blockIdx.x / (8 * NS)) * 8 + (w & 7);
            c0 = (w >> 3) * CW;
        } else {
            h = blockIdx.x / NS;
            c0 = (int)(blockIdx.x % NS) * CW;
        }
    }
    const int64_t slot = (int64_t)blockIdx.z * gridDim.y + blockIdx.y;
    cpx<T>* sb = buf + ((slot << lg) + (h << lgL)) * TC + c0;
    const cpx<T>* sp = spec + (h << lgL);
    const int c = threadIdx.x % CW;
    const int b = threadIdx.x / CW;
    cpx<T> x[1 << kC1MaxR];
    cpx<T> fs[kC1MaxR];
    const cpx<T> one[kC1MaxR] = {};
    // phase A: DIF of the high bits of the block index
    stage_factors(fs, RA, RB, b, tw, lgtw);
#pragma unroll
    for (int k = 0; k < (1 << kC1MaxR); ++k)
        if (k < (1 << RA)) x[k] = sb[((k << RB) + b) * TC + c];
    reg_fft<T, false, true>(x, RA, fs);
#pragma unroll
    for (int k = 0; k < (1 << kC1MaxR); ++k)
        if (k < (1 << RA)) z[lds_at<CW>(k, b, c, RB)] = x[k];
    // the kernel spectrum of phase B's points (a = b + j 2^RB, j < 2; at most
    // 32 values, slot j 16 + k) is requested before the barrier, once the
    // block's values have left the registers
    cpx<T> spv[1 << kC1MaxR];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 16 * (2 - j); ++k) {
            const int a = b + (j << RB);
            if (k < (1 << RB) && a < (1 << RA)) spv[j * 16 + k] = sp[(a << RB) + k];
        }
    __syncthreads();
    // phase B: DIF of the low bits, spectrum product, DIT of the low bits
    // (RA - RB <= 1, so a thread has at most two values of a)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int a = b + (j << RB);
        if (a >= (1 << RA)) continue;
#pragma unroll
        for (int k = 0; k < (1 << kC1MaxR); ++k)
            if (k < (1 << RB)) x[k] = z[lds_at<CW>(a, k, c, RB)];
        reg_fft<T, false, false>(x, RB, one);
#pragma unroll
        for (int k = 0; k < (1 << kC1MaxR); ++k)
            if (k < (1 << RB) && j * 16 + k < (1 << kC1MaxR)) x[k] = cmul(x[k], spv[j * 16 + k]);
        reg_fft<T, true, false>(x, RB, one);
#pragma unroll
        for (int k = 0; k < (1 << kC1MaxR); ++k)
            if (k < (1 << RB)) z[lds_at<CW>(a, k, c, RB)] = x[k];
    }
    __syncthreads();
    // phase A again: DIT of the high bits. The stage factors pass through an
    // empty register constraint so that the twiddle products of the forward
    // phase are formed again here rather than kept live across phase B.
#pragma unroll
    for (int u = 0; u < kC1MaxR; ++u) asm volatile("" : "+v"(fs[u].x), "+v"(fs[u].y));
#pragma unroll
    for (int k = 0; k < (1 << kC1MaxR); ++k)
        if (k < (1 << RA)) x[k] = z[lds_at<CW>(k, b, c, RB)];
    reg_fft<T, true, true>(x, RA, fs);
#pragma unroll
    for (int k = 0; k < (1 << kC1MaxR); ++k)
        if (k < (1 << RA)) sb[((k << RB) + b) * TC + c] = x[k];
}

}  // namespace tfi
