// kernels.hpp -- gfx950 device kernels of the tree field integrator.
//
// Stages of one integration (all calls of all recursion levels at once):
//   scatter  : b-cell sums b_alpha[r] (equation "stad-E") and A-cell sums
//              A_r[x] (Section 2.2) from the field rows of their vertices;
//   tables   : every table job evaluates, at its own occupied cells,
//                G(i) = sum_j f(r_i + r_j + |x_i - x_j|) * val(j)
//              by direct sums (small or sparse tables) or by one FFT
//              convolution on the padded lattice (equation
//              "stad-2d-convolution", lemma "stad-2d-fft");
//   gather   : out[v] = sum over the calls holding v of G - E
//              (lemma "stad-cross");
//   leaves   : dense f(D) F on small subtrees.
// No floating-point atomics: every sum has a fixed order, so results are
// bitwise reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tfi {

template <typename T>
struct cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // a * conj(b)
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// ------------------------------------------------------------- scatter ----
// Segmented sums with bounded fan-in. Segment s adds len[s] <= 32 source
// rows starting at src_beg[s] and writes row dst[s] of the value matrix.
// Level 0 reads field rows through the incidence vertex list; later levels
// add partial rows of longer segments (split on the host into pieces), so
// no thread walks an unbounded run and the summation order is fixed.
template <typename T, bool INDEXED>
__global__ void k_segsum(int64_t nseg, int32_t d, const int64_t* __restrict__ seg_src,
                         const int32_t* __restrict__ seg_len, const int64_t* __restrict__ seg_dst,
                         const int32_t* __restrict__ idx, const T* __restrict__ src,
                         T* __restrict__ val) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nseg * d) return;
    const int64_t s = tid / d;
    const int32_t c = (int32_t)(tid - s * d);
    const int64_t b = seg_src[s];
    const int32_t n = seg_len[s];
    T acc = 0;
#pragma unroll 4
    for (int32_t i = 0; i < n; ++i) {
        const int64_t row = INDEXED ? (int64_t)idx[b + i] : b + i;
        acc += src[row * d + c];
    }
    val[seg_dst[s] * d + c] = acc;
}

// ------------------------------------------------------ direct tables ----
// Direct evaluation G(i) = sum_{j in job(i)} f(r_i + r_j + |x_i - x_j|) v(j)
// for small or sparse tables. A workgroup owns a block of at most
// kDirOut output cells: either several whole small jobs (sources = the
// block's own cells) or a slice of one large job (sources = the whole job,
// streamed through LDS in tiles of kDirTile cells). Channels are processed
// in chunks of kDirCh. blk[4 b .. 4 b + 3] = (out_beg, out_end, src_beg,
// src_end) index the direct-cell list (dl_*); dl_jb/dl_je give each cell's
// job range in the same list.
constexpr int kDirOut = 64, kDirTile = 256, kDirCh = 16, kDirThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kDirThreads)
k_direct(int32_t d, const int32_t* __restrict__ blk, const int32_t* __restrict__ dl_r,
         const int32_t* __restrict__ dl_x, const int32_t* __restrict__ dl_row,
         const int32_t* __restrict__ dl_jb, const int32_t* __restrict__ dl_je,
         const T* __restrict__ f, int32_t flds, const T* __restrict__ val,
         T* __restrict__ g) {
    __shared__ T sv[kDirTile * kDirCh];
    __shared__ int32_t sr[kDirTile], sx[kDirTile];
    extern __shared__ unsigned char dyn_raw[];
    T* sf = reinterpret_cast<T*>(dyn_raw);
    const int32_t os = blk[4 * blockIdx.x], oe = blk[4 * blockIdx.x + 1];
    const int32_t ss = blk[4 * blockIdx.x + 2], se = blk[4 * blockIdx.x + 3];
    const T* fp = f;
    if (flds > 0) {
        for (int32_t k = threadIdx.x; k < flds; k += blockDim.x) sf[k] = f[k];
        fp = sf;
    }
    for (int32_t c0 = 0; c0 < d; c0 += kDirCh) {
        const int32_t nch = min(kDirCh, d - c0);
        const int32_t cpp = kDirThreads / nch;  // output cells per pass
        const int32_t ci0 = threadIdx.x / nch, c = threadIdx.x - ci0 * nch;
        const bool lane_ok = ci0 < cpp;
        T acc[4] = {0, 0, 0, 0};
        int32_t ri[4], xi[4], jb[4], je[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t i = os + ci0 + q * cpp;
            const bool ok = lane_ok && i < oe;
            ri[q] = ok ? dl_r[i] : 0;
            xi[q] = ok ? dl_x[i] : 0;
            jb[q] = ok ? dl_jb[i] : 0;
            je[q] = ok ? dl_je[i] : 0;
        }
        for (int32_t ts = ss; ts < se; ts += kDirTile) {
            const int32_t tn = min(kDirTile, se - ts);
            __syncthreads();
            for (int32_t k = threadIdx.x; k < tn; k += blockDim.x) {
                sr[k] = dl_r[ts + k];
                sx[k] = dl_x[ts + k];
            }
            for (int32_t e = threadIdx.x; e < tn * nch; e += blockDim.x) {
                const int32_t k = e / nch, cc = e - k * nch;
                sv[k * kDirCh + cc] = val[(int64_t)dl_row[ts + k] * d + c0 + cc];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t lo = max(jb[q], ts) - ts, hi = min(je[q], ts + tn) - ts;
                T a = acc[q];
                for (int32_t k = lo; k < hi; ++k) {
                    const int32_t dx = xi[q] - sx[k];
                    a += fp[ri[q] + sr[k] + (dx < 0 ? -dx : dx)] * sv[k * kDirCh + c];
                }
                acc[q] = a;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t i = os + ci0 + q * cpp;
            if (lane_ok && i < oe) g[(int64_t)dl_row[i] * d + c0 + c] = acc[q];
        }
    }
}

// ---------------------------------------------------------------- gather --
// One thread per (vertex, channel): adds, over the calls holding the
// vertex, the call's table value minus the component correction (row -1
// when the vertex is on the call's backbone). Writes every out row.
template <typename T>
__global__ void k_gather(int64_t N, int32_t d, const int64_t* __restrict__ v_off,
                         const int32_t* __restrict__ ga, const int32_t* __restrict__ gb,
                         const T* __restrict__ g, T* __restrict__ out) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= N * d) return;
    const int64_t v = tid / d;
    const int32_t c = (int32_t)(tid - v * d);
    T s = 0;
    const int64_t k1 = v_off[v + 1];
    for (int64_t k = v_off[v]; k < k1; ++k) {
        const int32_t b = gb[k];
        s += g[(int64_t)ga[k] * d + c];
        if (b >= 0) s -= g[(int64_t)b * d + c];
    }
    out[v * d + c] = s;
}

// ----------------------------------------------------------- leaf tiles --
// Dense f(D) F on small subtrees. A workgroup owns a group of consecutive
// tiles with at most kLeafMax vertices in total; the kernel values
// f(D[i, j]) of every tile and the field rows (kDirCh channels at a time)
// are staged in LDS, then out[v] += sum_j f(D[v, j]) F[j].
constexpr int kLeafMax = 64, kLeafThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kLeafThreads)
k_leaf(int32_t d, const int32_t* __restrict__ grp, const int64_t* __restrict__ leaf_off,
       const int32_t* __restrict__ leaf_v, const int64_t* __restrict__ leaf_doff,
       const int32_t* __restrict__ leaf_D, const T* __restrict__ f, const T* __restrict__ F,
       T* __restrict__ out) {
    __shared__ T sk[kLeafMax * kLeafMax];
    __shared__ T sF[kLeafMax * kDirCh];
    __shared__ int32_t sv[kLeafMax], stile_beg[kLeafMax], stile_n[kLeafMax], skoff[kLeafMax];
    const int32_t t0 = grp[blockIdx.x], t1 = grp[blockIdx.x + 1];
    const int64_t vbase = leaf_off[t0];
    const int32_t nv = (int32_t)(leaf_off[t1] - vbase);
    const int64_t dbase = leaf_doff[t0];
    // per-vertex tile bounds and kernel-row offsets
    for (int32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        const int32_t b = (int32_t)(leaf_off[t] - vbase), n = (int32_t)(leaf_off[t + 1] - leaf_off[t]);
        const int32_t ko = (int32_t)(leaf_doff[t] - dbase);
        for (int32_t i = 0; i < n; ++i) {
            stile_beg[b + i] = b;
            stile_n[b + i] = n;
            skoff[b + i] = ko + i * n;
        }
    }
    for (int32_t i = threadIdx.x; i < nv; i += blockDim.x) sv[i] = leaf_v[vbase + i];
    const int32_t nk = (int32_t)(leaf_doff[t1] - dbase);
    for (int32_t k = threadIdx.x; k < nk; k += blockDim.x) sk[k] = f[leaf_D[dbase + k]];
    for (int32_t c0 = 0; c0 < d; c0 += kDirCh) {
        const int32_t nch = min(kDirCh, d - c0);
        __syncthreads();
        for (int32_t e = threadIdx.x; e < nv * nch; e += blockDim.x) {
            const int32_t i = e / nch, cc = e - i * nch;
            sF[i * kDirCh + cc] = F[(int64_t)sv[i] * d + c0 + cc];
        }
        __syncthreads();
        for (int32_t e = threadIdx.x; e < nv * nch; e += blockDim.x) {
            const int32_t i = e / nch, cc = e - i * nch;
            const int32_t b = stile_beg[i], n = stile_n[i];
            const T* krow = sk + skoff[i];
            T a = 0;
            for (int32_t j = 0; j < n; ++j) a += krow[j] * sF[(b + j) * kDirCh + cc];
            out[(int64_t)sv[i] * d + c0 + cc] += a;
        }
    }
}

// ------------------------------------------------------------------- FFT --
// In-place radix-2 transforms along one axis of a 2-D array in LDS.
// Forward: decimation in frequency, natural order in, bit-reversed out.
// Inverse: decimation in time, bit-reversed in, natural order out
// (unnormalised). A convolution multiplies two forward spectra in the same
// bit-reversed layout, so no reordering pass is needed.
// Axis of length 2^lgL; `count` lines; element stride es, line stride ls.
// tw[k] = exp(-2 pi i k / 2^lgtw), k < 2^(lgtw-1), with lgtw >= lgL.
template <typename T, bool INV>
__device__ void fft_axis_lds(cpx<T>* z, int lgL, int count, int es, int ls,
                             const cpx<T>* __restrict__ tw, int lgtw) {
    if (lgL == 0) return;
    const int half = 1 << (lgL - 1);
    const int nb = count * half;
    for (int s = 0; s < lgL; ++s) {
        const int lh = INV ? s : (lgL - 1 - s);  // span h = 2^lh
        const int h = 1 << lh;
        for (int bi = threadIdx.x; bi < nb; bi += blockDim.x) {
            const int line = bi >> (lgL - 1);
            const int m = bi & (half - 1);
            const int j = m & (h - 1);
            const int blk = m >> lh;
            const int i0 = line * ls + ((blk << (lh + 1)) + j) * es;
            const int i1 = i0 + h * es;
            const cpx<T> w = tw[j << (lgtw - lh - 1)];
            const cpx<T> u = z[i0];
            const cpx<T> v = z[i1];
            if (!INV) {
                z[i0] = cadd(u, v);
                z[i1] = cmul(csub(u, v), w);
            } else {
                const cpx<T> vw = cmulc(v, w);
                z[i0] = cadd(u, vw);
                z[i1] = csub(u, vw);
            }
        }
        __syncthreads();
    }
}

// Kernel spectrum of one FFT bucket: k[a][b] = f(a + |b|) on the padded
// L1 x L2 grid (b taken as the signed circular offset), zero outside the
// bucket's reach a <= 2 Hmax, |b| <= Xmax; forward 2-D transform.
template <typename T>
__global__ void k_spectrum_lds(int lg1, int lg2, int32_t hmax, int32_t xmax,
                               const T* __restrict__ f, const cpx<T>* __restrict__ tw,
                               int lgtw, cpx<T>* __restrict__ spec) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_raw);
    const int L1 = 1 << lg1, L2 = 1 << lg2, P = L1 * L2;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        const int a = p >> lg2, b = p & (L2 - 1);
        const int bs = (b <= (L2 >> 1)) ? b : L2 - b;
        T v = 0;
        if (a <= 2 * hmax && bs <= xmax) v = f[a + bs];
        z[p] = {v, (T)0};
    }
    __syncthreads();
    fft_axis_lds<T, false>(z, lg2, L1, 1, L2, tw, lgtw);
    fft_axis_lds<T, false>(z, lg1, L2, L2, 1, tw, lgtw);
    for (int p = threadIdx.x; p < P; p += blockDim.x) spec[p] = z[p];
}

// FFT convolution of LDS-resident tables: one workgroup per (job, channel
// pair). Two real channels ride in the real and imaginary parts of one
// complex table (the kernel is real, so the two results separate again in
// the real and imaginary parts of the output). Source cell (r, x) goes to
// row (-r mod L1): the Hankel dependence on q + r becomes a circular
// convolution whose output row q needs no shift.
template <typename T>
__global__ void k_fft_conv_lds(int lg1, int lg2, const int32_t* __restrict__ jobs,
                               const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
                               const int32_t* __restrict__ jc_val, int32_t d,
                               const T* __restrict__ val, T* __restrict__ g,
                               const cpx<T>* __restrict__ spec, const cpx<T>* __restrict__ tw,
                               int lgtw) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_raw);
    const int L1 = 1 << lg1, L2 = 1 << lg2, P = L1 * L2;
    const int32_t cb = jobs[2 * blockIdx.x], ce = jobs[2 * blockIdx.x + 1];
    const int32_t c0 = 2 * blockIdx.y, c1 = c0 + 1;
    const bool has1 = c1 < d;
    for (int p = threadIdx.x; p < P; p += blockDim.x) z[p] = {(T)0, (T)0};
    __syncthreads();
    for (int32_t k = cb + threadIdx.x; k < ce; k += blockDim.x) {
        const int row = (L1 - jc_r[k]) & (L1 - 1);
        const int64_t vr = (int64_t)jc_val[k] * d;
        z[(row << lg2) + jc_x[k]] = {val[vr + c0], has1 ? val[vr + c1] : (T)0};
    }
    __syncthreads();
    fft_axis_lds<T, false>(z, lg2, L1, 1, L2, tw, lgtw);
    fft_axis_lds<T, false>(z, lg1, L2, L2, 1, tw, lgtw);
    for (int p = threadIdx.x; p < P; p += blockDim.x) z[p] = cmul(z[p], spec[p]);
    __syncthreads();
    fft_axis_lds<T, true>(z, lg1, L2, L2, 1, tw, lgtw);
    fft_axis_lds<T, true>(z, lg2, L1, 1, L2, tw, lgtw);
    const T scale = (T)1 / (T)P;
    for (int32_t k = cb + threadIdx.x; k < ce; k += blockDim.x) {
        const cpx<T> y = z[(jc_r[k] << lg2) + jc_x[k]];
        const int64_t vr = (int64_t)jc_val[k] * d;
        g[vr + c0] = y.x * scale;
        if (has1) g[vr + c1] = y.y * scale;
    }
}

// ---------------------------------------------- FFT through global memory --
// Tables too large for LDS: the same in-place DIF/DIT transforms, one
// radix-2 stage per launch over every (job, channel pair) line set of a
// bucket. Buffer layout: slot s = job * npairs + pair holds P complex.
template <typename T>
__global__ void k_fill_global(int lg1, int lg2, int32_t njobs, int32_t npairs,
                              const int32_t* __restrict__ jobs,
                              const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
                              const int32_t* __restrict__ jc_val, int32_t d,
                              const T* __restrict__ val, cpx<T>* __restrict__ buf) {
    const int64_t P = (int64_t)1 << (lg1 + lg2);
    const int64_t slot = blockIdx.y;
    const int32_t job = (int32_t)(slot / npairs), pair = (int32_t)(slot % npairs);
    const int32_t c0 = 2 * pair, c1 = c0 + 1;
    const int64_t L1 = (int64_t)1 << lg1;
    cpx<T>* z = buf + slot * P;
    const int32_t cb = jobs[2 * job], ce = jobs[2 * job + 1];
    for (int32_t k = cb + blockIdx.x * blockDim.x + threadIdx.x; k < ce;
         k += gridDim.x * blockDim.x) {
        const int64_t row = (L1 - jc_r[k]) & (L1 - 1);
        const int64_t vr = (int64_t)jc_val[k] * d;
        z[(row << lg2) + jc_x[k]] = {val[vr + c0], c1 < d ? val[vr + c1] : (T)0};
    }
}

template <typename T, bool INV>
__global__ void k_fft_stage_global(cpx<T>* __restrict__ buf, int64_t nslots, int lgP, int lgL,
                                   int lh, int64_t es, const cpx<T>* __restrict__ tw, int lgtw) {
    // Butterflies of span 2^lh along an axis of length 2^lgL with element
    // stride es; every slot holds one 2^lgP-element array.
    const int64_t P = (int64_t)1 << lgP;
    const int64_t per_slot = P >> 1;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nslots * per_slot) return;
    const int64_t slot = tid / per_slot;
    const int64_t bi = tid - slot * per_slot;
    const int64_t half = (int64_t)1 << (lgL - 1);
    const int64_t line = bi / half;
    const int64_t m = bi - line * half;
    const int64_t h = (int64_t)1 << lh;
    const int64_t j = m & (h - 1);
    const int64_t blk = m >> lh;
    // line index -> base offset: lines enumerate the other axis
    const int64_t base = (es == 1) ? line << lgL : line;
    const int64_t i0 = slot * P + base + ((blk << (lh + 1)) + j) * es;
    const int64_t i1 = i0 + h * es;
    const cpx<T> w = tw[j << (lgtw - lh - 1)];
    const cpx<T> u = buf[i0];
    const cpx<T> v = buf[i1];
    if (!INV) {
        buf[i0] = cadd(u, v);
        buf[i1] = cmul(csub(u, v), w);
    } else {
        const cpx<T> vw = cmulc(v, w);
        buf[i0] = cadd(u, vw);
        buf[i1] = csub(u, vw);
    }
}

template <typename T>
__global__ void k_spec_fill_global(int lg1, int lg2, int32_t hmax, int32_t xmax,
                                   const T* __restrict__ f, cpx<T>* __restrict__ z) {
    const int64_t P = (int64_t)1 << (lg1 + lg2);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t L2 = (int64_t)1 << lg2;
    const int64_t a = p >> lg2, b = p & (L2 - 1);
    const int64_t bs = (b <= (L2 >> 1)) ? b : L2 - b;
    T v = 0;
    if (a <= 2 * (int64_t)hmax && bs <= xmax) v = f[a + bs];
    z[p] = {v, (T)0};
}

template <typename T>
__global__ void k_spec_mul_global(cpx<T>* __restrict__ buf, int64_t nslots, int lgP,
                                  const cpx<T>* __restrict__ spec) {
    const int64_t P = (int64_t)1 << lgP;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nslots * P) return;
    buf[tid] = cmul(buf[tid], spec[tid & (P - 1)]);
}

template <typename T>
__global__ void k_extract_global(int lg1, int lg2, int32_t njobs, int32_t npairs,
                                 const int32_t* __restrict__ jobs,
                                 const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
                                 const int32_t* __restrict__ jc_val, int32_t d,
                                 const cpx<T>* __restrict__ buf, T* __restrict__ g) {
    const int64_t P = (int64_t)1 << (lg1 + lg2);
    const int64_t slot = blockIdx.y;
    const int32_t job = (int32_t)(slot / npairs), pair = (int32_t)(slot % npairs);
    const int32_t c0 = 2 * pair, c1 = c0 + 1;
    const cpx<T>* z = buf + slot * P;
    const T scale = (T)1 / (T)P;
    const int32_t cb = jobs[2 * job], ce = jobs[2 * job + 1];
    for (int32_t k = cb + blockIdx.x * blockDim.x + threadIdx.x; k < ce;
         k += gridDim.x * blockDim.x) {
        const cpx<T> y = z[((int64_t)jc_r[k] << lg2) + jc_x[k]];
        const int64_t vr = (int64_t)jc_val[k] * d;
        g[vr + c0] = y.x * scale;
        if (c1 < d) g[vr + c1] = y.y * scale;
    }
}

template <typename T>
__global__ void k_zero(T* __restrict__ p, int64_t n) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < n) p[tid] = T{};
}

}  // namespace tfi

namespace tfi {

// =================================================== kernel-table gradient ==
// For L = sum(gout * out), dL/df[k] = sum over pairs (v, w) at distance k
// of <gout[v], F[w]>. Through the decomposition, each table job adds
// sign * sum_{i, j} [r_i + r_j + |x_i - x_j| = k] <gbar_i, val_j>, where
// gbar and val are the same cell sums applied to gout and F (call jobs
// sign +1 on A-cell rows < NA, corrections sign -1 on b-cell rows), and
// every leaf tile adds its own dense pair histogram. Histograms accumulate
// in FP64 (LDS bins flushed with FP64 atomics): df is reproducible to FP64
// rounding, not bitwise.
constexpr int kDfTile = 64, kDfThreads = 256, kDfHistLds = 4096;

template <typename T>
__device__ __forceinline__ void hist_add(double* lh, double* gh, int32_t k, double v) {
    if (lh) atomicAdd(lh + k, v);
    else atomicAdd(gh + k, v);
}

// Direct jobs: same blocks as k_direct. Pair dot products are formed over
// channel chunks in registers (16 pairs per thread), then binned by
// surrogate distance.
template <typename T>
__global__ void __launch_bounds__(kDfThreads)
k_df_direct(int32_t d, int64_t NA, const int32_t* __restrict__ blk,
            const int32_t* __restrict__ dl_r, const int32_t* __restrict__ dl_x,
            const int32_t* __restrict__ dl_row, const int32_t* __restrict__ dl_jb,
            const int32_t* __restrict__ dl_je, const T* __restrict__ val,
            const T* __restrict__ valg, int32_t K, double* __restrict__ df) {
    __shared__ T sG[kDfTile * (kDirCh + 1)], sV[kDfTile * (kDirCh + 1)];
    __shared__ int32_t sr[kDfTile], sx[kDfTile];
    __shared__ double lh[kDfHistLds];
    const bool use_lds = K <= kDfHistLds;
    double* lhp = use_lds ? lh : nullptr;
    if (use_lds)
        for (int32_t k = threadIdx.x; k < K; k += blockDim.x) lh[k] = 0.0;
    const int32_t os = blk[4 * blockIdx.x], oe = blk[4 * blockIdx.x + 1];
    const int32_t ss = blk[4 * blockIdx.x + 2], se = blk[4 * blockIdx.x + 3];
    const int32_t ii = threadIdx.x & (kDfTile - 1), jj0 = threadIdx.x >> 6;
    const int32_t i = os + ii;
    const bool iok = i < oe;
    const int32_t ri = iok ? dl_r[i] : 0, xi = iok ? dl_x[i] : 0;
    const int32_t jb = iok ? dl_jb[i] : 0, je = iok ? dl_je[i] : 0;
    const double sign = (iok && dl_row[i] < NA) ? 1.0 : -1.0;
    for (int32_t ts = ss; ts < se; ts += kDfTile) {
        const int32_t tn = min(kDfTile, se - ts);
        T m[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) m[q] = 0;
        for (int32_t c0 = 0; c0 < d; c0 += kDirCh) {
            const int32_t nch = min(kDirCh, d - c0);
            __syncthreads();
            for (int32_t e = threadIdx.x; e < kDfTile * nch; e += blockDim.x) {
                const int32_t k = e / nch, cc = e - k * nch;
                sG[k * (kDirCh + 1) + cc] =
                    (os + k < oe) ? valg[(int64_t)dl_row[os + k] * d + c0 + cc] : (T)0;
                sV[k * (kDirCh + 1) + cc] =
                    (k < tn) ? val[(int64_t)dl_row[ts + k] * d + c0 + cc] : (T)0;
            }
            if (c0 == 0)
                for (int32_t k = threadIdx.x; k < tn; k += blockDim.x) {
                    sr[k] = dl_r[ts + k];
                    sx[k] = dl_x[ts + k];
                }
            __syncthreads();
            for (int32_t cc = 0; cc < nch; ++cc) {
                const T gv = sG[ii * (kDirCh + 1) + cc];
#pragma unroll
                for (int q = 0; q < 16; ++q) m[q] += gv * sV[(jj0 + 4 * q) * (kDirCh + 1) + cc];
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int32_t j = ts + jj0 + 4 * q;
            if (iok && j >= jb && j < je && jj0 + 4 * q < tn) {
                const int32_t dx = xi - sx[jj0 + 4 * q];
                hist_add<T>(lhp, df, ri + sr[jj0 + 4 * q] + (dx < 0 ? -dx : dx),
                            sign * (double)m[q]);
            }
        }
    }
    if (use_lds) {
        __syncthreads();
        for (int32_t k = threadIdx.x; k < K; k += blockDim.x)
            if (lh[k] != 0.0) atomicAdd(df + k, lh[k]);
    }
}

// Leaf tiles: pairs inside each tile of a group, distance from D.
template <typename T>
__global__ void __launch_bounds__(kLeafThreads)
k_df_leaf(int32_t d, const int32_t* __restrict__ grp, const int64_t* __restrict__ leaf_off,
          const int32_t* __restrict__ leaf_v, const int64_t* __restrict__ leaf_doff,
          const int32_t* __restrict__ leaf_D, const T* __restrict__ F,
          const T* __restrict__ gout, int32_t K, double* __restrict__ df) {
    __shared__ T sG[kLeafMax * (kDirCh + 1)], sF[kLeafMax * (kDirCh + 1)];
    __shared__ int32_t sv[kLeafMax], stile_beg[kLeafMax], stile_n[kLeafMax], skoff[kLeafMax];
    __shared__ double lh[kDfHistLds];
    const bool use_lds = K <= kDfHistLds;
    double* lhp = use_lds ? lh : nullptr;
    if (use_lds)
        for (int32_t k = threadIdx.x; k < K; k += blockDim.x) lh[k] = 0.0;
    const int32_t t0 = grp[blockIdx.x], t1 = grp[blockIdx.x + 1];
    const int64_t vbase = leaf_off[t0];
    const int32_t nv = (int32_t)(leaf_off[t1] - vbase);
    const int64_t dbase = leaf_doff[t0];
    for (int32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        const int32_t b = (int32_t)(leaf_off[t] - vbase), n = (int32_t)(leaf_off[t + 1] - leaf_off[t]);
        const int32_t ko = (int32_t)(leaf_doff[t] - dbase);
        for (int32_t i = 0; i < n; ++i) {
            stile_beg[b + i] = b;
            stile_n[b + i] = n;
            skoff[b + i] = ko + i * n;
        }
    }
    for (int32_t i = threadIdx.x; i < nv; i += blockDim.x) sv[i] = leaf_v[vbase + i];
    // thread -> (vertex i, sources j = jj0 + 4 q), 16 pairs per thread
    const int32_t ii = threadIdx.x & (kLeafMax - 1), jj0 = threadIdx.x >> 6;
    T m[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) m[q] = 0;
    for (int32_t c0 = 0; c0 < d; c0 += kDirCh) {
        const int32_t nch = min(kDirCh, d - c0);
        __syncthreads();
        for (int32_t e = threadIdx.x; e < nv * nch; e += blockDim.x) {
            const int32_t k = e / nch, cc = e - k * nch;
            sG[k * (kDirCh + 1) + cc] = gout[(int64_t)sv[k] * d + c0 + cc];
            sF[k * (kDirCh + 1) + cc] = F[(int64_t)sv[k] * d + c0 + cc];
        }
        __syncthreads();
        if (ii < nv) {
            const int32_t b = stile_beg[ii], n = stile_n[ii];
            for (int32_t cc = 0; cc < nch; ++cc) {
                const T gv = sG[ii * (kDirCh + 1) + cc];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int32_t j = jj0 + 4 * q;
                    if (j < n) m[q] += gv * sF[(b + j) * (kDirCh + 1) + cc];
                }
            }
        }
    }
    __syncthreads();
    if (ii < nv) {
        const int32_t n = stile_n[ii];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int32_t j = jj0 + 4 * q;
            if (j < n) hist_add<T>(lhp, df, leaf_D[dbase + skoff[ii] + j], (double)m[q]);
        }
    }
    if (use_lds) {
        __syncthreads();
        for (int32_t k = threadIdx.x; k < K; k += blockDim.x)
            if (lh[k] != 0.0) atomicAdd(df + k, lh[k]);
    }
}

// FFT jobs held in LDS: per channel pair, the forward transforms of the
// gout table (at output positions) and of the field table (at source
// positions); the products Zg * conj(Zv) are summed over channel pairs,
// one inverse transform gives the channel-summed cross-correlation
// Z[a][b] with a = q + r, b = s - x (mod L2), folded into df[a + |b|].
// Three LDS tables per workgroup; one workgroup per job.
template <typename T>
__global__ void k_df_fft_lds(int lg1, int lg2, int64_t NA, const int32_t* __restrict__ jobs,
                             const int32_t* __restrict__ job_hx,
                             const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
                             const int32_t* __restrict__ jc_val, int32_t d,
                             const T* __restrict__ val, const T* __restrict__ valg,
                             const cpx<T>* __restrict__ tw, int lgtw, double* __restrict__ df) {
    extern __shared__ unsigned char smem_raw[];
    const int L1 = 1 << lg1, L2 = 1 << lg2, P = L1 * L2;
    cpx<T>* zv = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* zg = zv + P;
    cpx<T>* acc = zg + P;
    const int32_t cb = jobs[2 * blockIdx.x], ce = jobs[2 * blockIdx.x + 1];
    const int32_t H = job_hx[2 * blockIdx.x], X = job_hx[2 * blockIdx.x + 1];
    const double sign = jc_val[cb] < NA ? 1.0 : -1.0;
    for (int p = threadIdx.x; p < P; p += blockDim.x) acc[p] = {(T)0, (T)0};
    const int32_t npairs = (d + 1) / 2;
    for (int32_t pr = 0; pr < npairs; ++pr) {
        const int32_t c0 = 2 * pr, c1 = c0 + 1;
        const bool has1 = c1 < d;
        for (int p = threadIdx.x; p < P; p += blockDim.x) {
            zv[p] = {(T)0, (T)0};
            zg[p] = {(T)0, (T)0};
        }
        __syncthreads();
        for (int32_t k = cb + threadIdx.x; k < ce; k += blockDim.x) {
            const int64_t vr = (int64_t)jc_val[k] * d;
            const int row = (L1 - jc_r[k]) & (L1 - 1);
            zv[(row << lg2) + jc_x[k]] = {val[vr + c0], has1 ? val[vr + c1] : (T)0};
            zg[(jc_r[k] << lg2) + jc_x[k]] = {valg[vr + c0], has1 ? valg[vr + c1] : (T)0};
        }
        __syncthreads();
        fft_axis_lds<T, false>(zv, lg2, L1, 1, L2, tw, lgtw);
        fft_axis_lds<T, false>(zv, lg1, L2, L2, 1, tw, lgtw);
        fft_axis_lds<T, false>(zg, lg2, L1, 1, L2, tw, lgtw);
        fft_axis_lds<T, false>(zg, lg1, L2, L2, 1, tw, lgtw);
        for (int p = threadIdx.x; p < P; p += blockDim.x) acc[p] = cadd(acc[p], cmulc(zg[p], zv[p]));
        __syncthreads();
    }
    fft_axis_lds<T, true>(acc, lg1, L2, L2, 1, tw, lgtw);
    fft_axis_lds<T, true>(acc, lg2, L1, 1, L2, tw, lgtw);
    const double scale = sign / (double)P;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        const int a = p >> lg2, b = p & (L2 - 1);
        const int bs = (b <= (L2 >> 1)) ? b : L2 - b;
        if (a <= 2 * H && bs <= X) {
            const double v = (double)acc[p].x * scale;
            if (v != 0.0) atomicAdd(df + a + bs, v);
        }
    }
}

// Global-memory variant for tables beyond LDS: fills of the two tables per
// (job, channel pair) slot, the pair-summed product per job, and the fold.
template <typename T>
__global__ void k_fill2_global(int lg1, int lg2, int32_t npairs, const int32_t* __restrict__ jobs,
                               const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
                               const int32_t* __restrict__ jc_val, int32_t d,
                               const T* __restrict__ val, const T* __restrict__ valg,
                               cpx<T>* __restrict__ bv, cpx<T>* __restrict__ bg) {
    const int64_t P = (int64_t)1 << (lg1 + lg2);
    const int64_t slot = blockIdx.y;
    const int32_t job = (int32_t)(slot / npairs), pair = (int32_t)(slot % npairs);
    const int32_t c0 = 2 * pair, c1 = c0 + 1;
    const int64_t L1 = (int64_t)1 << lg1;
    cpx<T>* zv = bv + slot * P;
    cpx<T>* zg = bg + slot * P;
    const int32_t cb = jobs[2 * job], ce = jobs[2 * job + 1];
    for (int32_t k = cb + blockIdx.x * blockDim.x + threadIdx.x; k < ce;
         k += gridDim.x * blockDim.x) {
        const int64_t vr = (int64_t)jc_val[k] * d;
        const int64_t row = (L1 - jc_r[k]) & (L1 - 1);
        zv[(row << lg2) + jc_x[k]] = {val[vr + c0], c1 < d ? val[vr + c1] : (T)0};
        zg[((int64_t)jc_r[k] << lg2) + jc_x[k]] = {valg[vr + c0], c1 < d ? valg[vr + c1] : (T)0};
    }
}

template <typename T>
__global__ void k_corr_accum_global(int64_t njobs, int32_t npairs, int lgP,
                                    const cpx<T>* __restrict__ bv, const cpx<T>* __restrict__ bg,
                                    cpx<T>* __restrict__ acc) {
    const int64_t P = (int64_t)1 << lgP;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= njobs * P) return;
    const int64_t job = tid >> lgP, p = tid & (P - 1);
    cpx<T> s = {(T)0, (T)0};
    for (int32_t pr = 0; pr < npairs; ++pr) {
        const int64_t o = (job * npairs + pr) * P + p;
        s = cadd(s, cmulc(bg[o], bv[o]));
    }
    acc[tid] = s;
}

template <typename T>
__global__ void k_fold_global(int64_t njobs, int lg1, int lg2, int64_t NA,
                              const int32_t* __restrict__ jobs, const int32_t* __restrict__ job_hx,
                              const int32_t* __restrict__ jc_val, const cpx<T>* __restrict__ acc,
                              double* __restrict__ df) {
    const int64_t P = (int64_t)1 << (lg1 + lg2);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= njobs * P) return;
    const int64_t job = tid / P, p = tid - job * P;
    const int64_t L2 = (int64_t)1 << lg2;
    const int64_t a = p >> lg2, b = p & (L2 - 1);
    const int64_t bs = (b <= (L2 >> 1)) ? b : L2 - b;
    const int32_t H = job_hx[2 * job], X = job_hx[2 * job + 1];
    if (a <= 2 * (int64_t)H && bs <= X) {
        const double sign = jc_val[jobs[2 * job]] < NA ? 1.0 : -1.0;
        const double v = sign * (double)acc[tid].x / (double)P;
        if (v != 0.0) atomicAdd(df + a + bs, v);
    }
}

}  // namespace tfi
