// kernels.hpp -- gfx950 device kernels of the tree field integrator.
//
// Stages of one integration (all calls of all recursion levels at once):
//   cells    : b-cell sums b_alpha[r] (equation "stad-E") and A-cell sums
//              A_r[x] (Section 2.2) from the field rows of their vertices
//              (kernels_cells.hpp);
//   tables   : every table job evaluates, at its own occupied cells,
//                G(i) = sum_j f(r_i + r_j + |x_i - x_j|) * val(j)
//              by direct sums (small or sparse tables) or by one FFT
//              convolution on the padded lattice (equation
//              "stad-2d-convolution", lemma "stad-2d-fft");
//   gather   : out[v] = sum over the calls holding v of G - E
//              (lemma "stad-cross");
//   leaves   : dense f(D) F on small subtrees.
// No floating-point atomics: every sum has a fixed order, or (the histograms
// of the kernel-table gradient) is an integer sum, so results are bitwise
// reproducible run to run.
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

// ----------------------------------------------------------- vectors ----
// Four consecutive channels of one row (16 B for float, 32 B for double).
template <typename T>
struct vec4 {
    T x, y, z, w;
};
template <typename T>
__device__ __forceinline__ vec4<T> ld4(const T* p) {
    return *reinterpret_cast<const vec4<T>*>(p);
}
template <>
__device__ __forceinline__ vec4<float> ld4<float>(const float* p) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    return {v.x, v.y, v.z, v.w};
}
template <typename T>
__device__ __forceinline__ void st4(T* p, vec4<T> v) {
    *reinterpret_cast<vec4<T>*>(p) = v;
}
template <>
__device__ __forceinline__ void st4<float>(float* p, vec4<float> v) {
    *reinterpret_cast<float4*>(p) = make_float4(v.x, v.y, v.z, v.w);
}
template <typename T>
__device__ __forceinline__ void add4(vec4<T>& a, vec4<T> b) {
    a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
}
template <typename T>
__device__ __forceinline__ void sub4(vec4<T>& a, vec4<T> b) {
    a.x -= b.x; a.y -= b.y; a.z -= b.z; a.w -= b.w;
}
template <typename T>
__device__ __forceinline__ void fma4(vec4<T>& a, T s, vec4<T> b) {
    a.x += s * b.x; a.y += s * b.y; a.z += s * b.z; a.w += s * b.w;
}

// ------------------------------------------------------------ row tiles ----
// Workgroups are dispatched to the 8 XCDs in turn, and each XCD has its own
// L2. Logical block of this workgroup such that every XCD takes one
// contiguous range of logical blocks, in order (a bijection on
// [0, gridDim.x)): rows that neighbouring logical blocks share are then
// fetched into one L2.
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t n = gridDim.x, b = blockIdx.x;
    const int64_t q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Thread -> (row index, first channel) under column tiling; false when the
// thread is past the end.
template <int VEC>
__device__ __forceinline__ bool tile_coords(int64_t tid, int64_t nrows, int32_t d, int32_t ct,
                                            int64_t& r, int32_t& c) {
    const int64_t per_tile = nrows * ct;
    const int64_t tile = tid / per_tile;
    const int64_t rem = tid - tile * per_tile;
    r = rem / ct;
    c = (int32_t)((tile * ct + (rem - r * ct)) * VEC);
    return c < d;
}

// -------------------------------------------------------- level scatter ----
// Segmented sums with bounded fan-in. Segment s adds len[s] <= 32 source
// rows starting at src_beg[s] and writes row dst[s] of the value matrix.
// Level 0 reads field rows through the incidence vertex list; later levels
// add partial rows of longer segments (split on the host into pieces), so
// no thread walks an unbounded run and the summation order is fixed.
// VEC = 4: one thread per (segment, 4 channels), requires d % 4 == 0.
// Rows are taken kSegBatch at a time: all their row indices are loaded,
// then all their values, so a batch waits for memory twice however long it
// is (the additions keep the order of the rows).
// Wide rows go in column tiles of ct VEC-groups, the tile index slowest:
// every segment's slice of one tile is summed before the next tile starts,
// so the rows read again by later segments are still in cache (ct = d/VEC
// is one tile, the whole row).
constexpr int kSegBatch = 8;

template <typename T, bool INDEXED, int VEC>
__global__ void k_segsum(int64_t nseg, int32_t d, int32_t ct, const int64_t* __restrict__ seg_src,
                         const int32_t* __restrict__ seg_len, const int64_t* __restrict__ seg_dst,
                         const int32_t* __restrict__ idx, const T* __restrict__ src,
                         T* __restrict__ val) {
    const int64_t tid = xcd_block() * blockDim.x + threadIdx.x;
    int64_t s;
    int32_t c;
    if (!tile_coords<VEC>(tid, nseg, d, ct, s, c) || s >= nseg) return;
    const int64_t b = seg_src[s];
    const int32_t n = seg_len[s];
    // rows per batch: the tail levels (consecutive partial rows, no index
    // loads) take twice as many, so a run of 32 needs two rounds
    constexpr int kSegBatch = INDEXED ? tfi::kSegBatch : 2 * tfi::kSegBatch;
    vec4<T> acc = {0, 0, 0, 0};
    for (int32_t i0 = 0; i0 < n; i0 += kSegBatch) {
        int64_t rows[kSegBatch];
#pragma unroll
        for (int u = 0; u < kSegBatch; ++u) {
            const int32_t i = min(i0 + u, n - 1);  // clamped: loads stay in the run
            rows[u] = INDEXED ? (int64_t)idx[b + i] : b + i;
        }
        // value loads predicated on the run length (issued together, no
        // load for rows past the end)
        if (VEC == 4) {
            vec4<T> v[kSegBatch];
#pragma unroll
            for (int u = 0; u < kSegBatch; ++u)
                v[u] = (i0 + u < n) ? ld4(src + rows[u] * d + c) : vec4<T>{0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < kSegBatch; ++u)
                if (i0 + u < n) add4(acc, v[u]);
        } else {
            T v[kSegBatch];
#pragma unroll
            for (int u = 0; u < kSegBatch; ++u) v[u] = (i0 + u < n) ? src[rows[u] * d + c] : (T)0;
#pragma unroll
            for (int u = 0; u < kSegBatch; ++u)
                if (i0 + u < n) acc.x += v[u];
        }
    }
    if (VEC == 4)
        st4(val + seg_dst[s] * d + c, acc);
    else
        val[seg_dst[s] * d + c] = acc.x;
}

// ------------------------------------------------------ direct tables ----
// Direct evaluation G(i) = sum_{j in job(i)} f(r_i + r_j + |x_i - x_j|) v(j)
// as small register-blocked products: a thread owns 4 cells x 4 channels
// (16 accumulators), so each kernel value read serves 4 channels and each
// 4-channel source vector serves 4 cells. Cells of a job are padded to a
// multiple of 4 (padding cells have row -1: zero source, no output), and
// jobs are sorted by size, so the lanes of a wavefront run loops of equal
// length. A workgroup owns kDirOut output cells: whole jobs packed
// together, or a slice of a larger job whose sources are streamed through
// LDS in tiles of kDirOut cells. Channels go in chunks of kDirCh.
// blk[4 b .. 4 b + 3] = (out_beg, out_end, src_beg, src_end) in the padded
// cell list; qjb/qje give each cell quad's job range in the same list.
constexpr int kDirOut = 256, kDirCh = 16, kDirThreads = 256;

// Stage tn (1 <= tn <= kDirOut) source cells ts .. ts + tn of the padded
// cell list into LDS: coordinates into sr/sx and value rows (channels
// c0 .. c0 + nch, nch <= 16) into sv at row stride SV, zero beyond tn and
// for padding cells. A workgroup of kDirThreads threads, 16 rows per
// thread: all row indices are loaded first, then all values (addresses
// clamped into range rather than branched around), so a tile waits for
// memory twice.
template <typename T, int SV>
__device__ __forceinline__ void stage_cells(const int32_t* __restrict__ dl_r,
                                            const int32_t* __restrict__ dl_x,
                                            const int32_t* __restrict__ dl_row, int32_t ts,
                                            int32_t tn, const T* __restrict__ val, int32_t d,
                                            int32_t c0, int32_t nch, int32_t* sr, int32_t* sx,
                                            T* sv) {
    const int32_t cc = threadIdx.x & 15, k0 = threadIdx.x >> 4;
    const int32_t ccs = min(cc, nch - 1);
    int32_t rows[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) rows[i] = dl_row[ts + min(k0 + 16 * i, tn - 1)];
    T v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = val[(int64_t)max(rows[i], 0) * d + c0 + ccs];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int32_t k = k0 + 16 * i;
        sv[k * SV + cc] = (k < tn && rows[i] >= 0 && cc < nch) ? v[i] : (T)0;
    }
    if ((int32_t)threadIdx.x < tn) {
        sr[threadIdx.x] = dl_r[ts + threadIdx.x];
        sx[threadIdx.x] = dl_x[ts + threadIdx.x];
    }
}

// FL: the kernel table is staged in LDS (flds = its length > 0). Kept a
// template argument so that every lookup is an LDS read: a pointer that may
// be either LDS or global compiles to flat loads, which wait on both
// counters and serialize the lookups.
template <typename T, bool FL>
__global__ void __launch_bounds__(kDirThreads)
k_direct(int32_t d, const int32_t* __restrict__ blk, const int32_t* __restrict__ dl_r,
         const int32_t* __restrict__ dl_x, const int32_t* __restrict__ dl_row,
         const int32_t* __restrict__ qjb, const int32_t* __restrict__ qje,
         const T* __restrict__ f, int32_t flds, const T* __restrict__ val,
         T* __restrict__ g) {
    __shared__ __attribute__((aligned(16))) T sv[kDirOut * kDirCh];
    __shared__ int32_t sr[kDirOut], sx[kDirOut];
    extern __shared__ unsigned char dyn_raw[];
    T* sf = reinterpret_cast<T*>(dyn_raw);
    const int32_t os = blk[4 * blockIdx.x], oe = blk[4 * blockIdx.x + 1];
    const int32_t ss = blk[4 * blockIdx.x + 2], se = blk[4 * blockIdx.x + 3];
    if (FL)
        for (int32_t k = threadIdx.x; k < flds; k += blockDim.x) sf[k] = f[k];
    const T* fp = FL ? sf : f;
    // channel chunks: this workgroup takes every gridDim.y-th one
    for (int32_t c0 = blockIdx.y * kDirCh; c0 < d; c0 += gridDim.y * kDirCh) {
        const int32_t nch = min(kDirCh, d - c0);
        const int32_t nq = (nch + 3) >> 2;             // channel quads
        const int32_t qpp = kDirThreads / nq;          // cell quads per pass
        const int32_t cq = threadIdx.x / nq, chq = threadIdx.x - cq * nq;
        const int32_t Q = (os >> 2) + cq;              // this thread's cell quad
        const bool act = cq < qpp && 4 * Q < oe;
        const int32_t Qs = act ? Q : (os >> 2);        // clamped: loads stay in range
        int32_t ri[4], xi[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            ri[c] = dl_r[4 * Qs + c];
            xi[c] = dl_x[4 * Qs + c];
        }
        const int32_t jb = act ? qjb[Qs] : 0, je = act ? qje[Qs] : 0;
        vec4<T> acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = {0, 0, 0, 0};
        for (int32_t ts = ss; ts < se; ts += kDirOut) {
            const int32_t tn = min(kDirOut, se - ts);
            __syncthreads();
            stage_cells<T, kDirCh>(dl_r, dl_x, dl_row, ts, tn, val, d, c0, nch, sr, sx, sv);
            __syncthreads();
            if (act) {
                const int32_t lo = max(jb, ts) - ts, hi = min(je, ts + tn) - ts;
                for (int32_t k = lo; k < hi; ++k) {
                    const int32_t rk = sr[k], xk = sx[k];
                    const vec4<T> v = ld4(sv + k * kDirCh + 4 * chq);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int32_t dx = xi[c] - xk;
                        fma4(acc[c], fp[ri[c] + rk + (dx < 0 ? -dx : dx)], v);
                    }
                }
            }
        }
        if (act) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int32_t row = dl_row[4 * Q + c];
                if (row < 0) continue;
                T* out = g + (int64_t)row * d + c0 + 4 * chq;
                const int32_t left = nch - 4 * chq;
                if (left >= 4 && ((d & 3) == 0)) {
                    st4(out, acc[c]);
                } else {
                    const T vv[4] = {acc[c].x, acc[c].y, acc[c].z, acc[c].w};
                    for (int cc = 0; cc < 4 && cc < left; ++cc) out[cc] = vv[cc];
                }
            }
        }
    }
}

// Direct tables on the matrix cores (FP32): per job, G = Kmat V with
// Kmat[i][k] = f(r_i + r_k + |x_i - x_k|) is a dense product, evaluated
// with v_mfma_f32_16x16x4f32 (D[16x16] += A[16x4] B[4x16]; lane l holds
// A[l%16][l/16] and B[l/16][l%16] and receives D[4(l/16)+r][l%16] in its
// r-th result register). A wave owns 16-cell row tiles of the block's
// output cells; for every k-step of 4 sources each lane forms its one
// kernel entry (0 outside its row's job) and uses it for the NCH 16-channel
// chunks of a pass, whose values come from an LDS tile of source cells x
// 16 NCH channels. Blocks, padding and job ranges are those of k_direct.
// NK = 2 evaluates two kernel tables (f, f1 into g, g1) over the same value
// tiles: each lane forms one entry per kernel and the B operand is shared.
typedef float v4f_t __attribute__((ext_vector_type(4)));
constexpr int kMfSrc = kDirOut;  // source cells per LDS tile (one chunk)

// LDS tile shape of a pass of NCH chunks: source rows, and a row stride
// that is 16 or 48 modulo 64 so that the 64 lanes of a B read hit distinct
// banks.
template <int NCH>
struct MfTile {
    static constexpr int rows = NCH == 1 ? kMfSrc : kMfSrc / 2;
    static constexpr int stride = NCH == 1 ? 16 : NCH <= 3 ? 48 : 80;
};

// FL as in k_direct: the kernel tables in LDS; the four row tiles' entries
// of a source step are then read (clamped into the table, zeroed outside
// the lane's job) before any of the step's products.
template <int NCH, int NK, bool FL>
__global__ void __launch_bounds__(kDirThreads)
k_direct_mfma(int32_t d, const int32_t* __restrict__ blk, const int32_t* __restrict__ dl_r,
              const int32_t* __restrict__ dl_x, const int32_t* __restrict__ dl_row,
              const int32_t* __restrict__ qjb, const int32_t* __restrict__ qje,
              const float* __restrict__ f, const float* __restrict__ f1, int32_t flds,
              const float* __restrict__ val, float* __restrict__ g, float* __restrict__ g1) {
    constexpr int ROWS = MfTile<NCH>::rows, SV = MfTile<NCH>::stride;
    constexpr int PER = ROWS / 16;  // staged rows per thread
    __shared__ __attribute__((aligned(16))) float sv[ROWS * SV];
    __shared__ int32_t sr[ROWS], sx[ROWS];
    // output rows of the block's cells, kept while their source tiles are
    // staged (every output cell is also a source cell of its block), so the
    // results need no further round trip for them
    __shared__ int32_t so[kDirOut];
    extern __shared__ unsigned char dyn_raw[];
    float* sf = reinterpret_cast<float*>(dyn_raw);
    const int32_t os = blk[4 * blockIdx.x], oe = blk[4 * blockIdx.x + 1];
    const int32_t ss = blk[4 * blockIdx.x + 2], se = blk[4 * blockIdx.x + 3];
    const float* fp[NK];
    fp[0] = f;
    if (NK > 1) fp[NK - 1] = f1;
    if (FL) {
        for (int32_t k = threadIdx.x; k < flds; k += blockDim.x) {
            sf[k] = f[k];
            if (NK > 1) sf[flds + k] = f1[k];
        }
#pragma unroll
        for (int u = 0; u < NK; ++u) fp[u] = sf + u * flds;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;  // A row / k of this lane
    const int32_t ntiles = (oe - os + 15) >> 4;
    // this wave's row tiles (at most 4 of the block's at most 16). Passes of
    // one chunk take a contiguous run t = wave tpw + q (q < tpw): the jobs of
    // its tiles, and with them the source range the wave walks, are
    // neighbours. Passes of several chunks, with more MFMA work per source
    // step, take t = wave + 4 q, which measured faster there.
    const int32_t tpw = (ntiles + 3) >> 2;
    auto row_tile = [&](int q) -> int32_t {
        if (NCH > 1) return wave + 4 * q;
        return q < tpw ? wave * tpw + q : ntiles;
    };
    int32_t ri[4], xi[4], jb[4], je[4], tjb[4], tje[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t t = row_tile(q);
        const int32_t i = os + 16 * t + lr;
        const bool ok = t < ntiles && i < oe;
        const int32_t is = ok ? i : os;  // clamped: loads stay in range
        ri[q] = dl_r[is];
        xi[q] = dl_x[is];
        jb[q] = ok ? qjb[is >> 2] : 0;
        je[q] = ok ? qje[is >> 2] : 0;
        const bool tok = t < ntiles;
        const int32_t tb = tok ? os + 16 * t : os;
        const int32_t tjb_ = qjb[tb >> 2], tje_ = qje[(min(oe, tb + 16) - 1) >> 2];
        tjb[q] = tok ? tjb_ : 0;
        tje[q] = tok ? tje_ : 0;
    }
    // passes of NCH chunks: this workgroup takes every gridDim.y-th one
    for (int32_t c0 = blockIdx.y * 16 * NCH; c0 < d; c0 += gridDim.y * 16 * NCH) {
        v4f_t acc[NK][NCH][4];
#pragma unroll
        for (int u = 0; u < NK; ++u)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[u][ch][q] = (v4f_t){0.f, 0.f, 0.f, 0.f};
        for (int32_t ts = ss; ts < se; ts += ROWS) {
            const int32_t tn = min(ROWS, se - ts);
            __syncthreads();
            {
                // stage the tile: all row indices, then all values of the
                // pass's channels (addresses clamped into range)
                const int32_t cc = threadIdx.x & 15, k0 = threadIdx.x >> 4;
                int32_t rows[PER];
#pragma unroll
                for (int i = 0; i < PER; ++i) rows[i] = dl_row[ts + min(k0 + 16 * i, tn - 1)];
                float v[NCH][PER];
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int32_t c = min(c0 + 16 * ch + cc, d - 1);
#pragma unroll
                    for (int i = 0; i < PER; ++i) v[ch][i] = val[(int64_t)max(rows[i], 0) * d + c];
                }
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const bool cok = c0 + 16 * ch + cc < d;
#pragma unroll
                    for (int i = 0; i < PER; ++i) {
                        const int32_t k = k0 + 16 * i;
                        sv[k * SV + 16 * ch + cc] = (k < tn && rows[i] >= 0 && cok) ? v[ch][i] : 0.f;
                    }
                }
                if ((int32_t)threadIdx.x < tn) {
                    sr[threadIdx.x] = dl_r[ts + threadIdx.x];
                    sx[threadIdx.x] = dl_x[ts + threadIdx.x];
                }
                if (cc == 0) {
#pragma unroll
                    for (int i = 0; i < PER; ++i) {
                        const int32_t src = ts + k0 + 16 * i;
                        if (k0 + 16 * i < tn && src >= os && src < oe) so[src - os] = rows[i];
                    }
                }
            }
            __syncthreads();
            int32_t kb[4], ke[4];
            int32_t lo = 1 << 30, hi = -1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                kb[q] = max(tjb[q], ts);
                ke[q] = min(tje[q], ts + tn);
                if (kb[q] < ke[q]) {
                    lo = min(lo, kb[q]);
                    hi = max(hi, ke[q]);
                }
            }
            // the four row tiles advance together: independent MFMA chains;
            // one kernel entry per lane and row tile serves every chunk
            for (int32_t k4 = lo; k4 < hi; k4 += 4) {
                const int32_t k = k4 + lk, kl = k - ts;
                const int32_t rk = sr[kl], xk = sx[kl];
                float b[NCH];
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) b[ch] = sv[kl * SV + 16 * ch + lr];
                if (FL) {
                    // every tile's entries first (LDS reads in flight
                    // together), then the products
                    float a[4][NK];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int32_t dx = xi[q] - xk;
                        const int32_t e = min(max(ri[q] + rk + (dx < 0 ? -dx : dx), 0), flds - 1);
                        const bool own = k >= jb[q] && k < je[q];  // the lane's own job only
#pragma unroll
                        for (int u = 0; u < NK; ++u) {
                            const float v = fp[u][e];
                            a[q][u] = own ? v : 0.f;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (k4 < kb[q] || k4 >= ke[q]) continue;  // uniform per wave
#pragma unroll
                        for (int u = 0; u < NK; ++u)
#pragma unroll
                            for (int ch = 0; ch < NCH; ++ch)
                                acc[u][ch][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                    a[q][u], b[ch], acc[u][ch][q], 0, 0, 0);
                    }
                    continue;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (k4 < kb[q] || k4 >= ke[q]) continue;  // uniform per wave
                    float a[NK];
#pragma unroll
                    for (int u = 0; u < NK; ++u) a[u] = 0.f;
                    if (k >= jb[q] && k < je[q]) {  // entries of the lane's own job only
                        const int32_t dx = xi[q] - xk;
                        const int32_t e = ri[q] + rk + (dx < 0 ? -dx : dx);
#pragma unroll
                        for (int u = 0; u < NK; ++u) a[u] = fp[u][e];
                    }
#pragma unroll
                    for (int u = 0; u < NK; ++u)
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch)
                            acc[u][ch][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                a[u], b[ch], acc[u][ch][q], 0, 0, 0);
                }
            }
        }
        // D[4 (l/16) + r][l % 16] of every row tile and chunk
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t t = row_tile(q);
            if (t >= ntiles) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int32_t i = os + 16 * t + 4 * lk + r;
                if (i >= oe) continue;
                const int32_t row = so[i - os];
                if (row < 0) continue;
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int32_t c = c0 + 16 * ch + lr;
                    if (c < d) {
                        g[(int64_t)row * d + c] = acc[0][ch][q][r];
                        if (NK > 1) g1[(int64_t)row * d + c] = acc[NK - 1][ch][q][r];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- gather --
// One thread per (vertex, VEC channels), in column tiles like the scatter
// (the table rows of one tile stay in cache across vertices): adds, over the
// calls holding the
// vertex, the call's table value minus the component correction (row -1
// when the vertex is on the call's backbone), on top of the leaf-tile value
// already stored in out for vertices of leaf tiles. Writes every out row.
// NK = 2 gathers the tables g, g1 of two kernels into out, out1 with one
// pass over the index lists (the summation order of each is unchanged).
constexpr int kGatherBatch = 4;

template <typename T, int VEC, int NK>
__global__ void k_gather(int64_t N, int32_t d, int32_t ct, const int64_t* __restrict__ v_off,
                         const int32_t* __restrict__ ga, const int32_t* __restrict__ gb,
                         const int8_t* __restrict__ vleaf, const T* __restrict__ g,
                         const T* __restrict__ g1, T* __restrict__ out, T* __restrict__ out1) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t v;
    int32_t c;
    if (!tile_coords<VEC>(tid, N, d, ct, v, c) || v >= N) return;
    const T* gk[NK];
    T* ok[NK];
    gk[0] = g;
    ok[0] = out;
    if (NK > 1) {
        gk[NK - 1] = g1;
        ok[NK - 1] = out1;
    }
    const int64_t k0 = v_off[v], k1 = v_off[v + 1];
    const bool leaf = vleaf[v] != 0;  // out already holds the leaf tile value
    vec4<T> s[NK];
#pragma unroll
    for (int u = 0; u < NK; ++u) {
        s[u] = {0, 0, 0, 0};
        if (leaf) {
            if (VEC == 4) s[u] = ld4(ok[u] + v * d + c);
            else s[u].x = ok[u][v * d + c];
        }
    }
    // calls taken kGatherBatch at a time: indices first, then table rows;
    // the next batch's indices are requested with this batch's rows
    int32_t an[kGatherBatch], bn[kGatherBatch];
    auto load_idx = [&](int64_t kk) {
#pragma unroll
        for (int w = 0; w < kGatherBatch; ++w) {
            const int64_t k = max(min(kk + w, k1 - 1), (int64_t)0);
            an[w] = ga[k];
            bn[w] = gb[k];
        }
    };
    if (k0 < k1) load_idx(k0);
    for (int64_t kk = k0; kk < k1; kk += kGatherBatch) {
        int32_t a[kGatherBatch], b[kGatherBatch];
#pragma unroll
        for (int w = 0; w < kGatherBatch; ++w) {
            a[w] = an[w];
            b[w] = bn[w];
        }
        if (kk + kGatherBatch < k1) load_idx(kk + kGatherBatch);
#pragma unroll
        for (int u = 0; u < NK; ++u) {
            if (VEC == 4) {
                vec4<T> ra[kGatherBatch], rb[kGatherBatch];
#pragma unroll
                for (int w = 0; w < kGatherBatch; ++w) {
                    ra[w] = ld4(gk[u] + (int64_t)a[w] * d + c);
                    rb[w] = ld4(gk[u] + (int64_t)(b[w] >= 0 ? b[w] : a[w]) * d + c);
                }
#pragma unroll
                for (int w = 0; w < kGatherBatch; ++w) {
                    if (kk + w >= k1) continue;
                    add4(s[u], ra[w]);
                    if (b[w] >= 0) sub4(s[u], rb[w]);
                }
            } else {
                T ra[kGatherBatch], rb[kGatherBatch];
#pragma unroll
                for (int w = 0; w < kGatherBatch; ++w) {
                    ra[w] = gk[u][(int64_t)a[w] * d + c];
                    rb[w] = gk[u][(int64_t)(b[w] >= 0 ? b[w] : a[w]) * d + c];
                }
#pragma unroll
                for (int w = 0; w < kGatherBatch; ++w) {
                    if (kk + w >= k1) continue;
                    s[u].x += ra[w];
                    if (b[w] >= 0) s[u].x -= rb[w];
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NK; ++u) {
        if (VEC == 4) st4(ok[u] + v * d + c, s[u]);
        else ok[u][v * d + c] = s[u].x;
    }
}

// ----------------------------------------------------------- leaf tiles --
// Dense f(D) F on small subtrees, blocked like the direct tables: a thread
// owns 4 vertices x 4 channels of one tile. A workgroup owns a group of
// consecutive tiles (at most kLeafQuads vertex quads and kLeafK kernel
// entries); f(D) of every tile and the field rows (kDirCh channels at a
// time) are staged in LDS, then out[v] = sum_j f(D[v, j]) F[j] (the gather
// adds the cross-call terms afterwards).
// lq[4 q .. 4 q + 3] describes quad q: (first vertex in leaf_v, tile start
// in leaf_v, tile size, offset of the quad's first kernel row in the
// group's f(D) block); grp holds quad ranges per group and koff the
// group's first leaf_D entry and count.
// NK = 2: two kernels f, f1 over the same tiles in one launch (the
// distances and field rows are staged once; out1 = f1(D) F); the threads
// take (kernel, quad) tasks, so the sums are those of two NK = 1 launches.
constexpr int kLeafMax = 64, kLeafQuads = 32, kLeafSlots = 128, kLeafK = 4096,
              kLeafThreads = 256;

template <typename T, int NK = 1>
__global__ void __launch_bounds__(kLeafThreads)
k_leaf(int32_t d, const int32_t* __restrict__ grp, const int64_t* __restrict__ gk,
       const int32_t* __restrict__ lq, const int32_t* __restrict__ leaf_v,
       const int32_t* __restrict__ leaf_D, const T* __restrict__ f, const T* __restrict__ F,
       T* __restrict__ out, const T* __restrict__ f1 = nullptr, T* __restrict__ out1 = nullptr) {
    static_assert(NK == 1 || NK == 2, "one or two kernels");
    __shared__ T sk[NK * kLeafK];
    __shared__ __attribute__((aligned(16))) T sF[kLeafSlots * kDirCh];
    const int32_t q0 = grp[blockIdx.x], q1 = grp[blockIdx.x + 1];
    const int64_t kb = gk[2 * blockIdx.x];
    const int32_t nk = (int32_t)gk[2 * blockIdx.x + 1];
    // vertex slots are leaf_v positions [vb, vb + nv): the group's tiles
    const int32_t vb = lq[4 * q0 + 1];
    const int32_t nv = lq[4 * (q1 - 1) + 1] + lq[4 * (q1 - 1) + 2] - vb;
    // the two independent load chains are issued together: distances, then
    // the kernel entries they select; vertex ids, then the field rows
    constexpr int kPerK = kLeafK / kLeafThreads;
    constexpr int kPerF = kLeafSlots / (kLeafThreads / 16);
    const int32_t lc = threadIdx.x & 15, k0 = threadIdx.x >> 4;
    int32_t di[kPerK];
#pragma unroll
    for (int i = 0; i < kPerK; ++i)
        di[i] = leaf_D[kb + min((int32_t)threadIdx.x + kLeafThreads * i, nk - 1)];
    int32_t vt[kPerF];
#pragma unroll
    for (int i = 0; i < kPerF; ++i) vt[i] = leaf_v[vb + min(k0 + 16 * i, nv - 1)];
    T fv[NK][kPerK];
#pragma unroll
    for (int u = 0; u < NK; ++u) {
        const T* fu = u ? f1 : f;
#pragma unroll
        for (int i = 0; i < kPerK; ++i) fv[u][i] = fu[di[i]];
    }
    // channel chunks: this workgroup takes every gridDim.y-th one. The field
    // rows of a chunk (all loads in flight at once) are requested before the
    // products of the previous chunk, so they arrive while it computes.
    const int32_t cstep = gridDim.y * kDirCh;
    T v[kPerF];
    auto load_rows = [&](int32_t c) {
        const int32_t ccs = min(lc, min(kDirCh, d - c) - 1);
#pragma unroll
        for (int i = 0; i < kPerF; ++i) v[i] = F[(int64_t)vt[i] * d + c + ccs];
    };
    if (blockIdx.y * kDirCh < d) load_rows(blockIdx.y * kDirCh);
    bool stage_k = true;
    for (int32_t c0 = blockIdx.y * kDirCh; c0 < d; c0 += cstep) {
        const int32_t nch = min(kDirCh, d - c0);
        const int32_t nq = (nch + 3) >> 2;
        const int32_t qpp = kLeafThreads / nq;
        if (stage_k) {
#pragma unroll
            for (int u = 0; u < NK; ++u)
#pragma unroll
                for (int i = 0; i < kPerK; ++i) {
                    const int32_t k = threadIdx.x + kLeafThreads * i;
                    if (k < nk) sk[u * kLeafK + k] = fv[u][i];
                }
            stage_k = false;
        }
        __syncthreads();  // the previous chunk's products are done with sF
#pragma unroll
        for (int i = 0; i < kPerF; ++i) {
            const int32_t k = k0 + 16 * i;
            if (k < nv) sF[k * kDirCh + lc] = (lc < nch) ? v[i] : (T)0;
        }
        __syncthreads();
        if (c0 + cstep < d) load_rows(c0 + cstep);
        const int32_t cq0 = threadIdx.x / nq;
        const int32_t nquads = q1 - q0;
        for (int32_t tq = cq0; cq0 < qpp && tq < NK * nquads; tq += qpp) {
            const int32_t u = NK > 1 && tq >= nquads ? 1 : 0;
            const int32_t qq = tq - u * nquads;
            const T* sku = sk + u * kLeafK;
            T* outu = u ? out1 : out;
            const int32_t chq = threadIdx.x % nq;
            const int32_t q = q0 + qq;
            const int32_t first = lq[4 * q], tb = lq[4 * q + 1], n = lq[4 * q + 2];
            // f(D) of a tile is symmetric: entry (row r, column j) is read
            // at column-major position j n + r, so the quads of one tile
            // read neighbouring LDS words instead of words n apart (which
            // share a bank); the values and their order are unchanged
            const int32_t r0 = first - tb;
            const int32_t kt = lq[4 * q + 3] - r0 * n + r0;
            vec4<T> acc[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = {0, 0, 0, 0};
            const int32_t rows = min(4, tb + n - first);
            for (int32_t j = 0; j < n; ++j) {
                const vec4<T> v = ld4(sF + (tb - vb + j) * kDirCh + 4 * chq);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c < rows) fma4(acc[c], sku[kt + j * n + c], v);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (c >= rows) continue;
                const int32_t vtx = leaf_v[first + c];
                T* o = outu + (int64_t)vtx * d + c0 + 4 * chq;
                const int32_t left = nch - 4 * chq;
                const T vv[4] = {acc[c].x, acc[c].y, acc[c].z, acc[c].w};
                for (int cc = 0; cc < 4 && cc < left; ++cc) o[cc] = vv[cc];
            }
        }
    }
}

// ------------------------------------------------------------------- FFT --
// In-place radix-2 transforms along one axis of a batch of lines in LDS.
// Forward: decimation in frequency, natural order in, bit-reversed out.
// Inverse: decimation in time, bit-reversed in, natural order out
// (unnormalised). A convolution multiplies two forward spectra in the same
// bit-reversed layout, so no reordering pass is needed.
//
// The stages run in passes of up to three (radix-8, radix-4 or radix-2
// groups): a thread loads the 2^R points of one group into registers, runs
// the group's R stages there and stores them back, so a transform of 2^lgL
// points takes ceil(lgL / 3) barriers instead of lgL. The stage of span 2^s
// pairs points e and e + 2^s with twiddle W_{2^(s+1)}^(e mod 2^s),
// W_n = exp(-2 pi i / n) (conjugated for the inverse). Within a pass over
// index bits [s0, s0 + R) that twiddle factors as a compile-time 8th root of
// unity times one table factor per stage, W_{2^(s+1)}^(e mod 2^s0). The
// stage factors of a pass are successive squares of the last one, so a
// group reads one table entry: f = W_{2^(s0+R)}^(e mod 2^s0), f^2, f^4.
//
// Twiddle table tw[k] = exp(-2 pi i k / 2^lgtw), k < 2^(lgtw-1), lgtw >= lgL.

// exp(-2 pi i m / 32), m < 16
constexpr double kW32re[16] = {
    1.0, 0.98078528040323043, 0.92387953251128674, 0.83146961230254524,
    0.70710678118654757, 0.55557023301960229, 0.38268343236508984, 0.19509032201612833,
    0.0, -0.19509032201612819, -0.38268343236508973, -0.55557023301960196,
    -0.70710678118654746, -0.83146961230254535, -0.92387953251128674, -0.98078528040323043};
constexpr double kW32im[16] = {
    -0.0, -0.19509032201612825, -0.38268343236508978, -0.55557023301960218,
    -0.70710678118654746, -0.83146961230254524, -0.92387953251128674, -0.98078528040323043,
    -1.0, -0.98078528040323043, -0.92387953251128674, -0.83146961230254546,
    -0.70710678118654757, -0.55557023301960218, -0.38268343236508989, -0.19509032201612861};

// z W_32^m and z conj(W_32^m) for m < 16 known at compile time once the
// butterfly loops are unrolled. The powers 1, W_8, -i and W_8^3 (m = 0, 4,
// 8, 12) take sign flips, adds and one scale by sqrt(1/2) rather than a
// full complex product with rounded constants.
template <typename T>
__device__ __forceinline__ cpx<T> mul_w32(cpx<T> z, int m) {
    const T h = (T)0.70710678118654752440;
    switch (m) {
        case 0: return z;
        case 4: return {(z.x + z.y) * h, (z.y - z.x) * h};
        case 8: return {z.y, -z.x};
        case 12: return {(z.y - z.x) * h, -(z.x + z.y) * h};
        default: return cmul(z, cpx<T>{(T)kW32re[m], (T)kW32im[m]});
    }
}
template <typename T>
__device__ __forceinline__ cpx<T> mul_w32c(cpx<T> z, int m) {
    const T h = (T)0.70710678118654752440;
    switch (m) {
        case 0: return z;
        case 4: return {(z.x - z.y) * h, (z.x + z.y) * h};
        case 8: return {-z.y, z.x};
        case 12: return {-(z.x + z.y) * h, (z.x - z.y) * h};
        default: return cmulc(z, cpx<T>{(T)kW32re[m], (T)kW32im[m]});
    }
}
// z^2, with the real part as (x - y)(x + y)
template <typename T>
__device__ __forceinline__ cpx<T> csq(cpx<T> z) {
    return {(z.x - z.y) * (z.x + z.y), (T)2 * z.x * z.y};
}

// A batch of lines in LDS: line l0 + 2^lgc0 l1 (l0 < 2^lgc0, l1 < c1)
// starts at l0 ls0 + l1 ls1; its points are es apart. lgtn: low bits of l0
// that select one of several separate transforms (see lds_pass).
struct LdsLines {
    int lgc0, ls0, c1, ls1, es, lgtn = 0;
};

// LDS position of point i of a block stored with one spare element after
// every 2^PAD (PAD = 0: none). A pass whose lanes read points 2^R apart
// (the groups of a line, lines one after another) then spreads them over
// the banks instead of hitting a few.
template <int PAD>
__device__ __forceinline__ int lds_at(int i) {
    return PAD ? i + (i >> PAD) : i;
}

// One pass: R stages over index bits [s0, s0 + R) of every line. Lines that
// are part of a longer transform (the blocked global passes) give their
// twiddles the global index: point e of line l0 stands for index
// (e << tsh) + tbase + (l0 >> lgtn) (tsh = 0: e itself). Ends with a
// barrier.
template <typename T, bool INV, int R, int PAD = 0>
__device__ __forceinline__ void lds_pass(cpx<T>* z, int lgL, int s0, const LdsLines& L, int tsh,
                                         int tbase, const cpx<T>* __restrict__ tw, int lgtw) {
    const int lgr = lgL - R;
    const int nitems = (L.c1 << L.lgc0) << lgr;
    const bool line_fast = L.ls0 < L.es;  // neighbouring lanes on neighbouring addresses
    const int mr = (1 << lgr) - 1, mc = (1 << L.lgc0) - 1;
    const int step = (1 << s0) * L.es;
    // item it: line (l0, l1) and the butterfly group (hi, lo) of index bits
    // below and above the pass's R bits
    auto split = [&](int it, int& l0, int& l1, int& lo, int& hi) {
        int rest;
        if (line_fast) {
            l0 = it & mc;
            rest = (it >> L.lgc0) & mr;
        } else {
            rest = it & mr;
            l0 = (it >> lgr) & mc;
        }
        l1 = it >> (lgr + L.lgc0);
        lo = rest & ((1 << s0) - 1);
        hi = rest >> s0;
    };
    // table factor of an item's last stage (see the twiddle note above)
    auto factor = [&](int l0, int lo) -> cpx<T> {
        const int J = (lo << tsh) + (tsh ? tbase + (l0 >> L.lgtn) : 0);
        const int t = J << (lgtw - tsh - s0 - R);
        if (tsh) {
            // A pass over the high bits of a long axis would touch the
            // whole table (megabytes, missing in L2 on every slot): split
            // t = th 2^lgb + tl, W^t = W^(th 2^lgb) W^tl, two factors
            // from 2^(lgtw-1-lgb) strided and 2^lgb leading entries.
            const int lgb = (lgtw + 1) >> 1;
            return cmul(tw[(t >> lgb) << lgb], tw[t & ((1 << lgb) - 1)]);
        }
        return tw[t];
    };
    const int nb = blockDim.x;
    cpx<T> f;
    int l0, l1, lo, hi;
    if ((int)threadIdx.x < nitems) {
        split(threadIdx.x, l0, l1, lo, hi);
        f = factor(l0, lo);
    }
    for (int it = threadIdx.x; it < nitems; it += nb) {
        split(it, l0, l1, lo, hi);
        // the next item's factor is requested before this item's work
        cpx<T> fn;
        if (it + nb < nitems) {
            int m0, m1, mlo, mhi;
            split(it + nb, m0, m1, mlo, mhi);
            fn = factor(m0, mlo);
        }
        cpx<T> fs[R];
        fs[R - 1] = f;
#pragma unroll
        for (int u = R - 2; u >= 0; --u) fs[u] = csq(fs[u + 1]);
        const int base = l0 * L.ls0 + l1 * L.ls1 + ((hi << (s0 + R)) | lo) * L.es;
        cpx<T> x[1 << R];
#pragma unroll
        for (int k = 0; k < (1 << R); ++k) x[k] = z[lds_at<PAD>(base + k * step)];
#pragma unroll
        for (int uu = 0; uu < R; ++uu) {
            const int u = INV ? uu : R - 1 - uu;
            const int h = 1 << u;
#pragma unroll
            for (int k = 0; k < (1 << R); ++k) {
                if (k & h) continue;
                const int m = (k & (h - 1)) << (4 - u);  // W_{2^(u+1)}^(k mod 2^u) = W_32^m
                const cpx<T> p = x[k], q = x[k + h];
                if (!INV) {
                    x[k] = cadd(p, q);
                    x[k + h] = cmul(csub(p, q), mul_w32(fs[u], m));
                } else {
                    const cpx<T> qw = cmulc(q, mul_w32(fs[u], m));
                    x[k] = cadd(p, qw);
                    x[k + h] = csub(p, qw);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < (1 << R); ++k) z[lds_at<PAD>(base + k * step)] = x[k];
        f = fn;
    }
    __syncthreads();
}

// The whole transform of 2^lgL points along every line of L: forward passes
// from the high index bits down, inverse passes from the low bits up.
template <typename T, bool INV, int PAD = 0>
__device__ void fft_lines(cpx<T>* z, int lgL, const LdsLines& L, int tsh, int tbase,
                          const cpx<T>* __restrict__ tw, int lgtw) {
    auto pass = [&](int s0, int R) {
        if (R == 3) lds_pass<T, INV, 3, PAD>(z, lgL, s0, L, tsh, tbase, tw, lgtw);
        else if (R == 2) lds_pass<T, INV, 2, PAD>(z, lgL, s0, L, tsh, tbase, tw, lgtw);
        else lds_pass<T, INV, 1, PAD>(z, lgL, s0, L, tsh, tbase, tw, lgtw);
    };
    if (INV) {
        for (int s0 = 0; s0 < lgL;) {
            const int R = min(3, lgL - s0);
            pass(s0, R);
            s0 += R;
        }
    } else {
        for (int s1 = lgL; s1 > 0;) {
            const int R = min(3, s1);
            pass(s1 - R, R);
            s1 -= R;
        }
    }
}

// One axis of a 2-D array: `count` (a power of two) lines of 2^lgL points,
// element stride es, line stride ls.
template <typename T, bool INV, int PAD = 0>
__device__ void fft_axis_lds(cpx<T>* z, int lgL, int count, int es, int ls,
                             const cpx<T>* __restrict__ tw, int lgtw) {
    fft_lines<T, INV, PAD>(z, lgL, LdsLines{31 - __clz(count), ls, 1, 0, es}, 0, 0, tw, lgtw);
}

// Bucket parameters of merged launches: bp[4 b .. 4 b + 3] = (lg1, lg2,
// Hmax, Xmax) and bo[b] = the bucket's offset in the spectrum arena.

// Kernel spectrum of FFT bucket blockIdx.x: k[a][b] = f(a + |b|) on the
// padded L1 x L2 grid (b taken as the signed circular offset), zero
// outside the bucket's reach a <= 2 Hmax, |b| <= Xmax; forward 2-D
// transform in LDS.
template <typename T>
__global__ void k_spectrum_multi(const int32_t* __restrict__ bp, const int64_t* __restrict__ bo,
                                 const T* __restrict__ f, const cpx<T>* __restrict__ tw, int lgtw,
                                 cpx<T>* __restrict__ spec) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_raw);
    const int lg1 = bp[4 * blockIdx.x], lg2 = bp[4 * blockIdx.x + 1];
    const int32_t hmax = bp[4 * blockIdx.x + 2], xmax = bp[4 * blockIdx.x + 3];
    cpx<T>* out = spec + bo[blockIdx.x];
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
    for (int p = threadIdx.x; p < P; p += blockDim.x) out[p] = z[p];
}

// FFT convolution of LDS-resident tables: one workgroup per (job, group of
// 2^lgnp channel pairs), one table per pair side by side in LDS (pair c at
// z + c P); fj[3 j .. 3 j + 2] = (first cell, end cell, bucket) of job j.
// Two real channels ride in the real and imaginary parts of one complex
// table (the kernel is real, so the two results separate again in the
// real and imaginary parts of the output). Source cell (r, x) goes to row
// (-r mod L1): the Hankel dependence on q + r becomes a circular
// convolution whose output row q needs no shift. The rows of all the
// group's tables transform as one batch of lines, then their columns.
// PAD: the block is stored with lds_at<PAD> (one spare element per 2^PAD),
// so that the row passes, whose lanes read points of one row 8 apart, do not
// share banks. Each thread issues the global loads of kConvBatch items
// before it uses the first.
constexpr int kConvBatch = 8;

constexpr unsigned kConvXcdGroups = 16;

template <typename T, int PAD = 0>
__global__ void k_fft_conv_multi(const int32_t* __restrict__ fj, const int32_t* __restrict__ bp,
                                 const int64_t* __restrict__ bo,
                                 const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
                                 const int32_t* __restrict__ jc_val, int32_t d,
                                 const T* __restrict__ val, T* __restrict__ g,
                                 const cpx<T>* __restrict__ spec_all,
                                 const cpx<T>* __restrict__ tw, int lgtw, int lgw, int lgcap,
                                 int32_t njobs) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_raw);
    // (job, group) of this workgroup. The groups of one job read the same
    // cell rows, a few pairs each. Workgroups are dealt to the 8 XCDs in
    // turn; with kConvXcdGroups groups or more (wide rows; the grid then
    // has a multiple of 8 job columns) job j goes to XCD j mod 8 and its
    // groups to consecutive slots there, so they run together and read the
    // rows from that XCD's L2, while neighbouring jobs (tables of similar
    // size) spread over the XCDs. With fewer groups, most of a small
    // table's groups exit at once and grid order measured faster.
    int32_t job = blockIdx.x, grp = blockIdx.y;
    if (gridDim.y >= kConvXcdGroups) {
        const int64_t w = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
        const int64_t k = w >> 3;
        job = (int32_t)((w & 7) + 8 * (k / gridDim.y));
        grp = (int32_t)(k % gridDim.y);
    }
    if (job >= njobs) return;
    const int32_t cb = fj[3 * job], ce = fj[3 * job + 1], bk = fj[3 * job + 2];
    const int lg1 = bp[4 * bk], lg2 = bp[4 * bk + 1];
    const cpx<T>* spec = spec_all + bo[bk];
    const int L1 = 1 << lg1, L2 = 1 << lg2, P = L1 * L2, lgP = lg1 + lg2;
    // channel pairs of this table's workgroups: as many as fill the block
    // of 2^lgw points (the launch's pairs for its largest table, more for
    // smaller ones), at most 2^lgcap; a job then needs fewer of the
    // launch's groups, and the others leave at once
    const int lgnp = max(0, min(lgw - lgP, lgcap));
    const int NP = 1 << lgnp;
    const int nb = blockDim.x;
    const int32_t ch0 = 2 * grp * NP;  // first channel of the group
    if (ch0 >= d) return;
    for (int p = threadIdx.x; p < NP * P; p += nb) z[lds_at<PAD>(p)] = {(T)0, (T)0};
    __syncthreads();
    // item it: cell cb + (it >> lgnp), pair it mod NP of the group
    const int32_t items = (ce - cb) << lgnp;
    for (int32_t i0 = threadIdx.x; i0 < items; i0 += kConvBatch * nb) {
        int at[kConvBatch];
        int64_t vr[kConvBatch];
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u) {
            const int32_t it = i0 + u * nb;
            at[u] = -1;
            if (it < items) {
                const int c = it & (NP - 1);
                const int32_t k = cb + (it >> lgnp);
                const int row = (L1 - jc_r[k]) & (L1 - 1);
                at[u] = (c << lgP) + (row << lg2) + jc_x[k];
                vr[u] = (int64_t)jc_val[k] * d + ch0 + 2 * c;
                if (ch0 + 2 * c >= d) at[u] = -1;
            }
        }
        cpx<T> v[kConvBatch];
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u) {
            const int32_t it = i0 + u * nb;
            if (at[u] >= 0) {
                const int ch = ch0 + 2 * (it & (NP - 1));
                v[u] = {val[vr[u]], ch + 1 < d ? val[vr[u] + 1] : (T)0};
            }
        }
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u)
            if (at[u] >= 0) z[lds_at<PAD>(at[u])] = v[u];
    }
    __syncthreads();
    const LdsLines rows{lg1 + lgnp, L2, 1, 0, 1}, cols{lg2, 1, NP, P, L2};
    fft_lines<T, false, PAD>(z, lg2, rows, 0, 0, tw, lgtw);
    fft_lines<T, false, PAD>(z, lg1, cols, 0, 0, tw, lgtw);
    for (int p0 = threadIdx.x; p0 < NP * P; p0 += kConvBatch * nb) {
        cpx<T> sv[kConvBatch];
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u)
            if (p0 + u * nb < NP * P) sv[u] = spec[(p0 + u * nb) & (P - 1)];
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u) {
            const int p = p0 + u * nb;
            if (p < NP * P) z[lds_at<PAD>(p)] = cmul(z[lds_at<PAD>(p)], sv[u]);
        }
    }
    __syncthreads();
    fft_lines<T, true, PAD>(z, lg1, cols, 0, 0, tw, lgtw);
    fft_lines<T, true, PAD>(z, lg2, rows, 0, 0, tw, lgtw);
    const T scale = (T)1 / (T)P;
    for (int32_t i0 = threadIdx.x; i0 < items; i0 += kConvBatch * nb) {
        int at[kConvBatch];
        int64_t vr[kConvBatch];
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u) {
            const int32_t it = i0 + u * nb;
            at[u] = -1;
            if (it < items) {
                const int c = it & (NP - 1);
                const int32_t k = cb + (it >> lgnp);
                at[u] = (c << lgP) + (jc_r[k] << lg2) + jc_x[k];
                vr[u] = (int64_t)jc_val[k] * d + ch0 + 2 * c;
                if (ch0 + 2 * c >= d) at[u] = -1;
            }
        }
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u) {
            if (at[u] < 0) continue;
            const cpx<T> y = z[lds_at<PAD>(at[u])];
            const int ch = ch0 + 2 * ((i0 + u * nb) & (NP - 1));
            g[vr[u]] = y.x * scale;
            if (ch + 1 < d) g[vr[u] + 1] = y.y * scale;
        }
    }
}

// One channel pair of a row as a single 8- or 16-byte access (the pair
// starts at an even channel of a row of even length, in a buffer aligned to
// two elements).
template <typename T>
__device__ __forceinline__ cpx<T> ld_pair(const T* p) {
    if constexpr (sizeof(T) == 4) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        return {v.x, v.y};
    } else {
        const double2 v = *reinterpret_cast<const double2*>(p);
        return {v.x, v.y};
    }
}
template <typename T>
__device__ __forceinline__ void st_pair(T* p, cpx<T> v) {
    if constexpr (sizeof(T) == 4)
        *reinterpret_cast<float2*>(p) = make_float2(v.x, v.y);
    else
        *reinterpret_cast<double2*>(p) = make_double2(v.x, v.y);
}

// ---------------------------------------------- FFT through global memory --
// Tables too large for LDS: the same in-place DIF/DIT transforms over every
// (job, channel pair) slot of a bucket, as blocked passes (k_fft_pass) of up
// to 12 radix-2 stages each, every pass staged through LDS. Buffer layout:
// slot s = job * npairs + pair holds P complex.
// rev != 0: source cell (r, x) at row -r mod L1 (the 2-D convolution);
// rev = 0: at row r (the per-depth rows of the 1-D path).
// Job blockIdx.y; a workgroup takes kXCells cells at a time and moves them
// through LDS in chunks of kXPairs channel pairs: the value rows are read
// whole (4 threads per cell, 4 pairs each) and every pair's points are
// written by consecutive lanes, one cell per lane.
constexpr int kXCells = 64, kXPairs = 16, kXStride = kXPairs + 1;

// The cell's table point (-1 past the job's end) and value row.
__device__ __forceinline__ void cell_point(int32_t k, int32_t ce, const int32_t* __restrict__ jc_r,
                                           const int32_t* __restrict__ jc_x,
                                           const int32_t* __restrict__ jc_val, int64_t L1, int lg2,
                                           int rev, int64_t& at, int64_t& vrow) {
    at = -1;
    vrow = 0;
    if (k < ce) {
        const int64_t row = rev ? (L1 - jc_r[k]) & (L1 - 1) : jc_r[k];
        at = (row << lg2) + jc_x[k];
        vrow = jc_val[k];
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_fill_global(int lg1, int lg2, int32_t npairs, const int32_t* __restrict__ jobs,
              const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
              const int32_t* __restrict__ jc_val, int32_t d, const T* __restrict__ val,
              cpx<T>* __restrict__ buf, int rev) {
    __shared__ cpx<T> sc[kXCells * kXStride];
    const int64_t P = (int64_t)1 << (lg1 + lg2);
    const int32_t job = blockIdx.y;
    const int64_t L1 = (int64_t)1 << lg1;
    cpx<T>* z = buf + (int64_t)job * npairs * P;
    const int32_t cb = jobs[2 * job], ce = jobs[2 * job + 1];
    const bool pairs = (d & 1) == 0 && ((uintptr_t)val & (2 * sizeof(T) - 1)) == 0;
    const int t = threadIdx.x;
    for (int32_t k0 = cb + blockIdx.x * kXCells; k0 < ce; k0 += gridDim.x * kXCells) {
        // lane view: cell t % 64 (points); row view: cell t / 4, pairs 4 (t % 4) ..
        int64_t at, vrow, at_r, vrow_r;
        cell_point(k0 + (t & 63), ce, jc_r, jc_x, jc_val, L1, lg2, rev, at, vrow);
        cell_point(k0 + (t >> 2), ce, jc_r, jc_x, jc_val, L1, lg2, rev, at_r, vrow_r);
        for (int32_t p0 = 0; p0 < npairs; p0 += kXPairs) {
            __syncthreads();
            if (at_r >= 0) {
                const T* v = val + vrow_r * d;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t pl = 4 * (t & 3) + q, c0 = 2 * (p0 + pl);
                    if (p0 + pl >= npairs) continue;
                    cpx<T> y;
                    if (pairs) y = ld_pair(v + c0);
                    else y = {v[c0], c0 + 1 < d ? v[c0 + 1] : (T)0};
                    sc[(t >> 2) * kXStride + pl] = y;
                }
            }
            __syncthreads();
            if (at >= 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t pl = (t >> 6) + 4 * q;
                    if (p0 + pl < npairs) z[(p0 + pl) * P + at] = sc[(t & 63) * kXStride + pl];
                }
            }
        }
    }
}

// Blocked pass of the in-place transform along one axis of length 2^lgL
// (element stride es) of every line (nlines per slot, line stride ls) of
// every slot (2^lgP elements apart): the stages whose butterfly spans are
// 2^lglo .. 2^(lglo+k-1), done in LDS by register passes. A workgroup owns
// one butterfly group -- the 2^k elements that differ in index bits
// [lglo, lglo + k) -- for C = 2^lgC consecutive values of the bits below
// lglo (consecutive addresses when es = 1) and N = 2^lgN neighbouring lines
// (consecutive addresses when ls = 1: the column passes of a 2-D table).
// The last pass (lglo = 0) takes 2^lgG consecutive groups instead, so that
// a workgroup still holds up to 4096 points when few bits are left (with
// es = 1 the groups are one contiguous run; lines that follow one another
// in memory are passed as one longer axis whose top bits no stage touches).
// Forward (DIF) passes go from the high bits down, inverse (DIT) passes from
// the low bits up, with the same twiddles exp(-+2 pi i j / 2h) as the LDS
// transform. MUL: the last forward pass of a convolution also multiplies by
// the kernel spectrum (spec, indexed by the point's offset in its table) and
// runs the first inverse pass, so the buffer is read and written once for
// the three.
constexpr int kPassThreads = 256;  // k_fft_pass block size
constexpr int kPassPer = 16;       // points per thread (at most 2^12 per workgroup)
constexpr int kPassPad = 4;        // one spare LDS element per 16 (lds_at)

// LDS elements of a k_fft_pass block of n points.
constexpr int64_t pass_lds_elems(int64_t n) { return n + (n >> kPassPad); }

template <typename T, bool INV, bool MUL = false>
__global__ void __launch_bounds__(kPassThreads)
k_fft_pass(cpx<T>* __restrict__ buf, int lgP, int lgL, int64_t es, int64_t ls,
           int64_t nlines, int lglo, int k, int lgC, int lgN, int lgG,
           const cpx<T>* __restrict__ tw, int lgtw,
           const cpx<T>* __restrict__ spec = nullptr) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_raw);
    const int64_t C = (int64_t)1 << lgC;
    const int64_t nlo = ((int64_t)1 << lglo) >> lgC;               // low-bit chunks
    const int64_t nhi = ((int64_t)1 << (lgL - lglo - k)) >> lgG;   // high-bit values (groups)
    const int64_t ngrp = nlines >> lgN;                             // groups of N lines
    int64_t g = blockIdx.x, slot = 0;
    const bool slots_fast = MUL && (gridDim.x & 7) == 0;
    if (slots_fast) {
        // Every slot multiplies by the same spectrum chunk. Workgroups are
        // dealt to the 8 XCDs in turn: renumber them so that each XCD runs a
        // contiguous range, slots fastest, and the slots of one chunk follow
        // one another on one XCD, reading the chunk from its L2.
        g = (g & 7) * (gridDim.x >> 3) + (g >> 3);
        const int64_t nslots = (int64_t)gridDim.x / (nlo * nhi * ngrp);
        slot = g % nslots;
        g /= nslots;
    }
    const int64_t lo_chunk = g % nlo;
    g /= nlo;
    const int64_t hi = (g % nhi) << lgG;
    g /= nhi;
    const int64_t line = (g % ngrp) << lgN;
    if (!slots_fast) slot = g / ngrp;
    cpx<T>* base = buf + (slot << lgP) + line * ls;
    const int64_t i0 = (hi << (lglo + k)) + lo_chunk * C;
    // Point e of the workgroup (e = threadIdx.x + u kPassThreads) sits at
    // off(e) from base. The lgG > 0 pass (lglo = lgC = lgN = 0) holds 2^lgG
    // groups of 2^k points, point e at i0 + e; the others hold C x N lines
    // of 2^k points, LDS e = ((j << lgC | lo) << lgN) | ln (line ln fastest)
    // at ln ls + (i0 + (j << lglo) + lo) es. Every load of the thread is
    // issued before the first is used.
    const int lgCN = lgC + lgN;
    const int n = 1 << (k + (lgG > 0 ? lgG : lgCN));
    auto off = [&](int e) -> int64_t {
        if (lgG > 0) return (i0 + e) * es;
        const int64_t ln = e & ((1 << lgN) - 1), lo = (e >> lgN) & (C - 1), j = e >> lgCN;
        return ln * ls + (i0 + (j << lglo) + lo) * es;
    };
    cpx<T> r[kPassPer], sv[kPassPer];
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) {
        const int e = threadIdx.x + u * kPassThreads;
        if (e < n) r[u] = base[off(e)];
    }
    if (MUL) {  // the last forward pass (lglo = 0): the spectrum at each point
#pragma unroll
        for (int u = 0; u < kPassPer; ++u) {
            const int e = threadIdx.x + u * kPassThreads;
            if (e < n) sv[u] = spec[line * ls + off(e)];
        }
    }
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) {
        const int e = threadIdx.x + u * kPassThreads;
        if (e < n) z[lds_at<kPassPad>(e)] = r[u];
    }
    __syncthreads();
    // lgG > 0: 2^lgG lines of 2^k points; else the C x N lines (l0 = lo N + ln)
    // of 2^k points j at stride C N, twiddles by the global index
    // (j << lglo) + lo_chunk C + lo
    const LdsLines L = lgG > 0 ? LdsLines{lgG, 1 << k, 1, 0, 1}
                               : LdsLines{lgCN, 1, 1, 0, 1 << lgCN, lgN};
    const int tsh = lgG > 0 ? 0 : lglo, tb = lgG > 0 ? 0 : (int)(lo_chunk * C);
    fft_lines<T, INV, kPassPad>(z, k, L, tsh, tb, tw, lgtw);
    if (MUL) {
#pragma unroll
        for (int u = 0; u < kPassPer; ++u) {
            const int e = threadIdx.x + u * kPassThreads;
            if (e < n) z[lds_at<kPassPad>(e)] = cmul(z[lds_at<kPassPad>(e)], sv[u]);
        }
        __syncthreads();
        fft_lines<T, true, kPassPad>(z, k, L, tsh, tb, tw, lgtw);
    }
#pragma unroll
    for (int u = 0; u < kPassPer; ++u) {
        const int e = threadIdx.x + u * kPassThreads;
        if (e < n) base[off(e)] = z[lds_at<kPassPad>(e)];
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

// Table rows of the cells from the inverse transforms, scaled by 2^-lgS
// (the points the inverse ran over: P for the 2-D transform, L2 for rows).
// Job blockIdx.y; the transpose of k_fill_global: every pair's points read
// by consecutive lanes, the rows written whole.
template <typename T>
__global__ void __launch_bounds__(256)
k_extract_global(int lg1, int lg2, int32_t npairs, const int32_t* __restrict__ jobs,
                 const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
                 const int32_t* __restrict__ jc_val, int32_t d, const cpx<T>* __restrict__ buf,
                 T* __restrict__ g, int lgS) {
    __shared__ cpx<T> sc[kXCells * kXStride];
    const int64_t P = (int64_t)1 << (lg1 + lg2);
    const int32_t job = blockIdx.y;
    const cpx<T>* z = buf + (int64_t)job * npairs * P;
    const T scale = (T)1 / (T)((int64_t)1 << lgS);
    const int32_t cb = jobs[2 * job], ce = jobs[2 * job + 1];
    const bool pairs = (d & 1) == 0 && ((uintptr_t)g & (2 * sizeof(T) - 1)) == 0;
    const int t = threadIdx.x;
    for (int32_t k0 = cb + blockIdx.x * kXCells; k0 < ce; k0 += gridDim.x * kXCells) {
        int64_t at, vrow, at_r, vrow_r;
        cell_point(k0 + (t & 63), ce, jc_r, jc_x, jc_val, 0, lg2, 0, at, vrow);
        cell_point(k0 + (t >> 2), ce, jc_r, jc_x, jc_val, 0, lg2, 0, at_r, vrow_r);
        for (int32_t p0 = 0; p0 < npairs; p0 += kXPairs) {
            __syncthreads();
            if (at >= 0) {
                cpx<T> y[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t pl = (t >> 6) + 4 * q;
                    if (p0 + pl < npairs) y[q] = z[(p0 + pl) * P + at];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t pl = (t >> 6) + 4 * q;
                    if (p0 + pl < npairs) sc[(t & 63) * kXStride + pl] = y[q];
                }
            }
            __syncthreads();
            if (at_r >= 0) {
                T* out = g + vrow_r * d;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t pl = 4 * (t & 3) + q, c0 = 2 * (p0 + pl);
                    if (p0 + pl >= npairs) continue;
                    const cpx<T> y = sc[(t >> 2) * kXStride + pl];
                    if (pairs) {
                        st_pair(out + c0, cpx<T>{y.x * scale, y.y * scale});
                    } else {
                        out[c0] = y.x * scale;
                        if (c0 + 1 < d) out[c0 + 1] = y.y * scale;
                    }
                }
            }
        }
    }
}

// Depth mixing of the per-depth path (algorithm "global-anchor"): with
// a[r] the backbone spectrum of depth row r of a slot (rows transformed
// along the backbone axis) and spec[s] that of kernel row s, f(s + |b|),
//     out[q][w] = sum_{r <= hmax} spec[q + r][w] a[r][w],   q <= hmax,
// the spectra of sum_r (f(q + r + |.|) * A_r), one 1-D convolution per
// depth pair summed before a single inverse transform per output row.
template <typename T>
__global__ void k_d1_mix(int lg1, int lg2, int32_t hmax, int64_t nslots,
                         const cpx<T>* __restrict__ a, const cpx<T>* __restrict__ spec,
                         cpx<T>* __restrict__ out) {
    const int64_t L2 = (int64_t)1 << lg2;
    const int64_t rows = (int64_t)hmax + 1;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nslots * rows * L2) return;
    const int64_t w = tid & (L2 - 1);
    const int64_t q = (tid >> lg2) % rows;
    const int64_t slot = (tid >> lg2) / rows;
    const cpx<T>* as = a + (slot << (lg1 + lg2)) + w;
    const cpx<T>* ks = spec + (q << lg2) + w;
    cpx<T> acc = {(T)0, (T)0};
    for (int64_t r = 0; r < rows; ++r) acc = cadd(acc, cmul(ks[r << lg2], as[r << lg2]));
    out[(slot << (lg1 + lg2)) + (q << lg2) + w] = acc;
}

template <typename T>
__global__ void k_zero(T* __restrict__ p, int64_t n) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < n) p[tid] = T{};
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < n) p[tid] = v;
}

// Channel tile [c0, c0 + w) of an [N x d] matrix into a dense [N x w] one
// (PUT = false), or back (PUT = true).
template <typename T, bool PUT>
__global__ void k_cols(const T* __restrict__ src, T* __restrict__ dst, int64_t N, int32_t d,
                       int32_t c0, int32_t w) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= N * w) return;
    const int64_t v = tid / w;
    const int32_t c = (int32_t)(tid - v * w);
    if (PUT)
        dst[v * d + c0 + c] = src[tid];
    else
        dst[tid] = src[v * d + c0 + c];
}

}  // namespace tfi

namespace tfi {

// =================================================== kernel-table gradient ==
// For L = sum(gout * out), dL/df[k] = sum over pairs (v, w) at distance k
// of <gout[v], F[w]>. Through the decomposition, each table job adds
// sign * sum_{i, j} [r_i + r_j + |x_i - x_j| = k] <gbar_i, val_j>, where
// gbar and val are the same cell sums applied to gout and F (call jobs
// sign +1 on A-cell rows < NA, corrections sign -1 on b-cell rows), and
// every leaf tile adds its own dense pair histogram.
//
// The histograms accumulate in fixed point, so that no sum depends on the
// order of its additions and df is bitwise reproducible: a contribution v
// splits into hi = floor(v 2^14) and lo = round(frac(v 2^14) 2^33), two
// 64-bit integers summed with integer atomics (in LDS bins per workgroup,
// normalised and added to the global accumulator), and df = hi 2^-14 +
// lo 2^-47 at the end (k_df_finish). Resolution 2^-47 (7e-15) per
// contribution; |df| below 2^49 (5.6e14).
constexpr int kDfTile = 64, kDfThreads = 256;
constexpr int kDfHiExp = 14, kDfLoBits = 33;
using u64 = unsigned long long;
// LDS histogram bins of 16 bytes: 16 KiB, 64 KiB for the matrix-core kernel
constexpr int kDfBins = 1024, kDfBinsMfma = 4096;

__device__ __forceinline__ void df_atomic(u64* acc, int32_t k, double v) {
    const double s = v * (double)(1 << kDfHiExp);  // exact
    const double fl = floor(s);
    const u64 hi = (u64)(long long)fl;
    const u64 lo = (u64)__double2ll_rn((s - fl) * (double)(1ull << kDfLoBits));
    if (hi) atomicAdd(acc + 2 * k, hi);
    if (lo) atomicAdd(acc + 2 * k + 1, lo);
}

// Histogram bin add: LDS bins when the block's bins fit, else the global
// accumulator.
template <typename T>
__device__ __forceinline__ void hist_add(u64* lh, u64* gh, int32_t k, T v) {
    df_atomic(lh ? lh : gh, k, (double)v);
}

__device__ __forceinline__ void hist_clear(u64* lh, int32_t K) {
    for (int32_t k = threadIdx.x; k < 2 * K; k += blockDim.x) lh[k] = 0;
}

// LDS bins into the global accumulator, each normalised (lo < 2^33) first.
__device__ __forceinline__ void hist_flush(const u64* lh, u64* gh, int32_t K) {
    __syncthreads();
    for (int32_t k = threadIdx.x; k < K; k += blockDim.x) {
        u64 hi = lh[2 * k], lo = lh[2 * k + 1];
        hi += lo >> kDfLoBits;
        lo &= (1ull << kDfLoBits) - 1;
        if (hi) atomicAdd(gh + 2 * k, hi);
        if (lo) atomicAdd(gh + 2 * k + 1, lo);
    }
}

// df[k] (or df[k] + the new value when accumulate) from the accumulator.
__global__ void k_df_finish(const u64* __restrict__ acc, int64_t K, double* __restrict__ df,
                            int accumulate) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    u64 hi = acc[2 * k], lo = acc[2 * k + 1];
    hi += lo >> kDfLoBits;
    lo &= (1ull << kDfLoBits) - 1;
    const double v = (double)(long long)hi * (1.0 / (double)(1 << kDfHiExp)) +
                     (double)lo * (1.0 / (double)(1ull << (kDfHiExp + kDfLoBits)));
    df[k] = accumulate ? df[k] + v : v;
}

// Direct jobs: same blocks as k_direct, output cells taken 64 at a time.
// Pair dot products are formed over channel chunks in registers (16 pairs
// per thread), then binned by surrogate distance.
template <typename T>
__global__ void __launch_bounds__(kDfThreads)
k_df_direct(int32_t d, int64_t NA, const int32_t* __restrict__ blk,
            const int32_t* __restrict__ dl_r, const int32_t* __restrict__ dl_x,
            const int32_t* __restrict__ dl_row, const int32_t* __restrict__ qjb,
            const int32_t* __restrict__ qje, const T* __restrict__ val,
            const T* __restrict__ valg, const int32_t* __restrict__ dbin,
            u64* __restrict__ df) {
    __shared__ T sG[kDfTile * (kDirCh + 1)], sV[kDfTile * (kDirCh + 1)];
    __shared__ int32_t sr[kDfTile], sx[kDfTile];
    __shared__ u64 lh[2 * kDfBins];
    const int32_t Kb = dbin[blockIdx.x];  // bins this block can reach
    const bool use_lds = Kb <= kDfBins;
    u64* lhp = use_lds ? lh : nullptr;
    if (use_lds) hist_clear(lh, Kb);
    const int32_t os = blk[4 * blockIdx.x], oe = blk[4 * blockIdx.x + 1];
    const int32_t ii = threadIdx.x & (kDfTile - 1), jj0 = threadIdx.x >> 6;
    for (int32_t oc = os; oc < oe; oc += kDfTile) {
        const int32_t on = min(kDfTile, oe - oc);
        const int32_t i = oc + ii;
        const bool iok = ii < on && dl_row[i] >= 0;
        const int32_t ri = iok ? dl_r[i] : 0, xi = iok ? dl_x[i] : 0;
        const int32_t jb = iok ? qjb[i >> 2] : 0, je = iok ? qje[i >> 2] : 0;
        const T sign = (iok && dl_row[i] < NA) ? (T)1 : (T)-1;
        // sources: the union of the job ranges of this chunk's cells
        const int32_t ss = qjb[oc >> 2], se = qje[(oc + on - 1) >> 2];
        for (int32_t ts = ss; ts < se; ts += kDfTile) {
            const int32_t tn = min(kDfTile, se - ts);
            T m[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) m[q] = 0;
            for (int32_t c0 = 0; c0 < d; c0 += kDirCh) {
                const int32_t nch = min(kDirCh, d - c0);
                __syncthreads();
                {
                    // both tiles' rows: all row indices first, then all values
                    constexpr int kPer = kDfTile / (kDfThreads / 16);
                    const int32_t cc = threadIdx.x & 15, k0 = threadIdx.x >> 4;
                    const int32_t ccs = min(cc, nch - 1);
                    int32_t ro[kPer], rs[kPer];
#pragma unroll
                    for (int i = 0; i < kPer; ++i) {
                        const int32_t k = k0 + 16 * i;
                        ro[i] = dl_row[oc + min(k, on - 1)];
                        rs[i] = dl_row[ts + min(k, tn - 1)];
                    }
                    T vg[kPer], vv[kPer];
#pragma unroll
                    for (int i = 0; i < kPer; ++i) {
                        vg[i] = valg[(int64_t)max(ro[i], 0) * d + c0 + ccs];
                        vv[i] = val[(int64_t)max(rs[i], 0) * d + c0 + ccs];
                    }
#pragma unroll
                    for (int i = 0; i < kPer; ++i) {
                        const int32_t k = k0 + 16 * i;
                        if (cc < nch) {
                            sG[k * (kDirCh + 1) + cc] = (k < on && ro[i] >= 0) ? vg[i] : (T)0;
                            sV[k * (kDirCh + 1) + cc] = (k < tn && rs[i] >= 0) ? vv[i] : (T)0;
                        }
                    }
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
                    for (int q = 0; q < 16; ++q)
                        m[q] += gv * sV[(jj0 + 4 * q) * (kDirCh + 1) + cc];
                }
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int32_t j = ts + jj0 + 4 * q;
                if (iok && j >= jb && j < je && jj0 + 4 * q < tn && m[q] != (T)0) {
                    const int32_t dx = xi - sx[jj0 + 4 * q];
                    hist_add<T>(lhp, df, ri + sr[jj0 + 4 * q] + (dx < 0 ? -dx : dx), sign * m[q]);
                }
            }
        }
    }
    if (use_lds) hist_flush(lh, df, Kb);
}

// Direct jobs on the matrix cores (FP32). The pair terms <gbar_i, val_j>
// of a job are its Gram matrix Gbar V^T, formed in 16 x 16 blocks with
// v_mfma_f32_16x16x4f32 and binned by surrogate distance. The sum runs over
// all channels, so any fixed assignment of channels to the four k-slots of
// an MFMA step works when both operands use the same one: in a chunk of
// 4 * CPL channels, lane (lr, lk) supplies channels c0 + lk * CPL + s at
// step s, for gbar of row lr of the row tile (A[lr][lk]) and val of source
// lr of the source tile (B[lk][lr]), so both come as contiguous runs of a
// row. Result register r of lane (lr, lk) is the pair (row 4 lk + r,
// source lr). A wave owns a contiguous run of up to 4 row tiles of the
// block's output cells (neighbouring jobs, so a short source range), keeps their gbar runs in registers, and streams
// source tiles of 16 cells straight from memory (sources of a job are
// consecutive value rows). Blocks, padding and job ranges are those of
// k_direct. dbin[b] bounds the distance bins of block b's pairs (one past
// the largest 2 r + x extent of its jobs): the LDS histogram is cleared and
// flushed over that range only, and a block whose bins do not fit in LDS
// adds straight to df.
template <int CPL>
__device__ __forceinline__ void load_run(const float* __restrict__ base, int32_t row, int32_t d,
                                         int32_t ch0, float (&v)[CPL]) {
    if (row < 0) {
#pragma unroll
        for (int s = 0; s < CPL; ++s) v[s] = 0.f;
        return;
    }
    const float* p = base + (int64_t)row * d + ch0;
    if ((CPL & 3) == 0 && (d & 3) == 0 && ch0 + CPL <= d) {
#pragma unroll
        for (int s = 0; s < CPL; s += 4) {
            const float4 q = *reinterpret_cast<const float4*>(p + s);
            v[s] = q.x;
            v[s + 1] = q.y;
            v[s + 2] = q.z;
            v[s + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int s = 0; s < CPL; ++s) v[s] = (ch0 + s < d) ? p[s] : 0.f;
    }
}

template <int CPL>
__global__ void __launch_bounds__(kDirThreads)
k_df_direct_mfma(int32_t d, int64_t NA, const int32_t* __restrict__ blk,
                 const int32_t* __restrict__ dl_r, const int32_t* __restrict__ dl_x,
                 const int32_t* __restrict__ dl_row, const int32_t* __restrict__ qjb,
                 const int32_t* __restrict__ qje, const float* __restrict__ val,
                 const float* __restrict__ valg, const int32_t* __restrict__ dbin,
                 u64* __restrict__ df) {
    __shared__ u64 lh[2 * kDfBinsMfma];
    const int32_t Kb = dbin[blockIdx.x];  // bins this block can reach
    const bool use_lds = Kb <= kDfBinsMfma;
    u64* lhp = use_lds ? lh : nullptr;
    if (use_lds) hist_clear(lh, Kb);
    __syncthreads();
    const int32_t os = blk[4 * blockIdx.x], oe = blk[4 * blockIdx.x + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int32_t ntiles = (oe - os + 15) >> 4;
    // per row tile: the A-side row (lr), the result-side rows 4 lk + r with
    // their coordinates and signs (0 for padding), the quad's job range and
    // the tile's source range
    int32_t arow[4], rr[4][4], rx[4][4], qb[4], qe[4], tjb[4], tje[4];
    float coef[4][4];
    const int32_t tpw = (ntiles + 3) >> 2;  // a contiguous run of row tiles per wave
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t t = q < tpw ? wave * tpw + q : ntiles;
        const int32_t tb = os + 16 * t;
        const bool tok = t < ntiles;
        arow[q] = (tok && tb + lr < oe) ? dl_row[tb + lr] : -1;
        const int32_t Q = (tb >> 2) + lk;
        const bool qok = tok && 4 * Q < oe;
        qb[q] = qok ? qjb[Q] : 0;
        qe[q] = qok ? qje[Q] : 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int32_t i = 4 * Q + r;
            const int32_t row = qok ? dl_row[i] : -1;
            rr[q][r] = qok ? dl_r[i] : 0;
            rx[q][r] = qok ? dl_x[i] : 0;
            coef[q][r] = row < 0 ? 0.f : (row < NA ? 1.f : -1.f);
        }
        if (tok) {
            tjb[q] = qjb[tb >> 2];
            tje[q] = qje[(min(oe, tb + 16) - 1) >> 2];
        } else {
            tjb[q] = tje[q] = 0;
        }
    }
    int32_t lo = 1 << 30, hi = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (tjb[q] < tje[q]) {
            lo = min(lo, tjb[q]);
            hi = max(hi, tje[q]);
        }
    for (int32_t c0 = 0; c0 < d; c0 += 4 * CPL) {
        const int32_t ch0 = c0 + lk * CPL;
        float gq[4][CPL];
#pragma unroll
        for (int q = 0; q < 4; ++q) load_run<CPL>(valg, arow[q], d, ch0, gq[q]);
        for (int32_t k16 = lo; k16 < hi; k16 += 16) {
            const int32_t j = k16 + lr;
            const bool jok = j < hi;
            const int32_t jrow = jok ? dl_row[j] : -1;
            const int32_t rj = jok ? dl_r[j] : 0, xj = jok ? dl_x[j] : 0;
            float vs[CPL];
            load_run<CPL>(val, jrow, d, ch0, vs);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (k16 + 16 <= tjb[q] || k16 >= tje[q]) continue;  // uniform per wave
                v4f_t acc = (v4f_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < CPL; ++s)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(gq[q][s], vs[s], acc, 0, 0, 0);
                if (jrow < 0 || j < qb[q] || j >= qe[q]) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (coef[q][r] == 0.f || acc[r] == 0.f) continue;
                    const int32_t dx = rx[q][r] - xj;
                    hist_add<float>(lhp, df, rr[q][r] + rj + (dx < 0 ? -dx : dx),
                                    coef[q][r] * acc[r]);
                }
            }
        }
    }
    if (use_lds) hist_flush(lh, df, Kb);
}

// Leaf tiles: pairs inside each tile, distance from D. The group's gout
// and F rows are staged in LDS kDirCh channels at a time; a thread owns up
// to kDfLeafRows (quad, source j) rows = 4 pair dot products each. lbin[g]
// is one past the largest distance inside group g's tiles: the LDS
// histogram is cleared and flushed over that range only.
constexpr int kDfLeafRows = 8;

template <typename T>
__global__ void __launch_bounds__(kLeafThreads)
k_df_leaf(int32_t d, const int32_t* __restrict__ grp, const int64_t* __restrict__ gk,
          const int32_t* __restrict__ lq, const int32_t* __restrict__ leaf_v,
          const int32_t* __restrict__ leaf_D, const T* __restrict__ F,
          const T* __restrict__ gout, const int32_t* __restrict__ lbin,
          u64* __restrict__ df) {
    // rows of kDirCh channels at a 16-byte aligned stride, read 4 channels
    // at a time
    constexpr int kStride = kDirCh + 4;
    __shared__ __attribute__((aligned(16))) T sG[kLeafSlots * kStride];
    __shared__ __attribute__((aligned(16))) T sF[kLeafSlots * kStride];
    __shared__ int32_t svtx[kLeafSlots], srow0[kLeafQuads + 1];
    __shared__ u64 lh[2 * kDfBins];
    const int32_t K = lbin[blockIdx.x];  // bins this group's pairs can reach
    const bool use_lds = K <= kDfBins;
    u64* lhp = use_lds ? lh : nullptr;
    if (use_lds) hist_clear(lh, K);
    const int32_t q0 = grp[blockIdx.x], q1 = grp[blockIdx.x + 1], nq_ = q1 - q0;
    const int64_t kb = gk[2 * blockIdx.x];
    const int32_t vb = lq[4 * q0 + 1];
    const int32_t nv = lq[4 * (q1 - 1) + 1] + lq[4 * (q1 - 1) + 2] - vb;
    for (int32_t i = threadIdx.x; i < nv; i += blockDim.x) svtx[i] = leaf_v[vb + i];
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int32_t q = 0; q < nq_; ++q) {
            srow0[q] = acc;
            acc += lq[4 * (q0 + q) + 2];
        }
        srow0[nq_] = acc;
    }
    __syncthreads();
    const int32_t rows_total = srow0[nq_];
    int32_t rq[kDfLeafRows], rj[kDfLeafRows];
#pragma unroll
    for (int r = 0; r < kDfLeafRows; ++r) {
        const int32_t row = threadIdx.x + r * blockDim.x;
        rq[r] = -1;
        rj[r] = 0;
        if (row < rows_total) {
            int32_t q = 0;
            while (srow0[q + 1] <= row) ++q;
            rq[r] = q;
            rj[r] = row - srow0[q];
        }
    }
    T m[kDfLeafRows][4];
#pragma unroll
    for (int r = 0; r < kDfLeafRows; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) m[r][c] = 0;
    // gout and field rows of the group's vertices, a chunk of kDirCh channels
    // at a time with all loads in flight at once; the next chunk's rows are
    // requested before the current chunk's products
    constexpr int kPer = kLeafSlots / (kLeafThreads / 16);
    const int32_t lc = threadIdx.x & 15, k0 = threadIdx.x >> 4;
    T vg[kPer], vf[kPer];
    auto load_rows = [&](int32_t c) {
        const int32_t ccs = min(lc, min(kDirCh, d - c) - 1);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int64_t o = (int64_t)svtx[min(k0 + 16 * i, nv - 1)] * d + c + ccs;
            vg[i] = gout[o];
            vf[i] = F[o];
        }
    };
    load_rows(0);
    for (int32_t c0 = 0; c0 < d; c0 += kDirCh) {
        const int32_t nch = min(kDirCh, d - c0);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int32_t k = k0 + 16 * i;
            if (k < nv) {  // channels past the chunk's end are zero
                sG[k * kStride + lc] = lc < nch ? vg[i] : (T)0;
                sF[k * kStride + lc] = lc < nch ? vf[i] : (T)0;
            }
        }
        __syncthreads();
        if (c0 + kDirCh < d) load_rows(c0 + kDirCh);
#pragma unroll
        for (int r = 0; r < kDfLeafRows; ++r) {
            if (rq[r] < 0) continue;
            const int32_t q = q0 + rq[r];
            const int32_t first = lq[4 * q], tb = lq[4 * q + 1], n = lq[4 * q + 2];
            const int32_t rows = min(4, tb + n - first);
            const T* fj = sF + (tb - vb + rj[r]) * kStride;
            for (int32_t cc = 0; cc < nch; cc += 4) {
                const vec4<T> fv = ld4(fj + cc);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c >= rows) continue;
                    const vec4<T> gv = ld4(sG + (first - vb + c) * kStride + cc);
                    // the channels in order, as one product each
                    m[r][c] += gv.x * fv.x;
                    m[r][c] += gv.y * fv.y;
                    m[r][c] += gv.z * fv.z;
                    m[r][c] += gv.w * fv.w;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kDfLeafRows; ++r) {
        if (rq[r] < 0) continue;
        const int32_t q = q0 + rq[r];
        const int32_t first = lq[4 * q], tb = lq[4 * q + 1], n = lq[4 * q + 2];
        const int32_t krow = lq[4 * q + 3];
        const int32_t rows = min(4, tb + n - first);
        for (int c = 0; c < rows; ++c)
            if (m[r][c] != (T)0) hist_add<T>(lhp, df, leaf_D[kb + krow + c * n + rj[r]], m[r][c]);
    }
    if (use_lds) hist_flush(lh, df, K);
}

// FFT jobs, pass 1: one workgroup per (job, group of ppg channel pairs)
// forms, per pair, the forward transforms of the gout table (at output
// positions) and of the field table (at source positions), and sums
// Zg * conj(Zv) over the group's pairs into a partial spectrum written to
// global memory (slot = job * groups + group). ppg is kDfPairs, or more
// when the bucket has jobs enough to fill the device with fewer groups
// (fewer partial spectra to write and sum).
constexpr int kDfPairs = 4;

// PAD: the transformed tables are one block stored with lds_at<PAD> (for
// pair b of a batch of 2^lgnb, zv point p at 2 b P + p, zg point p at
// (2 b + 1) P + p); the accumulator follows it. The
// cells' loads go out kDfBatch at a time (two tables per cell: a smaller
// batch than the forward kernel's keeps the registers of small tables'
// workgroups within occupancy).
constexpr int kDfBatch = 4;

//
// FOLD: the workgroup also applies the inverse transform to its own group
// sum and folds it into df as k_df_fft_fold does (the transform is linear
// and the fixed-point bins add in any order, so the per-group folds sum to
// the same df up to the rounding of each group's transform), with no
// partial spectrum in global memory. The bins (2 H + X + 1 of 16 bytes)
// reuse the LDS from the second table on, which holds at least 2 P complex
// values; the host checks that they fit.
template <typename T, int PAD = 0, bool FOLD = false>
__global__ void k_df_fft_partial(int lg1, int lg2, const int32_t* __restrict__ jobs,
                                 const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
                                 const int32_t* __restrict__ jc_val, int32_t d,
                                 const T* __restrict__ val, const T* __restrict__ valg,
                                 const cpx<T>* __restrict__ tw, int lgtw,
                                 cpx<T>* __restrict__ part, int32_t ppg, int lgnb,
                                 const int32_t* __restrict__ job_hx = nullptr, int64_t NA = 0,
                                 u64* __restrict__ df = nullptr) {
    extern __shared__ unsigned char smem_raw[];
    // (job, group) of this workgroup. Workgroups are dealt to the 8 XCDs in
    // turn; when their count allows, the groups of one job, which read the
    // same cell rows (2 ppg channels of each), take consecutive slots of one
    // XCD, so they run together and the rows come from that XCD's L2.
    int32_t job = blockIdx.x, grp = blockIdx.y;
    {
        const int64_t W = (int64_t)gridDim.x * gridDim.y;
        if (gridDim.y > 1 && (W & 7) == 0) {
            const int64_t w = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
            const int64_t lw = (w & 7) * (W >> 3) + (w >> 3);
            job = (int32_t)(lw / gridDim.y);
            grp = (int32_t)(lw % gridDim.y);
        }
    }
    const int32_t cb = jobs[2 * job], ce = jobs[2 * job + 1];
    const int L1 = 1 << lg1, L2 = 1 << lg2, P = L1 * L2, lgP = lg1 + lg2;
    const int nb = blockDim.x;
    // the tables of NB = 2^lgnb pairs at a time: pair b's field table at
    // 2 b P, its gout table at (2 b + 1) P
    const int NB = 1 << lgnb;
    cpx<T>* zv = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* acc = zv + (2 * P << lgnb) + (PAD ? (2 * P << lgnb) >> PAD : 0);
    const int32_t npairs = (d + 1) / 2;
    for (int p = threadIdx.x; p < P; p += nb) acc[p] = {(T)0, (T)0};
    const int32_t pe = min(npairs, (grp + 1) * ppg);
    const int32_t ncell = ce - cb;
    for (int32_t pb = grp * ppg; pb < pe; pb += NB) {
        const int32_t nbp = min(NB, pe - pb);
        for (int p = threadIdx.x; p < (2 * P << lgnb); p += nb) zv[lds_at<PAD>(p)] = {(T)0, (T)0};
        __syncthreads();
        // item it: cell cb + (it >> lgnb), pair pb + (it mod NB) (the pairs
        // of one cell row on neighbouring lanes)
        const int32_t items = ncell << lgnb;
        for (int32_t i0 = threadIdx.x; i0 < items; i0 += kDfBatch * nb) {
            int av[kDfBatch], ag[kDfBatch];
            int64_t vr[kDfBatch];
            bool h1[kDfBatch];
#pragma unroll
            for (int u = 0; u < kDfBatch; ++u) {
                const int32_t it = i0 + u * nb;
                const int b = it & (NB - 1);
                av[u] = -1;
                if (it < items && b < nbp) {
                    const int32_t k = cb + (it >> lgnb);
                    const int32_t c0 = 2 * (pb + b);
                    vr[u] = (int64_t)jc_val[k] * d + c0;
                    h1[u] = c0 + 1 < d;
                    const int r = jc_r[k], x = jc_x[k];
                    av[u] = (2 * b << lgP) + ((((L1 - r) & (L1 - 1)) << lg2) + x);
                    ag[u] = ((2 * b + 1) << lgP) + (r << lg2) + x;
                }
            }
            cpx<T> v[kDfBatch], w[kDfBatch];
#pragma unroll
            for (int u = 0; u < kDfBatch; ++u) {
                if (av[u] < 0) continue;
                v[u] = {val[vr[u]], h1[u] ? val[vr[u] + 1] : (T)0};
                w[u] = {valg[vr[u]], h1[u] ? valg[vr[u] + 1] : (T)0};
            }
#pragma unroll
            for (int u = 0; u < kDfBatch; ++u) {
                if (av[u] < 0) continue;
                zv[lds_at<PAD>(av[u])] = v[u];
                zv[lds_at<PAD>(ag[u])] = w[u];
            }
        }
        __syncthreads();
        // every table of the batch: their rows, then their columns
        fft_lines<T, false, PAD>(zv, lg2, LdsLines{lg1 + 1 + lgnb, L2, 1, 0, 1}, 0, 0, tw, lgtw);
        fft_lines<T, false, PAD>(zv, lg1, LdsLines{lg2, 1, 2 * NB, P, L2}, 0, 0, tw, lgtw);
        // pairs summed in pair order
        for (int p = threadIdx.x; p < P; p += nb) {
            cpx<T> a = acc[p];
            for (int b = 0; b < nbp; ++b)
                a = cadd(a, cmulc(zv[lds_at<PAD>(((2 * b + 1) << lgP) + p)],
                                  zv[lds_at<PAD>((2 * b << lgP) + p)]));
            acc[p] = a;
        }
        __syncthreads();
    }
    if (!FOLD) {
        cpx<T>* out = part + ((int64_t)job * gridDim.y + grp) * P;
        for (int p = threadIdx.x; p < P; p += nb) out[p] = acc[p];
        return;
    }
    for (int p = threadIdx.x; p < P; p += nb) zv[lds_at<PAD>(p)] = acc[p];
    __syncthreads();
    fft_axis_lds<T, true, PAD>(zv, lg1, L2, L2, 1, tw, lgtw);
    fft_axis_lds<T, true, PAD>(zv, lg2, L1, 1, L2, tw, lgtw);
    const int32_t H = job_hx[2 * job], X = job_hx[2 * job + 1];
    const int32_t nk = 2 * H + X + 1;
    u64* lh = reinterpret_cast<u64*>(zv + lds_at<PAD>(P));
    hist_clear(lh, nk);
    __syncthreads();
    const T scale = (jc_val[cb] < NA ? (T)1 : (T)-1) / (T)P;
    for (int p = threadIdx.x; p < P; p += nb) {
        const int a = p >> lg2, b = p & (L2 - 1);
        const int bs = (b <= (L2 >> 1)) ? b : L2 - b;
        if (a <= 2 * H && bs <= X) df_atomic(lh, a + bs, (double)(zv[lds_at<PAD>(p)].x * scale));
    }
    hist_flush(lh, df, nk);
}

// FFT jobs, pass 2: one workgroup per job sums the group spectra (fixed
// order), applies one inverse transform and folds Re Z[a][b] (a = q + r,
// b = s - x mod L2) into df[a + |b|], binned in LDS in fixed point.
template <typename T, int PAD = 0>
__global__ void k_df_fft_fold(int lg1, int lg2, const int32_t* __restrict__ jobs,
                              const int32_t* __restrict__ job_hx, int32_t groups, int64_t NA,
                              const int32_t* __restrict__ jc_val, const cpx<T>* __restrict__ part,
                              const cpx<T>* __restrict__ tw, int lgtw, u64* __restrict__ df) {
    extern __shared__ unsigned char smem_raw[];
    const int32_t cb = jobs[2 * blockIdx.x];
    const int L1 = 1 << lg1, L2 = 1 << lg2, P = L1 * L2;
    const int nb = blockDim.x;
    const int32_t H = job_hx[2 * blockIdx.x], X = job_hx[2 * blockIdx.x + 1];
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_raw);
    u64* lh = reinterpret_cast<u64*>(z + P + (PAD ? P >> PAD : 0));
    const int32_t nk = 2 * H + X + 1;  // bins this job can reach
    hist_clear(lh, nk);
    const cpx<T>* src = part + (int64_t)blockIdx.x * groups * P;
    // group spectra summed in group order; the loads of kConvBatch points
    // are issued together
    for (int p0 = threadIdx.x; p0 < P; p0 += kConvBatch * nb) {
        cpx<T> acc[kConvBatch];
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u) acc[u] = {(T)0, (T)0};
        for (int32_t gq = 0; gq < groups; ++gq) {
            cpx<T> v[kConvBatch];
#pragma unroll
            for (int u = 0; u < kConvBatch; ++u)
                if (p0 + u * nb < P) v[u] = src[(int64_t)gq * P + p0 + u * nb];
#pragma unroll
            for (int u = 0; u < kConvBatch; ++u)
                if (p0 + u * nb < P) acc[u] = cadd(acc[u], v[u]);
        }
#pragma unroll
        for (int u = 0; u < kConvBatch; ++u)
            if (p0 + u * nb < P) z[lds_at<PAD>(p0 + u * nb)] = acc[u];
    }
    __syncthreads();
    fft_axis_lds<T, true, PAD>(z, lg1, L2, L2, 1, tw, lgtw);
    fft_axis_lds<T, true, PAD>(z, lg2, L1, 1, L2, tw, lgtw);
    const T scale = (jc_val[cb] < NA ? (T)1 : (T)-1) / (T)P;
    for (int p = threadIdx.x; p < P; p += nb) {
        const int a = p >> lg2, b = p & (L2 - 1);
        const int bs = (b <= (L2 >> 1)) ? b : L2 - b;
        if (a <= 2 * H && bs <= X) df_atomic(lh, a + bs, (double)(z[lds_at<PAD>(p)].x * scale));
    }
    hist_flush(lh, df, nk);
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
    const int32_t job = blockIdx.y;
    const int64_t L1 = (int64_t)1 << lg1;
    cpx<T>* zv = bv + (int64_t)job * npairs * P;
    cpx<T>* zg = bg + (int64_t)job * npairs * P;
    const int32_t cb = jobs[2 * job], ce = jobs[2 * job + 1];
    for (int32_t k = cb + blockIdx.x * blockDim.x + threadIdx.x; k < ce;
         k += gridDim.x * blockDim.x) {
        const int64_t vr = (int64_t)jc_val[k] * d;
        const int64_t av = (((L1 - jc_r[k]) & (L1 - 1)) << lg2) + jc_x[k];
        const int64_t ag = ((int64_t)jc_r[k] << lg2) + jc_x[k];
        for (int32_t pair = 0; pair < npairs; ++pair) {
            const int32_t c0 = 2 * pair;
            const bool two = c0 + 1 < d;
            zv[pair * P + av] = {val[vr + c0], two ? val[vr + c0 + 1] : (T)0};
            zg[pair * P + ag] = {valg[vr + c0], two ? valg[vr + c0 + 1] : (T)0};
        }
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
                              u64* __restrict__ df) {
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
        if (v != 0.0) df_atomic(df, (int32_t)(a + bs), v);
    }
}

}  // namespace tfi
