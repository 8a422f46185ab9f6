// kernels_expsum.hpp -- table jobs for kernels given as sums of exponentials,
//     f(k) = sum_l c_l lam_l^k,   lam_l > 0,
// evaluated by backbone sweeps instead of direct sums or FFT (appendix
// "Specialized Kernels", lemma "stad-specialized-cross").
//
// For one term and a table job whose cells (r, x) carry values v:
//   a[t]  = sum over the cells at backbone position x_t of lam^r v
//   Y[x]  = sum_t lam^|x - x_t| a[t]            (forward + backward sweep)
//   table value at (r, x) = lam^r Y[x]
// (G_q[s] = lam^q G_0[s] and E[q] = lam^q E[0]: a correction job is a table
// with one position). Backbone positions are lattice coordinates, so a step
// between positions that are D apart multiplies by lam^D.
//
// Gradient moments of L = sum(gout * out), over all vertex pairs (v, w):
//   s0_l = sum lam_l^dist <gout_v, F_w>,   s1_l = sum dist lam_l^dist <gout_v, F_w>,
// so dL/dc_l = s0_l and dL/dlam_l = c_l s1_l / lam_l. Per job (with its
// sign), s0 = sum_cells <gbar, lam^r Y> and s1 = sum_cells <gbar, lam^r
// (r Y + Y^r + Z)>, where Y^r sweeps the profile of r lam^r v and
// Z[x] = sum_t |x - x_t| lam^|x - x_t| a[t] is the derivative sweep:
//   forward   M[p] = lam^D (M[p-1] + D L[p-1]),
//   backward  N[p] = lam^D (N[p+1] + D (a[p+1] + R[p+1])).
#pragma once

#include "kernels.hpp"

namespace tfi {

constexpr int kExpMaxTerms = 16;
constexpr int kExpThreads = 256;

// pw[l * K + k] = lam_l^k and ftab[k] = sum_l c_l lam_l^k for k < K; the
// powers are exp(k log lam_l) in double precision.
template <typename T>
__global__ void k_expsum_prep(int32_t nterm, const T* __restrict__ c, const T* __restrict__ lam,
                              int32_t K, T* __restrict__ pw, T* __restrict__ ftab) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double f = 0.0;
    for (int l = 0; l < nterm; ++l) {
        const double p = exp((double)k * log((double)lam[l]));
        pw[(int64_t)l * K + k] = (T)p;
        f += (double)c[l] * p;
    }
    ftab[k] = (T)f;
}

// Sum of a double over the workgroup (kExpThreads threads); every thread
// must call it. Returns the total in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kExpThreads / 64; ++w) t += red[w];
    return t;
}

// Jobs with several backbone positions (diameter backbones): one group of
// gs lanes (gs divides 64) per job, taken in the order ej (jobs sorted by
// size); lane c of a group handles channels c, c + gs, ... and sweeps the
// job's cells (sorted by backbone position) forward, then backward.
// jpos[job] is the job's first slot in `scratch`, which holds per position
// NQ quantities x nterm terms x d channels (forward: L, a; gradient: L, a,
// L^r, a^r, M).
// GRAD = false: writes the table value of every cell to g[row].
// GRAD = true: writes the workgroup's signed moments (sum over its jobs) to
// row mbase + blockIdx.x of mrow ([row][s0 | s1][nterm], FP64); valg holds
// the gout cell sums.
template <typename T, int NJ, bool GRAD>
__global__ void __launch_bounds__(kExpThreads)
k_expsum_jobs(int32_t nterm, int32_t d, int32_t gs, int32_t njobs,
              const int32_t* __restrict__ ej, const int64_t* __restrict__ joff,
              const int64_t* __restrict__ jpos, const int32_t* __restrict__ jsign,
              const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
              const int32_t* __restrict__ jc_val, const T* __restrict__ c,
              const T* __restrict__ pw, int32_t K, const T* __restrict__ val,
              const T* __restrict__ valg, T* __restrict__ g, T* __restrict__ scratch,
              double* __restrict__ mrow, int64_t mbase) {
    constexpr int NQ = GRAD ? 5 : 2;
    const int32_t gpb = kExpThreads / gs;
    const int32_t grp = threadIdx.x / gs, lc = threadIdx.x - grp * gs;
    const int32_t jn = blockIdx.x * gpb + grp;
    const bool active = jn < njobs;
    double m0[NJ], m1[NJ];  // gradient moments of this lane
#pragma unroll
    for (int l = 0; l < NJ; ++l) m0[l] = m1[l] = 0.0;
    T cl[NJ];
#pragma unroll
    for (int l = 0; l < NJ; ++l) cl[l] = (!GRAD && l < nterm) ? c[l] : (T)0;
    const int32_t job = active ? ej[jn] : 0;
    const int64_t cb = active ? joff[job] : 0, ce = active ? joff[job + 1] : 0;
    const T sgn = (GRAD && active && jsign[job] < 0) ? (T)-1 : (T)1;
    for (int32_t ch = lc; active && ch < d && cb < ce; ch += gs) {
        {
            const int64_t pos0 = jpos[job];
            auto slot = [&](int64_t p, int q, int l) -> T& {
                return scratch[((p * NQ + q) * nterm + l) * (int64_t)d + ch];
            };
            // ---- forward pass: profiles a (and a^r) per position, running L
            T L[NJ], A[NJ], Lr[NJ], Ar[NJ], M[NJ];
#pragma unroll
            for (int l = 0; l < NJ; ++l) L[l] = A[l] = Lr[l] = Ar[l] = M[l] = (T)0;
            int64_t p = pos0;
            int32_t xc = jc_x[cb];
            for (int64_t i = cb; i < ce; ++i) {
                const int32_t x = jc_x[i], r = jc_r[i];
                if (x != xc) {  // close the position at xc, step to x
                    const int32_t D = x - xc;
#pragma unroll
                    for (int l = 0; l < NJ; ++l) {
                        if (l >= nterm) continue;
                        L[l] += A[l];
                        slot(p, 0, l) = L[l];
                        slot(p, 1, l) = A[l];
                        if (GRAD) {
                            Lr[l] += Ar[l];
                            slot(p, 2, l) = Lr[l];
                            slot(p, 3, l) = Ar[l];
                            slot(p, 4, l) = M[l];
                        }
                        const T q = pw[(int64_t)l * K + D];
                        if (GRAD) M[l] = q * (M[l] + (T)D * L[l]);
                        L[l] *= q;
                        A[l] = (T)0;
                        if (GRAD) {
                            Lr[l] *= q;
                            Ar[l] = (T)0;
                        }
                    }
                    ++p;
                    xc = x;
                }
                const T v = val[(int64_t)jc_val[i] * d + ch];
#pragma unroll
                for (int l = 0; l < NJ; ++l) {
                    if (l >= nterm) continue;
                    const T w = pw[(int64_t)l * K + r] * v;
                    A[l] += w;
                    if (GRAD) Ar[l] += (T)r * w;
                }
            }
            // the last position: its values stay in registers
            T Lp[NJ], Ap[NJ], Lrp[NJ], Arp[NJ], Mp[NJ], R[NJ], Rr[NJ], N[NJ];
#pragma unroll
            for (int l = 0; l < NJ; ++l) {
                Lp[l] = L[l] + A[l];
                Ap[l] = A[l];
                Lrp[l] = Lr[l] + Ar[l];
                Arp[l] = Ar[l];
                Mp[l] = M[l];
                R[l] = Rr[l] = N[l] = (T)0;
            }
            // ---- backward pass: R (and R^r, N) from the right, then the cells
            for (int64_t i = ce - 1; i >= cb; --i) {
                const int32_t x = jc_x[i], r = jc_r[i];
                if (x != xc) {  // step left from the position at xc to x
                    const int32_t D = xc - x;
                    --p;
#pragma unroll
                    for (int l = 0; l < NJ; ++l) {
                        if (l >= nterm) continue;
                        const T q = pw[(int64_t)l * K + D];
                        if (GRAD) {
                            N[l] = q * (N[l] + (T)D * (Ap[l] + R[l]));
                            Rr[l] = q * (Arp[l] + Rr[l]);
                        }
                        R[l] = q * (Ap[l] + R[l]);
                        Lp[l] = slot(p, 0, l);
                        Ap[l] = slot(p, 1, l);
                        if (GRAD) {
                            Lrp[l] = slot(p, 2, l);
                            Arp[l] = slot(p, 3, l);
                            Mp[l] = slot(p, 4, l);
                        }
                    }
                    xc = x;
                }
                const int64_t o = (int64_t)jc_val[i] * d + ch;
                if (!GRAD) {
                    T sum = (T)0;
#pragma unroll
                    for (int l = 0; l < NJ; ++l)
                        if (l < nterm) sum += cl[l] * pw[(int64_t)l * K + r] * (Lp[l] + R[l]);
                    g[o] = sum;
                } else {
                    const T gv = sgn * valg[o];
#pragma unroll
                    for (int l = 0; l < NJ; ++l) {
                        if (l >= nterm) continue;
                        const T w = pw[(int64_t)l * K + r];
                        const T Y = Lp[l] + R[l];
                        m0[l] += (double)(gv * w * Y);
                        m1[l] += (double)(gv * w * ((T)r * Y + Lrp[l] + Rr[l] + Mp[l] + N[l]));
                    }
                }
            }
        }
    }
    if (GRAD) {
        __shared__ double red[kExpThreads / 64];
        double* row = mrow + (mbase + blockIdx.x) * 2 * nterm;
        for (int l = 0; l < nterm && l < NJ; ++l) {
            const double t0 = block_sum(m0[l], red);
            if (threadIdx.x == 0) row[l] = t0;
            const double t1 = block_sum(m1[l], red);
            if (threadIdx.x == 0) row[nterm + l] = t1;
        }
    }
}

// ---- single-position jobs, split into chunks of cells -------------------
// A job with one backbone position needs, per term l and channel c, the
// sums a_l = sum_i lam_l^{r_i} v_i (forward) or a_l, a^r_l (r-weighted) and
// their gout counterparts b_l, b^r_l (moments). Cells are taken in chunks
// of at most kExpChunk; chunk k covers cells ck[3k+1] .. ck[3k+2] of job
// ck[3k]. A workgroup per chunk: the chunk's weights lam_l^r go to LDS;
// thread (cell group g, lane c) sums the cells g, g + CG, ... for its
// channel; the partial sums are reduced over the cell groups (wave
// shuffles, then LDS across waves).
// cslot[k] < 0: the chunk is its whole job and the workgroup finishes it
// (forward: table values lam_l^r sum_l c_l a_l; moments: row mbase + k of
// mrow gets sign <b_l, a_l> and sign (<b^r_l, a_l> + <b_l, a^r_l>)). Else
// the sums go to partial slot cslot[k] ([NQ][nterm][d]) for
// k_expsum_jobsum (and the moment row is zero).
constexpr int kExpChunk = 256;

// Dynamic LDS bytes of k_expsum_chunks<T, NJ, *>.
template <typename T, int NJ>
constexpr int expsum_chunk_lds() {
    return (int)sizeof(T) * (NJ * kExpChunk + (kExpThreads / 64) * NJ * 64) + 8 * kExpChunk;
}

template <typename T, int NJ, bool GRAD>
__global__ void __launch_bounds__(kExpThreads)
k_expsum_chunks(int32_t nterm, int32_t d, int32_t gs, const int32_t* __restrict__ ck,
                const int32_t* __restrict__ cslot, const int32_t* __restrict__ jsign,
                const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_val,
                const T* __restrict__ c, const T* __restrict__ pw, int32_t K,
                const T* __restrict__ val, const T* __restrict__ valg, T* __restrict__ g,
                T* __restrict__ part, double* __restrict__ mrow, int64_t mbase) {
    constexpr int NQ = GRAD ? 4 : 1;
    // dynamic LDS (expsum_chunk_lds bytes): weights lam_l^r of the chunk's
    // cells [NJ][kExpChunk], the cross-wave reduction buffer [4][NJ][64],
    // cell rows and depths
    extern __shared__ unsigned char dyn_raw[];
    T* sw = reinterpret_cast<T*>(dyn_raw);
    T* red = sw + NJ * kExpChunk;
    int32_t* srow = reinterpret_cast<int32_t*>(red + (kExpThreads / 64) * NJ * 64);
    int32_t* sr = srow + kExpChunk;
    __shared__ double dred[kExpThreads / 64];
    const int32_t job = ck[3 * blockIdx.x];
    const int32_t cb = ck[3 * blockIdx.x + 1], ce = ck[3 * blockIdx.x + 2];
    const int32_t n = ce - cb;  // 1 .. kExpChunk
    const int32_t slot = cslot[blockIdx.x];
    const T sgn = (GRAD && jsign[job] < 0) ? (T)-1 : (T)1;
    if ((int32_t)threadIdx.x < n) {
        const int32_t i = cb + threadIdx.x;
        const int32_t r = jc_r[i];
        sr[threadIdx.x] = r;
        srow[threadIdx.x] = jc_val[i];
#pragma unroll
        for (int l = 0; l < NJ; ++l)
            sw[l * kExpChunk + threadIdx.x] = l < nterm ? pw[(int64_t)l * K + r] : (T)0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t lc = lane % gs, cgw = lane / gs;
    const int32_t cgpw = 64 / gs, CG = (kExpThreads / 64) * cgpw;
    const int32_t cg = wave * cgpw + cgw;
    double m0[NJ], m1[NJ];
#pragma unroll
    for (int l = 0; l < NJ; ++l) m0[l] = m1[l] = 0.0;
    for (int32_t c0 = 0; c0 < d; c0 += gs) {
        const int32_t ch = c0 + lc;
        const bool chok = ch < d;
        T acc[NQ][NJ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int l = 0; l < NJ; ++l) acc[q][l] = (T)0;
        // this thread's cells, loads four at a time
        for (int32_t k0 = cg; k0 < n; k0 += 4 * CG) {
            T v[4], gv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t k = k0 + u * CG;
                const bool ok = chok && k < n;
                const int64_t o = (int64_t)srow[min(k, n - 1)] * d + min(ch, d - 1);
                v[u] = ok ? val[o] : (T)0;
                if (GRAD) gv[u] = ok ? valg[o] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t k = min(k0 + u * CG, n - 1);
                const T rk = (T)sr[k];
#pragma unroll
                for (int l = 0; l < NJ; ++l) {
                    const T w = sw[l * kExpChunk + k];
                    acc[0][l] += w * v[u];
                    if (GRAD) {
                        acc[1][l] += rk * w * v[u];
                        acc[2][l] += w * gv[u];
                        acc[3][l] += rk * w * gv[u];
                    }
                }
            }
        }
        // reduce over the cell groups: inside the wave, then across waves
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int l = 0; l < NJ; ++l)
                for (int o = gs; o < 64; o <<= 1) acc[q][l] += __shfl_xor(acc[q][l], o, 64);
        // totals of this channel round, in every thread of the channel (one
        // quantity at a time through the reduction buffer)
        T tot[NQ][NJ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            __syncthreads();
            if (cgw == 0)
#pragma unroll
                for (int l = 0; l < NJ; ++l) red[(wave * NJ + l) * 64 + lc] = acc[q][l];
            __syncthreads();
#pragma unroll
            for (int l = 0; l < NJ; ++l) {
                T t = (T)0;
#pragma unroll
                for (int w = 0; w < kExpThreads / 64; ++w) t += red[(w * NJ + l) * 64 + lc];
                tot[q][l] = t;
            }
        }
        if (slot >= 0) {
            if (cg == 0 && chok)
#pragma unroll
                for (int q = 0; q < NQ; ++q)
#pragma unroll
                    for (int l = 0; l < NJ; ++l)
                        if (l < nterm) part[(((int64_t)slot * NQ + q) * nterm + l) * d + ch] = tot[q][l];
        } else if (!GRAD) {
            T cl[NJ];
#pragma unroll
            for (int l = 0; l < NJ; ++l) cl[l] = l < nterm ? c[l] * tot[0][l] : (T)0;
            for (int32_t k = cg; k < n && chok; k += CG) {
                T sum = (T)0;
#pragma unroll
                for (int l = 0; l < NJ; ++l) sum += cl[l] * sw[l * kExpChunk + k];
                g[(int64_t)srow[k] * d + ch] = sum;
            }
        } else if (cg == 0 && chok) {
#pragma unroll
            for (int l = 0; l < NJ; ++l) {
                m0[l] += (double)(sgn * tot[2][l] * tot[0][l]);
                m1[l] += (double)(sgn * (tot[3][l] * tot[0][l] + tot[2][l] * tot[1][l]));
            }
        }
    }
    if (GRAD) {  // every workgroup writes its row (zeros for partial chunks)
        double* row = mrow + (mbase + blockIdx.x) * 2 * nterm;
        for (int l = 0; l < nterm && l < NJ; ++l) {
            const double t0 = block_sum(m0[l], dred);
            if (threadIdx.x == 0) row[l] = t0;
            const double t1 = block_sum(m1[l], dred);
            if (threadIdx.x == 0) row[nterm + l] = t1;
        }
    }
}

// Jobs of several chunks: one workgroup per job sums its chunks' partial
// slots (jslot[2j] .. jslot[2j] + jslot[2j + 1] - 1, in order) into the
// first slot; with GRAD it then writes the job's moments (sign jsg[j]) to
// row mbase + j of mrow.
template <typename T, int NJ, bool GRAD>
__global__ void __launch_bounds__(kExpThreads)
k_expsum_jobsum(int32_t nterm, int32_t d, const int32_t* __restrict__ jslot,
                const int32_t* __restrict__ jsg, T* __restrict__ part,
                double* __restrict__ mrow, int64_t mbase) {
    constexpr int NQ = GRAD ? 4 : 1;
    __shared__ double dred[kExpThreads / 64];
    const int64_t first = jslot[2 * blockIdx.x];
    const int32_t cnt = jslot[2 * blockIdx.x + 1];
    const double sgn = jsg[blockIdx.x] < 0 ? -1.0 : 1.0;
    const int64_t per = (int64_t)NQ * nterm * d;
    for (int64_t e = threadIdx.x; e < per; e += blockDim.x) {
        T t = part[first * per + e];
        for (int32_t k = 1; k < cnt; ++k) t += part[(first + k) * per + e];
        part[first * per + e] = t;
    }
    if (!GRAD) return;
    __syncthreads();
    const T* P = part + first * per;
    for (int l = 0; l < nterm && l < NJ; ++l) {
        double a0 = 0.0, a1 = 0.0;
        for (int32_t ch = threadIdx.x; ch < d; ch += blockDim.x) {
            const double A = P[(0 * nterm + l) * d + ch], Ar = P[(1 * nterm + l) * d + ch];
            const double B = P[(2 * nterm + l) * d + ch], Br = P[(3 * nterm + l) * d + ch];
            a0 += B * A;
            a1 += Br * A + B * Ar;
        }
        const double t0 = block_sum(a0, dred);
        if (threadIdx.x == 0) mrow[(mbase + blockIdx.x) * 2 * nterm + l] = sgn * t0;
        const double t1 = block_sum(a1, dred);
        if (threadIdx.x == 0) mrow[(mbase + blockIdx.x) * 2 * nterm + nterm + l] = sgn * t1;
    }
}

// Table values of the chunks of several-chunk jobs (forward), from the
// job's summed slot: ck as in k_expsum_chunks, tslot[k] = that slot.
template <typename T, int NJ>
__global__ void __launch_bounds__(kExpThreads)
k_expsum_expand(int32_t nterm, int32_t d, const int32_t* __restrict__ ck,
                const int32_t* __restrict__ tslot, const int32_t* __restrict__ jc_r,
                const int32_t* __restrict__ jc_val, const T* __restrict__ c,
                const T* __restrict__ pw, int32_t K, const T* __restrict__ part,
                T* __restrict__ g) {
    const int32_t cb = ck[3 * blockIdx.x + 1], ce = ck[3 * blockIdx.x + 2];
    const T* P = part + (int64_t)tslot[blockIdx.x] * nterm * d;
    for (int64_t e = threadIdx.x; e < (int64_t)(ce - cb) * d; e += blockDim.x) {
        const int32_t i = cb + (int32_t)(e / d), ch = (int32_t)(e % d);
        const int32_t r = jc_r[i];
        T sum = (T)0;
        for (int l = 0; l < nterm && l < NJ; ++l)
            sum += c[l] * pw[(int64_t)l * K + r] * P[(int64_t)l * d + ch];
        g[(int64_t)jc_val[i] * d + ch] = sum;
    }
}

// Leaf-tile part of the moments from the leaf pair histogram h[k]:
// sum_k lam_l^k h[k] and sum_k k lam_l^k h[k]. One workgroup per term l,
// writing row mbase + l of mrow (its other entries zero).
template <typename T>
__global__ void __launch_bounds__(kExpThreads)
k_expsum_leaf_moments(int32_t nterm, int32_t K, const T* __restrict__ pw,
                      const double* __restrict__ h, double* __restrict__ mrow, int64_t mbase) {
    __shared__ double red[kExpThreads / 64];
    const int l = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int32_t k = threadIdx.x; k < K; k += blockDim.x) {
        const double w = (double)pw[(int64_t)l * K + k] * h[k];
        a += w;
        b += (double)k * w;
    }
    const double ta = block_sum(a, red);  // totals in thread 0
    const double tb = block_sum(b, red);
    if (threadIdx.x == 0) {
        double* row = mrow + (mbase + l) * 2 * nterm;
        for (int e = 0; e < 2 * nterm; ++e) row[e] = e == l ? ta : (e == nterm + l ? tb : 0.0);
    }
}

// s0[l] / s1[l] = column l / nterm + l of the moment rows mrow[0 .. rows),
// summed in a fixed order (one workgroup per column): reproducible bitwise.
__global__ void __launch_bounds__(kExpThreads)
k_expsum_moments(int32_t nterm, int64_t rows, const double* __restrict__ mrow,
                 double* __restrict__ s0, double* __restrict__ s1) {
    __shared__ double red[kExpThreads / 64];
    const int col = blockIdx.x;
    double a = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) a += mrow[r * 2 * nterm + col];
    const double t = block_sum(a, red);
    if (threadIdx.x == 0) {
        if (col < nterm) s0[col] = t;
        else s1[col - nterm] = t;
    }
}

}  // namespace tfi
