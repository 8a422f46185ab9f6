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

// One group of gs lanes (gs divides 64) per table job, taken in the order
// ej (jobs sorted by size); lane c of a group handles channels c, c + gs,
// ... Cells of a job are sorted by backbone position.
// MULTI = false: every job of the list has one backbone position (centroid
// backbones, corrections): a = sum lam^r v and the table value lam^r a.
// MULTI = true: jobs with several positions; jpos[job] is the job's first
// slot in `scratch`, which holds per position NQ quantities x nterm terms
// x d channels (forward: L, a; gradient: L, a, L^r, a^r, M).
// GRAD = false: writes the table value of every cell to g[row].
// GRAD = true: adds the job's signed moments to s0/s1 (FP64, one atomic
// per workgroup and term); valg holds the gout cell sums.
template <typename T, int NJ, bool GRAD, bool MULTI>
__global__ void __launch_bounds__(kExpThreads)
k_expsum_jobs(int32_t nterm, int32_t d, int32_t gs, int32_t njobs,
              const int32_t* __restrict__ ej, const int64_t* __restrict__ joff,
              const int64_t* __restrict__ jpos, const int32_t* __restrict__ jsign,
              const int32_t* __restrict__ jc_r, const int32_t* __restrict__ jc_x,
              const int32_t* __restrict__ jc_val, const T* __restrict__ c,
              const T* __restrict__ pw, int32_t K, const T* __restrict__ val,
              const T* __restrict__ valg, T* __restrict__ g, T* __restrict__ scratch,
              double* __restrict__ s0, double* __restrict__ s1) {
    constexpr int NQ = GRAD ? 5 : 2;
    constexpr int B = 4;  // cells per batch of loads (single-position jobs)
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
        if constexpr (!MULTI) {
            // a (and a^r) over the job's cells, loads in batches
            T A[NJ], Ar[NJ];
#pragma unroll
            for (int l = 0; l < NJ; ++l) A[l] = Ar[l] = (T)0;
            for (int64_t i0 = cb; i0 < ce; i0 += B) {
                int32_t rr[B];
                int64_t o[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int64_t i = min(i0 + u, ce - 1);
                    rr[u] = jc_r[i];
                    o[u] = (int64_t)jc_val[i] * d + ch;
                }
                T v[B];
#pragma unroll
                for (int u = 0; u < B; ++u) v[u] = (i0 + u < ce) ? val[o[u]] : (T)0;
#pragma unroll
                for (int u = 0; u < B; ++u)
#pragma unroll
                    for (int l = 0; l < NJ; ++l) {
                        if (l >= nterm) continue;
                        const T w = pw[(int64_t)l * K + rr[u]] * v[u];
                        A[l] += w;
                        if (GRAD) Ar[l] += (T)rr[u] * w;
                    }
            }
            // table values (or moments) at the cells
            for (int64_t i0 = cb; i0 < ce; i0 += B) {
                int32_t rr[B];
                int64_t o[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int64_t i = min(i0 + u, ce - 1);
                    rr[u] = jc_r[i];
                    o[u] = (int64_t)jc_val[i] * d + ch;
                }
                if (!GRAD) {
#pragma unroll
                    for (int u = 0; u < B; ++u) {
                        if (i0 + u >= ce) continue;
                        T sum = (T)0;
#pragma unroll
                        for (int l = 0; l < NJ; ++l)
                            if (l < nterm) sum += cl[l] * pw[(int64_t)l * K + rr[u]] * A[l];
                        g[o[u]] = sum;
                    }
                } else {
                    T gv[B];
#pragma unroll
                    for (int u = 0; u < B; ++u) gv[u] = (i0 + u < ce) ? sgn * valg[o[u]] : (T)0;
#pragma unroll
                    for (int u = 0; u < B; ++u)
#pragma unroll
                        for (int l = 0; l < NJ; ++l) {
                            if (l >= nterm) continue;
                            const T w = pw[(int64_t)l * K + rr[u]];
                            m0[l] += (double)(gv[u] * w * A[l]);
                            m1[l] += (double)(gv[u] * w * ((T)rr[u] * A[l] + Ar[l]));
                        }
                }
            }
        } else {
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
        for (int l = 0; l < nterm && l < NJ; ++l) {
            const double t0 = block_sum(m0[l], red);
            if (threadIdx.x == 0 && t0 != 0.0) atomicAdd(s0 + l, t0);
            const double t1 = block_sum(m1[l], red);
            if (threadIdx.x == 0 && t1 != 0.0) atomicAdd(s1 + l, t1);
        }
    }
}

// Leaf-tile part of the moments from the leaf pair histogram h[k]:
// s0_l += sum_k lam_l^k h[k], s1_l += sum_k k lam_l^k h[k]. One workgroup
// per term.
template <typename T>
__global__ void __launch_bounds__(kExpThreads)
k_expsum_leaf_moments(int32_t K, const T* __restrict__ pw, const double* __restrict__ h,
                      double* __restrict__ s0, double* __restrict__ s1) {
    __shared__ double red[kExpThreads / 64];
    const int l = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int32_t k = threadIdx.x; k < K; k += blockDim.x) {
        const double w = (double)pw[(int64_t)l * K + k] * h[k];
        a += w;
        b += (double)k * w;
    }
    const double ta = block_sum(a, red);
    if (threadIdx.x == 0) atomicAdd(s0 + l, ta);
    const double tb = block_sum(b, red);
    if (threadIdx.x == 0) atomicAdd(s1 + l, tb);
}

}  // namespace tfi
