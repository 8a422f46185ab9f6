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

// Value of lane src (uniform over the wavefront) in every lane, through the
// scalar registers.
template <typename T>
__device__ __forceinline__ T lane_value(T v, int src) {
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
    } else {
        const long long b = __double_as_longlong(v);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, src);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), src);
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
}
template <>
__device__ __forceinline__ int32_t lane_value<int32_t>(int32_t v, int src) {
    return __builtin_amdgcn_readlane(v, src);
}

// ---- one-position jobs, one wavefront each ------------------------------
// A job with one backbone position needs, per term l and channel c, the
// sums a_l = sum_i lam_l^{r_i} v_i (forward) or a_l, a^r_l (r-weighted) and
// their gout counterparts b_l, b^r_l (moments). One wavefront per job (jobs
// in the order ej, by size): lane (s, c) = (lane / gs, lane % gs), with gs
// the smallest power of two >= d (at most 64), handles channels c, c + gs,
// ... and, of every step of 64 cells, the cells s, s + S, ... (S = 64 / gs
// cell subgroups). In a step lane k reads cell k's depth, row and weights
// lam_l^r once; the others take them by cross-lane shuffle, so the walk
// needs neither LDS nor workgroup barriers (and every shuffle runs with the
// whole wavefront active). The subgroups' sums are combined by shuffles.
// Forward: a second walk writes the table values lam_l^r sum_l c_l a_l.
// Moments: subgroup 0 adds sign <b_l, a_l> and sign (<b^r_l, a_l> + <b_l,
// a^r_l>) over its channels; the workgroup total goes to row mbase +
// blockIdx.x of mrow ([s0 | s1][nterm]).
// WHOLE (gs = 64, i.e. d > 32): one cell subgroup, so the cell a step works
// on is the same in every lane; its row, depth and weights are read from the
// owning lane into scalar registers, and eight cell rows are loaded per step.
// DF (with GRAD): the same launch also writes the dF table values of the
// gout sums (the forward's second walk on b_l), bit-identical to a forward
// launch over valg.
template <typename T, int NJ, bool GRAD, bool WHOLE = false, bool DF = false>
__global__ void __launch_bounds__(kExpThreads)
k_expsum_wave(int32_t nterm, int32_t d, int32_t gs, int32_t njobs,
              const int32_t* __restrict__ ej, const int64_t* __restrict__ joff,
              const int32_t* __restrict__ jsign, const int32_t* __restrict__ jc_r,
              const int32_t* __restrict__ jc_val, const T* __restrict__ c,
              const T* __restrict__ pw, int32_t K, const T* __restrict__ val,
              const T* __restrict__ valg, T* __restrict__ g, double* __restrict__ mrow,
              int64_t mbase) {
    constexpr int NQ = GRAD ? 4 : 1;
    constexpr int B = WHOLE ? 8 : 4;  // cells per subgroup and batch of value loads
    const int lane = threadIdx.x & 63;
    const int32_t jn = blockIdx.x * (kExpThreads / 64) + (threadIdx.x >> 6);
    const bool active = jn < njobs;  // uniform per wavefront
    if (WHOLE) gs = 64;
    const int32_t S = WHOLE ? 1 : 64 / gs, sub = WHOLE ? 0 : lane / gs, lc = lane - sub * gs;
    const int32_t job = active ? ej[jn] : 0;
    const int64_t cb = active ? joff[job] : 0, ce = active ? joff[job + 1] : 0;
    const T sgn = (GRAD && active && jsign[job] < 0) ? (T)-1 : (T)1;
    T cl[NJ];
#pragma unroll
    for (int l = 0; l < NJ; ++l) cl[l] = ((!GRAD || DF) && l < nterm) ? c[l] : (T)0;
    double m0[NJ], m1[NJ];
#pragma unroll
    for (int l = 0; l < NJ; ++l) m0[l] = m1[l] = 0.0;
    for (int32_t c0 = 0; c0 < d; c0 += gs) {
        const int32_t ch = c0 + lc;
        const bool chok = ch < d;
        const int32_t chs = min(ch, d - 1);
        T acc[NQ][NJ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int l = 0; l < NJ; ++l) acc[q][l] = (T)0;
        for (int64_t k0 = cb; k0 < ce; k0 += 64) {
            const int32_t nk = (int32_t)min((int64_t)64, ce - k0);
            const int64_t mine = k0 + min(lane, nk - 1);
            const int32_t rmine = jc_r[mine], rowmine = jc_val[mine];
            T wmine[NJ];
#pragma unroll
            for (int l = 0; l < NJ; ++l) wmine[l] = l < nterm ? pw[(int64_t)l * K + rmine] : (T)0;
            for (int32_t k = 0; k < nk; k += S * B) {  // uniform in the wavefront
                int32_t kk[B], rowk[B];
                T rk[B], v[B], gv[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    kk[u] = k + u * S + sub;
                    const int32_t src = min(kk[u], nk - 1);
                    rowk[u] = WHOLE ? lane_value(rowmine, src) : __shfl(rowmine, src, 64);
                    rk[u] = !GRAD  ? (T)0
                            : WHOLE ? (T)lane_value(rmine, src)
                                    : (T)__shfl(rmine, src, 64);
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const bool ok = chok && kk[u] < nk;
                    const int64_t o = (int64_t)rowk[u] * d + chs;
                    v[u] = ok ? val[o] : (T)0;
                    gv[u] = (GRAD && ok) ? valg[o] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int32_t src = min(kk[u], nk - 1);
#pragma unroll
                    for (int l = 0; l < NJ; ++l) {
                        if (l >= nterm) continue;
                        const T w = WHOLE ? lane_value(wmine[l], src) : __shfl(wmine[l], src, 64);
                        acc[0][l] += w * v[u];
                        if (GRAD) {
                            acc[1][l] += rk[u] * w * v[u];
                            acc[2][l] += w * gv[u];
                            acc[3][l] += rk[u] * w * gv[u];
                        }
                    }
                }
            }
        }
        // combine the cell subgroups (lanes gs, 2 gs, ... apart)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int l = 0; l < NJ; ++l)
                for (int o = gs; o < 64; o <<= 1) acc[q][l] += __shfl_xor(acc[q][l], o, 64);
        if (GRAD && chok && sub == 0) {
#pragma unroll
            for (int l = 0; l < NJ; ++l) {
                m0[l] += (double)(sgn * acc[2][l] * acc[0][l]);
                m1[l] += (double)(sgn * (acc[3][l] * acc[0][l] + acc[2][l] * acc[1][l]));
            }
        }
        if (!GRAD || DF) {
            T ca[NJ];
#pragma unroll
            for (int l = 0; l < NJ; ++l) ca[l] = cl[l] * acc[GRAD ? 2 : 0][l];
            for (int64_t k0 = cb; k0 < ce; k0 += 64) {
                const int32_t nk = (int32_t)min((int64_t)64, ce - k0);
                const int64_t mine = k0 + min(lane, nk - 1);
                const int32_t rmine = jc_r[mine], rowmine = jc_val[mine];
                T wmine[NJ];
#pragma unroll
                for (int l = 0; l < NJ; ++l)
                    wmine[l] = l < nterm ? pw[(int64_t)l * K + rmine] : (T)0;
                for (int32_t k = 0; k < nk; k += S) {  // uniform in the wavefront
                    const int32_t kk = k + sub, src = min(kk, nk - 1);
                    const int32_t rowk =
                        WHOLE ? lane_value(rowmine, src) : __shfl(rowmine, src, 64);
                    T sum = (T)0;
#pragma unroll
                    for (int l = 0; l < NJ; ++l)
                        if (l < nterm)
                            sum += ca[l] * (WHOLE ? lane_value(wmine[l], src)
                                                  : __shfl(wmine[l], src, 64));
                    if (chok && kk < nk) g[(int64_t)rowk * d + ch] = sum;
                }
            }
        }
    }
    if (GRAD) {
        // workgroup totals in one pass: wave shuffles, then LDS across waves
        __shared__ double red[kExpThreads / 64][2 * NJ];
#pragma unroll
        for (int l = 0; l < NJ; ++l)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                m0[l] += __shfl_xor(m0[l], o, 64);
                m1[l] += __shfl_xor(m1[l], o, 64);
            }
        if (lane == 0)
#pragma unroll
            for (int l = 0; l < NJ; ++l) {
                red[threadIdx.x >> 6][l] = m0[l];
                red[threadIdx.x >> 6][NJ + l] = m1[l];
            }
        __syncthreads();
        if ((int32_t)threadIdx.x < 2 * nterm) {
            const int e = threadIdx.x < nterm ? threadIdx.x : NJ + threadIdx.x - nterm;
            double t = 0.0;
            for (int w = 0; w < kExpThreads / 64; ++w) t += red[w][e];
            mrow[(mbase + blockIdx.x) * 2 * nterm + threadIdx.x] = t;
        }
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
