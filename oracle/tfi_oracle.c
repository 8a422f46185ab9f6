/*
 * tfi_oracle.c -- CPU FP64 reference for tree field integration.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library's compute path links,
 * loads or calls this file; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it. It shares no code with the device
 * path.
 *
 * What it computes is the plain definition of the problem (Section 1,
 * equation "integration"; Section 2, equation "stad-target"):
 *
 *     out[v, c] = sum_{w in V} f(dist_T(v, w)) * F[w, c]
 *
 * for every vertex v of a forest given by parent pointers, where dist_T is
 * the sum of the positive integer edge lengths on the unique v-w path
 * (the quantised lattice metric of the appendix on distance quantisation;
 * unit lengths give the hop distance the main text uses). The v = w term
 * f(0) F[v] is included. Vertices of different trees do not interact.
 * No decomposition, FFT, blocking or reordering is used: one traversal per
 * source row gives exact int64 distances, then a compensated FP64 sum.
 *
 * Also here:
 *  - oracle_pair_hist: h[k] = sum_{v,w : dist = k} <G[v,:], F[w,:]>, the
 *    gradient of sum(G * out) with respect to the kernel table f[k];
 *  - oracle_expdp: the textbook two-pass rooted-tree recursion for kernels
 *    f(d) = sum_j c_j lambda_j^d (the exponential kernels the paper's
 *    specialised-kernel section and its exact-DP baseline target). It is a
 *    different algorithm and serves as an independent pin of
 *    oracle_integrate at sizes where all-pairs traversal is too slow.
 *
 * Return codes: 0 ok, -1 bad argument, -2 malformed tree (parent out of
 * range or a cycle), -3 non-positive weight or distance overflow, -4 the
 * kernel table is shorter than a distance that occurs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n;
    int64_t *off;   /* CSR offsets, n+1 */
    int64_t *nbr;   /* neighbours */
    int64_t *len;   /* edge lengths */
} adj_t;

static void adj_free(adj_t *a)
{
    free(a->off);
    free(a->nbr);
    free(a->len);
    a->off = a->nbr = a->len = NULL;
}

/* Undirected adjacency of the forest; validates parent pointers (range,
 * acyclicity) and weights. */
static int adj_build(int64_t n, const int64_t *parent, const int32_t *weight,
                     adj_t *a)
{
    int64_t v, edges = 0;
    memset(a, 0, sizeof(*a));
    if (n < 0 || (n > 0 && (!parent || !weight)))
        return -1;
    a->n = n;
    a->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!a->off)
        return -1;
    for (v = 0; v < n; ++v) {
        int64_t p = parent[v];
        if (p < -1 || p >= n || p == v) {
            adj_free(a);
            return -2;
        }
        if (p >= 0) {
            if (weight[v] < 1) {
                adj_free(a);
                return -3;
            }
            a->off[v + 1]++;
            a->off[p + 1]++;
            edges++;
        }
    }
    for (v = 0; v < n; ++v)
        a->off[v + 1] += a->off[v];
    a->nbr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * edges + 1));
    a->len = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * edges + 1));
    if (!a->nbr || !a->len) {
        adj_free(a);
        return -1;
    }
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        if (!fill) {
            adj_free(a);
            return -1;
        }
        memcpy(fill, a->off, sizeof(int64_t) * (size_t)n);
        for (v = 0; v < n; ++v) {
            int64_t p = parent[v];
            if (p >= 0) {
                a->nbr[fill[v]] = p;
                a->len[fill[v]++] = weight[v];
                a->nbr[fill[p]] = v;
                a->len[fill[p]++] = weight[v];
            }
        }
        free(fill);
    }
    /* acyclicity: following parents from every vertex must reach a root
     * within n steps; equivalently the edge count equals n - #roots and a
     * traversal from the roots reaches every vertex once. */
    {
        int64_t roots = 0, seen = 0, head = 0, tail = 0;
        int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        char *mark = (char *)calloc((size_t)n + 1, 1);
        if (!queue || !mark) {
            free(queue);
            free(mark);
            adj_free(a);
            return -1;
        }
        for (v = 0; v < n; ++v)
            if (parent[v] < 0) {
                roots++;
                mark[v] = 1;
                queue[tail++] = v;
            }
        while (head < tail) {
            int64_t x = queue[head++], k;
            seen++;
            for (k = a->off[x]; k < a->off[x + 1]; ++k) {
                int64_t y = a->nbr[k];
                if (!mark[y]) {
                    mark[y] = 1;
                    queue[tail++] = y;
                }
            }
        }
        free(queue);
        free(mark);
        if (seen != n || edges != n - roots) {
            adj_free(a);
            return -2;
        }
    }
    return 0;
}

/* Distances from src to every vertex of its tree; dist[] must hold -1 on
 * entry for all vertices and is left with the distances of the visited
 * vertices, listed in order[0..*cnt). */
static int bfs(const adj_t *a, int64_t src, int64_t *dist, int64_t *order,
               int64_t *cnt)
{
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    order[tail++] = src;
    while (head < tail) {
        int64_t x = order[head++], k;
        for (k = a->off[x]; k < a->off[x + 1]; ++k) {
            int64_t y = a->nbr[k];
            if (dist[y] < 0) {
                int64_t dy = dist[x] + a->len[k];
                if (dy < dist[x])
                    return -3; /* overflow */
                dist[y] = dy;
                order[tail++] = y;
            }
        }
    }
    *cnt = tail;
    return 0;
}

static int resolve_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    return nthreads < 1 ? 1 : nthreads;
}

/* Neumaier's compensated addition of x into (s, comp). */
static inline void neumaier(double *s, double *comp, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *comp += (*s - t) + x;
    else
        *comp += (x - t) + *s;
    *s = t;
}

int oracle_num_threads(int nthreads)
{
    return resolve_threads(nthreads);
}

/*
 * out[i, c] = sum_w f(dist(rows[i], w)) F[w, c] for i < nrows (all
 * vertices in order when rows == NULL, nrows ignored). F is row-major
 * [N x d], out is row-major [nrows x d]. f has flen entries.
 */
int oracle_integrate(int64_t n, const int64_t *parent, const int32_t *weight,
                     const double *f, int64_t flen, const double *F,
                     int64_t d, const int64_t *rows, int64_t nrows,
                     double *out, int nthreads)
{
    adj_t a;
    int rc, status = 0;
    int64_t nr;
    if (d < 0 || flen < 0 || (n > 0 && (!f || (d > 0 && (!F || !out)))))
        return -1;
    rc = adj_build(n, parent, weight, &a);
    if (rc)
        return rc;
    nr = rows ? nrows : n;
    if (rows) {
        int64_t i;
        for (i = 0; i < nr; ++i)
            if (rows[i] < 0 || rows[i] >= n) {
                adj_free(&a);
                return -1;
            }
    }
    nthreads = resolve_threads(nthreads);
#pragma omp parallel num_threads(nthreads)
    {
        int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        double *s = (double *)malloc(sizeof(double) * (size_t)(2 * d + 1));
        int64_t i, j;
        int local = 0;
        if (!dist || !order || !s)
            local = -1;
        else
            for (j = 0; j < n; ++j)
                dist[j] = -1;
#pragma omp for schedule(dynamic, 4)
        for (i = 0; i < nr; ++i) {
            int64_t src = rows ? rows[i] : i, cnt = 0, k, c;
            double *sum = s, *comp = s + d;
            if (local)
                continue;
            if (bfs(&a, src, dist, order, &cnt)) {
                local = -3;
                continue;
            }
            for (c = 0; c < d; ++c)
                sum[c] = comp[c] = 0.0;
            for (k = 0; k < cnt; ++k) {
                int64_t w = order[k], dw = dist[w];
                double fv;
                if (dw >= flen) {
                    local = -4;
                    break;
                }
                fv = f[dw];
                for (c = 0; c < d; ++c)
                    neumaier(&sum[c], &comp[c], fv * F[w * d + c]);
            }
            for (c = 0; c < d; ++c)
                out[i * d + c] = sum[c] + comp[c];
            for (k = 0; k < cnt; ++k)
                dist[order[k]] = -1;
        }
#pragma omp critical
        {
            if (local && !status)
                status = local;
        }
        free(dist);
        free(order);
        free(s);
    }
    adj_free(&a);
    return status;
}

/*
 * h[k] += sum over v in rows (all vertices when rows == NULL) and all w
 * with dist(v, w) = k of <G[v, :], F[w, :]>; h has hlen entries and is
 * overwritten. G is indexed by vertex id (row-major [N x d]).
 */
int oracle_pair_hist(int64_t n, const int64_t *parent, const int32_t *weight,
                     const double *G, const double *F, int64_t d,
                     const int64_t *rows, int64_t nrows, double *h,
                     int64_t hlen, int nthreads)
{
    adj_t a;
    int rc, status = 0;
    int64_t nr, k0;
    if (d < 0 || hlen < 0 || !h || (n > 0 && d > 0 && (!G || !F)))
        return -1;
    rc = adj_build(n, parent, weight, &a);
    if (rc)
        return rc;
    nr = rows ? nrows : n;
    for (k0 = 0; k0 < hlen; ++k0)
        h[k0] = 0.0;
    nthreads = resolve_threads(nthreads);
#pragma omp parallel num_threads(nthreads)
    {
        int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        double *hs = (double *)calloc((size_t)(2 * hlen + 1), sizeof(double));
        int64_t i, j;
        int local = 0;
        if (!dist || !order || !hs)
            local = -1;
        else
            for (j = 0; j < n; ++j)
                dist[j] = -1;
#pragma omp for schedule(dynamic, 4)
        for (i = 0; i < nr; ++i) {
            int64_t src = rows ? rows[i] : i, cnt = 0, k, c;
            if (local)
                continue;
            if (src < 0 || src >= n) {
                local = -1;
                continue;
            }
            if (bfs(&a, src, dist, order, &cnt)) {
                local = -3;
                continue;
            }
            for (k = 0; k < cnt; ++k) {
                int64_t w = order[k], dw = dist[w];
                double dot = 0.0;
                if (dw >= hlen) {
                    local = -4;
                    break;
                }
                for (c = 0; c < d; ++c)
                    dot += G[src * d + c] * F[w * d + c];
                neumaier(&hs[dw], &hs[hlen + dw], dot);
            }
            for (k = 0; k < cnt; ++k)
                dist[order[k]] = -1;
        }
#pragma omp critical
        {
            int64_t k;
            if (local && !status)
                status = local;
            if (hs)
                for (k = 0; k < hlen; ++k)
                    h[k] += hs[k] + hs[hlen + k];
        }
        free(dist);
        free(order);
        free(hs);
    }
    adj_free(&a);
    return status;
}

/* Row-major distance matrix D[nrows x N] (-1 across trees of a forest). */
int oracle_distances(int64_t n, const int64_t *parent, const int32_t *weight,
                     const int64_t *rows, int64_t nrows, int64_t *D)
{
    adj_t a;
    int rc;
    int64_t i, j, nr;
    int64_t *order;
    rc = adj_build(n, parent, weight, &a);
    if (rc)
        return rc;
    nr = rows ? nrows : n;
    order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!order) {
        adj_free(&a);
        return -1;
    }
    for (i = 0; i < nr; ++i) {
        int64_t src = rows ? rows[i] : i, cnt;
        int64_t *row = D + i * n;
        if (src < 0 || src >= n) {
            rc = -1;
            break;
        }
        for (j = 0; j < n; ++j)
            row[j] = -1;
        rc = bfs(&a, src, row, order, &cnt);
        if (rc)
            break;
    }
    free(order);
    adj_free(&a);
    return rc;
}

/* Largest distance between two vertices of one tree (two traversals per
 * tree: the farthest vertex from any vertex is an end of a diameter). */
int oracle_diameter(int64_t n, const int64_t *parent, const int32_t *weight,
                    int64_t *diam)
{
    adj_t a;
    int rc;
    int64_t v, best = 0;
    int64_t *dist, *order;
    rc = adj_build(n, parent, weight, &a);
    if (rc)
        return rc;
    dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!dist || !order) {
        free(dist);
        free(order);
        adj_free(&a);
        return -1;
    }
    for (v = 0; v < n; ++v)
        dist[v] = -1;
    for (v = 0; v < n && !rc; ++v) {
        int64_t cnt, k, far, fd;
        if (parent[v] >= 0)
            continue;
        rc = bfs(&a, v, dist, order, &cnt);
        if (rc)
            break;
        far = v;
        fd = 0;
        for (k = 0; k < cnt; ++k)
            if (dist[order[k]] > fd) {
                fd = dist[order[k]];
                far = order[k];
            }
        for (k = 0; k < cnt; ++k)
            dist[order[k]] = -1;
        rc = bfs(&a, far, dist, order, &cnt);
        if (rc)
            break;
        for (k = 0; k < cnt; ++k) {
            if (dist[order[k]] > best)
                best = dist[order[k]];
            dist[order[k]] = -1;
        }
    }
    free(dist);
    free(order);
    adj_free(&a);
    *diam = best;
    return rc;
}

/*
 * Exponential-sum kernels f(d) = sum_j c[j] * lam[j]^d, all vertices:
 * root every tree, then for each term
 *   up[v]   = F[v] + sum_{children u} lam^{w(u)} up[u]      (leaves first)
 *   full[r] = up[r] at a root r,
 *   full[u] = up[u] + lam^{w(u)} (full[p] - lam^{w(u)} up[u])   (root first)
 * so that full[v] = sum_w lam^{dist(v,w)} F[w]; out = sum_j c[j] full_j.
 * Requires 0 < lam[j] <= 1.
 */
int oracle_expdp(int64_t n, const int64_t *parent, const int32_t *weight,
                 const double *c, const double *lam, int64_t J,
                 const double *F, int64_t d, double *out)
{
    adj_t a;
    int rc;
    int64_t *order, head = 0, tail = 0, v, j, k;
    double *up, *full;
    if (J < 0 || d < 0 || (n > 0 && (!F || !out || (J > 0 && (!c || !lam)))))
        return -1;
    for (j = 0; j < J; ++j)
        if (!(lam[j] > 0.0 && lam[j] <= 1.0))
            return -1;
    rc = adj_build(n, parent, weight, &a);
    if (rc)
        return rc;
    order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    up = (double *)malloc(sizeof(double) * (size_t)(n * d + 1));
    full = (double *)malloc(sizeof(double) * (size_t)(n * d + 1));
    if (!order || !up || !full) {
        free(order);
        free(up);
        free(full);
        adj_free(&a);
        return -1;
    }
    /* parents before children */
    for (v = 0; v < n; ++v)
        if (parent[v] < 0)
            order[tail++] = v;
    {
        char *seen = (char *)calloc((size_t)n + 1, 1);
        for (k = 0; k < tail; ++k)
            seen[order[k]] = 1;
        while (head < tail) {
            int64_t x = order[head++];
            for (k = a.off[x]; k < a.off[x + 1]; ++k) {
                int64_t y = a.nbr[k];
                if (!seen[y]) {
                    seen[y] = 1;
                    order[tail++] = y;
                }
            }
        }
        free(seen);
    }
    for (k = 0; k < n * d; ++k)
        out[k] = 0.0;
    for (j = 0; j < J; ++j) {
        int64_t i, ch;
        for (k = 0; k < n * d; ++k)
            up[k] = F[k];
        for (i = n - 1; i >= 0; --i) {
            int64_t u = order[i], p = parent[u];
            if (p >= 0) {
                double g = pow(lam[j], (double)weight[u]);
                for (ch = 0; ch < d; ++ch)
                    up[p * d + ch] += g * up[u * d + ch];
            }
        }
        for (i = 0; i < n; ++i) {
            int64_t u = order[i], p = parent[u];
            if (p < 0) {
                for (ch = 0; ch < d; ++ch)
                    full[u * d + ch] = up[u * d + ch];
            } else {
                double g = pow(lam[j], (double)weight[u]);
                for (ch = 0; ch < d; ++ch)
                    full[u * d + ch] =
                        up[u * d + ch] +
                        g * (full[p * d + ch] - g * up[u * d + ch]);
            }
        }
        for (k = 0; k < n * d; ++k)
            out[k] += c[j] * full[k];
    }
    free(order);
    free(up);
    free(full);
    adj_free(&a);
    return 0;
}
