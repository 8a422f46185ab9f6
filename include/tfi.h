/*
 * tfi.h -- C ABI of the MI355X tree field integrator (libtfi.so).
 *
 * Problem (Section 1, equation "integration"; Section 2, equation
 * "stad-target"): for every vertex v of a forest with positive integer
 * edge lengths,
 *
 *     out[v, c] = sum_{w in same tree} f(dist(v, w)) * F[w, c],
 *
 * where dist is the sum of edge lengths on the v-w path and f is a table on
 * the integer lattice (f : Z>=0 -> R; real lengths are quantised to lattice
 * units first, appendix "Distance quantization"). The self term f(0) F[v]
 * is included; vertices of different trees do not interact.
 *
 * Method (Section 2 and its appendix algorithms): the tree is decomposed
 * recursively around backbones -- a diameter path or a single centroid,
 * chosen per call by the adaptive score (equation "stad-score"). Each
 * call's cross-component interactions are the interaction table
 * G_q[s] (equation "sumofFFTterms") minus the per-component corrections
 * E_alpha (equation "stad-E", lemma "stad-cross"), with G evaluated as one
 * 2-D convolution of the depth-reversed aggregate table with the kernel
 * K[a, b] = f(H + a + |b|) (equation "stad-2d-convolution", lemma
 * "stad-2d-fft"). Backbone coordinates and depths are weighted lattice
 * distances. Small subtrees are evaluated densely.
 *
 * Conventions for every entry point:
 *  - return 0 on success, a negative tfi_status otherwise; the message of
 *    the last failure on the calling thread is tfi_last_error();
 *  - no entry point throws or aborts; invalid arguments are reported;
 *  - "device" pointers are HIP device allocations of the handle's device;
 *    "host" pointers are ordinary CPU memory;
 *  - device work is enqueued on `stream` (0 = the null stream) and is
 *    asynchronous with respect to the host; a handle must not be used on
 *    two streams at the same time (it owns scratch arenas);
 *  - element types follow `dtype` (TFI_F32 = float, TFI_F64 = double);
 *  - matrices are row-major: element (v, c) of an [N x d] matrix is at
 *    offset v * d + c.
 */
#ifndef TFI_H
#define TFI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tfi_plan *tfi_handle;

typedef enum {
    TFI_F32 = 0,
    TFI_F64 = 1
} tfi_dtype;

typedef enum {
    TFI_OK = 0,
    TFI_ERR_ARG = -1,     /* null pointer, bad size, bad option          */
    TFI_ERR_TREE = -2,    /* parent out of range, self loop or cycle      */
    TFI_ERR_WEIGHT = -3,  /* weight < 1, or a distance exceeds int32      */
    TFI_ERR_DTYPE = -4,   /* unknown dtype                               */
    TFI_ERR_OOM = -5,     /* host or device allocation failed            */
    TFI_ERR_BUDGET = -6,  /* device memory budget too small              */
    TFI_ERR_HIP = -7,     /* HIP runtime error (no device, launch error)  */
    TFI_ERR_STATE = -8    /* handle built host-only, or wrong device      */
} tfi_status;

/* Backbone selection policy per recursive call. */
typedef enum {
    TFI_POLICY_ADAPTIVE = 0, /* diameter or centroid by the adaptive score  */
    TFI_POLICY_DIAMETER = 1, /* always a (weighted) diameter path           */
    TFI_POLICY_CENTROID = 2, /* always a single centroid vertex             */
    TFI_POLICY_CHANNEL = 3   /* diameter or centroid by the channel-aware
                                cost model (appendix "Channel-aware backbone
                                selection"): fields chan_width and cost_*  */
} tfi_policy;

/* Build options; pass NULL for the defaults (all fields 0 = default). */
typedef struct {
    int32_t policy;              /* tfi_policy; default adaptive            */
    int32_t leaf_max;            /* subtrees with at most this many
                                    vertices are integrated densely;
                                    0 = default (32), 1 = only single
                                    vertices (the plain recursion); at
                                    most 64                               */
    int32_t device;              /* HIP device ordinal; -1 = host-only
                                    plan (no device upload; for planning
                                    statistics and host-side tests)        */
    int32_t table_method;        /* 0 = per-job choice, 1 = force direct
                                    sums, 2 = force FFT for every table,
                                    3 = tables with several depths and
                                    several backbone positions as one 1-D
                                    FFT convolution along the backbone per
                                    pair of depths (algorithm
                                    "global-anchor"), the others by FFT,
                                    4 = such tables with depth H <= 127 by
                                    the product with the Hankel matrix
                                    f(l + r) and walks along the backbone
                                    (attention-width appendix
                                    "Hankel-GEMM"), the others by FFT      */
    uint64_t memory_budget_bytes;/* cap on device bytes held by the handle
                                    and its per-call scratch; 0 = none.
                                    tfi_integrate and tfi_backward (without
                                    kept cell sums) split a call whose
                                    scratch would not fit into tiles of
                                    channels that do, each a full pass;
                                    TFI_ERR_BUDGET when not even one
                                    channel fits                           */
    int32_t no_graphs;           /* 1 = launch kernels directly instead of
                                    replaying captured hipGraphs           */
    float fft_cost;              /* per-job rule: direct sums if
                                    cells^2 <= fft_cost * P log2 P, FFT
                                    otherwise (P = padded table cells);
                                    0 = default (4). A table with depths
                                    0 < H <= 127 and backbone positions
                                    X > 0 takes the Hankel product
                                    (table_method 4) when (H + X + 1)
                                    (X + 1)(H + 3) is below both           */
    int32_t direct_kernel;       /* direct sums: 0 = matrix cores for FP32
                                    with d >= 8, vector ALU otherwise;
                                    1 = vector ALU; 2 = matrix cores when
                                    the dtype is FP32                      */
    /* TFI_POLICY_CHANNEL only. A candidate backbone of a call costs
     *   cost_call x (table jobs of the call: 1 + components)
     *   + chan_width x (cost_vertex x (|V(S)| + sum_a n_a log2(n_a + 1))
     *                   + its table + every correction table),
     * each table at the cheaper of cost_direct x cells^2 and
     * cost_fft x P log2 P (occupied cells; P = padded FFT cells). The centroid
     * is taken when it costs strictly less. Costs are in seconds per unit
     * (tfi_calibrate measures them); all four 0 = defaults (1, 1, 4, 0). With
     * measured costs and fft_cost 0, the per-table rule uses
     * fft_cost = cost_fft / cost_direct.                                     */
    int32_t chan_width;          /* channel count C the plan is made for;
                                    0 = 1                                  */
    float cost_vertex;           /* per incidence and channel (scatter and
                                    gather)                                */
    float cost_direct;           /* per direct-sum cell pair and channel   */
    float cost_fft;              /* per P log2 P of an FFT table and channel */
    float cost_call;             /* per table job, independent of C        */
} tfi_build_opts;

/*
 * Plan a forest on the host and upload the plan to the device.
 *   parent  host int64[N]: parent[v] in [-1, N), -1 marks a root; the
 *           parent pointers must form a forest (no cycles, no self loops)
 *   weight  host int32[N]: weight[v] >= 1 is the length of edge
 *           (v, parent[v]); ignored at roots
 *   N       number of vertices, N >= 1
 *   opts    NULL or build options
 *   out     receives the handle (owned by the caller; free with
 *           tfi_destroy)
 * The arrays are read during the call only. Errors: TFI_ERR_ARG,
 * TFI_ERR_TREE, TFI_ERR_WEIGHT, TFI_ERR_OOM, TFI_ERR_HIP, TFI_ERR_BUDGET.
 */
int tfi_build(const int64_t *parent, const int32_t *weight, int64_t N,
              const tfi_build_opts *opts, tfi_handle *out);

/* Number of vertices of the handle's forest. */
int64_t tfi_num_vertices(tfi_handle h);

/*
 * Number of kernel-table entries f[0 .. K-1] that tfi_integrate and
 * tfi_backward read. K exceeds the forest diameter: the interaction tables
 * evaluate f at surrogate (through-the-backbone) distances and on the
 * padded convolution grid (appendix algorithm "ComputeGTerm2DFFT" indexes
 * f up to 2H + m - 1). Those extra entries cancel exactly in exact
 * arithmetic but must be finite. Returns -1 for a null handle.
 */
int64_t tfi_kernel_length(tfi_handle h);

/*
 * Forward integration: out = K F with K[v, w] = f(dist(v, w)).
 *   f    device dtype[tfi_kernel_length(h)]
 *   F    device dtype[N x d]
 *   d    channels, d >= 1
 *   out  device dtype[N x d]; must not alias F
 * Errors: TFI_ERR_ARG, TFI_ERR_DTYPE, TFI_ERR_STATE, TFI_ERR_HIP,
 * TFI_ERR_BUDGET, TFI_ERR_OOM.
 */
int tfi_integrate(tfi_handle h, const void *f, const void *F, int64_t d,
                  tfi_dtype dtype, void *out, void *stream);

/*
 * Several kernels over one field: out[i] = K_i F with K_i[v, w] =
 * f[i](dist(v, w)), for i < nk (Section 1, equation "integration", once per
 * kernel). The cell sums of F (equation "stad-E" and the A-cells of
 * Section 2.2) do not depend on the kernel, so they are formed once; each
 * kernel then has its own spectra, tables, leaf tiles and gather. Each
 * out[i] equals what tfi_integrate(h, f[i], F, ...) writes, bit for bit.
 *   nk   1 <= nk <= TFI_MULTI_MAX
 *   f    host array of nk device pointers, each dtype[tfi_kernel_length(h)]
 *   F    device dtype[N x d]
 *   out  host array of nk device pointers, each dtype[N x d]; distinct, none
 *        aliasing F
 * Scratch grows with nk: nk table arrays and nk spectrum arenas.
 * Errors: as tfi_integrate.
 */
#define TFI_MULTI_MAX 4
int tfi_integrate_multi(tfi_handle h, int32_t nk, const void *const *f, const void *F,
                        int64_t d, tfi_dtype dtype, void *const *out, void *stream);

/*
 * tfi_integrate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result from the same kernels, with every scratch buffer of the
 * pass (cell sums, table rows, kernel spectra, FFT slots) carved out of one
 * fixed device array of TFI_NOALLOC_SCRATCH_BYTES bytes per GPU, held from
 * the library's first use of that GPU until the process ends. The call
 * allocates nothing and captures no graph: the kernels are launched
 * directly on `stream` and the handle's two side streams, joined back into
 * `stream` before the pass ends. Stage profiling is off during the call.
 *  - Arguments, layouts and ownership as tfi_integrate; the caller still
 *    provides f, F and out.
 *  - TFI_ERR_BUDGET (before anything is launched) when the plan needs more
 *    scratch at this d and dtype than the array holds.
 *  - Every call on one GPU shares that GPU's array, which keeps the last
 *    call's contents. Calls whose work overlaps on one GPU (two streams, or
 *    two handles used at the same time) race on it: order them.
 */
#define TFI_NOALLOC_SCRATCH_BYTES (128u << 20)
int tfi_integrate_noalloc(tfi_handle h, const void *f, const void *F, int64_t d,
                          tfi_dtype dtype, void *out, void *stream);

/*
 * Adjoint of tfi_integrate for the loss L = sum(gout * out):
 *   dF = K gout (K is symmetric), device dtype[N x d], may be NULL;
 *   df[k] = sum_{v, w : dist(v, w) = k} <gout[v, :], F[w, :]>, the
 *   gradient with respect to the kernel table, device double[K] with
 *   K = tfi_kernel_length(h) (entries beyond the diameter are 0), may be
 *   NULL.
 *   f, F, gout as in tfi_integrate (gout device dtype[N x d]).
 * Errors as tfi_integrate.
 */
int tfi_backward(tfi_handle h, const void *f, const void *F,
                 const void *gout, int64_t d, tfi_dtype dtype, void *dF,
                 double *df, void *stream);

/*
 * Kernels given as sums of exponentials (appendix "Specialized Kernels",
 * lemma "stad-specialized-cross" and algorithm "CrossSubRoutineExp"):
 *   f(k) = sum_{l < nterm} c[l] * lambda[l]^k,   lambda[l] > 0,
 * on the integer lattice distances of the tree. Every table job is
 * evaluated by two backbone sweeps per term, in time linear in its cells,
 * instead of direct sums or FFT; the leaf tiles use f tabulated on the
 * device. Results equal tfi_integrate with that f table (up to rounding).
 *   nterm   1 <= nterm <= TFI_EXPSUM_MAX_TERMS
 *   c       device dtype[nterm]
 *   lambda  device dtype[nterm], every entry > 0
 *   F, d, out, stream as in tfi_integrate.
 * Errors as tfi_integrate.
 */
#define TFI_EXPSUM_MAX_TERMS 16
int tfi_integrate_expsum(tfi_handle h, int32_t nterm, const void *c,
                         const void *lambda, const void *F, int64_t d,
                         tfi_dtype dtype, void *out, void *stream);

/*
 * Adjoint of tfi_integrate_expsum for L = sum(gout * out):
 *   dF  = K gout, device dtype[N x d], may be NULL;
 *   s0[l] = sum_{v, w} lambda[l]^dist(v,w) <gout[v, :], F[w, :]>,
 *   s1[l] = sum_{v, w} dist(v,w) lambda[l]^dist(v,w) <gout[v, :], F[w, :]>,
 *   device double[nterm] each (overwritten), both NULL or both given.
 * Then dL/dc[l] = s0[l] and dL/dlambda[l] = c[l] * s1[l] / lambda[l]; with
 * lambda = exp(-b), dL/db[l] = -c[l] * s1[l]. s0/s1 are FP64 sums of
 * per-workgroup rows in a fixed order, but their leaf-tile part comes from
 * a pair histogram binned with atomics (LDS bins in the field's precision,
 * then FP64): reproducible to that rounding, not bitwise.
 * Errors as tfi_integrate.
 */
int tfi_backward_expsum(tfi_handle h, int32_t nterm, const void *c,
                        const void *lambda, const void *F, const void *gout,
                        int64_t d, tfi_dtype dtype, void *dF, double *s0,
                        double *s1, void *stream);

/*
 * Cell sums kept from the forward for the backward (a training step saves
 * them instead of scattering F a second time). The cell sums are the
 * per-cell field totals of every table job (the A-cells of a call, the
 * b-cells of its components) that both passes start from: the
 * accumulation of F by depth and backbone position in the pseudocode for
 * the cross terms (appendix "Algorithmic Details and Deferred Proofs").
 *
 * tfi_cell_rows: rows of the cell-sum array of h (>= 1), or a negative
 * status.
 *
 * tfi_integrate_expsum_cells: tfi_integrate_expsum that also leaves the
 * cell sums of F in cells, device dtype[tfi_cell_rows(h) x d] owned by the
 * caller (overwritten; must not alias F or out).
 *
 * tfi_backward_expsum_cells: tfi_backward_expsum that takes the cell sums
 * of F from cells, as written by tfi_integrate_expsum_cells on the same
 * handle with the same F and d, instead of forming them again. F is still
 * read (leaf tiles). dF is bitwise that of tfi_backward_expsum, s0/s1 the
 * same to the rounding of the leaf histogram.
 *
 * Errors as tfi_integrate_expsum; cells == NULL is TFI_ERR_ARG.
 */
int64_t tfi_cell_rows(tfi_handle h);

/*
 * The same for kernel tables: tfi_integrate_cells is tfi_integrate that
 * also leaves the cell sums of F in cells (device dtype[tfi_cell_rows(h) x
 * d], caller-owned, overwritten; must not alias F or out; the plan's
 * whole-path shortcut is not taken, since it forms no cell sums).
 * tfi_backward_cells is tfi_backward that takes them for df instead of
 * scattering F again (same handle, F and d as the forward; dF must not
 * alias cells). dF is bitwise that of tfi_backward, df the same to the
 * rounding of its atomic histograms. Errors as tfi_integrate; cells ==
 * NULL is TFI_ERR_ARG.
 */
int tfi_integrate_cells(tfi_handle h, const void *f, const void *F, int64_t d,
                        tfi_dtype dtype, void *out, void *cells, void *stream);
int tfi_backward_cells(tfi_handle h, const void *f, const void *F,
                       const void *cells, const void *gout, int64_t d,
                       tfi_dtype dtype, void *dF, double *df, void *stream);
int tfi_integrate_expsum_cells(tfi_handle h, int32_t nterm, const void *c,
                               const void *lambda, const void *F, int64_t d,
                               tfi_dtype dtype, void *out, void *cells,
                               void *stream);
int tfi_backward_expsum_cells(tfi_handle h, int32_t nterm, const void *c,
                              const void *lambda, const void *F,
                              const void *cells, const void *gout, int64_t d,
                              tfi_dtype dtype, void *dF, double *s0, double *s1,
                              void *stream);

/*
 * Plan statistics as a JSON object written to the host buffer json[cap]
 * (NUL-terminated, truncated to fit). Returns the full length needed
 * (excluding the NUL), or a negative status.
 */
int64_t tfi_plan_stats(tfi_handle h, char *json, size_t cap);

/*
 * Copy a named plan array to the host buffer buf[cap bytes] for host-side
 * inspection and tests. Returns the array's size in bytes (copying only
 * when buf != NULL and cap is large enough), or a negative status for an
 * unknown name. Names and element types are listed in the plan-stats JSON
 * under "arrays".
 */
int64_t tfi_plan_export(tfi_handle h, const char *name, void *buf,
                        size_t cap);

/*
 * Autotuning of the per-table evaluation method. Each candidate value of
 * the cost constant of tfi_build_opts.fft_cost (0.25, 1, 2, 4, 8, 16, 32,
 * 64) re-assigns every table job to direct sums or FFT, rebuilds the
 * device job lists, and times passes of d channels of dtype with the kernel
 * table f (device, tfi_kernel_length entries) on `stream` (HIP events).
 * with_backward = 0 times forward integrations; with_backward != 0 times a
 * forward integration followed by the adjoint with both dF and df (the
 * work of one training step). The timed fields hold ones. The fastest
 * value stays in effect and is written to *best_cost (host). The kernel
 * length does not change. Uses temporary device memory for three [N x d]
 * fields and one FP64 kernel-length histogram. With the chosen constant it
 * then times both strategies of the cell sums (tfi_set_scatter) and keeps
 * the faster. A handle whose table method was forced at build keeps it (no
 * cost constant is scanned; *best_cost is the handle's constant) and tunes
 * the cell sums only. The FFT kernels' shapes are tuned separately
 * (tfi_autotune_fft).
 * Errors: TFI_ERR_ARG, TFI_ERR_DTYPE, TFI_ERR_STATE, TFI_ERR_HIP,
 * TFI_ERR_BUDGET, TFI_ERR_OOM.
 */
int tfi_autotune(tfi_handle h, const void *f, int64_t d, tfi_dtype dtype,
                 int with_backward, float *best_cost, void *stream);

/* Apply a cost constant (e.g. a cached tuning result) without timing. */
int tfi_set_fft_cost(tfi_handle h, float cost);

/*
 * Strategy of the cell sums b_alpha[r] (equation "stad-E") and A_r[x]
 * (Section 2.2) that every pass forms first:
 *   0  pieces: the incidences in segments of at most 16, runs of 64
 *      segments per workgroup summed through LDS, cells cut between
 *      workgroups added by a second launch (two launches);
 *   1  levels: every segment of at most 32 incidences its own thread group,
 *      longer runs summed level by level (one launch per level);
 *  -1  by width (the default): pieces up to 16 channels, levels above.
 * Both give the same cell sums up to the order of the additions.
 * Errors: TFI_ERR_ARG (method outside [-1, 1]), TFI_ERR_STATE, TFI_ERR_HIP.
 */
int tfi_set_scatter(tfi_handle h, int32_t method);

/*
 * Shapes of the FFT convolution kernels (lemma "stad-2d-fft", algorithm
 * "global-anchor-2dfft"); tfi_autotune picks them by timing. They change
 * how the transforms are blocked, not what they compute: results agree up
 * to rounding order.
 *   lds_pairs[t]      channel pairs transformed together by one workgroup
 *                     of LDS tier t (tables up to 16 KiB, up to 64 KiB,
 *                     larger) for the tier's largest table; smaller tables
 *                     take proportionally more (the same points per
 *                     workgroup). A power of two <= 64, or 0 = enough pairs
 *                     for about 2048 points per workgroup (4096 when d
 *                     exceeds 64 channels). Reduced to the pairs there are
 *                     and to what fits LDS.
 *   conv1d_min_lg     one-row and one-column tables of at least
 *                     2^conv1d_min_lg lattice points take the channel-tiled
 *                     1-D convolution kernels even when they fit LDS
 *                     (default 10; tables beyond LDS always do), in [2, 31].
 *   conv1d_pairs      channel pairs per 1-D tile: 0 = one 128-byte line
 *                     per point (16 FP32 or 8 FP64 pairs), or a power of
 *                     two <= 16 as a cap.
 *   conv1d_group_mib  work buffer of one group of 1-D tiles in MiB (the
 *                     passes run group by group); 0 = 2048.
 *   col_lines         neighbouring columns per workgroup of the blocked
 *                     global passes along the first table axis; a power of
 *                     two <= 64 (default 16).
 * tfi_set_fft_params waits for the device, drops captured launches and,
 * when conv1d_min_lg changes, rebuilds the device job lists.
 * Errors: TFI_ERR_ARG (a field out of range), TFI_ERR_STATE, TFI_ERR_HIP,
 * TFI_ERR_OOM, TFI_ERR_BUDGET.
 */
typedef struct tfi_fft_params {
    int32_t lds_pairs[3];
    int32_t conv1d_min_lg;
    int32_t conv1d_pairs;
    int32_t conv1d_group_mib;
    int32_t col_lines;
} tfi_fft_params;

int tfi_set_fft_params(tfi_handle h, const tfi_fft_params *p);

/* The handle's current FFT kernel shapes (host struct). Errors: TFI_ERR_ARG. */
int tfi_get_fft_params(tfi_handle h, tfi_fft_params *p);

/*
 * Search the FFT kernel shapes (tfi_fft_params) that passes of d channels
 * of dtype run under the handle's current method rule: one parameter at a
 * time (pairs per workgroup of each LDS tier in use, conv1d_min_lg when
 * one-row or one-column FFT tables exist, the 1-D tile width and group
 * buffer when 1-D kernels run, col_lines when blocked global passes run),
 * every candidate timed as in tfi_autotune (kernel table f, fields of ones,
 * `stream`, with_backward as there); the fastest setting stays in effect.
 * Does nothing when the passes run no FFT kernels.
 * Errors: TFI_ERR_ARG, TFI_ERR_DTYPE, TFI_ERR_STATE, TFI_ERR_HIP,
 * TFI_ERR_BUDGET, TFI_ERR_OOM.
 */
int tfi_autotune_fft(tfi_handle h, const void *f, int64_t d, tfi_dtype dtype,
                     int with_backward, void *stream);

/*
 * Measure the channel-aware cost model of TFI_POLICY_CHANNEL on this
 * handle's plan at d channels of dtype (kernel table f: device,
 * tfi_kernel_length entries; fields of ones on `stream`). Two passes are
 * profiled stage by stage: one with every table job evaluated by direct sums
 * (skipped when its direct work, sum over jobs of cells^2 x d, exceeds
 * 4e11 multiply-adds) and one with every table job by FFT. Then
 *   costs[0] = cost_vertex = (scatter + gather time) / (d x incidences),
 *   costs[1] = cost_direct = direct-sum time / (d x sum of cells^2),
 *   costs[2] = cost_fft    = FFT table time / (d x sum of P log2 P),
 *   costs[3] = cost_call   = 0 (the job lists are batched: no per-call
 *                              launch),
 * in seconds (host float[4]); without the direct pass, cost_direct =
 * cost_fft / the handle's fft_cost. The handle's method rule is restored.
 * Uses the temporary device memory of tfi_autotune.
 * Errors: TFI_ERR_ARG, TFI_ERR_DTYPE, TFI_ERR_STATE (host-only handle,
 * method forced at build), TFI_ERR_HIP, TFI_ERR_BUDGET, TFI_ERR_OOM.
 */
int tfi_calibrate(tfi_handle h, const void *f, int64_t d, tfi_dtype dtype, float costs[4],
                  void *stream);

/*
 * Stage timing. With enable != 0, every later tfi_integrate/tfi_backward
 * on the handle records a HIP event pair around each stage (on the same
 * stream as the stage's kernels) and adds the stage's algorithmic bytes
 * (the bytes the stage must move: inputs read once, outputs written once,
 * index arrays; independent of caching) and, for the stages that are
 * dense contractions (direct table sums, dense leaf tiles and their df
 * counterparts), their arithmetic (2 flops per multiply-add over the
 * unpadded cell or vertex pairs; 0 for the other stages) to a per-stage
 * tally.
 * tfi_profile_report waits for the recorded events, writes a JSON object
 * {"stage": {"launches": n, "ms": total, "bytes": total, "flops": total},
 * ...} into
 * json[cap] (truncated to fit), resets the tally and returns the full
 * length needed, or a negative status.
 */
int tfi_profile(tfi_handle h, int enable);
int64_t tfi_profile_report(tfi_handle h, char *json, size_t cap);

/* Release the handle and all its host and device memory. NULL is a no-op.
 * Work enqueued with the handle must have completed. */
void tfi_destroy(tfi_handle h);

/* Message of the last failed call on this thread ("" if none). */
const char *tfi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TFI_H */
