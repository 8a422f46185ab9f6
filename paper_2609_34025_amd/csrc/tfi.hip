// tfi.hip -- runtime and C ABI of libtfi.so (declared in include/tfi.h).
//
// tfi_build plans on the host (plan.cpp) and uploads the plan once.
// tfi_integrate enqueues one forward pass as a small DAG over three
// streams of the handle:
//   main : scatter -> direct tables ----------------> gather
//   side1: kernel spectra -> (after scatter) FFT tables --^
//   side2: leaf tiles (store into out) -------------------^
// joined before the gather, which adds the cross-call terms onto the leaf
// rows. The DAG is captured once per (dtype, d, pointers) into a hipGraph
// and replayed (a small LRU cache of executable graphs per handle).
// tfi_backward runs the same forward on gout for dF (the kernel matrix f(D)
// is symmetric) and the pair histograms for df as a second DAG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>
#include <new>
#include <set>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/tfi.h"
#include "kernels.hpp"
#include "kernels_expsum.hpp"
#include "kernels_conv1d.hpp"
#include "kernels_cells.hpp"
#include "kernels_hankel.hpp"
#include "plan.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define TFI_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(TFI_ERR_HIP, std::string(#call) + ": " +              \
                                         hipGetErrorString(e_));               \
    } while (0)

constexpr int kThreads = 256;
constexpr int kGraphCache = 16;

// Workgroups per job of the per-cell fill and extract kernels (grid-stride
// over the job's cells): about 4096 in all.
inline unsigned cell_blocks(int64_t njobs) {
    return (unsigned)std::max<int64_t>(4, std::min<int64_t>(1024, 4096 / std::max<int64_t>(1, njobs)));
}

inline unsigned blocks_for(int64_t n, int threads = kThreads) {
    return (unsigned)((n + threads - 1) / threads);
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

struct Bucket {
    int lg1 = 0, lg2 = 0;
    int32_t hmax = 0, xmax = 0;
    std::vector<int32_t> jobs;  // pairs [cell_beg, cell_end)
    std::vector<int32_t> hx;    // pairs (H, X) per job
    int32_t* d_jobs = nullptr;
    int32_t* d_hx = nullptr;
    // 1-D buckets for the channel-tiled convolution: per job, the value row of
    // the cell at each coordinate c <= cmax, or -1 (stride mstride = cmax+1).
    // One row (lg1 = 0): c = backbone coordinate x. One column (lg2 = 0,
    // single-position jobs): c = depth r; the source sits at point -r mod P
    // (reflect) and the output at point r.
    int32_t* d_map = nullptr;
    int32_t* d_vmap = nullptr;  // the same with the cell's vertex (whole-path plans)
    int64_t mstride = 0;
    int32_t cmax = 0;
    bool reflect = false;
    int64_t spec_off = 0;       // element offset into the spectrum arena
    int64_t cells = 0;          // table cells over the bucket's jobs
    bool d1 = false;            // per-depth 1-D convolutions (METHOD_FFT1D jobs)
    int tc_cap = 0;             // FftParams::conv1d_pairs
    int64_t group_bytes = 0;    // FftParams::conv1d_group_mib in bytes (0 = kConvGroupBytes)
    int64_t P() const { return (int64_t)1 << (lg1 + lg2); }
    int64_t njobs() const { return (int64_t)jobs.size() / 2; }
};

// FFT buckets that fit LDS are launched together per tier of LDS size.
struct Tier {
    int64_t lds_bytes = 0;      // dynamic LDS of the merged launch
    int64_t nbuckets = 0, njobs = 0;
    int32_t* d_bp = nullptr;    // (lg1, lg2, Hmax, Xmax) per bucket
    int64_t* d_bo = nullptr;    // spectrum offset per bucket
    int32_t* d_fj = nullptr;    // (cell_beg, cell_end, bucket) per job
    double bytes_per_d = 0, bytes_fixed = 0, spec_bytes = 0;
};

struct DeviceBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Shapes of the FFT kernels, set by tfi_set_fft_params or tfi_autotune
// (the fields of tfi_fft_params).
struct FftParams {
    int lds_pairs[3] = {0, 0, 0};  // channel pairs per workgroup of the LDS tiers; 0 = by size
    int conv1d_min_lg = 10;        // one-row/one-column tables of >= 2^this points: 1-D kernels
    int conv1d_pairs = 0;          // channel pairs per 1-D tile; 0 = one 128-byte line
    int conv1d_group_mib = 0;      // 1-D work buffer per group of tiles; 0 = 2048
    int col_lines = 16;            // columns per workgroup of the blocked column passes
};

// Direct-sum tables of a set of jobs: padded cell list (jobs by size),
// per-quad job ranges, blocks of output cells.
struct DirectSet {
    int32_t *d_dl_r = nullptr, *d_dl_x = nullptr, *d_dl_row = nullptr;
    int32_t *d_qjb = nullptr, *d_qje = nullptr, *d_dblk = nullptr;
    int32_t* d_dbin = nullptr;  // per direct block: bound of its pair distances
    int32_t dbin_max = 0;
    int64_t ndirect = 0, ndblk = 0;
    double direct_pairs = 0;  // sum over the jobs of cells^2 (unpadded)
};

// Tables evaluated by the Hankel product and backbone walks
// (kernels_hankel.hpp), in groups whose B rows share one buffer.
struct HankelSet {
    int64_t njobs = 0;
    int64_t* d_jh = nullptr;        // per job: H, X, map offset, B row offset in its group
    int32_t* d_map = nullptr;       // per job: (H + 1) x (X + 1) value rows, or -1
    int32_t* d_bt = nullptr;        // product items (job, t)
    int32_t* d_ln = nullptr;        // walk items (job, line)
    std::vector<int64_t> grp_bt, grp_ln;  // item ranges of the groups
    int64_t max_rows = 0;           // B rows of the largest group
    double pairs = 0;               // Hankel-product multiply-adds per channel
    double cells = 0;               // table cells of the jobs
};

// Pieces of the cell-sum kernel (k_cells): their segments, b-cell and
// A-cell entries, and the cells cut between pieces (see kernels_cells.hpp).
struct CellPlan {
    int64_t npieces = 0, nsegs = 0, nbent = 0, naent = 0;
    int64_t part_rows = 0;  // partial rows of the cells cut between pieces
    int64_t ncomb = 0;      // cells cut between pieces
    int64_t max_rows = 0;   // LDS rows (segments + b-cells) of the largest piece
    int32_t *d_piece = nullptr, *d_seg = nullptr, *d_bent = nullptr, *d_aent = nullptr,
            *d_comb = nullptr;
};

// The cell-sum kernel's arrays on the host (uploaded into CellPlan).
struct CellHost {
    CellPlan stats;
    std::vector<int32_t> piece, seg, bent, aent, comb;
};

struct GraphKey {
    int kind = 0, dtype = 0, n = 0;
    int64_t d = 0;
    const void* p[12] = {};
    bool operator==(const GraphKey& o) const {
        if (kind != o.kind || dtype != o.dtype || n != o.n || d != o.d) return false;
        for (int i = 0; i < 12; ++i)
            if (p[i] != o.p[i]) return false;
        return true;
    }
};

}  // namespace

struct tfi_plan {
    tfi::Plan plan;
    tfi::PlanOptions popt;
    int device = -1;
    uint64_t budget = 0;
    size_t dev_bytes = 0;
    std::vector<void*> allocs;   // plan arrays for the handle's lifetime
    std::vector<void*> mallocs;  // method-dependent arrays (rebuilt on tuning)
    std::vector<size_t> mbytes;

    // plan arrays on the device
    int32_t *d_inc_v = nullptr, *d_jc_r = nullptr, *d_jc_x = nullptr, *d_jc_val = nullptr;
    int64_t* d_v_off = nullptr;
    // direct tables: every direct job (adjoint, cell-keeping forward), and
    // those of the calls the fused call kernel leaves to the table kernels
    DirectSet dall;
    HankelSet hk;                   // Hankel-product tables (METHOD_HANKEL)
    DirectSet dhank;                // the same tables as direct sums, for df
    // cell sums: pieces of the cell-sum kernel
    CellPlan cells;
    // cell sums: levels of bounded segment sums (the other strategy)
    struct SegLevel {
        bool indexed = false;
        int64_t n = 0;
        int64_t* d_src = nullptr;
        int32_t* d_len = nullptr;
        int64_t* d_dst = nullptr;
        int64_t rows_read = 0;
    };
    std::vector<SegLevel> seg_levels;
    // cell-sum strategy: -1 by width (pieces up to 16 channels), 0 pieces,
    // 1 levels (tfi_autotune times both)
    int scatter_pick = -1;
    int64_t val_rows = 0;  // A-cells, b-cells, then partial rows of the levels
    // gather rows, leaf flags and leaf groups
    int32_t *d_ga = nullptr, *d_gb = nullptr, *d_lgrp = nullptr, *d_lq = nullptr;
    int8_t* d_vleaf = nullptr;
    int64_t* d_lgk = nullptr;
    int32_t* d_lbin = nullptr;  // per leaf group: bound of its distances
    int64_t nlgrp = 0;
    // per dtype: every job is a 1-D job beyond LDS whose cells are single
    // vertices held by no other call, with no corrections and no leaf tiles
    // (e.g. a forest of paths, each its own backbone); the convolution kernels
    // then read the field and write the output directly
    bool path_mode[2] = {false, false};
    int64_t gather_reads = 0;  // table values read by the gather
    int32_t *d_leaf_v = nullptr, *d_leaf_D = nullptr;
    std::vector<Bucket> buckets;
    Tier tiers[2][3];               // [float/double][LDS tier]
    std::vector<int> global_b[2];   // buckets beyond LDS, per dtype
    int64_t spec_elems = 0;
    int lgtw = 1;
    void* d_tw[2] = {nullptr, nullptr};  // float / double twiddles
    int64_t lds_max = 65536;        // bytes of LDS a workgroup may use
    FftParams fp;                   // shapes of the FFT kernels (tfi_set_fft_params)

    // per-dtype scratch (grow-only)
    DeviceBuf val[2], g[2], spec[2], fftbuf[2], valg[2], dfbuf[2], part[2], partg[2];
    // exponential sums: per-term power table and f table, sweep scratch,
    // leaf pair histogram (FP64)
    DeviceBuf expw[2], exps[2], hleaf;
    DeviceBuf dfacc;                // fixed-point df accumulator, [2 x kernel length] u64
    // channel tiles of a call over the memory budget: the tile of F (and of
    // gout) and of the result
    DeviceBuf tin[2], tgin[2], tout[2];
    // table jobs for the sweep evaluator: ids sorted by size, cell offsets,
    // first scratch position (-1: one backbone position), signs
    int32_t *d_ej1 = nullptr, *d_ejm = nullptr, *d_jsign = nullptr;
    int64_t *d_joff = nullptr, *d_jpos = nullptr;
    int64_t nej1 = 0, nejm = 0, npos_multi = 0;
    DeviceBuf mrows;    // per-workgroup gradient moments (FP64)

    // streams, fork/join events, graph cache
    hipStream_t s1 = nullptr, s2 = nullptr, cs0 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_a = nullptr, ev_b = nullptr, ev_c = nullptr,
               ev_d = nullptr;
    bool use_graphs = true;
    int direct_kernel = 0;  // 0 auto, 1 vector, 2 matrix cores (FP32)
    struct GraphEntry {
        GraphKey key;
        hipGraphExec_t exec;
        uint64_t last;
    };
    std::vector<GraphEntry> graphs;
    uint64_t tick = 0;

    // stage profiling: event pairs recorded on the launch streams
    struct Tally {
        int64_t launches = 0;
        double ms = 0, bytes = 0, flops = 0;
    };
    struct Pending {
        std::string stage;
        hipEvent_t e0, e1;
        double bytes, flops;
    };
    bool prof = false;
    std::map<std::string, Tally> tally;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;

    hipEvent_t take_event() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    hipEvent_t begin(hipStream_t st) {
        if (!prof) return nullptr;
        hipEvent_t e = take_event();
        if (e) (void)hipEventRecord(e, st);
        return e;
    }
    // bytes: algorithmic HBM bytes of the stage; flops: its arithmetic
    // (2 per multiply-add) where the stage is a contraction, else 0
    void end(hipStream_t st, hipEvent_t e0, const char* stage, double bytes,
             double flops = 0) {
        if (!prof || !e0) return;
        hipEvent_t e1 = take_event();
        if (!e1) return;
        (void)hipEventRecord(e1, st);
        pending.push_back({stage, e0, e1, bytes, flops});
    }

    void drop_graphs() {
        for (auto& g_ : graphs) (void)hipGraphExecDestroy(g_.exec);
        graphs.clear();
    }

    ~tfi_plan() {
        if (device < 0) return;
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess) return;
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize();
        drop_graphs();
        for (auto& q : pending) {
            pool.push_back(q.e0);
            pool.push_back(q.e1);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        for (hipEvent_t e : {ev_fork, ev_a, ev_b, ev_c, ev_d})
            if (e) (void)hipEventDestroy(e);
        for (hipStream_t s : {s1, s2, cs0})
            if (s) (void)hipStreamDestroy(s);
        for (void* p : allocs) (void)hipFree(p);
        for (void* p : mallocs) (void)hipFree(p);
        for (int t = 0; t < 2; ++t)
            for (DeviceBuf* b : {&val[t], &g[t], &spec[t], &fftbuf[t], &valg[t], &dfbuf[t], &part[t],
                                 &partg[t], &expw[t], &exps[t], &tin[t], &tgin[t], &tout[t]})
                if (b->p) (void)hipFree(b->p);
        if (hleaf.p) (void)hipFree(hleaf.p);
        if (dfacc.p) (void)hipFree(dfacc.p);
        if (mrows.p) (void)hipFree(mrows.p);
        (void)hipSetDevice(prev);
    }

    int dalloc(void** p, size_t bytes) {
        if (bytes == 0) bytes = 16;
        if (budget && dev_bytes + bytes > budget)
            return fail(TFI_ERR_BUDGET, "device memory budget exceeded (need " +
                                            std::to_string(dev_bytes + bytes) + " bytes)");
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess)
            return fail(TFI_ERR_OOM, std::string("hipMalloc(") + std::to_string(bytes) +
                                         "): " + hipGetErrorString(e));
        dev_bytes += bytes;
        return TFI_OK;
    }

    template <typename V>
    int upload(V** dst, const std::vector<V>& src) {
        void* p = nullptr;
        int rc = dalloc(&p, src.size() * sizeof(V));
        if (rc) return rc;
        allocs.push_back(p);
        if (!src.empty())
            TFI_HIP(hipMemcpy(p, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
        *dst = (V*)p;
        return TFI_OK;
    }

    template <typename V>
    int upload_m(V** dst, const std::vector<V>& src) {
        void* p = nullptr;
        int rc = dalloc(&p, src.size() * sizeof(V));
        if (rc) return rc;
        mallocs.push_back(p);
        mbytes.push_back(src.empty() ? 16 : src.size() * sizeof(V));  // as dalloc counted
        if (!src.empty())
            TFI_HIP(hipMemcpy(p, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
        *dst = (V*)p;
        return TFI_OK;
    }

    // Every per-call scratch buffer, and their bytes.
    std::vector<DeviceBuf*> scratch_bufs() {
        std::vector<DeviceBuf*> v;
        for (int t = 0; t < 2; ++t)
            for (DeviceBuf* b : {&val[t], &g[t], &spec[t], &fftbuf[t], &valg[t], &dfbuf[t], &part[t],
                                 &partg[t], &expw[t], &exps[t], &tin[t], &tgin[t], &tout[t]})
                v.push_back(b);
        v.push_back(&hleaf);
        v.push_back(&dfacc);
        v.push_back(&mrows);
        return v;
    }
    size_t scratch_bytes() {
        size_t n = 0;
        for (DeviceBuf* b : scratch_bufs()) n += b->p ? b->bytes : 0;
        return n;
    }
    // Release every scratch buffer (after the device drained).
    int free_scratch() {
        TFI_HIP(hipDeviceSynchronize());
        drop_graphs();
        for (DeviceBuf* b : scratch_bufs())
            if (b->p) {
                (void)hipFree(b->p);
                dev_bytes -= b->bytes;
                b->p = nullptr;
                b->bytes = 0;
            }
        return TFI_OK;
    }

    // Release the method-dependent structures (after the device drained).
    int free_methods() {
        TFI_HIP(hipDeviceSynchronize());
        drop_graphs();
        for (size_t i = 0; i < mallocs.size(); ++i) {
            (void)hipFree(mallocs[i]);
            dev_bytes -= mbytes[i];
        }
        mallocs.clear();
        mbytes.clear();
        buckets.clear();
        for (int t = 0; t < 2; ++t) {
            global_b[t].clear();
            path_mode[t] = false;
            for (int k = 0; k < 3; ++k) tiers[t][k] = Tier();
        }
        dall = DirectSet();
        hk = HankelSet();
        dhank = DirectSet();
        spec_elems = 0;
        return TFI_OK;
    }

    // Grow a scratch buffer; graphs that captured the old address are
    // dropped after the device has drained.
    int ensure(DeviceBuf& b, size_t bytes) {
        if (b.bytes >= bytes && b.p) return TFI_OK;
        if (b.p) {
            TFI_HIP(hipDeviceSynchronize());
            drop_graphs();
            TFI_HIP(hipFree(b.p));
            dev_bytes -= b.bytes;
            b.p = nullptr;
            b.bytes = 0;
        }
        int rc = dalloc(&b.p, bytes);
        if (rc) return rc;
        b.bytes = bytes;
        return TFI_OK;
    }
};

namespace {

int check_handle(tfi_handle h, bool need_device) {
    if (!h) return fail(TFI_ERR_ARG, "null handle");
    if (need_device && h->device < 0)
        return fail(TFI_ERR_STATE, "handle was built host-only (opts.device = -1)");
    if (need_device) {
        hipError_t e = hipSetDevice(h->device);
        if (e != hipSuccess)
            return fail(TFI_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    return TFI_OK;
}

template <typename T>
int conv1d_lds_optin(int lds);

// LDS beyond 64 KiB needs an opt-in per kernel. The attribute belongs to
// the kernel in this process on the current device, so it is set once per
// device, not per handle.
int lds_optin_once(int device, int lds) {
    static std::mutex mu;
    static std::set<int> done;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count(device)) return TFI_OK;
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_fft_conv_multi<float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_fft_conv_multi<double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_fft_conv_multi<float, tfi::kPassPad>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_fft_conv_multi<double, tfi::kPassPad>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_spectrum_multi<float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_spectrum_multi<double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_partial<float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_partial<double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_fold<float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_fold<double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_partial<float, tfi::kPassPad>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_partial<double, tfi::kPassPad>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_fold<float, tfi::kPassPad>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_fold<double, tfi::kPassPad>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_partial<float, 0, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_partial<double, 0, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_partial<float, tfi::kPassPad, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_df_fft_partial<double, tfi::kPassPad, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    int rc1 = conv1d_lds_optin<float>(lds);
    if (!rc1) rc1 = conv1d_lds_optin<double>(lds);
    if (rc1) return rc1;
    done.insert(device);
    return TFI_OK;
}

// ---- cell-sum pieces ----------------------------------------------------------
// Segments per piece of the cell-sum kernel.
constexpr int64_t kPieceSegs = 64;

// Pieces of the cell-sum kernel (kernels_cells.hpp): every b-cell cut into
// segments of at most kCallSeg incidences, the segment list of all calls (in
// b-cell order) cut into pieces of kPieceSegs segments; a cell that a
// piece's ends cut is written as partial rows (one per piece holding part of
// it) that the combine launch adds in piece order.
int plan_cells(const tfi::Plan& p, CellHost& H) {
    H = CellHost();
    CellPlan& C = H.stats;
    const int64_t NB = p.NB;
    std::vector<int32_t>&piece = H.piece, &seg = H.seg, &bent = H.bent, &aent = H.aent,
                           &comb = H.comb;
    std::vector<int64_t> bseg0(NB + 1, 0);  // first segment of each b-cell
    for (int64_t b = 0; b < NB; ++b) {
        bseg0[b] = (int64_t)seg.size() / 2;
        for (int64_t i = p.b_inc_off[b]; i < p.b_inc_off[b + 1]; i += tfi::kCallSeg) {
            seg.push_back((int32_t)i);
            seg.push_back((int32_t)std::min<int64_t>(tfi::kCallSeg, p.b_inc_off[b + 1] - i));
        }
    }
    const int64_t nseg = (int64_t)seg.size() / 2;
    bseg0[NB] = nseg;
    for (int64_t b = 0; b < NB; ++b)
        if (bseg0[b + 1] <= bseg0[b])
            return fail(TFI_ERR_STATE, "internal: a b-cell without incidences");
    // cut cells: (0 b-cell / 1 A-cell, id) -> their entries, in piece order
    std::map<std::pair<int, int64_t>, std::vector<int64_t>> cut;
    std::vector<std::pair<int, int64_t>> cut_order;
    int64_t part_rows = 0, mrows = 1, b = 0;
    for (int64_t ps0 = 0; ps0 < nseg; ps0 += kPieceSegs) {
        const int64_t ps1 = std::min(nseg, ps0 + kPieceSegs);
        while (bseg0[b + 1] <= ps0) ++b;  // the b-cell holding segment ps0
        const int64_t e0 = (int64_t)bent.size() / tfi::kCallBEnt,
                      q0 = (int64_t)aent.size() / tfi::kCallAEnt;
        int64_t bb = b;
        for (; bb < NB && bseg0[bb] < ps1; ++bb) {
            const int64_t lo = std::max(bseg0[bb], ps0), hi = std::min(bseg0[bb + 1], ps1);
            bent.insert(bent.end(), {(int32_t)bb, (int32_t)(lo - ps0), (int32_t)(hi - ps0), -1});
            if (lo != bseg0[bb] || hi != bseg0[bb + 1]) {
                const auto key = std::make_pair(0, bb);
                if (!cut.count(key)) cut_order.push_back(key);
                cut[key].push_back((int64_t)bent.size() / tfi::kCallBEnt - 1);
            }
        }
        const int64_t e1 = (int64_t)bent.size() / tfi::kCallBEnt;
        // the A-cells of the b-cells touched (each A-cell is a run of b-cells)
        for (int64_t a = p.b2a[b]; a <= p.b2a[bb - 1]; ++a) {
            const int64_t ab0 = p.a_b_off[a], ab1 = p.a_b_off[a + 1];
            const int64_t alo = std::max<int64_t>(ab0, b) - b, ahi = std::min<int64_t>(ab1, bb) - b;
            aent.insert(aent.end(), {(int32_t)a, (int32_t)alo, (int32_t)ahi, -1});
            if (bseg0[ab0] < ps0 || bseg0[ab1] > ps1) {
                const auto key = std::make_pair(1, a);
                if (!cut.count(key)) cut_order.push_back(key);
                cut[key].push_back((int64_t)aent.size() / tfi::kCallAEnt - 1);
            }
        }
        const int64_t q1 = (int64_t)aent.size() / tfi::kCallAEnt;
        piece.insert(piece.end(), {(int32_t)ps0, (int32_t)ps1, (int32_t)e0, (int32_t)e1,
                                   (int32_t)q0, (int32_t)q1, 0, 0});
        mrows = std::max(mrows, (ps1 - ps0) + (e1 - e0));
    }
    // partial rows of each cut cell, consecutive in piece order
    for (const auto& key : cut_order) {
        const std::vector<int64_t>& ents = cut[key];
        comb.insert(comb.end(), {key.first, (int32_t)key.second, (int32_t)part_rows,
                                 (int32_t)ents.size()});
        for (int64_t ent : ents) {
            if (key.first == 0)
                bent[ent * tfi::kCallBEnt + 3] = (int32_t)part_rows++;
            else
                aent[ent * tfi::kCallAEnt + 3] = (int32_t)part_rows++;
        }
    }
    // pieces by blocks of 2^12 vertex ids (of their first incidence), in
    // order within a block: the pieces of all levels over one region of the
    // forest (one tree of a batch) run together and share its field rows in
    // cache; the kernel gives each XCD a contiguous range of this order
    {
        const int64_t np = (int64_t)piece.size() / tfi::kCallRec;
        std::vector<int64_t> order(np), key(np);
        for (int64_t k = 0; k < np; ++k) {
            order[k] = k;
            key[k] = p.inc_v[seg[2 * (size_t)piece[k * tfi::kCallRec]]] >> 12;
        }
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        std::vector<int32_t> sorted(piece.size());
        for (int64_t k = 0; k < np; ++k)
            std::copy(piece.begin() + order[k] * tfi::kCallRec,
                      piece.begin() + (order[k] + 1) * tfi::kCallRec,
                      sorted.begin() + k * tfi::kCallRec);
        piece.swap(sorted);
    }
    C.npieces = (int64_t)piece.size() / tfi::kCallRec;
    C.nsegs = (int64_t)seg.size() / 2;
    C.nbent = (int64_t)bent.size() / tfi::kCallBEnt;
    C.naent = (int64_t)aent.size() / tfi::kCallAEnt;
    C.part_rows = part_rows;
    C.ncomb = (int64_t)comb.size() / 4;
    C.max_rows = mrows;
    if (part_rows > INT32_MAX || (int64_t)seg.size() > INT32_MAX)
        return fail(TFI_ERR_STATE, "internal: cell-sum indices exceed 32 bits");
    return TFI_OK;
}

int build_cells(tfi_plan* h) {
    CellHost H;
    int rc = plan_cells(h->plan, H);
    if (rc) return rc;
    CellPlan& C = h->cells;
    C = H.stats;
    if ((rc = h->upload(&C.d_piece, H.piece))) return rc;
    if ((rc = h->upload(&C.d_seg, H.seg))) return rc;
    if ((rc = h->upload(&C.d_bent, H.bent))) return rc;
    if ((rc = h->upload(&C.d_aent, H.aent))) return rc;
    if ((rc = h->upload(&C.d_comb, H.comb))) return rc;
    return TFI_OK;
}

int upload_static(tfi_plan* h) {
    const tfi::Plan& p = h->plan;
    int rc;
    if ((rc = h->upload(&h->d_inc_v, p.inc_v))) return rc;
    if ((rc = h->upload(&h->d_v_off, p.v_off))) return rc;
    if ((rc = h->upload(&h->d_jc_r, p.jc_r))) return rc;
    if ((rc = h->upload(&h->d_jc_x, p.jc_x))) return rc;
    if ((rc = h->upload(&h->d_jc_val, p.jc_val))) return rc;
    if ((rc = h->upload(&h->d_leaf_v, p.leaf_v))) return rc;
    if ((rc = h->upload(&h->d_leaf_D, p.leaf_D))) return rc;
    {
        std::vector<int8_t> vleaf(p.N, 0);
        for (int32_t v : p.leaf_v) vleaf[v] = 1;
        if ((rc = h->upload(&h->d_vleaf, vleaf))) return rc;
    }

    int maxlg = 1;
    for (size_t j = 0; j < p.job_lg1.size(); ++j)
        maxlg = std::max(maxlg, std::max(p.job_lg1[j], p.job_lg2[j]));
    // scatter levels: every b-cell and A-cell is a run of incidences; runs
    // longer than kSeg are cut into pieces summed into partial rows, which
    // the next level adds up (again in pieces of at most kSeg)
    {
        constexpr int64_t kSeg = 32;
        struct Seg { int64_t beg, end, dst; };
        std::vector<Seg> cur;
        cur.reserve(p.NA + p.NB);
        for (int64_t b = 0; b < p.NB; ++b)
            cur.push_back({p.b_inc_off[b], p.b_inc_off[b + 1], p.NA + b});
        for (int64_t a = 0; a < p.NA; ++a)
            cur.push_back({p.b_inc_off[p.a_b_off[a]], p.b_inc_off[p.a_b_off[a + 1]], a});
        int64_t next_row = p.NA + p.NB;
        bool indexed = true;
        while (!cur.empty()) {
            std::vector<Seg> next;
            std::vector<std::pair<int64_t, int64_t>> order;  // (len, idx)
            std::vector<int64_t> src, dst;
            std::vector<int32_t> len;
            for (const Seg& sg : cur) {
                const int64_t n = sg.end - sg.beg;
                if (n <= kSeg) {
                    src.push_back(sg.beg);
                    len.push_back((int32_t)n);
                    dst.push_back(sg.dst);
                    continue;
                }
                const int64_t np = (n + kSeg - 1) / kSeg, r0 = next_row;
                next_row += np;
                for (int64_t q = 0; q < np; ++q) {
                    src.push_back(sg.beg + q * kSeg);
                    len.push_back((int32_t)std::min(kSeg, n - q * kSeg));
                    dst.push_back(r0 + q);
                }
                next.push_back({r0, r0 + np, sg.dst});
            }
            // longest segments first so that a wavefront's lanes finish
            // together; the field-row level goes by blocks of 2^12 vertex
            // ids first (the first row's vertex), so that the cells of all
            // levels over one region of the forest (one tree of a batch)
            // run together and share its rows in cache. The order does not
            // change any sum.
            std::vector<int64_t> perm(src.size());
            for (size_t k = 0; k < perm.size(); ++k) perm[k] = (int64_t)k;
            if (indexed) {
                std::vector<int32_t> vblk(src.size());
                for (size_t k = 0; k < src.size(); ++k) vblk[k] = p.inc_v[src[k]] >> 12;
                std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) {
                    return vblk[a] != vblk[b] ? vblk[a] < vblk[b] : len[a] > len[b];
                });
            } else {
                std::stable_sort(perm.begin(), perm.end(),
                                 [&](int64_t a, int64_t b) { return len[a] > len[b]; });
            }
            std::vector<int64_t> s2(src.size()), d2(src.size());
            std::vector<int32_t> l2(src.size());
            int64_t rows = 0;
            for (size_t k = 0; k < perm.size(); ++k) {
                s2[k] = src[perm[k]];
                l2[k] = len[perm[k]];
                d2[k] = dst[perm[k]];
                rows += l2[k];
            }
            tfi_plan::SegLevel L;
            L.indexed = indexed;
            L.n = (int64_t)s2.size();
            L.rows_read = rows;
            if ((rc = h->upload(&L.d_src, s2))) return rc;
            if ((rc = h->upload(&L.d_len, l2))) return rc;
            if ((rc = h->upload(&L.d_dst, d2))) return rc;
            h->seg_levels.push_back(L);
            cur.swap(next);
            indexed = false;
        }
        h->val_rows = next_row;
    }
    // cell sums, the other strategy: pieces of the cell-sum kernel
    if ((rc = build_cells(h))) return rc;

    // gather: table row and correction row (or -1) per vertex incidence
    {
        std::vector<int32_t> ga(p.v_b.size()), gb(p.v_b.size());
        h->gather_reads = 0;
        for (size_t k = 0; k < p.v_b.size(); ++k) {
            const int32_t b = p.v_b[k];
            ga[k] = p.b2a[b];
            gb[k] = p.b_corr[b] ? (int32_t)(p.NA + b) : -1;
            h->gather_reads += 1 + (p.b_corr[b] ? 1 : 0);
        }
        if ((rc = h->upload(&h->d_ga, ga))) return rc;
        if ((rc = h->upload(&h->d_gb, gb))) return rc;
    }
    // leaf quads (4 vertices of one tile) and groups of consecutive tiles
    // within the kernel's LDS limits
    {
        std::vector<int32_t> lq, grp{0};
        std::vector<int64_t> gk;
        std::vector<int32_t> lbin;  // per group: 1 + largest distance in its tiles
        const int64_t nt = (int64_t)p.leaf_off.size() - 1;
        int64_t t = 0;
        while (t < nt) {
            const int64_t dbase = p.leaf_doff[t];
            int64_t quads = 0, verts = 0, kk = 0, e = t;
            while (e < nt) {
                const int64_t n = p.leaf_off[e + 1] - p.leaf_off[e];
                const int64_t nq = (n + 3) / 4;
                if (e > t && (quads + nq > tfi::kLeafQuads || verts + n > tfi::kLeafSlots ||
                              kk + n * n > tfi::kLeafK))
                    break;
                const int32_t tb = (int32_t)p.leaf_off[e];
                const int32_t koff = (int32_t)(p.leaf_doff[e] - dbase);
                for (int64_t q = 0; q < nq; ++q) {
                    lq.push_back(tb + (int32_t)(4 * q));
                    lq.push_back(tb);
                    lq.push_back((int32_t)n);
                    lq.push_back(koff + (int32_t)(4 * q * n));
                }
                quads += nq;
                verts += n;
                kk += n * n;
                ++e;
            }
            grp.push_back((int32_t)(lq.size() / 4));
            gk.push_back(dbase);
            gk.push_back(kk);
            int32_t dmax = 0;
            for (int64_t u = dbase; u < dbase + kk; ++u) dmax = std::max(dmax, p.leaf_D[u]);
            lbin.push_back((int32_t)std::min<int64_t>((int64_t)dmax + 1, p.kernel_len));
            t = e;
        }
        h->nlgrp = (int64_t)grp.size() - 1;
        if ((rc = h->upload(&h->d_lgrp, grp))) return rc;
        if ((rc = h->upload(&h->d_lq, lq))) return rc;
        if ((rc = h->upload(&h->d_lgk, gk))) return rc;
        if ((rc = h->upload(&h->d_lbin, lbin))) return rc;
    }
    if (h->lds_max > 65536) {
        const int rc1 = lds_optin_once(h->device, (int)h->lds_max);
        if (rc1) return rc1;
    }
    // sweep evaluator job lists (exponential-sum kernels)
    {
        const int64_t J = (int64_t)p.job_H.size();
        std::vector<int32_t> ej1, ejm;  // one backbone position / several
        std::vector<int64_t> jpos(J, -1);
        int64_t npos = 0;
        for (int64_t j = 0; j < J; ++j) {
            const int64_t cb = p.job_cell_off[j], ce = p.job_cell_off[j + 1];
            if (ce <= cb) continue;
            int64_t np = 1;
            for (int64_t i = cb + 1; i < ce; ++i) {
                if (p.jc_x[i] < p.jc_x[i - 1])
                    return fail(TFI_ERR_STATE, "internal: job cells not sorted by position");
                np += p.jc_x[i] != p.jc_x[i - 1];
            }
            if (np > 1) {
                jpos[j] = npos;
                npos += np;
                ejm.push_back((int32_t)j);
            } else {
                ej1.push_back((int32_t)j);
            }
        }
        auto by_size = [&](int32_t a, int32_t b) {
            return p.job_cell_off[a + 1] - p.job_cell_off[a] >
                   p.job_cell_off[b + 1] - p.job_cell_off[b];
        };
        std::stable_sort(ej1.begin(), ej1.end(), by_size);
        std::stable_sort(ejm.begin(), ejm.end(), by_size);
        h->nej1 = (int64_t)ej1.size();
        h->nejm = (int64_t)ejm.size();
        h->npos_multi = npos;
        if ((rc = h->upload(&h->d_ej1, ej1))) return rc;
        if ((rc = h->upload(&h->d_ejm, ejm))) return rc;
        if ((rc = h->upload(&h->d_joff, p.job_cell_off))) return rc;
        if ((rc = h->upload(&h->d_jpos, jpos))) return rc;
        if ((rc = h->upload(&h->d_jsign, p.job_sign))) return rc;
    }
    // twiddles exp(-2 pi i k / 2^lgtw), k < 2^(lgtw-1), from long double
    h->lgtw = maxlg;
    const int64_t TW = (int64_t)1 << h->lgtw, nt = TW / 2;
    std::vector<tfi::cpx<float>> twf(nt);
    std::vector<tfi::cpx<double>> twd(nt);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int64_t k = 0; k < nt; ++k) {
        long double a = -2.0L * pi * (long double)k / (long double)TW;
        twd[k] = {(double)cosl(a), (double)sinl(a)};
        twf[k] = {(float)cosl(a), (float)sinl(a)};
    }
    tfi::cpx<float>* tf = nullptr;
    tfi::cpx<double>* td = nullptr;
    if ((rc = h->upload(&tf, twf))) return rc;
    if ((rc = h->upload(&td, twd))) return rc;
    h->d_tw[0] = tf;
    h->d_tw[1] = td;
    // side streams (default priority) and fork/join events
    TFI_HIP(hipStreamCreateWithFlags(&h->s1, hipStreamNonBlocking));
    TFI_HIP(hipStreamCreateWithFlags(&h->s2, hipStreamNonBlocking));
    TFI_HIP(hipStreamCreateWithFlags(&h->cs0, hipStreamNonBlocking));
    for (hipEvent_t* e :
         {&h->ev_fork, &h->ev_a, &h->ev_b, &h->ev_c, &h->ev_d})
        TFI_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return TFI_OK;
}

// Device structures that depend on the per-job method (direct blocks, FFT
// buckets and their LDS tiers); rebuilt when the methods are re-assigned.
// LDS beyond 64 KiB for the 1-D convolution kernels of every channel tile.
template <typename T, int TC, int LG>
int conv1d_lds_optin_lg(int lds) {
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_conv1d_hi<T, TC, false, LG>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_conv1d_hi<T, TC, true, LG>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_conv1d_lo<T, TC, LG>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    return TFI_OK;
}

// Block splits compiled with fixed sizes (straight-line register stages):
// FP32 with full-line tiles, blocks of 2^5 .. 2^10 points, and FP32 with
// half-line tiles at the 2^10 x 2^10 split of 2^20-point tables (whose
// full-line blocks would pass 64 KiB of LDS). FP64 at these sizes runs out
// of registers unrolled and keeps the runtime split.
constexpr int kC1FixedMin = 5, kC1FixedMax = 10;
template <typename T, int TC>
constexpr bool conv1d_fixed() {
    return std::is_same<T, float>::value && TC == 16;
}
template <typename T, int TC>
constexpr bool conv1d_fixed_half() {
    return std::is_same<T, float>::value && TC == 8;
}

template <typename T, int TC>
int conv1d_lds_optin_tc(int lds) {
    int rc = conv1d_lds_optin_lg<T, TC, 0>(lds);
    if constexpr (conv1d_fixed<T, TC>()) {
        if (!rc) rc = conv1d_lds_optin_lg<T, TC, 5>(lds);
        if (!rc) rc = conv1d_lds_optin_lg<T, TC, 6>(lds);
        if (!rc) rc = conv1d_lds_optin_lg<T, TC, 7>(lds);
        if (!rc) rc = conv1d_lds_optin_lg<T, TC, 8>(lds);
        if (!rc) rc = conv1d_lds_optin_lg<T, TC, 9>(lds);
        if (!rc) rc = conv1d_lds_optin_lg<T, TC, 10>(lds);
        if (!rc)
            TFI_HIP(hipFuncSetAttribute((const void*)tfi::k_conv1d_lo<T, TC, 10, TC / 2>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    }
    if constexpr (conv1d_fixed_half<T, TC>()) {
        if (!rc) rc = conv1d_lds_optin_lg<T, TC, 10>(lds);
    }
    return rc;
}

template <typename T>
int conv1d_lds_optin(int lds) {
    int rc = conv1d_lds_optin_tc<T, 16>(lds);
    if (!rc) rc = conv1d_lds_optin_tc<T, 8>(lds);
    if (!rc) rc = conv1d_lds_optin_tc<T, 4>(lds);
    if (!rc) rc = conv1d_lds_optin_tc<T, 2>(lds);
    if (!rc) rc = conv1d_lds_optin_tc<T, 1>(lds);
    return rc;
}

// Plan shape of whole-path mode: no leaf tiles, every vertex in exactly one
// b-cell of one incidence, no corrections, every A-cell one b-cell, and every
// job a call job of one row (H = 0) evaluated by FFT.
bool whole_path_plan(const tfi::Plan& p) {
    if (p.leaf_off.size() > 1 || p.NB != p.N || p.NA != p.NB) return false;
    for (int64_t v = 0; v < p.N; ++v)
        if (p.v_off[v + 1] - p.v_off[v] != 1) return false;
    for (int64_t b = 0; b < p.NB; ++b)
        if (p.b_corr[b] || p.b_inc_off[b + 1] - p.b_inc_off[b] != 1) return false;
    for (int64_t a = 0; a < p.NA; ++a)
        if (p.a_b_off[a + 1] - p.a_b_off[a] != 1) return false;
    for (size_t j = 0; j < p.job_sign.size(); ++j)
        if (p.job_sign[j] != 1 || p.job_lg1[j] != 0 || p.job_method[j] != tfi::METHOD_FFT)
            return false;
    return true;
}

// Direct tables of a list of jobs: jobs sorted by size (largest first) so
// that lanes of a wavefront run equal loops, each padded to whole quads of 4
// cells (padding: r = x = 0, row -1); blocks pack whole jobs up to kDirOut
// cells, larger jobs are cut into kDirOut-cell output slices whose sources
// are the whole job.
int build_direct(tfi_plan* h, std::vector<int64_t> djobs, DirectSet& ds) {
    const tfi::Plan& p = h->plan;
    int rc;
    ds = DirectSet();
    std::stable_sort(djobs.begin(), djobs.end(), [&](int64_t a, int64_t b) {
        return p.job_cell_off[a + 1] - p.job_cell_off[a] >
               p.job_cell_off[b + 1] - p.job_cell_off[b];
    });
    std::vector<int32_t> dl_r, dl_x, dl_row, qjb, qje, dblk, dbin;
    std::vector<std::pair<int32_t, int32_t>> jr;  // padded job ranges
    std::vector<int32_t> jbin;                    // per job: 1 + largest pair distance
    for (int64_t j : djobs) {
        const int32_t cb = (int32_t)p.job_cell_off[j], ce = (int32_t)p.job_cell_off[j + 1];
        const int32_t jb = (int32_t)dl_r.size();
        const int32_t n = ce - cb, np = (n + 3) & ~3;
        ds.direct_pairs += (double)n * n;
        {
            int32_t rmax = 0, xmin = INT32_MAX, xmax = INT32_MIN;
            for (int32_t i = cb; i < ce; ++i) {
                rmax = std::max(rmax, p.jc_r[i]);
                xmin = std::min(xmin, p.jc_x[i]);
                xmax = std::max(xmax, p.jc_x[i]);
            }
            const int64_t b = n > 0 ? 2 * (int64_t)rmax + (xmax - xmin) + 1 : 1;
            jbin.push_back((int32_t)std::min<int64_t>(b, p.kernel_len));
        }
        for (int32_t i = 0; i < np; ++i) {
            const bool real = i < n;
            dl_r.push_back(real ? p.jc_r[cb + i] : 0);
            dl_x.push_back(real ? p.jc_x[cb + i] : 0);
            dl_row.push_back(real ? p.jc_val[cb + i] : -1);
        }
        const int32_t je = jb + np;
        for (int32_t q = 0; q < np / 4; ++q) {
            qjb.push_back(jb);
            qje.push_back(je);
        }
        jr.emplace_back(jb, je);
    }
    size_t k = 0;
    while (k < jr.size()) {
        const int32_t jb = jr[k].first, je = jr[k].second;
        if (je - jb > tfi::kDirOut) {
            for (int32_t o = jb; o < je; o += tfi::kDirOut) {
                dblk.insert(dblk.end(), {o, std::min(je, o + tfi::kDirOut), jb, je});
                dbin.push_back(jbin[k]);
            }
            ++k;
            continue;
        }
        size_t e = k + 1;
        while (e < jr.size() && jr[e].second - jb <= tfi::kDirOut) ++e;
        const int32_t end = jr[e - 1].second;
        dblk.insert(dblk.end(), {jb, end, jb, end});
        int32_t bmax = 1;
        for (size_t u = k; u < e; ++u) bmax = std::max(bmax, jbin[u]);
        dbin.push_back(bmax);
        k = e;
    }
    ds.ndirect = (int64_t)dl_r.size();
    ds.ndblk = (int64_t)dblk.size() / 4;
    if ((rc = h->upload_m(&ds.d_dl_r, dl_r))) return rc;
    if ((rc = h->upload_m(&ds.d_dl_x, dl_x))) return rc;
    if ((rc = h->upload_m(&ds.d_dl_row, dl_row))) return rc;
    if ((rc = h->upload_m(&ds.d_qjb, qjb))) return rc;
    if ((rc = h->upload_m(&ds.d_qje, qje))) return rc;
    if ((rc = h->upload_m(&ds.d_dblk, dblk))) return rc;
    if ((rc = h->upload_m(&ds.d_dbin, dbin))) return rc;
    ds.dbin_max = dbin.empty() ? 0 : *std::max_element(dbin.begin(), dbin.end());
    return TFI_OK;
}

// B rows of one group of Hankel tables (a larger table is a group alone).
constexpr int64_t kHankGroupRows = (int64_t)1 << 21;

int build_hankel(tfi_plan* h, const std::vector<int64_t>& hjobs) {
    const tfi::Plan& p = h->plan;
    HankelSet& k = h->hk;
    k = HankelSet();
    if (hjobs.empty()) return TFI_OK;
    std::vector<int64_t> jh;
    std::vector<int32_t> map, bt, ln;
    int64_t rows_in = 0;
    k.grp_bt.push_back(0);
    k.grp_ln.push_back(0);
    auto close = [&]() {
        k.grp_bt.push_back((int64_t)bt.size() / 2);
        k.grp_ln.push_back((int64_t)ln.size() / 2);
        k.max_rows = std::max(k.max_rows, rows_in);
        rows_in = 0;
    };
    for (int64_t j : hjobs) {
        const int32_t H = p.job_H[j], X = p.job_X[j];
        const int64_t rows = (int64_t)(H + X + 1) * (X + 1);
        if (H > tfi::kHankHmax || H < 0 || X < 0)
            return fail(TFI_ERR_STATE, "Hankel table outside the kernel's limits");
        if (rows_in > 0 && rows_in + rows > kHankGroupRows) close();
        const int64_t mapoff = (int64_t)map.size();
        map.resize((size_t)(mapoff + (int64_t)(H + 1) * (X + 1)), -1);
        for (int64_t c = p.job_cell_off[j]; c < p.job_cell_off[j + 1]; ++c) {
            if (p.jc_r[c] < 0 || p.jc_r[c] > H || p.jc_x[c] < 0 || p.jc_x[c] > X)
                return fail(TFI_ERR_STATE, "Hankel table cell outside its job's range");
            map[(size_t)(mapoff + (int64_t)p.jc_r[c] * (X + 1) + p.jc_x[c])] = p.jc_val[c];
        }
        const int32_t jid = (int32_t)(jh.size() / 4);
        jh.insert(jh.end(), {(int64_t)H, (int64_t)X, mapoff, rows_in});
        for (int32_t t = 0; t <= X; ++t) bt.insert(bt.end(), {jid, t});
        for (int32_t l = 0; l <= H + X; ++l) ln.insert(ln.end(), {jid, l});
        rows_in += rows;
        k.pairs += (double)(H + X + 1) * (H + 1) * (X + 1);
        k.cells += (double)(p.job_cell_off[j + 1] - p.job_cell_off[j]);
    }
    close();
    k.njobs = (int64_t)hjobs.size();
    int rc;
    if ((rc = h->upload_m(&k.d_jh, jh))) return rc;
    if ((rc = h->upload_m(&k.d_map, map))) return rc;
    if ((rc = h->upload_m(&k.d_bt, bt))) return rc;
    if ((rc = h->upload_m(&k.d_ln, ln))) return rc;
    return TFI_OK;
}

int upload_methods(tfi_plan* h) {
    const tfi::Plan& p = h->plan;
    int rc;
    std::vector<int64_t> djobs;  // direct-method jobs
    std::vector<int64_t> hjobs;  // Hankel-product jobs
    std::map<std::tuple<int, int, bool>, size_t> bidx;
    const int64_t J = (int64_t)p.job_H.size();
    for (int64_t j = 0; j < J; ++j) {
        const int32_t cb = (int32_t)p.job_cell_off[j], ce = (int32_t)p.job_cell_off[j + 1];
        if (p.job_method[j] == tfi::METHOD_DIRECT) {
            djobs.push_back(j);
        } else if (p.job_method[j] == tfi::METHOD_HANKEL) {
            hjobs.push_back(j);
        } else {
            const bool d1 = p.job_method[j] == tfi::METHOD_FFT1D;
            auto key = std::make_tuple((int)p.job_lg1[j], (int)p.job_lg2[j], d1);
            auto it = bidx.find(key);
            if (it == bidx.end()) {
                it = bidx.emplace(key, h->buckets.size()).first;
                Bucket b;
                b.lg1 = std::get<0>(key);
                b.lg2 = std::get<1>(key);
                b.d1 = d1;
                b.tc_cap = h->fp.conv1d_pairs;
                b.group_bytes = (int64_t)h->fp.conv1d_group_mib << 20;
                h->buckets.push_back(b);
            }
            Bucket& b = h->buckets[it->second];
            b.hmax = std::max(b.hmax, p.job_H[j]);
            b.xmax = std::max(b.xmax, p.job_X[j]);
            b.jobs.push_back(cb);
            b.jobs.push_back(ce);
            b.hx.push_back(p.job_H[j]);
            b.hx.push_back(p.job_X[j]);
            b.cells += ce - cb;
        }
    }
    if ((rc = build_direct(h, djobs, h->dall))) return rc;
    if ((rc = build_hankel(h, hjobs))) return rc;
    if ((rc = build_direct(h, hjobs, h->dhank))) return rc;

    h->spec_elems = 0;
    for (Bucket& b : h->buckets) {
        if ((rc = h->upload_m(&b.d_jobs, b.jobs))) return rc;
        if ((rc = h->upload_m(&b.d_hx, b.hx))) return rc;
        b.spec_off = h->spec_elems;
        h->spec_elems += b.P();
    }
    // LDS tiers per dtype: up to 16 KiB, up to 64 KiB, up to the device
    // limit; larger tables take the global-memory passes
    for (int ti = 0; ti < 2; ++ti) {
        const int64_t cs = ti ? (int64_t)sizeof(tfi::cpx<double>) : (int64_t)sizeof(tfi::cpx<float>);
        const int64_t lim[3] = {16384, 65536, h->lds_max};
        std::vector<int32_t> bp[3], fj[3];
        std::vector<int64_t> bo[3];
        for (size_t bi = 0; bi < h->buckets.size(); ++bi) {
            const Bucket& b = h->buckets[bi];
            const int64_t bytes = b.P() * cs;
            int t = 0;
            while (t < 3 && bytes > lim[t]) ++t;
            // long 1-D tables take the channel-tiled convolution kernels even
            // when one channel pair would fit LDS (the LDS kernels read one
            // pair per workgroup: 8 bytes of every row)
            if ((b.lg1 == 0 || b.lg2 == 0) && b.lg1 + b.lg2 >= h->fp.conv1d_min_lg) t = 3;
            if (b.d1) t = 3;  // the per-depth path runs through global memory
            if (t == 3) {
                h->global_b[ti].push_back((int)bi);
                continue;
            }
            Tier& T = h->tiers[ti][t];
            const int32_t local = (int32_t)(bp[t].size() / 4);
            bp[t].insert(bp[t].end(), {b.lg1, b.lg2, b.hmax, b.xmax});
            bo[t].push_back(b.spec_off);
            for (int64_t j = 0; j < b.njobs(); ++j)
                fj[t].insert(fj[t].end(), {b.jobs[2 * j], b.jobs[2 * j + 1], local});
            T.lds_bytes = std::max(T.lds_bytes, bytes);
            T.bytes_per_d += 2.0 * (double)b.cells;
            T.bytes_fixed += 12.0 * (double)b.cells;
            T.spec_bytes += 2.0 * (double)b.P();
        }
        for (int bi : h->global_b[ti]) {
            Bucket& b = h->buckets[bi];
            if ((b.lg1 != 0 && b.lg2 != 0) || b.d_map) continue;
            const bool col = b.lg1 != 0;  // one column: cells by depth
            const int32_t cmax = col ? b.hmax : b.xmax;
            std::vector<int32_t> map((size_t)b.njobs() * (cmax + 1), -1);
            bool ok = true;
            for (int64_t j = 0; j < b.njobs() && ok; ++j)
                for (int32_t k = b.jobs[2 * j]; k < b.jobs[2 * j + 1]; ++k) {
                    const int32_t c = col ? p.jc_r[k] : p.jc_x[k];
                    const int32_t other = col ? p.jc_x[k] : p.jc_r[k];
                    if (other != 0 || c < 0 || c > cmax) {
                        ok = false;
                        break;
                    }
                    map[(size_t)j * (cmax + 1) + c] = p.jc_val[k];
                }
            if (!ok) continue;
            if ((rc = h->upload_m(&b.d_map, map))) return rc;
            b.mstride = cmax + 1;
            b.cmax = cmax;
            b.reflect = col;
        }
        h->path_mode[ti] = fj[0].empty() && fj[1].empty() && fj[2].empty() &&
                           h->dall.ndirect == 0 && whole_path_plan(p);
        for (int bi : h->global_b[ti])
            if (!h->buckets[bi].d_map) h->path_mode[ti] = false;
        if (h->path_mode[ti])
            for (int bi : h->global_b[ti]) {
                Bucket& b = h->buckets[bi];
                if (b.d_vmap) continue;
                std::vector<int32_t> vmap((size_t)b.njobs() * b.mstride, -1);
                for (int64_t j = 0; j < b.njobs(); ++j)
                    for (int32_t k = b.jobs[2 * j]; k < b.jobs[2 * j + 1]; ++k) {
                        const int32_t a = p.jc_val[k];
                        vmap[(size_t)j * b.mstride + p.jc_x[k]] =
                            p.inc_v[p.b_inc_off[p.a_b_off[a]]];
                    }
                if ((rc = h->upload_m(&b.d_vmap, vmap))) return rc;
            }
        for (int t = 0; t < 3; ++t) {
            Tier& T = h->tiers[ti][t];
            T.nbuckets = (int64_t)bo[t].size();
            T.njobs = (int64_t)fj[t].size() / 3;
            if (!T.nbuckets) continue;
            if ((rc = h->upload_m(&T.d_bp, bp[t]))) return rc;
            if ((rc = h->upload_m(&T.d_bo, bo[t]))) return rc;
            if ((rc = h->upload_m(&T.d_fj, fj[t]))) return rc;
        }
    }
    return TFI_OK;
}

int upload_plan(tfi_plan* h) {
    int rc = upload_static(h);
    if (rc) return rc;
    return upload_methods(h);
}

// Cell sums of the rows of `src` ([N x d]) into val: A-cells, b-cells and
// the partial rows of long runs.
// Column tile, in groups of vec channels, of the row kernels (scatter,
// gather): a 256-byte slice for rows wider than 512 bytes, else the whole
// row; and the thread count that covers nrows rows in such tiles.
template <typename T>
int32_t col_tile(int32_t d, int vec) {
    const int32_t dv = d / vec;
    if ((int64_t)d * (int64_t)sizeof(T) <= 512) return dv;
    return std::max<int32_t>(1, 256 / (vec * (int32_t)sizeof(T)));
}

inline int64_t tiled_threads(int64_t nrows, int32_t dv, int32_t ct) {
    return (int64_t)((dv + ct - 1) / ct) * nrows * ct;
}

// Threads per row (up to 16) and VEC of the cell-sum kernel at d channels:
// chunks of up to 64 channels.
inline void cell_shape(int32_t d, bool v4, int* lanes, int* vec) {
    *vec = v4 ? 4 : 1;
    const int32_t w = std::min<int32_t>(64, d);
    const int32_t need = w / *vec + (w % *vec != 0);
    int l = 1;
    while (l < need) l <<= 1;
    *lanes = std::min(l, 16);
}

// Cell sums of the rows of src ([N x d]) into val: A-cells at rows
// [0, NA), b-cells at NA + b (kernels_cells.hpp); part holds the partial
// rows of the cells cut between pieces (part_rows x d).
template <typename T>
void launch_scatter_pieces(tfi_plan* h, const T* src, T* val, T* part, int32_t d,
                           hipStream_t st) {
    const CellPlan& C = h->cells;
    if (C.npieces == 0) return;
    const tfi::Plan& p = h->plan;
    hipEvent_t ev = h->begin(st);
    const bool v4 = d % 4 == 0 && aligned16(src);
    int lanes = 1, vec = 1;
    cell_shape(d, v4, &lanes, &vec);
    const unsigned lds = (unsigned)((size_t)C.max_rows * lanes * vec * sizeof(T));
    if (v4)
        hipLaunchKernelGGL((tfi::k_cells<T, 4>), dim3((unsigned)C.npieces), dim3(tfi::kCallThreads),
                           lds, st, d, (int32_t)lanes, C.d_piece, C.d_seg, C.d_bent, C.d_aent,
                           h->d_inc_v, src, (int64_t)p.NA, part, val);
    else
        hipLaunchKernelGGL((tfi::k_cells<T, 1>), dim3((unsigned)C.npieces), dim3(tfi::kCallThreads),
                           lds, st, d, (int32_t)lanes, C.d_piece, C.d_seg, C.d_bent, C.d_aent,
                           h->d_inc_v, src, (int64_t)p.NA, part, val);
    const double sz = (double)sizeof(T);
    h->end(st, ev, "scatter",
           sz * d * ((double)p.incidences + (double)(C.nbent + C.naent)) + 4.0 * p.incidences +
               8.0 * C.nsegs + 16.0 * (C.nbent + C.naent) + 4.0 * tfi::kCallRec * C.npieces);
    if (C.ncomb > 0) {  // cells cut between pieces: their partial rows in order
        hipEvent_t ev2 = h->begin(st);
        const dim3 grid(blocks_for(C.ncomb * lanes, tfi::kCallThreads));
        if (v4)
            hipLaunchKernelGGL((tfi::k_cells_combine<T, 4>), grid, dim3(tfi::kCallThreads), 0, st,
                               d, (int32_t)lanes, (int32_t)C.ncomb, C.d_comb, (const T*)part, val,
                               (int64_t)p.NA);
        else
            hipLaunchKernelGGL((tfi::k_cells_combine<T, 1>), grid, dim3(tfi::kCallThreads), 0, st,
                               d, (int32_t)lanes, (int32_t)C.ncomb, C.d_comb, (const T*)part, val,
                               (int64_t)p.NA);
        h->end(st, ev2, "scatter_combine",
               sz * d * ((double)C.part_rows + (double)C.ncomb) + 16.0 * C.ncomb);
    }
}

// Cell sums by levels of bounded segment sums (k_segsum): field rows per
// segment of at most 32 incidences, then partial rows level by level.
template <typename T>
void launch_scatter_levels(tfi_plan* h, const T* src, T* val, int32_t d, hipStream_t st) {
    const double sz = (double)sizeof(T);
    for (size_t l = 0; l < h->seg_levels.size(); ++l) {
        const tfi_plan::SegLevel& L = h->seg_levels[l];
        hipEvent_t ev = h->begin(st);
        const bool v4 = (d % 4 == 0) && (L.indexed ? aligned16(src) : aligned16(val));
        const int vec = v4 ? 4 : 1;
        const int32_t ct = col_tile<T>(d, vec);
        const int64_t nt = tiled_threads(L.n, d / vec, ct);
        if (L.indexed && v4)
            hipLaunchKernelGGL((tfi::k_segsum<T, true, 4>), dim3(blocks_for(nt)), dim3(kThreads),
                               0, st, L.n, d, ct, L.d_src, L.d_len, L.d_dst, h->d_inc_v, src, val);
        else if (L.indexed)
            hipLaunchKernelGGL((tfi::k_segsum<T, true, 1>), dim3(blocks_for(nt)), dim3(kThreads),
                               0, st, L.n, d, ct, L.d_src, L.d_len, L.d_dst, h->d_inc_v, src, val);
        else if (v4)
            hipLaunchKernelGGL((tfi::k_segsum<T, false, 4>), dim3(blocks_for(nt)),
                               dim3(kThreads), 0, st, L.n, d, ct, L.d_src, L.d_len, L.d_dst,
                               (const int32_t*)nullptr, (const T*)val, val);
        else
            hipLaunchKernelGGL((tfi::k_segsum<T, false, 1>), dim3(blocks_for(nt)),
                               dim3(kThreads), 0, st, L.n, d, ct, L.d_src, L.d_len, L.d_dst,
                               (const int32_t*)nullptr, (const T*)val, val);
        h->end(st, ev, l == 0 ? "scatter" : "scatter_tail",
               sz * d * (double)(L.rows_read + L.n) + (L.indexed ? 4.0 * L.rows_read : 0.0) +
                   20.0 * L.n);
    }
}

// Whether the cell sums at d channels go through the pieces (k_cells) or
// the levels (k_segsum): pieces put fewer launches and round trips on the
// chain and suit larger cells; levels run every segment as its own thread
// group and suit many tiny cells at wide rows. tfi_autotune times both.
inline bool scatter_pieces(const tfi_plan* h, int32_t d) {
    return h->scatter_pick >= 0 ? h->scatter_pick == 0 : d <= 16;
}

// Cell sums of the rows of src ([N x d]) into val (A-cells at [0, NA),
// b-cells at NA + b); part: partial rows of the pieces.
template <typename T>
void launch_scatter(tfi_plan* h, const T* src, T* val, T* part, int32_t d, hipStream_t st) {
    if (scatter_pieces(h, d))
        launch_scatter_pieces<T>(h, src, val, part, d, st);
    else
        launch_scatter_levels<T>(h, src, val, d, st);
}

// Pass schedule of a transform along an axis of 2^lgL points, 2^lgN
// neighbouring lines per workgroup: at most 2^lgW points per workgroup, as
// groups of index bits with 16 consecutive low indices per workgroup (rows,
// lgN = 0) or with the lines giving the contiguous runs (columns), or one
// pass when the axis fits. Listed in DIF order (high bits first); the
// inverse runs them in reverse.
struct PassSpec {
    int lglo, k, lgC, lgG;
};

// log2 of the points of a k_fft_pass workgroup: 2^12 in FP32; 2^11 in FP64,
// whose padded block of 2^12 would pass the 64 KiB LDS a launch may take
// without opting in.
template <typename T>
constexpr int pass_lgw() {
    return sizeof(T) == 8 ? 11 : 12;
}

// lgT: index bits of the (possibly merged) axis above which no stage runs
// but which the last pass may batch into one workgroup (lgT >= lgL).
inline std::vector<PassSpec> fft_passes(int lgL, int lgN, int lgT, int lgW) {
    std::vector<PassSpec> v;
    const int kmax = lgW - lgN;
    int hi = lgL;
    while (hi > 0) {
        if (hi <= kmax) {
            // the last pass: consecutive groups fill the workgroup (not with
            // line groups, whose lines are not consecutive)
            const int lgG = lgN ? 0 : std::min(kmax - hi, lgT - hi);
            v.push_back({0, hi, 0, std::max(lgG, 0)});
            break;
        }
        const int lgC = lgN ? 0 : 4, k = kmax - lgC;
        v.push_back({hi - k, k, lgC, 0});
        hi -= k;
    }
    return v;
}

// One axis of a batch of tables: its (possibly merged) index bits, line
// groups and pass schedule.
struct AxisPlan {
    int lgL = 0, lgA = 0, lgN = 0;
    int64_t es = 1, ls = 1, nlines = 1;
    std::vector<PassSpec> ps;  // DIF order
};

inline AxisPlan plan_axis(int lgL, int64_t es, int64_t ls, int64_t nlines, int lgN, int lgW) {
    AxisPlan a;
    while (lgN > 0 && ((int64_t)1 << lgN) > nlines) --lgN;
    // lines that follow one another in memory form one longer axis: its top
    // bits (the line) are never transformed, only batched by the last pass
    int lgA = lgL;
    if (es == 1 && ls == ((int64_t)1 << lgL) && lgN == 0 && (nlines & (nlines - 1)) == 0) {
        while (((int64_t)1 << (lgA - lgL)) < nlines) ++lgA;
        nlines = 1;
    }
    a.lgL = lgL;
    a.lgA = lgA;
    a.lgN = lgN;
    a.es = es;
    a.ls = ls;
    a.nlines = nlines;
    a.ps = fft_passes(lgL, lgN, lgA, lgW);
    return a;
}

template <typename T, bool INV, bool MUL = false>
void launch_pass(tfi::cpx<T>* buf, int64_t nslots, int lgP, const AxisPlan& a, const PassSpec& q,
                 const tfi::cpx<T>* tw, int lgtw, hipStream_t st,
                 const tfi::cpx<T>* spec = nullptr) {
    const int64_t groups = nslots * (a.nlines >> a.lgN) *
                           (((int64_t)1 << (a.lgA - q.lglo - q.k)) >> q.lgG) *
                           (((int64_t)1 << q.lglo) >> q.lgC);
    const unsigned lds = (unsigned)(tfi::pass_lds_elems((int64_t)1 << (q.k + q.lgC + a.lgN + q.lgG)) *
                                    sizeof(tfi::cpx<T>));
    hipLaunchKernelGGL((tfi::k_fft_pass<T, INV, MUL>), dim3((unsigned)groups), dim3(tfi::kPassThreads), lds,
                       st, buf, lgP, a.lgA, a.es, a.ls, a.nlines, q.lglo, q.k, q.lgC, a.lgN, q.lgG,
                       tw, lgtw, spec);
}

template <typename T, bool INV>
void launch_axis(tfi::cpx<T>* buf, int64_t nslots, int lgP, int lgL, int64_t es, int64_t ls,
                 int64_t nlines, int lgN, const tfi::cpx<T>* tw, int lgtw, hipStream_t st) {
    AxisPlan a = plan_axis(lgL, es, ls, nlines, lgN, pass_lgw<T>());
    std::vector<PassSpec> ps = a.ps;
    if (INV) std::reverse(ps.begin(), ps.end());
    for (const PassSpec& q : ps) launch_pass<T, INV>(buf, nslots, lgP, a, q, tw, lgtw, st);
}

// The forward DIF passes of the axis, the spectrum product, and its inverse
// DIT passes, with the last forward pass, the product and the first inverse
// pass in one launch.
template <typename T>
void launch_axis_conv(tfi::cpx<T>* buf, int64_t nslots, int lgP, int lgL, int64_t es, int64_t ls,
                      int64_t nlines, int lgN, const tfi::cpx<T>* spec, const tfi::cpx<T>* tw,
                      int lgtw, hipStream_t st) {
    const AxisPlan a = plan_axis(lgL, es, ls, nlines, lgN, pass_lgw<T>());
    const size_t np = a.ps.size();
    for (size_t i = 0; i + 1 < np; ++i) launch_pass<T, false>(buf, nslots, lgP, a, a.ps[i], tw, lgtw, st);
    launch_pass<T, false, true>(buf, nslots, lgP, a, a.ps[np - 1], tw, lgtw, st, spec);
    for (size_t i = np - 1; i-- > 0;) launch_pass<T, true>(buf, nslots, lgP, a, a.ps[i], tw, lgtw, st);
}

inline int ilog2_floor(int64_t v) {
    int lg = 0;
    while (((int64_t)2 << lg) <= v) ++lg;
    return lg;
}

// Forward 2-D transform (rows, then columns) or inverse (columns, then
// rows) of nslots tables of 2^lg1 x 2^lg2 points; the column passes take
// col_lines neighbouring columns per workgroup.
template <typename T, bool INV>
void launch_fft2(tfi::cpx<T>* buf, int64_t nslots, int lg1, int lg2, const tfi::cpx<T>* tw,
                 int lgtw, int col_lines, hipStream_t st) {
    const int lgP = lg1 + lg2;
    const int64_t L1 = (int64_t)1 << lg1, L2 = (int64_t)1 << lg2;
    const int lgN = ilog2_floor(std::max(1, col_lines));
    if (!INV) {
        if (lg2) launch_axis<T, false>(buf, nslots, lgP, lg2, 1, L2, L1, 0, tw, lgtw, st);
        if (lg1) launch_axis<T, false>(buf, nslots, lgP, lg1, L2, 1, L2, lgN, tw, lgtw, st);
    } else {
        if (lg1) launch_axis<T, true>(buf, nslots, lgP, lg1, L2, 1, L2, lgN, tw, lgtw, st);
        if (lg2) launch_axis<T, true>(buf, nslots, lgP, lg2, 1, L2, L1, 0, tw, lgtw, st);
    }
}

// Convolution of nslots tables with one spectrum: forward 2-D transform
// (rows, then columns), product, inverse (columns, then rows), the last axis
// fused around the product (launch_axis_conv).
template <typename T>
void launch_conv2(tfi::cpx<T>* buf, int64_t nslots, int lg1, int lg2, const tfi::cpx<T>* spec,
                  const tfi::cpx<T>* tw, int lgtw, int col_lines, hipStream_t st) {
    const int lgP = lg1 + lg2;
    const int64_t L1 = (int64_t)1 << lg1, L2 = (int64_t)1 << lg2;
    const int lgN = ilog2_floor(std::max(1, col_lines));
    if (lg1 == 0) {  // one row: the row axis carries the product
        launch_axis_conv<T>(buf, nslots, lgP, lg2, 1, L2, L1, 0, spec, tw, lgtw, st);
        return;
    }
    if (lg2) launch_axis<T, false>(buf, nslots, lgP, lg2, 1, L2, L1, 0, tw, lgtw, st);
    launch_axis_conv<T>(buf, nslots, lgP, lg1, L2, 1, L2, lgN, spec, tw, lgtw, st);
    if (lg2) launch_axis<T, true>(buf, nslots, lgP, lg2, 1, L2, L1, 0, tw, lgtw, st);
}

// Shape of the 1-D convolution kernels for a bucket: TC channel pairs per
// slot point and the split lg = lgH + lgL of the point index. TC starts at
// one 128-byte line per point (the high-bit passes read and write points
// 2^lgL apart, and a partial line would be fetched once per workgroup that
// reads a part of it); the strided high-bit blocks (2^lgH points x TC) stay
// within 64 KiB of LDS, the contiguous low-bit blocks within 128 KiB, and
// both within 2^10 points. Returns 0 when the bucket takes the blocked 2-D
// passes instead.
template <typename T>
int conv1d_tc(const Bucket& b, int32_t d, int* lgL_out = nullptr) {
    if (!b.d_map) return 0;
    const int lg = b.lg1 + b.lg2;
    if (lg < 2 || lg > 20) return 0;
    const int64_t cs = (int64_t)sizeof(tfi::cpx<T>);
    const int64_t npairs = (d + 1) / 2;
    int tc = (int)(128 / cs);
    while (b.tc_cap > 0 && tc > b.tc_cap) tc >>= 1;
    while (tc > 1 && tc / 2 >= npairs) tc >>= 1;
    for (; tc >= 1; tc >>= 1) {
        int lgH = lg - lg / 2;
        while (lgH > 1 && ((int64_t)1 << lgH) * tc * cs > 65536) --lgH;
        const int lgL = lg - lgH;
        if (lgH > 10 || lgL > 10 || ((int64_t)1 << lgL) * tc * cs > 131072) continue;
        if ((npairs + tc - 1) / tc > 65535) return 0;
        if (lgL_out) *lgL_out = lgL;
        return tc;
    }
    return 0;
}

// Bytes of one job's slots in the FFT work buffer.
template <typename T>
int64_t fft_job_bytes(const Bucket& b, int32_t d) {
    const int64_t npairs = (d + 1) / 2;
    const int tc = conv1d_tc<T>(b, d);
    const int64_t pairs = tc ? (npairs + tc - 1) / tc * tc : npairs;
    // the per-depth path keeps the depth-row spectra and the mixed rows
    return (b.d1 ? 2 : 1) * pairs * b.P() * (int64_t)sizeof(tfi::cpx<T>);
}

// Work buffer a bucket needs: for the channel-tiled 1-D convolution, the
// slots of all jobs and tiles, or of one group of tiles of about
// kConvGroupBytes when that is less (the passes then run group by group);
// else chunks of at most 2 GiB, or one job's slots when a job alone is
// larger.
template <typename T>
size_t fft_buf_bytes(const Bucket& b, int32_t d) {
    const int64_t one_job = fft_job_bytes<T>(b, d);
    const int64_t all = one_job * b.njobs();
    if (const int tc = conv1d_tc<T>(b, d)) {
        const int64_t slot = (int64_t)tc * b.P() * (int64_t)sizeof(tfi::cpx<T>);
        const int64_t gb = b.group_bytes > 0 ? b.group_bytes : tfi::kConvGroupBytes;
        const int64_t group = std::max<int64_t>(1, gb / slot) * slot;
        return (size_t)std::min(all, group);
    }
    return (size_t)std::max(one_job, std::min(all, (int64_t)2 << 30));
}

template <typename T, int TC>
void launch_conv1d_tc(tfi_plan* h, const Bucket& b, const int32_t* bmap, int32_t d, const T* val,
                      T* g, const tfi::cpx<T>* spec, const tfi::cpx<T>* tw, tfi::cpx<T>* buf,
                      size_t buf_bytes, hipStream_t st) {
    int lgL = 0;
    (void)conv1d_tc<T>(b, d, &lgL);
    const int lg = b.lg1 + b.lg2, lgH = lg - lgL;
    const int32_t ntiles = ((d + 1) / 2 + TC - 1) / TC;
    const int64_t slot_bytes = (int64_t)TC * b.P() * (int64_t)sizeof(tfi::cpx<T>);
    const int64_t nslots = std::max<int64_t>(1, (int64_t)buf_bytes / slot_bytes);
    // tiles per group: all of them when the buffer holds a job's slots, else
    // as many as it holds (one job per group then)
    const int32_t gt = (int32_t)std::min<int64_t>(ntiles, nslots);
    const int64_t jpc = gt == ntiles ? std::max<int64_t>(1, std::min<int64_t>(65535, nslots / ntiles))
                                     : 1;
    // LDS block: 2^RA rows of (2^RB x TC + pad) complex; 2^RB x TC threads
    const int hRB = lgH / 2, hRA = lgH - hRB, lRB = lgL / 2, lRA = lgL - lRB;
    const unsigned lds_hi = (unsigned)(((int64_t)1 << hRA) * ((TC << hRB) + tfi::kC1Pad) *
                                       sizeof(tfi::cpx<T>));
    // the low-bit blocks of 2^10 points take their TC pairs in two workgroups
    // of TC / 2 (two per CU instead of one)
    int lo_parts = 1;
    if constexpr (conv1d_fixed<T, TC>()) lo_parts = lgL == 10 ? 2 : 1;
    const int lo_cw = TC / lo_parts;
    const unsigned lds_lo = (unsigned)(((int64_t)1 << lRA) * ((lo_cw << lRB) + tfi::kC1Pad) *
                                       sizeof(tfi::cpx<T>));
    const unsigned thr_hi = (unsigned)(TC << hRB), thr_lo = (unsigned)(lo_cw << lRB);
    // kernel instances: the fixed split where one is compiled, else runtime
    using HiK = void (*)(int, int, int32_t, int, const int32_t*, int64_t, int32_t, const T*, T*,
                         tfi::cpx<T>*, const tfi::cpx<T>*, int, int32_t);
    using LoK = void (*)(int, int, tfi::cpx<T>*, const tfi::cpx<T>*, const tfi::cpx<T>*, int);
    HiK hi_fwd = tfi::k_conv1d_hi<T, TC, false, 0>, hi_inv = tfi::k_conv1d_hi<T, TC, true, 0>;
    LoK lo = tfi::k_conv1d_lo<T, TC, 0>;
    if constexpr (conv1d_fixed<T, TC>()) {
#define TFI_C1_FIXED(LG)                                         \
    if (lgH == LG) {                                             \
        hi_fwd = tfi::k_conv1d_hi<T, TC, false, LG>;             \
        hi_inv = tfi::k_conv1d_hi<T, TC, true, LG>;              \
    }                                                            \
    if (lgL == LG) lo = tfi::k_conv1d_lo<T, TC, LG>;
        TFI_C1_FIXED(5)
        TFI_C1_FIXED(6)
        TFI_C1_FIXED(7)
        TFI_C1_FIXED(8)
        TFI_C1_FIXED(9)
        TFI_C1_FIXED(10)
#undef TFI_C1_FIXED
        if (lo_parts == 2) lo = tfi::k_conv1d_lo<T, TC, 10, TC / 2>;
        static_assert(kC1FixedMin == 5 && kC1FixedMax == 10, "fixed splits listed above");
    }
    if constexpr (conv1d_fixed_half<T, TC>()) {
        if (lgH == 10) {
            hi_fwd = tfi::k_conv1d_hi<T, TC, false, 10>;
            hi_inv = tfi::k_conv1d_hi<T, TC, true, 10>;
        }
        if (lgL == 10) lo = tfi::k_conv1d_lo<T, TC, 10>;
    }
    for (int64_t j0 = 0; j0 < b.njobs(); j0 += jpc) {
        const int64_t nj = std::min(jpc, b.njobs() - j0);
        const int32_t* map = bmap + j0 * b.mstride;
        for (int32_t t0 = 0; t0 < ntiles; t0 += gt) {
            const unsigned nt = (unsigned)std::min(gt, ntiles - t0);
            hipLaunchKernelGGL(hi_fwd, dim3(1u << lgL, nt, (unsigned)nj), dim3(thr_hi), lds_hi, st,
                               lg, lgL, b.cmax, (int)b.reflect, map, b.mstride, d, val, (T*)nullptr,
                               buf, tw, h->lgtw, t0);
            hipLaunchKernelGGL(lo, dim3((1u << lgH) * lo_parts, nt, (unsigned)nj), dim3(thr_lo),
                               lds_lo, st, lg, lgL, buf, spec + b.spec_off, tw, h->lgtw);
            hipLaunchKernelGGL(hi_inv, dim3(1u << lgL, nt, (unsigned)nj), dim3(thr_hi), lds_hi, st,
                               lg, lgL, b.cmax, 0, map, b.mstride, d, (const T*)nullptr, g, buf, tw,
                               h->lgtw, t0);
        }
    }
}

// src rows -> dst rows through bmap (b.d_map: value and table rows;
// b.d_vmap: field and output rows).
template <typename T>
void launch_conv1d(tfi_plan* h, int tc, const Bucket& b, const int32_t* bmap, int32_t d,
                   const T* src, T* dst, const tfi::cpx<T>* spec, const tfi::cpx<T>* tw,
                   tfi::cpx<T>* buf, size_t buf_bytes, hipStream_t st) {
    switch (tc) {
#define TFI_C1(TCV)                                                                         \
    case TCV:                                                                               \
        launch_conv1d_tc<T, TCV>(h, b, bmap, d, src, dst, spec, tw, buf, buf_bytes, st);    \
        break;
        TFI_C1(16)
        TFI_C1(8)
        TFI_C1(4)
        TFI_C1(2)
#undef TFI_C1
        default: launch_conv1d_tc<T, 1>(h, b, bmap, d, src, dst, spec, tw, buf, buf_bytes, st);
    }
}

// Transform along the second table axis only (every row of nrows rows of
// each of nslots tables of 2^lg1 x 2^lg2 points).
template <typename T, bool INV>
void launch_rows(tfi::cpx<T>* buf, int64_t nslots, int lg1, int lg2, int64_t nrows,
                 const tfi::cpx<T>* tw, int lgtw, hipStream_t st) {
    if (lg2) launch_axis<T, INV>(buf, nslots, lg1 + lg2, lg2, 1, (int64_t)1 << lg2, nrows, 0, tw,
                                 lgtw, st);
}

// Per-depth path of one bucket (algorithm "global-anchor"): the depth rows
// of every (job, channel pair) slot are transformed along the backbone,
// mixed with the kernel-row spectra (k_d1_mix), and the hmax + 1 output rows
// transformed back. The work buffer holds the row spectra and the mixed
// rows of each chunk of slots.
template <typename T>
void launch_d1_global(tfi_plan* h, const Bucket& b, int32_t d, const T* val, T* g,
                      const tfi::cpx<T>* spec, const tfi::cpx<T>* tw, tfi::cpx<T>* buf,
                      size_t buf_bytes, hipStream_t st) {
    const int32_t npairs = (d + 1) / 2;
    const int64_t P = b.P();
    const int64_t slots_cap =
        std::min<int64_t>(65535, (int64_t)(buf_bytes / sizeof(tfi::cpx<T>)) / (2 * P));
    const int64_t jobs_per_chunk = std::max<int64_t>(1, slots_cap / npairs);
    for (int64_t j0 = 0; j0 < b.njobs(); j0 += jobs_per_chunk) {
        const int64_t nj = std::min(jobs_per_chunk, b.njobs() - j0);
        const int64_t nslots = nj * npairs;
        const int32_t* jobs = b.d_jobs + 2 * j0;
        tfi::cpx<T>* mixed = buf + nslots * P;
        hipLaunchKernelGGL(tfi::k_zero<tfi::cpx<T>>, dim3(blocks_for(nslots * P)), dim3(kThreads),
                           0, st, buf, nslots * P);
        hipLaunchKernelGGL(tfi::k_fill_global<T>, dim3(cell_blocks(nj), (unsigned)nj),
                           dim3(kThreads), 0, st, b.lg1, b.lg2, npairs, jobs, h->d_jc_r,
                           h->d_jc_x, h->d_jc_val, d, val, buf, 0);
        launch_rows<T, false>(buf, nslots, b.lg1, b.lg2, (int64_t)b.hmax + 1, tw, h->lgtw, st);
        const int64_t n = nslots * ((int64_t)b.hmax + 1) << b.lg2;
        hipLaunchKernelGGL(tfi::k_d1_mix<T>, dim3(blocks_for(n)), dim3(kThreads), 0, st, b.lg1,
                           b.lg2, b.hmax, nslots, (const tfi::cpx<T>*)buf, spec + b.spec_off,
                           mixed);
        launch_rows<T, true>(mixed, nslots, b.lg1, b.lg2, (int64_t)b.hmax + 1, tw, h->lgtw, st);
        hipLaunchKernelGGL(tfi::k_extract_global<T>, dim3(cell_blocks(nj), (unsigned)nj),
                           dim3(kThreads), 0, st, b.lg1, b.lg2, npairs, jobs, h->d_jc_r,
                           h->d_jc_x, h->d_jc_val, d, (const tfi::cpx<T>*)mixed, g, b.lg2);
    }
}

// Global-memory FFT passes of one bucket (tables beyond LDS): forward
// transform of (job, channel pair) slots, product with the spectrum,
// inverse, read-back.
template <typename T>
void launch_fft_global(tfi_plan* h, const Bucket& b, int32_t d, const T* val, T* g,
                       const tfi::cpx<T>* spec, const tfi::cpx<T>* tw, tfi::cpx<T>* buf,
                       size_t buf_bytes, hipStream_t st) {
    if (const int tc = conv1d_tc<T>(b, d)) {
        launch_conv1d<T>(h, tc, b, b.d_map, d, val, g, spec, tw, buf, buf_bytes, st);
        return;
    }
    if (b.d1) {
        launch_d1_global<T>(h, b, d, val, g, spec, tw, buf, buf_bytes, st);
        return;
    }
    const int32_t npairs = (d + 1) / 2;
    const int64_t slots_cap =
        std::min<int64_t>(65535, (int64_t)(buf_bytes / sizeof(tfi::cpx<T>)) / b.P());
    const int64_t jobs_per_chunk = std::max<int64_t>(1, slots_cap / npairs);
    const int lgP = b.lg1 + b.lg2;
    for (int64_t j0 = 0; j0 < b.njobs(); j0 += jobs_per_chunk) {
        const int64_t nj = std::min(jobs_per_chunk, b.njobs() - j0);
        const int64_t nslots = nj * npairs;
        const int32_t* jobs = b.d_jobs + 2 * j0;
        hipLaunchKernelGGL(tfi::k_zero<tfi::cpx<T>>, dim3(blocks_for(nslots * b.P())),
                           dim3(kThreads), 0, st, buf, nslots * b.P());
        hipLaunchKernelGGL(tfi::k_fill_global<T>, dim3(cell_blocks(nj), (unsigned)nj),
                           dim3(kThreads), 0, st, b.lg1, b.lg2, npairs, jobs, h->d_jc_r,
                           h->d_jc_x, h->d_jc_val, d, val, buf, 1);
        launch_conv2<T>(buf, nslots, b.lg1, b.lg2, spec + b.spec_off, tw, h->lgtw,
                        h->fp.col_lines, st);
        hipLaunchKernelGGL(tfi::k_extract_global<T>, dim3(cell_blocks(nj), (unsigned)nj),
                           dim3(kThreads), 0, st, b.lg1, b.lg2, npairs, jobs, h->d_jc_r,
                           h->d_jc_x, h->d_jc_val, d, buf, g, lgP);
    }
}

// Whole-path mode applies to this dtype and channel count.
template <typename T>
bool path_direct(const tfi_plan* h, int32_t d) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    if (!h->path_mode[ti] || h->global_b[ti].empty()) return false;
    for (int bi : h->global_b[ti])
        if (!conv1d_tc<T>(h->buckets[bi], d) || !h->buckets[bi].d_vmap) return false;
    return true;
}

// Scratch of one forward pass (or of dF): cell sums, table rows, kernel
// spectra and the FFT work buffer of the buckets beyond LDS.
struct Work {
    void* val = nullptr;   // [NA + NB, d] cell sums
    void* g = nullptr;     // [nk x (NA + NB) x d] table rows
    void* spec = nullptr;  // [nk x spec_elems] complex spectra
    void* fft = nullptr;   // FFT slots of the global buckets
    size_t fft_bytes = 0;
    void* part = nullptr;  // [part_rows x d] partial rows of cells cut between pieces
};

// Bytes of each part of Work; `general` asks for the value and table rows
// even where whole-path mode would not use them; nk kernels in one call
// take nk table arrays and nk spectrum arenas. The FFT workspace holds
// chunks of at most 2 GiB, or one job's slots when a job alone is larger.
struct WorkSizes {
    size_t val = 0, g = 0, spec = 0, fft = 0, part = 0;
};

template <typename T>
WorkSizes forward_sizes(const tfi_plan* h, int32_t d, bool general = false, int nk = 1) {
    const tfi::Plan& p = h->plan;
    const int ti = sizeof(T) == 8 ? 1 : 0;
    WorkSizes z;
    const bool rows = general || !path_direct<T>(h, d);
    if (rows) {
        z.val = (size_t)std::max<int64_t>(h->val_rows, 1) * d * sizeof(T);
        z.g = (size_t)nk * std::max<int64_t>(p.NA + p.NB, 1) * d * sizeof(T);
        if (scatter_pieces(h, d))
            z.part = (size_t)std::max<int64_t>(h->cells.part_rows, 1) * d * sizeof(T);
    }
    z.spec = (size_t)nk * std::max<int64_t>(h->spec_elems, 1) * sizeof(tfi::cpx<T>);
    for (int bi : h->global_b[ti]) z.fft = std::max(z.fft, fft_buf_bytes<T>(h->buckets[bi], d));
    // the Hankel tables' B rows share the buffer (same stream, after the FFTs)
    if (h->hk.njobs)
        z.fft = std::max(z.fft, (size_t)h->hk.max_rows * std::min<int32_t>(d, tfi::kHankCh) *
                                    sizeof(T));
    return z;
}

// The handle's own scratch buffers as a Work (after prepare_forward).
template <typename T>
Work handle_work(const tfi_plan* h) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    Work w;
    w.val = h->val[ti].p;
    w.g = h->g[ti].p;
    w.spec = h->spec[ti].p;
    w.fft = h->fftbuf[ti].p;
    w.fft_bytes = h->fftbuf[ti].bytes;
    w.part = h->part[ti].p;
    return w;
}

// Grow the handle's scratch to the sizes of a forward.
template <typename T>
int prepare_forward(tfi_plan* h, int32_t d, bool general = false, int nk = 1) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const WorkSizes z = forward_sizes<T>(h, d, general, nk);
    int rc = 0;
    if (z.val && (rc = h->ensure(h->val[ti], z.val))) return rc;
    if (z.g && (rc = h->ensure(h->g[ti], z.g))) return rc;
    if ((rc = h->ensure(h->spec[ti], z.spec))) return rc;
    if (z.fft && (rc = h->ensure(h->fftbuf[ti], z.fft))) return rc;
    if (z.part && (rc = h->ensure(h->part[ti], z.part))) return rc;
    return TFI_OK;
}

// ---- stage helpers (enqueue only; buffers prepared beforehand) ----------

// Channel split of the row-block kernels (leaf tiles, direct tables): with
// few workgroups along x, the chunks of step channels go to gridDim.y
// workgroups so that the launch still fills the device (4096 workgroups);
// a workgroup walks its chunks in order either way.
inline unsigned chan_split(int64_t xblocks, int32_t d, int32_t step) {
    const int64_t chunks = (d + step - 1) / step;
    const int64_t want = (4096 + std::max<int64_t>(xblocks, 1) - 1) / std::max<int64_t>(xblocks, 1);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>({chunks, want, 65535}));
}

template <typename T>
void enq_leaf(tfi_plan* h, const T* f, const T* F, int32_t d, T* out, hipStream_t st,
              const T* f1 = nullptr, T* out1 = nullptr) {
    if (h->nlgrp == 0) return;
    const tfi::Plan& p = h->plan;
    hipEvent_t ev = h->begin(st);
    const dim3 grid((unsigned)h->nlgrp, chan_split(h->nlgrp, d, tfi::kDirCh));
    const int nk = f1 ? 2 : 1;
    if (nk == 2) {
        if constexpr (sizeof(T) == 4) {
            hipLaunchKernelGGL((tfi::k_leaf<T, 2>), grid, dim3(tfi::kLeafThreads), 0, st, d,
                               h->d_lgrp, h->d_lgk, h->d_lq, h->d_leaf_v, h->d_leaf_D, f, F,
                               out, f1, out1);
        } else {  // FP64: one launch per kernel
            for (int u = 0; u < 2; ++u)
                hipLaunchKernelGGL((tfi::k_leaf<T, 1>), grid, dim3(tfi::kLeafThreads), 0, st, d,
                                   h->d_lgrp, h->d_lgk, h->d_lq, h->d_leaf_v, h->d_leaf_D,
                                   u ? f1 : f, F, u ? out1 : out, (const T*)nullptr,
                                   (T*)nullptr);
        }
    } else {
        hipLaunchKernelGGL((tfi::k_leaf<T, 1>), grid, dim3(tfi::kLeafThreads), 0, st, d,
                           h->d_lgrp, h->d_lgk, h->d_lq, h->d_leaf_v, h->d_leaf_D, f, F, out,
                           (const T*)nullptr, (T*)nullptr);
    }
    const double nv = (double)p.leaf_v.size();
    h->end(st, ev, "leaf",
           sizeof(T) * d * nv * (1.0 + nk) + 4.0 * nv + 4.0 * (double)p.leaf_D.size(),
           2.0 * d * nk * (double)p.leaf_pairs);
}

// Kernel spectra of every FFT bucket into spec (default: the handle's arena;
// several kernels of one call use consecutive arenas).
template <typename T>
void enq_spectra(tfi_plan* h, const T* f, hipStream_t st, tfi::cpx<T>* spec = nullptr) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    if (!spec) spec = (tfi::cpx<T>*)h->spec[ti].p;
    const tfi::cpx<T>* tw = (const tfi::cpx<T>*)h->d_tw[ti];
    for (int t = 0; t < 3; ++t) {
        const Tier& T_ = h->tiers[ti][t];
        if (!T_.nbuckets) continue;
        hipEvent_t ev = h->begin(st);
        hipLaunchKernelGGL(tfi::k_spectrum_multi<T>, dim3((unsigned)T_.nbuckets), dim3(kThreads),
                           (unsigned)T_.lds_bytes, st, T_.d_bp, T_.d_bo, f, tw, h->lgtw, spec);
        h->end(st, ev, "spectrum", sizeof(T) * T_.spec_bytes);
    }
    for (int bi : h->global_b[ti]) {
        const Bucket& b = h->buckets[bi];
        hipEvent_t ev = h->begin(st);
        tfi::cpx<T>* z = spec + b.spec_off;
        hipLaunchKernelGGL(tfi::k_spec_fill_global<T>, dim3(blocks_for(b.P())), dim3(kThreads), 0,
                           st, b.lg1, b.lg2, b.hmax, b.xmax, f, z);
        if (b.d1)  // kernel rows f(s + |b|), s <= 2 hmax, along the backbone axis only
            launch_rows<T, false>(z, 1, b.lg1, b.lg2, (int64_t)1 << b.lg1, tw, h->lgtw, st);
        else
            launch_fft2<T, false>(z, 1, b.lg1, b.lg2, tw, h->lgtw, h->fp.col_lines, st);
        h->end(st, ev, "spectrum_global", 2.0 * sizeof(T) * (double)b.P());
    }
}

// log2 of the channel pairs one workgroup of LDS tier t transforms for the
// tier's largest table (smaller tables take proportionally more, see
// k_fft_conv_multi): the handle's setting, else enough for about 2048
// points per workgroup (a radix-8 pass then has one group per thread), or
// 4096 for rows of more than 32 pairs (a job's many groups then read
// longer slices of each row); at most the pairs there are and what fits
// the LDS limit.
inline int fft_lgnp(const tfi_plan* h, int ti, int t, int32_t npairs) {
    const Tier& T_ = h->tiers[ti][t];
    const int64_t cs = ti ? 16 : 8;
    const int64_t pmax = std::max<int64_t>(1, T_.lds_bytes / cs);
    int lg = 0;
    if (h->fp.lds_pairs[t] > 0) {
        while ((2 << lg) <= h->fp.lds_pairs[t]) ++lg;
    } else {
        const int64_t points = (npairs > 32 ? 16 : 8) * kThreads;
        while (((int64_t)2 << lg) * pmax <= points) ++lg;
    }
    while (lg > 0 && (1 << lg) > npairs) --lg;
    while (lg > 0 && ((int64_t)1 << lg) * T_.lds_bytes > h->lds_max) --lg;
    return lg;
}

template <typename T>
void enq_fft(tfi_plan* h, int32_t d, const T* val, T* g, hipStream_t st, const Work& w,
             const tfi::cpx<T>* spec = nullptr) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    if (!spec) spec = (const tfi::cpx<T>*)w.spec;
    const tfi::cpx<T>* tw = (const tfi::cpx<T>*)h->d_tw[ti];
    const int32_t npairs = (d + 1) / 2;
    const double sz = (double)sizeof(T);
    for (int t = 0; t < 3; ++t) {
        const Tier& T_ = h->tiers[ti][t];
        if (!T_.njobs) continue;
        const int lgnp = fft_lgnp(h, ti, t, npairs);
        const unsigned groups = (unsigned)((npairs + (1 << lgnp) - 1) >> lgnp);
        // the padded block where it fits the LDS limit
        const int64_t lds = T_.lds_bytes << lgnp;
        const int64_t lds_pad = tfi::pass_lds_elems(lds / (int64_t)sizeof(tfi::cpx<T>)) *
                                (int64_t)sizeof(tfi::cpx<T>);
        const bool pad = lds_pad <= h->lds_max;
        // points per workgroup (lgnp pairs of the tier's largest table),
        // which smaller tables fill with more pairs, up to npairs
        int lgw = lgnp, lgcap = 0;
        while (((int64_t)sizeof(tfi::cpx<T>) << lgw) < lds) ++lgw;
        while ((2 << lgcap) <= npairs) ++lgcap;
        // with 16 groups or more the job columns are padded to a multiple
        // of 8 (the kernel's XCD order; the extra workgroups exit at once)
        const int64_t nj = T_.njobs;
        const unsigned gx = (unsigned)(groups >= tfi::kConvXcdGroups ? (nj + 7) / 8 * 8 : nj);
        hipEvent_t ev = h->begin(st);
        if (pad)
            hipLaunchKernelGGL((tfi::k_fft_conv_multi<T, tfi::kPassPad>), dim3(gx, groups),
                               dim3(kThreads), (unsigned)lds_pad, st, T_.d_fj, T_.d_bp, T_.d_bo,
                               h->d_jc_r, h->d_jc_x, h->d_jc_val, d, val, g, spec, tw, h->lgtw,
                               lgw, lgcap, (int32_t)nj);
        else
            hipLaunchKernelGGL(tfi::k_fft_conv_multi<T>, dim3(gx, groups), dim3(kThreads),
                               (unsigned)lds, st, T_.d_fj, T_.d_bp, T_.d_bo, h->d_jc_r, h->d_jc_x,
                               h->d_jc_val, d, val, g, spec, tw, h->lgtw, lgw, lgcap,
                               (int32_t)nj);
        h->end(st, ev, "fft_lds", sz * d * T_.bytes_per_d + T_.bytes_fixed + sz * T_.spec_bytes);
    }
    for (int bi : h->global_b[ti]) {
        const Bucket& b = h->buckets[bi];
        hipEvent_t ev = h->begin(st);
        launch_fft_global<T>(h, b, d, val, g, spec, tw, (tfi::cpx<T>*)w.fft, w.fft_bytes, st);
        h->end(st, ev, conv1d_tc<T>(b, d) ? "fft_conv1d" : (b.d1 ? "fft1d_global" : "fft_global"),
               2.0 * sz * d * (double)b.cells + 12.0 * b.cells + 2.0 * sz * b.P());
    }
}

// Hankel-product tables (kernels_hankel.hpp): per chunk of at most 64
// channels and group of tables, the product B (one workgroup per backbone
// column) and the two walks; B lives in the FFT work buffer.
template <typename T>
void enq_hankel(tfi_plan* h, const T* f, int32_t d, const T* val, T* g, hipStream_t st,
                const Work& w) {
    const HankelSet& k = h->hk;
    if (!k.njobs) return;
    hipEvent_t ev = h->begin(st);
    T* B = (T*)w.fft;
    for (int32_t c0 = 0; c0 < d; c0 += tfi::kHankCh) {
        const int32_t cw = std::min<int32_t>(tfi::kHankCh, d - c0);
        for (size_t gi = 0; gi + 1 < k.grp_bt.size(); ++gi) {
            const int64_t b0 = k.grp_bt[gi], nb = k.grp_bt[gi + 1] - b0;
            const int64_t l0 = k.grp_ln[gi], nl = k.grp_ln[gi + 1] - l0;
            const unsigned wb = (unsigned)((nl + 3) / 4);  // 4 items of 64 lanes per block
            hipLaunchKernelGGL(tfi::k_hankel_b<T>, dim3((unsigned)nb), dim3(256), 0, st,
                               k.d_bt + 2 * b0, k.d_jh, k.d_map, f, val, d, c0, cw, B);
            hipLaunchKernelGGL((tfi::k_hankel_walk<T, true>), dim3(wb), dim3(256), 0, st, nl,
                               k.d_ln + 2 * l0, k.d_jh, k.d_map, (const T*)B, d, c0, cw, g);
            hipLaunchKernelGGL((tfi::k_hankel_walk<T, false>), dim3(wb), dim3(256), 0, st, nl,
                               k.d_ln + 2 * l0, k.d_jh, k.d_map, (const T*)B, d, c0, cw, g);
        }
    }
    const double sz = (double)sizeof(T);
    h->end(st, ev, "hankel", 2.0 * sz * d * k.cells + 8.0 * k.cells, 2.0 * d * k.pairs);
}

// Direct tables of one kernel (f into g), or of two (also f1 into g1): on
// the matrix cores both share one launch and its value tiles; otherwise one
// launch each.
template <typename T>
void enq_direct(tfi_plan* h, const DirectSet& ds, const T* f, int32_t d, const T* val, T* g,
                hipStream_t st, const T* f1 = nullptr, T* g1 = nullptr) {
    if (ds.ndblk == 0) return;
    const tfi::Plan& p = h->plan;
    const int nk = f1 ? 2 : 1;
    const bool mfma = sizeof(T) == 4 && (h->direct_kernel == 2 || (h->direct_kernel == 0 && d >= 8));
    if (!mfma && f1) {
        enq_direct<T>(h, ds, f, d, val, g, st);
        enq_direct<T>(h, ds, f1, d, val, g1, st);
        return;
    }
    hipEvent_t ev = h->begin(st);
    const int32_t flds =
        (nk * p.kernel_len * (int64_t)sizeof(T) <= 16384) ? (int32_t)p.kernel_len : 0;
    if (mfma) {
        // 16-channel chunks per pass: one kernel entry serves all of them
        const int nch = d > 48 ? 4 : d > 32 ? 3 : d > 16 ? 2 : 1;
        const unsigned ys = chan_split(ds.ndblk, d, 16 * nch);
        const unsigned lds = (unsigned)(nk * flds * sizeof(float));
        auto launch = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)ds.ndblk, ys), dim3(tfi::kDirThreads), lds, st,
                               d, ds.d_dblk, ds.d_dl_r, ds.d_dl_x, ds.d_dl_row, ds.d_qjb,
                               ds.d_qje, (const float*)f, (const float*)f1, flds,
                               (const float*)val, (float*)g, (float*)g1);
        };
        // instances: kernel tables staged in LDS (flds > 0) or read from HBM
        auto launch_nk = [&](auto fl) {
            constexpr bool FL = decltype(fl)::value;
            if (nk == 2) {
                switch (nch) {
                    case 4: launch(tfi::k_direct_mfma<4, 2, FL>); break;
                    case 3: launch(tfi::k_direct_mfma<3, 2, FL>); break;
                    case 2: launch(tfi::k_direct_mfma<2, 2, FL>); break;
                    default: launch(tfi::k_direct_mfma<1, 2, FL>); break;
                }
            } else {
                switch (nch) {
                    case 4: launch(tfi::k_direct_mfma<4, 1, FL>); break;
                    case 3: launch(tfi::k_direct_mfma<3, 1, FL>); break;
                    case 2: launch(tfi::k_direct_mfma<2, 1, FL>); break;
                    default: launch(tfi::k_direct_mfma<1, 1, FL>); break;
                }
            }
        };
        if (flds > 0) launch_nk(std::true_type{});
        else launch_nk(std::false_type{});
    } else {
        auto kern = flds > 0 ? tfi::k_direct<T, true> : tfi::k_direct<T, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)ds.ndblk, chan_split(ds.ndblk, d, tfi::kDirCh)),
                           dim3(tfi::kDirThreads), (unsigned)(flds * sizeof(T)), st, d, ds.d_dblk,
                           ds.d_dl_r, ds.d_dl_x, ds.d_dl_row, ds.d_qjb, ds.d_qje, f, flds, val,
                           g);
    }
    // bytes: the value rows once, the table rows of every kernel
    h->end(st, ev, mfma ? "direct_mfma" : "direct",
           sizeof(T) * d * (double)ds.ndirect * (1 + nk) + 20.0 * ds.ndirect,
           2.0 * nk * d * ds.direct_pairs);
}

// Gather of one kernel's tables (g into out), or of two (also g1 into out1)
// in one pass over the index lists.
template <typename T>
void enq_gather(tfi_plan* h, int32_t d, const T* g, T* out, hipStream_t st,
                const T* g1 = nullptr, T* out1 = nullptr) {
    const tfi::Plan& p = h->plan;
    const int nk = g1 ? 2 : 1;
    const int32_t* ga = h->d_ga;
    const int32_t* gb = h->d_gb;
    const double reads = (double)h->gather_reads;
    hipEvent_t ev = h->begin(st);
    const bool v4 = d % 4 == 0 && aligned16(out) && (!out1 || aligned16(out1));
    const int vec = v4 ? 4 : 1;
    const int32_t ct = col_tile<T>(d, vec);
    const dim3 grid(blocks_for(tiled_threads(p.N, d / vec, ct)));
    if (v4 && nk == 2)
        hipLaunchKernelGGL((tfi::k_gather<T, 4, 2>), grid, dim3(kThreads), 0, st, p.N, d, ct,
                           h->d_v_off, ga, gb, h->d_vleaf, g, g1, out, out1);
    else if (v4)
        hipLaunchKernelGGL((tfi::k_gather<T, 4, 1>), grid, dim3(kThreads), 0, st, p.N, d, ct,
                           h->d_v_off, ga, gb, h->d_vleaf, g, (const T*)nullptr, out,
                           (T*)nullptr);
    else if (nk == 2)
        hipLaunchKernelGGL((tfi::k_gather<T, 1, 2>), grid, dim3(kThreads), 0, st, p.N, d, ct,
                           h->d_v_off, ga, gb, h->d_vleaf, g, g1, out, out1);
    else
        hipLaunchKernelGGL((tfi::k_gather<T, 1, 1>), grid, dim3(kThreads), 0, st, p.N, d, ct,
                           h->d_v_off, ga, gb, h->d_vleaf, g, (const T*)nullptr, out,
                           (T*)nullptr);
    h->end(st, ev, "gather",
           nk * sizeof(T) * d * (reads + 2 * p.N) +
               8.0 * (double)p.v_b.size() + 9.0 * p.N);
}

// LDS budget of the df FFT passes for one bucket (3 tables), 0 if the
// bucket needs the global-memory path.
template <typename T>
int64_t df_lds_bytes(const tfi_plan* h, const Bucket& b) {
    const int64_t need = 3 * b.P() * (int64_t)sizeof(tfi::cpx<T>);
    return need <= h->lds_max ? need : 0;
}

// Whether the LDS df pass of a bucket folds each group's spectrum in the
// same workgroup (no partial spectra in global memory): when a job has at
// most two groups (beyond that, the extra inverse transforms and bin
// flushes per group cost more than the partial spectra's round trip) and
// the bins of its largest job fit the LDS from the second table on (2 P
// complex values).
template <typename T>
bool df_group_folds(const Bucket& b, int32_t groups) {
    const int64_t hist = (2 * (int64_t)b.hmax + b.xmax + 1) * 2 * (int64_t)sizeof(tfi::u64);
    return groups <= 2 && hist <= 2 * b.P() * (int64_t)sizeof(tfi::cpx<T>);
}

// Channel pairs per workgroup of the LDS df pass for a bucket: kDfPairs,
// doubled while the bucket still has at least 4096 (job, group) workgroups.
inline int32_t df_pairs_per_group(int64_t njobs, int32_t npairs) {
    int32_t ppg = tfi::kDfPairs;
    while (ppg < npairs && njobs * ((npairs + 2 * ppg - 1) / (2 * ppg)) >= 4096) ppg *= 2;
    return ppg;
}

template <typename T>
void enq_df_tables(tfi_plan* h, int32_t d, const T* val, const T* valg, tfi::u64* df,
                   hipStream_t st) {
    const tfi::Plan& p = h->plan;
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const tfi::cpx<T>* tw = (const tfi::cpx<T>*)h->d_tw[ti];
    const int32_t npairs = (d + 1) / 2;
    const double sz = (double)sizeof(T);
    for (const Bucket& b : h->buckets) {
        const int64_t P = b.P();
        const int32_t ppg = df_pairs_per_group(b.njobs(), npairs);
        const int32_t groups = (npairs + ppg - 1) / ppg;
        const double bytes = 2.0 * sz * d * (double)b.cells + 12.0 * b.cells;
        const int64_t lds = df_lds_bytes<T>(h, b);
        if (lds) {
            hipEvent_t ev = h->begin(st);
            tfi::cpx<T>* part = (tfi::cpx<T>*)h->dfbuf[ti].p;
            const int64_t cs = (int64_t)sizeof(tfi::cpx<T>);
            // pairs transformed together: 2^lgnb of the group's, while their
            // tables hold at most one radix-8 group per thread (more would
            // only cost occupancy) and the padded block fits the limit
            int lgnb = 0;
            while ((2 << lgnb) <= ppg && (4 * P << lgnb) <= 8 * kThreads &&
                   (tfi::pass_lds_elems(4 * P << lgnb) + P) * cs <= h->lds_max)
                ++lgnb;
            // padded LDS blocks (lds_at) where they fit the limit
            const int64_t lds_pad = (tfi::pass_lds_elems(2 * P << lgnb) + P) * cs;
            const int64_t hist = (2 * (int64_t)b.hmax + b.xmax + 1) * 2 * (int64_t)sizeof(tfi::u64);
            if (df_group_folds<T>(b, groups)) {
                if (lds_pad <= h->lds_max)
                    hipLaunchKernelGGL((tfi::k_df_fft_partial<T, tfi::kPassPad, true>),
                                       dim3((unsigned)b.njobs(), groups), dim3(kThreads),
                                       (unsigned)lds_pad, st, b.lg1, b.lg2, b.d_jobs, h->d_jc_r,
                                       h->d_jc_x, h->d_jc_val, d, val, valg, tw, h->lgtw,
                                       (tfi::cpx<T>*)nullptr, ppg, lgnb, b.d_hx, p.NA, df);
                else
                    hipLaunchKernelGGL((tfi::k_df_fft_partial<T, 0, true>),
                                       dim3((unsigned)b.njobs(), groups), dim3(kThreads),
                                       (unsigned)lds, st, b.lg1, b.lg2, b.d_jobs, h->d_jc_r,
                                       h->d_jc_x, h->d_jc_val, d, val, valg, tw, h->lgtw,
                                       (tfi::cpx<T>*)nullptr, ppg, lgnb, b.d_hx, p.NA, df);
                h->end(st, ev, "df_fft_lds", bytes);
                continue;
            }
            if (lds_pad <= h->lds_max)
                hipLaunchKernelGGL((tfi::k_df_fft_partial<T, tfi::kPassPad>),
                                   dim3((unsigned)b.njobs(), groups), dim3(kThreads),
                                   (unsigned)lds_pad, st, b.lg1, b.lg2, b.d_jobs, h->d_jc_r,
                                   h->d_jc_x, h->d_jc_val, d, val, valg, tw, h->lgtw, part, ppg,
                                   lgnb);
            else
                hipLaunchKernelGGL(tfi::k_df_fft_partial<T>, dim3((unsigned)b.njobs(), groups),
                                   dim3(kThreads), (unsigned)lds, st, b.lg1, b.lg2, b.d_jobs,
                                   h->d_jc_r, h->d_jc_x, h->d_jc_val, d, val, valg, tw, h->lgtw,
                                   part, ppg, lgnb);
            const int64_t fold_lds = P * cs + hist, fold_pad = tfi::pass_lds_elems(P) * cs + hist;
            if (fold_pad <= h->lds_max)
                hipLaunchKernelGGL((tfi::k_df_fft_fold<T, tfi::kPassPad>),
                                   dim3((unsigned)b.njobs()), dim3(kThreads), (unsigned)fold_pad,
                                   st, b.lg1, b.lg2, b.d_jobs, b.d_hx, groups, p.NA, h->d_jc_val,
                                   (const tfi::cpx<T>*)part, tw, h->lgtw, df);
            else
                hipLaunchKernelGGL(tfi::k_df_fft_fold<T>, dim3((unsigned)b.njobs()),
                                   dim3(kThreads), (unsigned)fold_lds, st, b.lg1, b.lg2, b.d_jobs,
                                   b.d_hx, groups, p.NA, h->d_jc_val, (const tfi::cpx<T>*)part,
                                   tw, h->lgtw, df);
            h->end(st, ev, "df_fft_lds", bytes);
            continue;
        }
        const int64_t per_job = (2 * (int64_t)npairs + 1) * P * (int64_t)sizeof(tfi::cpx<T>);
        const int64_t cap = (int64_t)2 << 30;
        const int64_t jpc = std::max<int64_t>(
            1, std::min<int64_t>(cap / per_job, 65535 / std::max<int32_t>(npairs, 1)));
        tfi::cpx<T>* bv = (tfi::cpx<T>*)h->dfbuf[ti].p;
        hipEvent_t ev = h->begin(st);
        const int lgP = b.lg1 + b.lg2;
        for (int64_t j0 = 0; j0 < b.njobs(); j0 += jpc) {
            const int64_t nj = std::min(jpc, b.njobs() - j0);
            const int64_t nslots = nj * npairs;
            tfi::cpx<T>* bg = bv + nslots * P;
            tfi::cpx<T>* acc = bg + nslots * P;
            const int32_t* jobs = b.d_jobs + 2 * j0;
            hipLaunchKernelGGL(tfi::k_zero<tfi::cpx<T>>, dim3(blocks_for(2 * nslots * P)),
                               dim3(kThreads), 0, st, bv, 2 * nslots * P);
            hipLaunchKernelGGL(tfi::k_fill2_global<T>, dim3(cell_blocks(nj), (unsigned)nj),
                               dim3(kThreads), 0, st, b.lg1, b.lg2, npairs, jobs, h->d_jc_r,
                               h->d_jc_x, h->d_jc_val, d, val, valg, bv, bg);
            launch_fft2<T, false>(bv, 2 * nslots, b.lg1, b.lg2, tw, h->lgtw, h->fp.col_lines, st);
            hipLaunchKernelGGL(tfi::k_corr_accum_global<T>, dim3(blocks_for(nj * P)),
                               dim3(kThreads), 0, st, nj, npairs, lgP, (const tfi::cpx<T>*)bv,
                               (const tfi::cpx<T>*)bg, acc);
            launch_fft2<T, true>(acc, nj, b.lg1, b.lg2, tw, h->lgtw, h->fp.col_lines, st);
            hipLaunchKernelGGL(tfi::k_fold_global<T>, dim3(blocks_for(nj * P)), dim3(kThreads), 0,
                               st, nj, b.lg1, b.lg2, p.NA, jobs, b.d_hx + 2 * j0, h->d_jc_val,
                               (const tfi::cpx<T>*)acc, df);
        }
        h->end(st, ev, "df_fft_global", bytes);
    }
}

template <typename T>
void enq_df_direct(tfi_plan* h, const DirectSet& ds, int32_t d, const T* val, const T* valg,
                   tfi::u64* df, hipStream_t st) {
    if (ds.ndblk == 0) return;
    const tfi::Plan& p = h->plan;
    hipEvent_t ev = h->begin(st);
    const bool mfma = sizeof(T) == 4 && (h->direct_kernel == 2 || (h->direct_kernel == 0 && d >= 8));
    if (mfma) {
        // channels per lane per chunk: the smallest run that covers d (up to 16)
        const int cpl = d > 32 ? 16 : d > 16 ? 8 : d > 8 ? 4 : d > 4 ? 2 : 1;
        // histogram copies: as many as fit (up to 16) in 80 KiB of LDS, so
        // that two blocks share a CU; none when one copy does not fit
        auto launch = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)ds.ndblk), dim3(tfi::kDirThreads), 0, st, d,
                               p.NA, ds.d_dblk, ds.d_dl_r, ds.d_dl_x, ds.d_dl_row, ds.d_qjb,
                               ds.d_qje, (const float*)val, (const float*)valg, ds.d_dbin, df);
        };
        switch (cpl) {
            case 16: launch(tfi::k_df_direct_mfma<16>); break;
            case 8: launch(tfi::k_df_direct_mfma<8>); break;
            case 4: launch(tfi::k_df_direct_mfma<4>); break;
            case 2: launch(tfi::k_df_direct_mfma<2>); break;
            default: launch(tfi::k_df_direct_mfma<1>); break;
        }
    } else {
        hipLaunchKernelGGL(tfi::k_df_direct<T>, dim3((unsigned)ds.ndblk), dim3(tfi::kDfThreads), 0,
                           st, d, p.NA, ds.d_dblk, ds.d_dl_r, ds.d_dl_x, ds.d_dl_row, ds.d_qjb,
                           ds.d_qje, val, valg, ds.d_dbin, df);
    }
    h->end(st, ev, mfma ? "df_direct_mfma" : "df_direct",
           2.0 * sizeof(T) * d * (double)ds.ndirect + 20.0 * ds.ndirect,
           2.0 * d * ds.direct_pairs);
}

template <typename T>
void enq_df_leaf(tfi_plan* h, int32_t d, const T* F, const T* gout, tfi::u64* df, hipStream_t st) {
    if (h->nlgrp == 0) return;
    const tfi::Plan& p = h->plan;
    hipEvent_t ev = h->begin(st);
    hipLaunchKernelGGL(tfi::k_df_leaf<T>, dim3((unsigned)h->nlgrp), dim3(tfi::kLeafThreads), 0, st,
                       d, h->d_lgrp, h->d_lgk, h->d_lq, h->d_leaf_v, h->d_leaf_D, F, gout,
                       h->d_lbin, df);
    const double nv = (double)p.leaf_v.size();
    h->end(st, ev, "df_leaf", 2.0 * sizeof(T) * d * nv + 4.0 * nv + 4.0 * (double)p.leaf_D.size(),
           2.0 * d * (double)p.leaf_pairs);
}

inline void fork3(tfi_plan* h, hipStream_t s0, hipStream_t s1, hipStream_t s2) {
    (void)hipEventRecord(h->ev_fork, s0);
    (void)hipStreamWaitEvent(s1, h->ev_fork, 0);
    (void)hipStreamWaitEvent(s2, h->ev_fork, 0);
}

// Whether the plan has FFT tables in dtype T (LDS tiers or global buckets):
// without them the forward leaves the FFT side stream out of the DAG, so
// that a captured graph holds no empty branch (each cross-queue edge costs
// microseconds at replay).
template <typename T>
bool fft_work(const tfi_plan* h) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    for (int t = 0; t < 3; ++t)
        if (h->tiers[ti][t].nbuckets || h->tiers[ti][t].njobs) return true;
    return !h->global_b[ti].empty() || h->hk.njobs > 0;
}

// Fork the side streams that have work from s0.
inline void fork_sides(tfi_plan* h, hipStream_t s0, hipStream_t s1, hipStream_t s2, bool use1,
                       bool use2) {
    if (!use1 && !use2) return;
    (void)hipEventRecord(h->ev_fork, s0);
    if (use1) (void)hipStreamWaitEvent(s1, h->ev_fork, 0);
    if (use2) (void)hipStreamWaitEvent(s2, h->ev_fork, 0);
}

// Enqueue out = f(D) F: `s0` is the main stream, s1/s2 the side streams.
// Whole-path mode: kernel spectra, then the convolution of every job from the
// field rows straight into the output rows.
template <typename T>
void enqueue_path(tfi_plan* h, const T* f, const T* F, int32_t d, T* out, hipStream_t st,
                  const Work& w, tfi::cpx<T>* spec = nullptr) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    if (!spec) spec = (tfi::cpx<T>*)w.spec;
    enq_spectra<T>(h, f, st, spec);
    const tfi::cpx<T>* tw = (const tfi::cpx<T>*)h->d_tw[ti];
    const double sz = (double)sizeof(T);
    for (int bi : h->global_b[ti]) {
        const Bucket& b = h->buckets[bi];
        hipEvent_t ev = h->begin(st);
        launch_conv1d<T>(h, conv1d_tc<T>(b, d), b, b.d_vmap, d, F, out, spec, tw,
                         (tfi::cpx<T>*)w.fft, w.fft_bytes, st);
        h->end(st, ev, "fft_conv1d_path",
               2.0 * sz * d * (double)b.cells + 4.0 * b.cells + 2.0 * sz * b.P());
    }
}

template <typename T>
void enqueue_forward(tfi_plan* h, const T* f, const T* F, int32_t d, T* out, hipStream_t s0,
                     hipStream_t s1, hipStream_t s2, const Work& w, T* cells = nullptr) {
    // cells: caller's buffer for the cell sums of F (kept for a backward with
    // df), which whole-path mode would not form
    if (!cells && path_direct<T>(h, d)) {
        enqueue_path<T>(h, f, F, d, out, s0, w);
        return;
    }
    T* val = cells ? cells : (T*)w.val;
    T* g = (T*)w.g;
    const bool use1 = fft_work<T>(h), use2 = h->nlgrp > 0;
    fork_sides(h, s0, s1, s2, use1, use2);
    if (use2) {
        enq_leaf<T>(h, f, F, d, out, s2);      // side2: leaf rows into out
        (void)hipEventRecord(h->ev_c, s2);
    }
    if (use1) enq_spectra<T>(h, f, s1, (tfi::cpx<T>*)w.spec);  // side1: kernel spectra
    launch_scatter<T>(h, F, val, (T*)w.part, d, s0);  // main: cell sums
    if (use1) {
        (void)hipEventRecord(h->ev_a, s0);
        (void)hipStreamWaitEvent(s1, h->ev_a, 0);
        enq_fft<T>(h, d, val, g, s1, w);        // side1: FFT tables
        enq_hankel<T>(h, f, d, val, g, s1, w);  // side1: Hankel-product tables
        (void)hipEventRecord(h->ev_b, s1);
    }
    enq_direct<T>(h, h->dall, f, d, val, g, s0);  // main: direct tables
    if (use1) (void)hipStreamWaitEvent(s0, h->ev_b, 0);
    if (use2) (void)hipStreamWaitEvent(s0, h->ev_c, 0);
    enq_gather<T>(h, d, g, out, s0);            // main: out = leaf + calls
}

// Several kernels over one field: the cell sums depend only on F, so the
// scatter runs once; kernel i has its own spectra, tables (rows i of the
// table arrays), leaf rows and gather into out[i].
template <typename T>
void enqueue_forward_multi(tfi_plan* h, int nk, const T* const* f, const T* F, int32_t d,
                           T* const* out, hipStream_t s0, hipStream_t s1, hipStream_t s2) {
    const tfi::Plan& p = h->plan;
    const Work w = handle_work<T>(h);
    tfi::cpx<T>* spec0 = (tfi::cpx<T>*)w.spec;
    const int64_t sstride = std::max<int64_t>(h->spec_elems, 1);
    if (path_direct<T>(h, d)) {
        for (int i = 0; i < nk; ++i)
            enqueue_path<T>(h, f[i], F, d, out[i], s0, w, spec0 + i * sstride);
        return;
    }
    T* val = (T*)w.val;
    T* g0 = (T*)w.g;
    const int64_t gstride = std::max<int64_t>(p.NA + p.NB, 1) * (int64_t)d;
    const bool use1 = fft_work<T>(h), use2 = h->nlgrp > 0;
    fork_sides(h, s0, s1, s2, use1, use2);
    // the main chain is enqueued first (in a captured graph the first chain
    // keeps the launch queue, so the gather follows the direct tables on
    // one queue and its wait for the side streams finds them done)
    launch_scatter<T>(h, F, val, (T*)w.part, d, s0);
    // leaf tiles in pairs of kernels (FP32: two FP64 f(D) blocks would not
    // fit the LDS of one workgroup)
    if (use2) {
        for (int i = 0; i < nk;) {
            const bool two = sizeof(T) == 4 && i + 1 < nk;
            enq_leaf<T>(h, f[i], F, d, out[i], s2, two ? f[i + 1] : nullptr,
                        two ? out[i + 1] : nullptr);
            i += two ? 2 : 1;
        }
        (void)hipEventRecord(h->ev_c, s2);
    }
    if (use1)
        for (int i = 0; i < nk; ++i) enq_spectra<T>(h, f[i], s1, spec0 + i * sstride);
    if (use1) {
        (void)hipEventRecord(h->ev_a, s0);
        (void)hipStreamWaitEvent(s1, h->ev_a, 0);
        for (int i = 0; i < nk; ++i) {
            enq_fft<T>(h, d, val, g0 + i * gstride, s1, w, spec0 + i * sstride);
            enq_hankel<T>(h, f[i], d, val, g0 + i * gstride, s1, w);
        }
        (void)hipEventRecord(h->ev_b, s1);
    }
    // kernels in pairs: one launch per pair for the direct tables and the
    // gather
    for (int i = 0; i < nk; i += 2) {
        const bool two = i + 1 < nk;
        enq_direct<T>(h, h->dall, f[i], d, val, g0 + i * gstride, s0, two ? f[i + 1] : nullptr,
                      two ? g0 + (i + 1) * gstride : nullptr);
    }
    if (use1) (void)hipStreamWaitEvent(s0, h->ev_b, 0);
    if (use2) (void)hipStreamWaitEvent(s0, h->ev_c, 0);
    for (int i = 0; i < nk; i += 2) {
        const bool two = i + 1 < nk;
        enq_gather<T>(h, d, g0 + i * gstride, out[i], s0,
                      two ? g0 + (i + 1) * gstride : nullptr, two ? out[i + 1] : nullptr);
    }
}

// Enqueue the adjoint: dF = f(D) gout (when dF != null) and the kernel-table
// gradient df (when df != null). gout is scattered once (it feeds both),
// F once (df only).
template <typename T>
void enqueue_backward(tfi_plan* h, const T* f, const T* F, const T* gout, int32_t d, T* dF,
                      double* df, hipStream_t s0, hipStream_t s1, hipStream_t s2,
                      const T* cells = nullptr, bool zero_df = true) {
    const Work w = handle_work<T>(h);
    if (!df) {  // dF alone is the forward applied to gout
        if (dF) enqueue_forward<T>(h, f, gout, d, dF, s0, s1, s2, w);
        return;
    }
    const tfi::Plan& p = h->plan;
    const int ti = sizeof(T) == 8 ? 1 : 0;
    T* val = (T*)w.val;
    T* valg = (T*)h->valg[ti].p;
    T* g = (T*)w.g;
    tfi::u64* acc = (tfi::u64*)h->dfacc.p;
    hipLaunchKernelGGL(tfi::k_zero<tfi::u64>, dim3(blocks_for(2 * p.kernel_len)), dim3(kThreads), 0,
                       s0, acc, 2 * (int64_t)p.kernel_len);
    fork3(h, s0, s1, s2);
    if (dF) enq_leaf<T>(h, f, gout, d, dF, s2);
    enq_df_leaf<T>(h, d, F, gout, acc, s2);
    (void)hipEventRecord(h->ev_c, s2);
    // the cell sums of F: kept from the forward, or formed here
    const T* valF = cells ? cells : val;
    if (df && !cells) launch_scatter<T>(h, F, val, (T*)w.part, d, s1);
    (void)hipEventRecord(h->ev_d, s1);
    if (dF) enq_spectra<T>(h, f, s1, (tfi::cpx<T>*)w.spec);
    launch_scatter<T>(h, gout, valg, (T*)h->partg[ti].p, d, s0);
    (void)hipEventRecord(h->ev_a, s0);
    (void)hipStreamWaitEvent(s1, h->ev_a, 0);
    if (dF) {
        enq_fft<T>(h, d, valg, g, s1, w);
        enq_hankel<T>(h, f, d, valg, g, s1, w);
    }
    enq_df_tables<T>(h, d, valF, valg, acc, s1);
    (void)hipEventRecord(h->ev_b, s1);
    if (dF) enq_direct<T>(h, h->dall, f, d, valg, g, s0);
    (void)hipStreamWaitEvent(s0, h->ev_d, 0);
    enq_df_direct<T>(h, h->dall, d, valF, valg, acc, s0);
    enq_df_direct<T>(h, h->dhank, d, valF, valg, acc, s0);
    (void)hipStreamWaitEvent(s0, h->ev_b, 0);
    (void)hipStreamWaitEvent(s0, h->ev_c, 0);
    if (dF) enq_gather<T>(h, d, g, dF, s0);
    // df from the integer sums (added to df after the first channel tile)
    hipLaunchKernelGGL(tfi::k_df_finish, dim3(blocks_for(p.kernel_len)), dim3(kThreads), 0, s0,
                       (const tfi::u64*)acc, (int64_t)p.kernel_len, df, zero_df ? 0 : 1);
}

// Bytes of the adjoint's scratch beyond the forward's when df is wanted:
// the cell sums of gout (and their partial rows), and the df FFT slots.
struct DfSizes {
    size_t valg = 0, partg = 0, dfbuf = 0, dfacc = 0;
};

template <typename T>
DfSizes df_sizes(const tfi_plan* h, int32_t d) {
    DfSizes z;
    z.valg = (size_t)std::max<int64_t>(h->val_rows, 1) * d * sizeof(T);
    z.dfacc = (size_t)h->plan.kernel_len * 2 * sizeof(tfi::u64);
    if (scatter_pieces(h, d))
        z.partg = (size_t)std::max<int64_t>(h->cells.part_rows, 1) * d * sizeof(T);
    const int32_t npairs = (d + 1) / 2;
    for (const Bucket& b : h->buckets) {
        const int64_t P = b.P();
        if (df_lds_bytes<T>(h, b)) {
            const int32_t ppg = df_pairs_per_group(b.njobs(), npairs);
            const int32_t groups = (npairs + ppg - 1) / ppg;
            if (df_group_folds<T>(b, groups)) continue;
            z.dfbuf = std::max(z.dfbuf, (size_t)(b.njobs() * groups * P * sizeof(tfi::cpx<T>)));
            continue;
        }
        const int64_t per_job = (2 * (int64_t)npairs + 1) * P * (int64_t)sizeof(tfi::cpx<T>);
        const int64_t cap = (int64_t)2 << 30;
        const int64_t jpc = std::max<int64_t>(
            1, std::min<int64_t>(cap / per_job, 65535 / std::max<int32_t>(npairs, 1)));
        z.dfbuf = std::max(z.dfbuf, (size_t)(std::min(jpc, b.njobs()) * per_job));
    }
    return z;
}

template <typename T>
int prepare_backward(tfi_plan* h, int32_t d, bool need_df) {
    int rc = prepare_forward<T>(h, d, need_df);
    if (rc) return rc;
    if (!need_df) return TFI_OK;  // dF alone runs the forward on gout
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const DfSizes z = df_sizes<T>(h, d);
    if ((rc = h->ensure(h->valg[ti], z.valg))) return rc;
    if (z.partg && (rc = h->ensure(h->partg[ti], z.partg))) return rc;
    if (z.dfbuf && (rc = h->ensure(h->dfbuf[ti], z.dfbuf))) return rc;
    if ((rc = h->ensure(h->dfacc, z.dfacc))) return rc;
    return TFI_OK;
}

// Run a DAG either eagerly on (caller stream, s1, s2) or as a cached graph
// replayed on the handle's capture stream, ordered after the caller's
// stream and before its later work.
template <typename Enq>
int run_dag(tfi_plan* h, const GraphKey& key, hipStream_t caller, Enq enq) {
    if (h->prof) {
        // stage timing: every stage on the caller's stream, one after the
        // other, so that each event pair brackets that stage's kernels alone
        enq(caller, caller, caller);
        TFI_HIP(hipGetLastError());
        return TFI_OK;
    }
    if (!h->use_graphs) {
        enq(caller, h->s1, h->s2);
        TFI_HIP(hipGetLastError());
        return TFI_OK;
    }
    hipGraphExec_t exec = nullptr;
    for (auto& e : h->graphs)
        if (e.key == key) {
            exec = e.exec;
            e.last = ++h->tick;
            break;
        }
    if (!exec) {
        hipGraph_t graph = nullptr;
        TFI_HIP(hipStreamBeginCapture(h->cs0, hipStreamCaptureModeThreadLocal));
        enq(h->cs0, h->s1, h->s2);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(h->cs0, &graph);
        if (le != hipSuccess || ce != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(TFI_ERR_HIP, std::string("graph capture: ") +
                                         hipGetErrorString(le != hipSuccess ? le : ce));
        }
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess)
            return fail(TFI_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        if ((int)h->graphs.size() >= kGraphCache) {
            auto it = std::min_element(h->graphs.begin(), h->graphs.end(),
                                       [](const tfi_plan::GraphEntry& a,
                                          const tfi_plan::GraphEntry& b) { return a.last < b.last; });
            TFI_HIP(hipDeviceSynchronize());  // the evicted graph may still run
            (void)hipGraphExecDestroy(it->exec);
            h->graphs.erase(it);
        }
        h->graphs.push_back({key, exec, ++h->tick});
    }
    // the executable graph runs in order on the caller's stream (its side
    // branches fork from and join back into that stream)
    TFI_HIP(hipGraphLaunch(exec, caller));
    return TFI_OK;
}

template <typename T>
int run_forward(tfi_plan* h, const T* f, const T* F, int32_t d, T* out, hipStream_t st,
                T* cells = nullptr) {
    int rc = prepare_forward<T>(h, d, cells != nullptr);
    if (rc) return rc;
    GraphKey key;
    key.kind = 1;
    key.dtype = sizeof(T) == 8;
    key.d = d;
    key.p[0] = f;
    key.p[1] = F;
    key.p[2] = out;
    key.p[3] = cells;
    const Work w = handle_work<T>(h);
    return run_dag(h, key, st, [&](hipStream_t a, hipStream_t b, hipStream_t c) {
        enqueue_forward<T>(h, f, F, d, out, a, b, c, w, cells);
    });
}

// ---- forward without allocation -------------------------------------------
// Scratch of tfi_integrate_noalloc: one fixed array in the code object, so
// each GPU the library runs on holds its own copy until the process ends.
// Host code never uses the array's name as an address: its device address
// is taken once per device with hipGetSymbolAddress and kept here.
constexpr size_t kNoAllocBytes = (size_t)TFI_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on `device`, which must be current.
int scratch_address(int device, unsigned char** out) {
    static std::mutex mu;
    static std::map<int, unsigned char*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *out = it->second;
        return TFI_OK;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(TFI_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
    addr[device] = (unsigned char*)ptr;
    *out = (unsigned char*)ptr;
    return TFI_OK;
}

// The forward of run_forward, launched directly on (caller, s1, s2) with its
// Work carved out of the device's scratch array: no allocation, no graph.
template <typename T>
int run_forward_noalloc(tfi_plan* h, const T* f, const T* F, int32_t d, T* out,
                        hipStream_t st) {
    const WorkSizes z = forward_sizes<T>(h, d);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_val = take(z.val), o_g = take(z.g), o_spec = take(z.spec),
                 o_fft = take(z.fft), o_part = take(z.part);
    if (off > kNoAllocBytes)
        return fail(TFI_ERR_BUDGET,
                    "tfi_integrate_noalloc: this plan needs " + std::to_string(off) +
                        " bytes of scratch at d = " + std::to_string(d) + ", more than the " +
                        std::to_string(kNoAllocBytes) + " bytes of the fixed scratch array");
    unsigned char* base = nullptr;
    int rc = scratch_address(h->device, &base);
    if (rc) return rc;
    Work w;
    w.val = z.val ? base + o_val : nullptr;
    w.g = z.g ? base + o_g : nullptr;
    w.spec = base + o_spec;
    w.fft = z.fft ? base + o_fft : nullptr;
    w.fft_bytes = z.fft;
    w.part = z.part ? base + o_part : nullptr;
    // stage events would be created on demand: none while this runs
    const bool keep_prof = h->prof;
    h->prof = false;
    enqueue_forward<T>(h, f, F, d, out, st, h->s1, h->s2, w);
    h->prof = keep_prof;
    TFI_HIP(hipGetLastError());
    return TFI_OK;
}

template <typename T>
int run_forward_multi(tfi_plan* h, int nk, const T* const* f, const T* F, int32_t d,
                      T* const* out, hipStream_t st) {
    int rc = prepare_forward<T>(h, d, false, nk);
    if (rc) return rc;
    GraphKey key;
    key.kind = 5;
    key.dtype = sizeof(T) == 8;
    key.n = nk;
    key.d = d;
    key.p[0] = F;
    for (int i = 0; i < nk; ++i) {
        key.p[1 + 2 * i] = f[i];
        key.p[2 + 2 * i] = out[i];
    }
    return run_dag(h, key, st, [&](hipStream_t a, hipStream_t b, hipStream_t c) {
        enqueue_forward_multi<T>(h, nk, f, F, d, out, a, b, c);
    });
}

template <typename T>
int run_backward(tfi_plan* h, const T* f, const T* F, const T* gout, int32_t d, T* dF,
                 double* df, hipStream_t st, const T* cells = nullptr, bool zero_df = true) {
    int rc = prepare_backward<T>(h, d, df != nullptr);
    if (rc) return rc;
    GraphKey key;
    key.kind = 2;
    key.dtype = sizeof(T) == 8;
    key.n = zero_df ? 0 : 1;
    key.d = d;
    key.p[0] = f;
    key.p[1] = F;
    key.p[2] = gout;
    key.p[3] = dF;
    key.p[4] = df;
    key.p[5] = cells;
    return run_dag(h, key, st, [&](hipStream_t a, hipStream_t b, hipStream_t c) {
        enqueue_backward<T>(h, f, F, gout, d, dF, df, a, b, c, cells, zero_df);
    });
}

// ---- channel tiles under the memory budget ----------------------------------
// Channels are independent, so a call whose scratch would not fit the
// handle's budget runs on tiles of the channels, each tile a full pass
// (kernel spectra formed again, no state kept between tiles) on a dense
// copy of its columns; df adds up over the tiles. Returns the widest tile
// that fits: d when the whole call fits, 0 when not even one channel does.
template <typename T>
int32_t budget_tile(tfi_plan* h, int32_t d, bool bwd, bool need_df) {
    if (!h->budget) return d;
    const size_t base = h->dev_bytes - h->scratch_bytes();
    const size_t N = (size_t)h->plan.N;
    auto need = [&](int32_t w, bool tiled) {
        const WorkSizes z = forward_sizes<T>(h, w, need_df);
        size_t n = z.val + z.g + z.spec + z.fft + z.part + 5 * 16;
        if (need_df) {
            const DfSizes e = df_sizes<T>(h, w);
            n += e.valg + e.partg + e.dfbuf + e.dfacc + 4 * 16;
        }
        if (tiled) n += (bwd ? 3 : 2) * N * (size_t)w * sizeof(T);  // tiles in and out
        return base + n;
    };
    if (need(d, false) <= h->budget) return d;
    int32_t lo = 0, hi = d;  // need(lo) fits (lo = 0 trivially), need(hi) does not
    while (hi - lo > 1) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (need(mid, true) <= h->budget) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Run fn; if it stops at the budget (before launching anything) because
// buffers of other passes are held, release every scratch buffer and run it
// once more.
template <typename Fn>
int budget_retry(tfi_plan* h, Fn fn) {
    int rc = fn();
    if (rc != TFI_ERR_BUDGET || !h->budget) return rc;
    if ((rc = h->free_scratch())) return rc;
    rc = fn();
    if (rc == TFI_OK) g_err.clear();
    return rc;
}

// The forward (tfi_integrate) on channel tiles of width dt < d.
template <typename T>
int run_forward_tiled(tfi_plan* h, const T* f, const T* F, int32_t d, T* out, hipStream_t st,
                      int32_t dt) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const size_t tb = (size_t)h->plan.N * dt * sizeof(T);
    int rc = budget_retry(h, [&]() {
        int r = h->ensure(h->tin[ti], tb);
        if (!r) r = h->ensure(h->tout[ti], tb);
        if (!r) r = prepare_forward<T>(h, dt);
        return r;
    });
    if (rc) return rc;
    T* tin = (T*)h->tin[ti].p;
    T* tout = (T*)h->tout[ti].p;
    const int64_t N = h->plan.N;
    for (int32_t c0 = 0; c0 < d && !rc; c0 += dt) {
        const int32_t w = std::min(dt, d - c0);
        hipLaunchKernelGGL((tfi::k_cols<T, false>), dim3(blocks_for(N * w)), dim3(kThreads), 0, st,
                           F, tin, N, d, c0, w);
        rc = run_forward<T>(h, f, tin, w, tout, st);
        if (!rc)
            hipLaunchKernelGGL((tfi::k_cols<T, true>), dim3(blocks_for(N * w)), dim3(kThreads), 0,
                               st, (const T*)tout, out, N, d, c0, w);
    }
    if (rc) return rc;
    TFI_HIP(hipGetLastError());
    return TFI_OK;
}

// The adjoint (tfi_backward) on channel tiles of width dt < d: dF tile by
// tile, df summed over the tiles (cleared by the first).
template <typename T>
int run_backward_tiled(tfi_plan* h, const T* f, const T* F, const T* gout, int32_t d, T* dF,
                       double* df, hipStream_t st, int32_t dt) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const size_t tb = (size_t)h->plan.N * dt * sizeof(T);
    int rc = budget_retry(h, [&]() {
        int r = h->ensure(h->tin[ti], tb);
        if (!r) r = h->ensure(h->tgin[ti], tb);
        if (!r) r = h->ensure(h->tout[ti], tb);
        if (!r) r = prepare_backward<T>(h, dt, df != nullptr);
        return r;
    });
    if (rc) return rc;
    T* tin = (T*)h->tin[ti].p;
    T* tg = (T*)h->tgin[ti].p;
    T* tout = (T*)h->tout[ti].p;
    const int64_t N = h->plan.N;
    for (int32_t c0 = 0; c0 < d && !rc; c0 += dt) {
        const int32_t w = std::min(dt, d - c0);
        if (df)
            hipLaunchKernelGGL((tfi::k_cols<T, false>), dim3(blocks_for(N * w)), dim3(kThreads), 0,
                               st, F, tin, N, d, c0, w);
        hipLaunchKernelGGL((tfi::k_cols<T, false>), dim3(blocks_for(N * w)), dim3(kThreads), 0, st,
                           gout, tg, N, d, c0, w);
        rc = run_backward<T>(h, f, tin, tg, w, dF ? tout : nullptr, df, st, nullptr, c0 == 0);
        if (!rc && dF)
            hipLaunchKernelGGL((tfi::k_cols<T, true>), dim3(blocks_for(N * w)), dim3(kThreads), 0,
                               st, (const T*)tout, dF, N, d, c0, w);
    }
    if (rc) return rc;
    TFI_HIP(hipGetLastError());
    return TFI_OK;
}


// ---- kernels given as sums of exponentials: sweep evaluator -------------

// Lanes per table job: the smallest power of two >= d, at most 64.
inline int32_t exp_group(int32_t d) {
    int32_t gs = 1;
    while (gs < d && gs < 64) gs <<= 1;
    return gs;
}

// Gradient moment rows: one per workgroup of the one-position and
// multi-position job kernels, one per term for the leaf tiles.
inline int64_t expsum_moment_rows(const tfi_plan* h, int32_t d, int32_t nterm) {
    const int64_t gpb = tfi::kExpThreads / exp_group(d), wpb = tfi::kExpThreads / 64;
    return (h->nej1 + wpb - 1) / wpb + (h->nejm + gpb - 1) / gpb + nterm;
}

template <typename T>
int prepare_expsum(tfi_plan* h, int32_t nterm, int32_t d, bool bwd, bool grad) {
    const tfi::Plan& p = h->plan;
    const int ti = sizeof(T) == 8 ? 1 : 0;
    int rc;
    const size_t rowbytes = (size_t)std::max<int64_t>(h->val_rows, 1) * d * sizeof(T);
    const size_t partbytes = (size_t)std::max<int64_t>(h->cells.part_rows, 1) * d * sizeof(T);
    if ((rc = h->ensure(h->val[ti], rowbytes))) return rc;
    const bool pieces = scatter_pieces(h, d);
    if (pieces && (rc = h->ensure(h->part[ti], partbytes))) return rc;
    if ((rc = h->ensure(h->g[ti], (size_t)std::max<int64_t>(p.NA + p.NB, 1) * d * sizeof(T))))
        return rc;
    if ((rc = h->ensure(h->expw[ti], (size_t)(nterm + 1) * p.kernel_len * sizeof(T)))) return rc;
    const size_t nq = grad ? 5 : 2;
    if (h->npos_multi > 0 &&
        (rc = h->ensure(h->exps[ti], (size_t)h->npos_multi * nq * nterm * d * sizeof(T))))
        return rc;
    if (bwd && (rc = h->ensure(h->valg[ti], rowbytes))) return rc;
    if (bwd && pieces && (rc = h->ensure(h->partg[ti], partbytes))) return rc;
    if (grad && (rc = h->ensure(h->hleaf, (size_t)p.kernel_len * sizeof(double)))) return rc;
    if (grad && (rc = h->ensure(h->dfacc, (size_t)p.kernel_len * 2 * sizeof(tfi::u64))))
        return rc;
    if (grad && (rc = h->ensure(h->mrows, (size_t)expsum_moment_rows(h, d, nterm) * 2 * nterm *
                                              sizeof(double))))
        return rc;
    return TFI_OK;
}

// Power table lam_l^k and f table for the leaf tiles.
template <typename T>
void enq_expsum_prep(tfi_plan* h, int32_t nterm, const T* c, const T* lam, hipStream_t st) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const int64_t K = h->plan.kernel_len;
    T* pw = (T*)h->expw[ti].p;
    hipEvent_t ev = h->begin(st);
    hipLaunchKernelGGL(tfi::k_expsum_prep<T>, dim3(blocks_for(K)), dim3(kThreads), 0, st, nterm, c,
                       lam, (int32_t)K, pw, pw + (size_t)nterm * K);
    h->end(st, ev, "expsum_prep", sizeof(T) * (double)(nterm + 1) * K);
}

template <typename T, bool GRAD, bool DF = false>
void launch_expsum_wave(tfi_plan* h, int32_t nterm, const T* c, int32_t d, const T* val,
                        const T* valg, T* g, double* mrow, int64_t& mbase, hipStream_t st) {
    const int64_t nj = h->nej1;
    if (nj == 0) return;
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const int32_t gs = exp_group(d), wpb = tfi::kExpThreads / 64;  // one job per wavefront
    const unsigned blocks = (unsigned)((nj + wpb - 1) / wpb);
    const T* pw = (const T*)h->expw[ti].p;
    auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(tfi::kExpThreads), 0, st, nterm, d, gs,
                           (int32_t)nj, h->d_ej1, h->d_joff, h->d_jsign, h->d_jc_r, h->d_jc_val, c,
                           pw, (int32_t)h->plan.kernel_len, val, valg, g, mrow, mbase);
    };
    if (gs == 64) {  // one cell subgroup: the lane-uniform walk
        if (nterm <= 1) launch(tfi::k_expsum_wave<T, 1, GRAD, true, DF>);
        else if (nterm <= 2) launch(tfi::k_expsum_wave<T, 2, GRAD, true, DF>);
        else if (nterm <= 4) launch(tfi::k_expsum_wave<T, 4, GRAD, true, DF>);
        else if (nterm <= 8) launch(tfi::k_expsum_wave<T, 8, GRAD, true, DF>);
        else launch(tfi::k_expsum_wave<T, 16, GRAD, true, DF>);
    } else if (nterm <= 1) launch(tfi::k_expsum_wave<T, 1, GRAD, false, DF>);
    else if (nterm <= 2) launch(tfi::k_expsum_wave<T, 2, GRAD, false, DF>);
    else if (nterm <= 4) launch(tfi::k_expsum_wave<T, 4, GRAD, false, DF>);
    else if (nterm <= 8) launch(tfi::k_expsum_wave<T, 8, GRAD, false, DF>);
    else launch(tfi::k_expsum_wave<T, 16, GRAD, false, DF>);
    mbase += blocks;
}

template <typename T, bool GRAD>
void launch_expsum_multi(tfi_plan* h, int32_t nterm, const T* c, int32_t d, const T* val,
                         const T* valg, T* g, double* mrow, int64_t& mbase, hipStream_t st) {
    const int64_t nj = h->nejm;
    if (nj == 0) return;
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const int32_t gs = exp_group(d), gpb = tfi::kExpThreads / gs;
    const unsigned blocks = (unsigned)((nj + gpb - 1) / gpb);
    const T* pw = (const T*)h->expw[ti].p;
    T* scr = (T*)h->exps[ti].p;
    auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(tfi::kExpThreads), 0, st, nterm, d, gs,
                           (int32_t)nj, h->d_ejm, h->d_joff, h->d_jpos,
                           h->d_jsign, h->d_jc_r, h->d_jc_x, h->d_jc_val, c, pw,
                           (int32_t)h->plan.kernel_len, val, valg, g, scr, mrow, mbase);
    };
    if (nterm <= 1) launch(tfi::k_expsum_jobs<T, 1, GRAD>);
    else if (nterm <= 2) launch(tfi::k_expsum_jobs<T, 2, GRAD>);
    else if (nterm <= 4) launch(tfi::k_expsum_jobs<T, 4, GRAD>);
    else if (nterm <= 8) launch(tfi::k_expsum_jobs<T, 8, GRAD>);
    else launch(tfi::k_expsum_jobs<T, 16, GRAD>);
    mbase += blocks;
}

// Table values (forward) or gradient moment rows (leaf rows excluded) of
// every table job: one-position jobs (a wavefront each), then the jobs with
// several backbone positions.
template <typename T, bool GRAD>
void enq_expsum_jobs(tfi_plan* h, int32_t nterm, const T* c, int32_t d, const T* val,
                     const T* valg, T* g, double* mrow, hipStream_t st) {
    if (h->nej1 + h->nejm == 0) return;
    const tfi::Plan& p = h->plan;
    hipEvent_t ev = h->begin(st);
    int64_t mbase = 0;
    launch_expsum_wave<T, GRAD>(h, nterm, c, d, val, valg, g, mrow, mbase, st);
    launch_expsum_multi<T, GRAD>(h, nterm, c, d, val, valg, g, mrow, mbase, st);
    const double cells = (double)p.jc_r.size();
    h->end(st, ev, GRAD ? "expsum_grad" : "expsum",
           2.0 * sizeof(T) * d * cells + 12.0 * cells, (GRAD ? 10.0 : 4.0) * nterm * d * cells);
}

// Backward with both dF and the moments: the one-position jobs in one launch
// that reads the F and gout cell sums once and writes the moment rows and
// the dF tables; the multi-position jobs as in the separate passes.
template <typename T>
void enq_expsum_jobs_fused(tfi_plan* h, int32_t nterm, const T* c, int32_t d, const T* val,
                           const T* valg, T* g, double* mrow, hipStream_t st) {
    if (h->nej1 + h->nejm == 0) return;
    const tfi::Plan& p = h->plan;
    hipEvent_t ev = h->begin(st);
    int64_t mbase = 0, unused = 0;
    launch_expsum_wave<T, true, true>(h, nterm, c, d, val, valg, g, mrow, mbase, st);
    launch_expsum_multi<T, false>(h, nterm, c, d, valg, nullptr, g, nullptr, unused, st);
    launch_expsum_multi<T, true>(h, nterm, c, d, val, valg, nullptr, mrow, mbase, st);
    const double cells = (double)p.jc_r.size();
    h->end(st, ev, "expsum_grad_df", 3.0 * sizeof(T) * d * cells + 12.0 * cells,
           14.0 * nterm * d * cells);
}

// out = f(D) F for f(k) = sum_l c_l lam_l^k.
template <typename T>
void enqueue_forward_expsum(tfi_plan* h, int32_t nterm, const T* c, const T* lam, const T* F,
                            int32_t d, T* out, T* cells, hipStream_t s0, hipStream_t s1,
                            hipStream_t s2) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    T* val = cells ? cells : (T*)h->val[ti].p;  // the cell sums of F
    T* g = (T*)h->g[ti].p;
    const T* ftab = (const T*)h->expw[ti].p + (size_t)nterm * h->plan.kernel_len;
    enq_expsum_prep<T>(h, nterm, c, lam, s0);
    fork3(h, s0, s1, s2);
    enq_leaf<T>(h, ftab, F, d, out, s2);  // side2: leaf rows into out
    (void)hipEventRecord(h->ev_c, s2);
    (void)hipEventRecord(h->ev_b, s1);
    launch_scatter<T>(h, F, val, (T*)h->part[ti].p, d, s0);  // main: cell sums, sweeps
    enq_expsum_jobs<T, false>(h, nterm, c, d, val, nullptr, g, nullptr, s0);
    (void)hipStreamWaitEvent(s0, h->ev_b, 0);
    (void)hipStreamWaitEvent(s0, h->ev_c, 0);
    enq_gather<T>(h, d, g, out, s0);
}

// dF = f(D) gout (when dF != null) and the moments m0/m1 (when non-null).
// cells: the cell sums of F left by the forward (then F is not scattered
// again), or null.
template <typename T>
void enqueue_backward_expsum(tfi_plan* h, int32_t nterm, const T* c, const T* lam, const T* F,
                             const T* cells, const T* gout, int32_t d, T* dF, double* m0,
                             double* m1, hipStream_t s0, hipStream_t s1, hipStream_t s2) {
    const tfi::Plan& p = h->plan;
    const int ti = sizeof(T) == 8 ? 1 : 0;
    T* val = (T*)h->val[ti].p;
    const T* valF = cells ? cells : val;
    T* valg = (T*)h->valg[ti].p;
    T* g = (T*)h->g[ti].p;
    const T* pw = (const T*)h->expw[ti].p;
    const T* ftab = pw + (size_t)nterm * p.kernel_len;
    double* hl = (double*)h->hleaf.p;
    double* mrow = (double*)h->mrows.p;
    const bool grad = m0 != nullptr;
    const int64_t rows = grad ? expsum_moment_rows(h, d, nterm) : 0;
    enq_expsum_prep<T>(h, nterm, c, lam, s0);
    tfi::u64* acc = (tfi::u64*)h->dfacc.p;
    if (grad)
        hipLaunchKernelGGL(tfi::k_zero<tfi::u64>, dim3(blocks_for(2 * p.kernel_len)),
                           dim3(kThreads), 0, s0, acc, 2 * (int64_t)p.kernel_len);
    fork3(h, s0, s1, s2);
    if (dF) enq_leaf<T>(h, ftab, gout, d, dF, s2);
    if (grad) {
        enq_df_leaf<T>(h, d, F, gout, acc, s2);  // leaf pair histogram -> the last rows
        hipLaunchKernelGGL(tfi::k_df_finish, dim3(blocks_for(p.kernel_len)), dim3(kThreads), 0,
                           s2, (const tfi::u64*)acc, (int64_t)p.kernel_len, hl, 0);
        hipLaunchKernelGGL(tfi::k_expsum_leaf_moments<T>, dim3((unsigned)nterm),
                           dim3(tfi::kExpThreads), 0, s2, nterm, (int32_t)p.kernel_len, pw, hl,
                           mrow, rows - nterm);
    }
    (void)hipEventRecord(h->ev_c, s2);
    if (grad && !cells) launch_scatter<T>(h, F, val, (T*)h->part[ti].p, d, s1);
    (void)hipEventRecord(h->ev_d, s1);
    launch_scatter<T>(h, gout, valg, (T*)h->partg[ti].p, d, s0);
    if (dF && !grad) enq_expsum_jobs<T, false>(h, nterm, c, d, valg, nullptr, g, nullptr, s0);
    (void)hipStreamWaitEvent(s0, h->ev_d, 0);
    if (grad && dF) enq_expsum_jobs_fused<T>(h, nterm, c, d, valF, valg, g, mrow, s0);
    else if (grad) enq_expsum_jobs<T, true>(h, nterm, c, d, valF, valg, nullptr, mrow, s0);
    (void)hipStreamWaitEvent(s0, h->ev_c, 0);
    if (grad)
        hipLaunchKernelGGL(tfi::k_expsum_moments, dim3((unsigned)(2 * nterm)),
                           dim3(tfi::kExpThreads), 0, s0, nterm, rows, (const double*)mrow, m0,
                           m1);
    if (dF) enq_gather<T>(h, d, g, dF, s0);
}

template <typename T>
int run_forward_expsum(tfi_plan* h, int32_t nterm, const T* c, const T* lam, const T* F,
                       int32_t d, T* out, T* cells, hipStream_t st) {
    int rc = prepare_expsum<T>(h, nterm, d, false, false);
    if (rc) return rc;
    GraphKey key;
    key.kind = 3;
    key.dtype = sizeof(T) == 8;
    key.n = nterm;
    key.d = d;
    key.p[0] = c;
    key.p[1] = lam;
    key.p[2] = F;
    key.p[3] = out;
    key.p[4] = cells;
    return run_dag(h, key, st, [&](hipStream_t a, hipStream_t b, hipStream_t cc) {
        enqueue_forward_expsum<T>(h, nterm, c, lam, F, d, out, cells, a, b, cc);
    });
}

template <typename T>
int run_backward_expsum(tfi_plan* h, int32_t nterm, const T* c, const T* lam, const T* F,
                        const T* cells, const T* gout, int32_t d, T* dF, double* m0,
                        double* m1, hipStream_t st) {
    int rc = prepare_expsum<T>(h, nterm, d, true, m0 != nullptr);
    if (rc) return rc;
    GraphKey key;
    key.kind = 4;
    key.dtype = sizeof(T) == 8;
    key.n = nterm;
    key.d = d;
    key.p[0] = c;
    key.p[1] = lam;
    key.p[2] = F;
    key.p[3] = gout;
    key.p[4] = dF;
    key.p[5] = m0;
    key.p[6] = m1;
    key.p[7] = cells;
    return run_dag(h, key, st, [&](hipStream_t a, hipStream_t b, hipStream_t cc) {
        enqueue_backward_expsum<T>(h, nterm, c, lam, F, cells, gout, d, dF, m0, m1, a, b, cc);
    });
}

// Fold the recorded stage events into the per-stage tallies.
int drain_profile(tfi_plan* h) {
    for (auto& q : h->pending) {
        TFI_HIP(hipEventSynchronize(q.e1));
        float ms = 0;
        TFI_HIP(hipEventElapsedTime(&ms, q.e0, q.e1));
        auto& t = h->tally[q.stage];
        t.launches++;
        t.ms += ms;
        t.bytes += q.bytes;
        t.flops += q.flops;
        h->pool.push_back(q.e0);
        h->pool.push_back(q.e1);
    }
    h->pending.clear();
    return TFI_OK;
}

int reassign_methods(tfi_plan* h, double cost) {
    h->popt.fft_cost = cost;
    tfi::assign_methods(h->plan, h->popt);
    int rc = h->free_methods();
    if (rc) return rc;
    return upload_methods(h);
}

// Average time of `reps` passes (after two untimed ones) on fields of ones:
// forward integrations, or forward + adjoint (dF and df) when with_bwd.
template <typename T>
int time_pass(tfi_plan* h, const T* f, int32_t d, hipStream_t st, int reps, bool with_bwd,
              float* ms) {
    const int64_t n = h->plan.N * (int64_t)d;
    const size_t fb = (size_t)n * sizeof(T), hb = (size_t)h->plan.kernel_len * sizeof(double);
    void* buf[4] = {nullptr, nullptr, nullptr, nullptr};  // F, gout, out/dF, df
    const size_t sz[4] = {fb, fb, fb, hb};
    int rc = TFI_OK;
    for (int i = 0; i < 4 && !rc; ++i)
        if (i < 2 || i == 2 || with_bwd) rc = h->dalloc(&buf[i], sz[i]);
    auto release = [&]() {
        for (int i = 0; i < 4; ++i)
            if (buf[i]) {
                (void)hipFree(buf[i]);
                h->dev_bytes -= sz[i];
            }
    };
    if (rc) {
        release();
        return rc;
    }
    hipLaunchKernelGGL(tfi::k_fill<T>, dim3(blocks_for(n)), dim3(kThreads), 0, st, (T*)buf[0], n,
                       (T)1);
    hipLaunchKernelGGL(tfi::k_fill<T>, dim3(blocks_for(n)), dim3(kThreads), 0, st, (T*)buf[1], n,
                       (T)1);
    auto pass = [&]() {
        int r = run_forward<T>(h, f, (const T*)buf[0], d, (T*)buf[2], st);
        if (!r && with_bwd)
            r = run_backward<T>(h, f, (const T*)buf[0], (const T*)buf[1], d, (T*)buf[2],
                                (double*)buf[3], st);
        return r;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (int i = 0; i < 2 && !rc; ++i) rc = pass();
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps && !rc; ++i) rc = pass();
    (void)hipEventRecord(e1, st);
    if (!rc && hipEventSynchronize(e1) == hipSuccess) {
        (void)hipEventElapsedTime(ms, e0, e1);
        *ms /= (float)reps;
    }
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // graphs are dropped after the whole device has drained, as everywhere
    // else (they captured the temporary buffers)
    (void)hipDeviceSynchronize();
    h->drop_graphs();
    release();
    return rc;
}


// Apply FFT kernel shapes: tables move between the LDS tiers and the 1-D
// kernels when conv1d_min_lg changes (the device job lists are rebuilt);
// graphs holding the old launches are dropped.
int apply_fft_params(tfi_plan* h, const FftParams& p) {
    TFI_HIP(hipDeviceSynchronize());
    h->drop_graphs();
    const bool retier = p.conv1d_min_lg != h->fp.conv1d_min_lg;
    h->fp = p;
    if (retier) {
        int rc = h->free_methods();
        if (rc) return rc;
        return upload_methods(h);
    }
    for (Bucket& b : h->buckets) {
        b.tc_cap = p.conv1d_pairs;
        b.group_bytes = (int64_t)p.conv1d_group_mib << 20;
    }
    return TFI_OK;
}

// Coordinate search over the FFT kernel shapes that this dtype and width
// use: channel pairs per workgroup of each LDS tier, the size from which
// one-row and one-column tables take the 1-D kernels, the 1-D tile width
// and tile-group buffer, and the columns per workgroup of the blocked
// column passes. Each candidate is timed like the method rule; the fastest
// setting of each parameter is kept before the next is tried.
template <typename T>
int tune_fft(tfi_plan* h, const T* f, int32_t d, hipStream_t st, bool with_bwd) {
    const int ti = sizeof(T) == 8 ? 1 : 0;
    const int32_t npairs = (d + 1) / 2;
    auto uses = [&](bool* lds, bool* c1, bool* g2) {
        for (int t = 0; t < 3; ++t) lds[t] = h->tiers[ti][t].njobs > 0;
        *c1 = *g2 = false;
        for (int bi : h->global_b[ti]) (conv1d_tc<T>(h->buckets[bi], d) ? *c1 : *g2) = true;
    };
    bool lds[3], c1, g2;
    uses(lds, &c1, &g2);
    bool line_tables = false;  // one-row/one-column tables the 1-D threshold can move
    for (const Bucket& b : h->buckets)
        if ((b.lg1 == 0 || b.lg2 == 0) && b.lg1 + b.lg2 >= 6) line_tables = true;
    if (!lds[0] && !lds[1] && !lds[2] && !c1 && !g2) return TFI_OK;
    FftParams best = h->fp;
    float best_ms = 1e30f;
    int rc = time_pass<T>(h, f, d, st, 5, with_bwd, &best_ms);
    if (rc) return rc;
    auto trial = [&](const FftParams& cand) -> int {
        int r = apply_fft_params(h, cand);
        if (r) return r;
        float ms = 1e30f;
        r = time_pass<T>(h, f, d, st, 5, with_bwd, &ms);
        if (r) return r;
        if (ms < best_ms) {
            best_ms = ms;
            best = cand;
        }
        return TFI_OK;
    };
    for (int t = 0; t < 3 && !rc; ++t) {
        if (!lds[t]) continue;
        // candidates by the pair count they give (after the LDS and pair limits)
        auto eff = [&](const FftParams& c) {
            const FftParams keep = h->fp;
            h->fp = c;
            const int lg = fft_lgnp(h, ti, t, npairs);
            h->fp = keep;
            return lg;
        };
        std::set<int> tried = {eff(best)};
        for (int np : {1, 2, 4, 8, 16, 32}) {
            FftParams c = best;
            c.lds_pairs[t] = np;
            if (!tried.insert(eff(c)).second) continue;
            if ((rc = trial(c))) break;
        }
    }
    if (!rc && line_tables)
        for (int lg : {6, 8, 12, 15}) {
            if (lg == best.conv1d_min_lg) continue;
            FftParams c = best;
            c.conv1d_min_lg = lg;
            if ((rc = trial(c))) break;
        }
    if (!rc) rc = apply_fft_params(h, best);
    uses(lds, &c1, &g2);
    if (!rc && c1)
        for (int tc : {8, 4}) {
            if (tc * (int)sizeof(tfi::cpx<T>) >= 128) continue;
            FftParams c = best;
            c.conv1d_pairs = tc;
            if ((rc = trial(c))) break;
        }
    if (!rc && c1)
        for (int mib : {512, 128}) {
            FftParams c = best;
            c.conv1d_group_mib = mib;
            if ((rc = trial(c))) break;
        }
    if (!rc && g2)
        for (int n : {1, 4, 32}) {
            FftParams c = best;
            c.col_lines = n;
            if ((rc = trial(c))) break;
        }
    const int rc2 = apply_fft_params(h, best);
    return rc ? rc : rc2;
}

}  // namespace

extern "C" {

int tfi_build(const int64_t* parent, const int32_t* weight, int64_t N,
              const tfi_build_opts* opts, tfi_handle* out) {
    g_err.clear();
    if (!out) return fail(TFI_ERR_ARG, "tfi_build: null output handle");
    *out = nullptr;
    tfi_build_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    tfi::PlanOptions po;
    po.policy = o.policy;
    po.leaf_max = o.leaf_max == 0 ? 32 : o.leaf_max;
    if (po.leaf_max < 1 || po.leaf_max > tfi::kLeafMax)
        return fail(TFI_ERR_ARG, "tfi_build: leaf_max must be in [0, " +
                                     std::to_string(tfi::kLeafMax) + "]");
    if (o.table_method < 0 || o.table_method > 4)
        return fail(TFI_ERR_ARG, "tfi_build: table_method must be in [0, 4]");
    po.table_method = o.table_method;
    po.fft_cost = o.fft_cost == 0.0f ? 4.0 : (double)o.fft_cost;
    po.chan_width = o.chan_width == 0 ? 1 : o.chan_width;
    if (o.cost_vertex != 0.0f || o.cost_direct != 0.0f || o.cost_fft != 0.0f ||
        o.cost_call != 0.0f) {
        po.cost_vertex = o.cost_vertex;
        po.cost_direct = o.cost_direct;
        po.cost_fft = o.cost_fft;
        po.cost_call = o.cost_call;
        if (o.policy == TFI_POLICY_CHANNEL && o.fft_cost == 0.0f && o.cost_direct > 0.0f)
            po.fft_cost = (double)o.cost_fft / (double)o.cost_direct;
    }
    if (o.device < -1) return fail(TFI_ERR_ARG, "tfi_build: device must be >= -1");
    std::unique_ptr<tfi_plan> h;
    try {
        h.reset(new tfi_plan());
    } catch (const std::bad_alloc&) {
        return fail(TFI_ERR_OOM, "tfi_build: host allocation failed");
    }
    std::string err;
    int rc = tfi::build_plan(parent, weight, N, po, h->plan, err);
    if (rc) return fail(rc, err);
    h->popt = po;
    h->budget = o.memory_budget_bytes;
    h->use_graphs = o.no_graphs == 0;
    if (o.direct_kernel < 0 || o.direct_kernel > 2)
        return fail(TFI_ERR_ARG, "tfi_build: direct_kernel must be 0, 1 or 2");
    h->direct_kernel = o.direct_kernel;
    if (const char* e = std::getenv("TFI_NO_GRAPHS"))
        if (e[0] && e[0] != '0') h->use_graphs = false;

    if (o.device >= 0) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || count <= o.device)
            return fail(TFI_ERR_HIP, "tfi_build: HIP device " + std::to_string(o.device) +
                                         " not available");
        TFI_HIP(hipSetDevice(o.device));
        h->device = o.device;
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, o.device) ==
                hipSuccess &&
            lds > 0)
            h->lds_max = lds;
        rc = upload_plan(h.get());
        if (rc) return rc;
    }
    *out = h.release();
    return TFI_OK;
}

int64_t tfi_num_vertices(tfi_handle h) { return h ? h->plan.N : -1; }

int64_t tfi_kernel_length(tfi_handle h) { return h ? h->plan.kernel_len : -1; }

namespace {
// A forward, on channel tiles when the whole call would exceed the budget
// (not for the cell-keeping forward, whose cell sums span every channel).
extern "C++" template <typename T>
int forward_entry(const std::string& fs, tfi_plan* h, const T* f, const T* F, int32_t d, T* out,
                  hipStream_t st, T* cells) {
    if (!cells && h->budget) {
        const int32_t dt = budget_tile<T>(h, d, false, false);
        if (dt == 0)
            return fail(TFI_ERR_BUDGET, fs + ": the budget does not hold one channel of the pass");
        if (dt < d) return run_forward_tiled<T>(h, f, F, d, out, st, dt);
    }
    return budget_retry(h, [&]() { return run_forward<T>(h, f, F, d, out, st, cells); });
}

int integrate_impl(const char* fn, tfi_handle h, const void* f, const void* F, int64_t d,
                   tfi_dtype dtype, void* out, void* cells, void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    const std::string fs(fn);
    if (!f || !F || !out) return fail(TFI_ERR_ARG, fs + ": null pointer");
    if (d < 1 || d > (1 << 20)) return fail(TFI_ERR_ARG, fs + ": need 1 <= d <= 2^20");
    if (F == out) return fail(TFI_ERR_ARG, fs + ": out must not alias F");
    if (cells && (cells == F || cells == out))
        return fail(TFI_ERR_ARG, fs + ": cells must not alias F or out");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == TFI_F32)
        return forward_entry<float>(fs, h, (const float*)f, (const float*)F, (int32_t)d,
                                    (float*)out, st, (float*)cells);
    if (dtype == TFI_F64)
        return forward_entry<double>(fs, h, (const double*)f, (const double*)F, (int32_t)d,
                                     (double*)out, st, (double*)cells);
    return fail(TFI_ERR_DTYPE, fs + ": unknown dtype");
}
}  // namespace

int tfi_integrate(tfi_handle h, const void* f, const void* F, int64_t d, tfi_dtype dtype,
                  void* out, void* stream) {
    return integrate_impl("tfi_integrate", h, f, F, d, dtype, out, nullptr, stream);
}

int tfi_integrate_cells(tfi_handle h, const void* f, const void* F, int64_t d, tfi_dtype dtype,
                        void* out, void* cells, void* stream) {
    if (!cells) {
        g_err.clear();
        return fail(TFI_ERR_ARG, "tfi_integrate_cells: null pointer");
    }
    return integrate_impl("tfi_integrate_cells", h, f, F, d, dtype, out, cells, stream);
}

int tfi_integrate_multi(tfi_handle h, int32_t nk, const void* const* f, const void* F,
                        int64_t d, tfi_dtype dtype, void* const* out, void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (nk < 1 || nk > TFI_MULTI_MAX)
        return fail(TFI_ERR_ARG, "tfi_integrate_multi: need 1 <= nk <= TFI_MULTI_MAX");
    if (!f || !F || !out) return fail(TFI_ERR_ARG, "tfi_integrate_multi: null pointer");
    if (d < 1 || d > (1 << 20))
        return fail(TFI_ERR_ARG, "tfi_integrate_multi: need 1 <= d <= 2^20");
    for (int i = 0; i < nk; ++i) {
        if (!f[i] || !out[i]) return fail(TFI_ERR_ARG, "tfi_integrate_multi: null pointer");
        if (out[i] == F) return fail(TFI_ERR_ARG, "tfi_integrate_multi: out must not alias F");
        for (int j = 0; j < i; ++j)
            if (out[j] == out[i])
                return fail(TFI_ERR_ARG, "tfi_integrate_multi: outputs must be distinct");
    }
    hipStream_t st = (hipStream_t)stream;
    if (dtype == TFI_F32)
        return run_forward_multi<float>(h, nk, (const float* const*)f, (const float*)F,
                                        (int32_t)d, (float* const*)out, st);
    if (dtype == TFI_F64)
        return run_forward_multi<double>(h, nk, (const double* const*)f, (const double*)F,
                                         (int32_t)d, (double* const*)out, st);
    return fail(TFI_ERR_DTYPE, "tfi_integrate_multi: unknown dtype");
}

namespace {
// The adjoint, on channel tiles when the whole call would exceed the budget
// (not with kept cell sums, which span every channel).
extern "C++" template <typename T>
int backward_entry(const std::string& fs, tfi_plan* h, const T* f, const T* F, const T* gout,
                   int32_t d, T* dF, double* df, hipStream_t st, const T* cells) {
    if (!cells && h->budget) {
        const int32_t dt = budget_tile<T>(h, d, true, df != nullptr);
        if (dt == 0)
            return fail(TFI_ERR_BUDGET, fs + ": the budget does not hold one channel of the pass");
        if (dt < d) return run_backward_tiled<T>(h, f, F, gout, d, dF, df, st, dt);
    }
    return budget_retry(h, [&]() { return run_backward<T>(h, f, F, gout, d, dF, df, st, cells); });
}

int backward_impl(const char* fn, tfi_handle h, const void* f, const void* F, const void* cells,
                  const void* gout, int64_t d, tfi_dtype dtype, void* dF, double* df,
                  void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    const std::string fs(fn);
    if (!f || !F || !gout) return fail(TFI_ERR_ARG, fs + ": null pointer");
    if (d < 1 || d > (1 << 20)) return fail(TFI_ERR_ARG, fs + ": need 1 <= d <= 2^20");
    if (dtype != TFI_F32 && dtype != TFI_F64) return fail(TFI_ERR_DTYPE, fs + ": unknown dtype");
    if (dF && (dF == F || dF == gout || dF == cells))
        return fail(TFI_ERR_ARG, fs + ": dF must not alias F, cells or gout");
    if (!dF && !df) return TFI_OK;
    hipStream_t st = (hipStream_t)stream;
    // f(D) is symmetric: dF = f(D) gout
    if (dtype == TFI_F32)
        return backward_entry<float>(fs, h, (const float*)f, (const float*)F, (const float*)gout,
                                     (int32_t)d, (float*)dF, df, st, (const float*)cells);
    return backward_entry<double>(fs, h, (const double*)f, (const double*)F, (const double*)gout,
                                  (int32_t)d, (double*)dF, df, st, (const double*)cells);
}
}  // namespace

int tfi_backward(tfi_handle h, const void* f, const void* F, const void* gout, int64_t d,
                 tfi_dtype dtype, void* dF, double* df, void* stream) {
    return backward_impl("tfi_backward", h, f, F, nullptr, gout, d, dtype, dF, df, stream);
}

int tfi_backward_cells(tfi_handle h, const void* f, const void* F, const void* cells,
                       const void* gout, int64_t d, tfi_dtype dtype, void* dF, double* df,
                       void* stream) {
    if (!cells) {
        g_err.clear();
        return fail(TFI_ERR_ARG, "tfi_backward_cells: null pointer");
    }
    return backward_impl("tfi_backward_cells", h, f, F, cells, gout, d, dtype, dF, df, stream);
}

namespace {
int integrate_expsum_impl(const char* fn, tfi_handle h, int32_t nterm, const void* c,
                          const void* lambda, const void* F, int64_t d, tfi_dtype dtype,
                          void* out, void* cells, void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    const std::string f(fn);
    if (!c || !lambda || !F || !out) return fail(TFI_ERR_ARG, f + ": null pointer");
    if (nterm < 1 || nterm > tfi::kExpMaxTerms)
        return fail(TFI_ERR_ARG, f + ": need 1 <= nterm <= 16");
    if (d < 1 || d > (1 << 20)) return fail(TFI_ERR_ARG, f + ": need 1 <= d <= 2^20");
    if (F == out) return fail(TFI_ERR_ARG, f + ": out must not alias F");
    if (cells && (cells == F || cells == out))
        return fail(TFI_ERR_ARG, f + ": cells must not alias F or out");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == TFI_F32)
        return run_forward_expsum<float>(h, nterm, (const float*)c, (const float*)lambda,
                                         (const float*)F, (int32_t)d, (float*)out,
                                         (float*)cells, st);
    if (dtype == TFI_F64)
        return run_forward_expsum<double>(h, nterm, (const double*)c, (const double*)lambda,
                                          (const double*)F, (int32_t)d, (double*)out,
                                          (double*)cells, st);
    return fail(TFI_ERR_DTYPE, f + ": unknown dtype");
}
}  // namespace

int tfi_integrate_expsum(tfi_handle h, int32_t nterm, const void* c, const void* lambda,
                         const void* F, int64_t d, tfi_dtype dtype, void* out, void* stream) {
    return integrate_expsum_impl("tfi_integrate_expsum", h, nterm, c, lambda, F, d, dtype, out,
                                 nullptr, stream);
}

int tfi_integrate_expsum_cells(tfi_handle h, int32_t nterm, const void* c, const void* lambda,
                               const void* F, int64_t d, tfi_dtype dtype, void* out,
                               void* cells, void* stream) {
    if (!cells) {
        g_err.clear();
        return fail(TFI_ERR_ARG, "tfi_integrate_expsum_cells: null pointer");
    }
    return integrate_expsum_impl("tfi_integrate_expsum_cells", h, nterm, c, lambda, F, d, dtype,
                                 out, cells, stream);
}

namespace {
int backward_expsum_impl(const char* fn, tfi_handle h, int32_t nterm, const void* c,
                         const void* lambda, const void* F, const void* cells,
                         const void* gout, int64_t d, tfi_dtype dtype, void* dF, double* s0,
                         double* s1, void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    const std::string f(fn);
    if (!c || !lambda || !F || !gout) return fail(TFI_ERR_ARG, f + ": null pointer");
    if (nterm < 1 || nterm > tfi::kExpMaxTerms)
        return fail(TFI_ERR_ARG, f + ": need 1 <= nterm <= 16");
    if (d < 1 || d > (1 << 20)) return fail(TFI_ERR_ARG, f + ": need 1 <= d <= 2^20");
    if (dtype != TFI_F32 && dtype != TFI_F64) return fail(TFI_ERR_DTYPE, f + ": unknown dtype");
    if ((s0 == nullptr) != (s1 == nullptr))
        return fail(TFI_ERR_ARG, f + ": s0 and s1 are both given or both null");
    if (s0 && s0 == s1) return fail(TFI_ERR_ARG, f + ": s0 must not alias s1");
    if (dF && (dF == F || dF == gout || dF == cells))
        return fail(TFI_ERR_ARG, f + ": dF must not alias F, cells or gout");
    if (!dF && !s0) return TFI_OK;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == TFI_F32)
        return run_backward_expsum<float>(h, nterm, (const float*)c, (const float*)lambda,
                                          (const float*)F, (const float*)cells,
                                          (const float*)gout, (int32_t)d, (float*)dF, s0, s1,
                                          st);
    return run_backward_expsum<double>(h, nterm, (const double*)c, (const double*)lambda,
                                       (const double*)F, (const double*)cells,
                                       (const double*)gout, (int32_t)d, (double*)dF, s0, s1,
                                       st);
}
}  // namespace

int tfi_backward_expsum(tfi_handle h, int32_t nterm, const void* c, const void* lambda,
                        const void* F, const void* gout, int64_t d, tfi_dtype dtype, void* dF,
                        double* s0, double* s1, void* stream) {
    return backward_expsum_impl("tfi_backward_expsum", h, nterm, c, lambda, F, nullptr, gout, d,
                                dtype, dF, s0, s1, stream);
}

int tfi_backward_expsum_cells(tfi_handle h, int32_t nterm, const void* c, const void* lambda,
                              const void* F, const void* cells, const void* gout, int64_t d,
                              tfi_dtype dtype, void* dF, double* s0, double* s1, void* stream) {
    if (!cells) {
        g_err.clear();
        return fail(TFI_ERR_ARG, "tfi_backward_expsum_cells: null pointer");
    }
    return backward_expsum_impl("tfi_backward_expsum_cells", h, nterm, c, lambda, F, cells, gout,
                                d, dtype, dF, s0, s1, stream);
}

int64_t tfi_cell_rows(tfi_handle h) {
    g_err.clear();
    int rc = check_handle(h, false);
    if (rc) return rc;
    return std::max<int64_t>(h->val_rows, 1);
}

int64_t tfi_plan_stats(tfi_handle h, char* json, size_t cap) {
    g_err.clear();
    if (!h) return fail(TFI_ERR_ARG, "tfi_plan_stats: null handle");
    std::string s = tfi::plan_stats_json(h->plan);
    char fp[32];
    std::snprintf(fp, sizeof(fp), "%016llx", (unsigned long long)tfi::plan_fingerprint(h->plan));
    s += ",\"fingerprint\":\"" + std::string(fp) + "\",\"fft_cost\":" +
         std::to_string(h->popt.fft_cost);
    s += ",\"scatter_pick\":" + std::to_string(h->scatter_pick) +
         ",\"cell_pieces\":" + std::to_string(h->cells.npieces) +
         ",\"cell_cuts\":" + std::to_string(h->cells.ncomb) +
         ",\"hankel_jobs\":" + std::to_string(h->hk.njobs);
    s += ",\"device\":" + std::to_string(h->device) +
         ",\"device_bytes\":" + std::to_string(h->dev_bytes) +
         ",\"arrays\":{\"job_H\":\"i32\",\"job_X\":\"i32\",\"job_sign\":\"i32\","
         "\"job_method\":\"i32\",\"job_level\":\"i32\",\"job_lg1\":\"i32\",\"job_lg2\":\"i32\","
         "\"job_cell_off\":\"i64\",\"jc_r\":\"i32\",\"jc_x\":\"i32\",\"jc_val\":\"i32\","
         "\"inc_v\":\"i32\",\"b_inc_off\":\"i64\",\"a_b_off\":\"i64\",\"b2a\":\"i32\","
         "\"b_corr\":\"i8\",\"v_off\":\"i64\",\"v_b\":\"i32\",\"leaf_off\":\"i64\","
         "\"leaf_v\":\"i32\",\"leaf_doff\":\"i64\",\"leaf_D\":\"i32\","
         "\"cells_piece\":\"i32\",\"cells_seg\":\"i32\",\"cells_bent\":\"i32\","
         "\"cells_aent\":\"i32\",\"cells_comb\":\"i32\"}}";
    if (json && cap > 0) {
        size_t n = std::min(cap - 1, s.size());
        std::memcpy(json, s.data(), n);
        json[n] = 0;
    }
    return (int64_t)s.size();
}

int64_t tfi_plan_export(tfi_handle h, const char* name, void* buf, size_t cap) {
    g_err.clear();
    if (!h || !name) return fail(TFI_ERR_ARG, "tfi_plan_export: null argument");
    const tfi::Plan& p = h->plan;
    const void* src = nullptr;
    size_t bytes = 0;
    auto pick = [&](const auto& v) {
        src = v.data();
        bytes = v.size() * sizeof(v[0]);
    };
    std::string n(name);
    if (n == "job_H") pick(p.job_H);
    else if (n == "job_X") pick(p.job_X);
    else if (n == "job_sign") pick(p.job_sign);
    else if (n == "job_method") pick(p.job_method);
    else if (n == "job_level") pick(p.job_level);
    else if (n == "job_lg1") pick(p.job_lg1);
    else if (n == "job_lg2") pick(p.job_lg2);
    else if (n == "job_cell_off") pick(p.job_cell_off);
    else if (n == "jc_r") pick(p.jc_r);
    else if (n == "jc_x") pick(p.jc_x);
    else if (n == "jc_val") pick(p.jc_val);
    else if (n == "inc_v") pick(p.inc_v);
    else if (n == "b_inc_off") pick(p.b_inc_off);
    else if (n == "a_b_off") pick(p.a_b_off);
    else if (n == "b2a") pick(p.b2a);
    else if (n == "b_corr") pick(p.b_corr);
    else if (n == "v_off") pick(p.v_off);
    else if (n == "v_b") pick(p.v_b);
    else if (n == "leaf_off") pick(p.leaf_off);
    else if (n == "leaf_v") pick(p.leaf_v);
    else if (n == "leaf_doff") pick(p.leaf_doff);
    else if (n == "leaf_D") pick(p.leaf_D);
    else if (n.rfind("cells_", 0) == 0) {
        // the cell-sum kernel's piece arrays (planned again here, so
        // host-only handles export them too)
        static thread_local CellHost H;
        const int rc = plan_cells(p, H);
        if (rc) return rc;
        const std::string k = n.substr(6);
        if (k == "piece") pick(H.piece);
        else if (k == "seg") pick(H.seg);
        else if (k == "bent") pick(H.bent);
        else if (k == "aent") pick(H.aent);
        else if (k == "comb") pick(H.comb);
        else return fail(TFI_ERR_ARG, "tfi_plan_export: unknown array '" + n + "'");
    }
    else return fail(TFI_ERR_ARG, "tfi_plan_export: unknown array '" + n + "'");
    if (buf && cap >= bytes && bytes) std::memcpy(buf, src, bytes);
    return (int64_t)bytes;
}

int tfi_integrate_noalloc(tfi_handle h, const void* f, const void* F, int64_t d,
                          tfi_dtype dtype, void* out, void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!f || !F || !out) return fail(TFI_ERR_ARG, "tfi_integrate_noalloc: null pointer");
    if (d < 1 || d > (1 << 20))
        return fail(TFI_ERR_ARG, "tfi_integrate_noalloc: need 1 <= d <= 2^20");
    if (F == out) return fail(TFI_ERR_ARG, "tfi_integrate_noalloc: out must not alias F");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == TFI_F32)
        return run_forward_noalloc<float>(h, (const float*)f, (const float*)F, (int32_t)d,
                                          (float*)out, st);
    if (dtype == TFI_F64)
        return run_forward_noalloc<double>(h, (const double*)f, (const double*)F, (int32_t)d,
                                           (double*)out, st);
    return fail(TFI_ERR_DTYPE, "tfi_integrate_noalloc: unknown dtype");
}

int tfi_set_scatter(tfi_handle h, int32_t method) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (method < -1 || method > 1) return fail(TFI_ERR_ARG, "tfi_set_scatter: method must be -1, 0 or 1");
    if (h->scatter_pick != method) {
        TFI_HIP(hipDeviceSynchronize());
        h->drop_graphs();  // they hold the other strategy's launches
        h->scatter_pick = method;
    }
    return TFI_OK;
}

int tfi_set_fft_cost(tfi_handle h, float cost) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!(cost > 0.0f)) return fail(TFI_ERR_ARG, "tfi_set_fft_cost: cost must be > 0");
    return reassign_methods(h, cost);
}

}  // extern "C"

namespace {

// Cost model of the channel-aware policy, measured on the handle's plan
// (see tfi_calibrate): stage times of profiled passes with every table job
// on one evaluator, per unit of that evaluator's work.
template <typename T>
int calibrate(tfi_plan* h, const T* f, int32_t d, hipStream_t st, float* costs) {
    const tfi::Plan& p = h->plan;
    const double keep = h->popt.fft_cost;
    double c2 = 0, plp = 0;
    for (size_t j = 0; j + 1 < p.job_cell_off.size(); ++j) {
        const double c = (double)(p.job_cell_off[j + 1] - p.job_cell_off[j]);
        c2 += c * c;
        const double P = std::ldexp(1.0, p.job_lg1[j] + p.job_lg2[j]);
        plp += P * std::log2(std::max(P, 2.0));
    }
    // every table through the scatter/gather path while measuring (the
    // restoring reassignment below recomputes the whole-path flags)
    const bool keep_prof = h->prof;
    int rc = drain_profile(h);
    if (rc) return rc;
    h->tally.clear();
    double rows_s = 0, dir_s = -1, fft_s = -1;
    for (int mode = 0; mode < 2 && !rc; ++mode) {
        if (mode == 0 && c2 * (double)d > 4e11) continue;  // all-direct too large
        if ((rc = reassign_methods(h, mode == 0 ? 1e30 : 1e-30))) break;
        h->path_mode[0] = h->path_mode[1] = false;
        h->prof = true;
        float ms = 0;
        rc = time_pass<T>(h, f, d, st, 1, false, &ms);  // 3 profiled passes
        h->prof = keep_prof;
        if (!rc) rc = drain_profile(h);
        if (rc) break;
        double rows = 0, tab = 0;
        for (auto& kv : h->tally) {
            const std::string& k = kv.first;
            if (k == "scatter" || k == "scatter_tail" || k == "gather") rows += kv.second.ms;
            const bool is_dir = k == "direct" || k == "direct_mfma";
            const bool is_fft = k.rfind("fft", 0) == 0 || k.rfind("spectrum", 0) == 0;
            if (mode == 0 ? is_dir : is_fft) tab += kv.second.ms;
        }
        h->tally.clear();
        rows_s = 1e-3 * rows / 3.0;
        (mode == 0 ? dir_s : fft_s) = 1e-3 * tab / 3.0;
    }
    h->prof = keep_prof;
    int rc2 = reassign_methods(h, keep);
    if (rc) return rc;
    if (rc2) return rc2;
    const double dd = (double)d;
    costs[0] = p.incidences > 0 ? (float)(rows_s / (dd * (double)p.incidences)) : 0.0f;
    costs[2] = (fft_s > 0 && plp > 0) ? (float)(fft_s / (dd * plp)) : 4.0f;
    costs[1] = (dir_s > 0 && c2 > 0) ? (float)(dir_s / (dd * c2)) : (float)(costs[2] / keep);
    costs[3] = 0.0f;
    return TFI_OK;
}

}  // namespace

extern "C" {

int tfi_calibrate(tfi_handle h, const void* f, int64_t d, tfi_dtype dtype, float* costs,
                  void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!f || !costs) return fail(TFI_ERR_ARG, "tfi_calibrate: null pointer");
    if (d < 1 || d > (1 << 20)) return fail(TFI_ERR_ARG, "tfi_calibrate: need 1 <= d <= 2^20");
    if (dtype != TFI_F32 && dtype != TFI_F64)
        return fail(TFI_ERR_DTYPE, "tfi_calibrate: unknown dtype");
    if (h->popt.table_method != 0)
        return fail(TFI_ERR_STATE, "tfi_calibrate: table method is forced for this handle");
    hipStream_t st = (hipStream_t)stream;
    return dtype == TFI_F32 ? calibrate<float>(h, (const float*)f, (int32_t)d, st, costs)
                            : calibrate<double>(h, (const double*)f, (int32_t)d, st, costs);
}

int tfi_autotune(tfi_handle h, const void* f, int64_t d, tfi_dtype dtype, int with_backward,
                 float* best_cost, void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!f || !best_cost) return fail(TFI_ERR_ARG, "tfi_autotune: null pointer");
    if (d < 1 || d > (1 << 20)) return fail(TFI_ERR_ARG, "tfi_autotune: need 1 <= d <= 2^20");
    if (dtype != TFI_F32 && dtype != TFI_F64)
        return fail(TFI_ERR_DTYPE, "tfi_autotune: unknown dtype");
    hipStream_t st = (hipStream_t)stream;
    const float cands[] = {0.25f, 1.0f, 2.0f, 4.0f, 8.0f, 16.0f, 32.0f, 64.0f};
    float best = (float)h->popt.fft_cost, best_ms = 1e30f;
    // a forced table method keeps its assignment: no cost constant to scan
    for (float c : cands) {
        if (h->popt.table_method != 0) break;
        if ((rc = reassign_methods(h, c))) return rc;
        float ms = 1e30f;
        rc = dtype == TFI_F32 ? time_pass<float>(h, (const float*)f, (int32_t)d, st, 5,
                                                 with_backward != 0, &ms)
                              : time_pass<double>(h, (const double*)f, (int32_t)d, st, 5,
                                                  with_backward != 0, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    if (h->popt.table_method == 0 && (rc = reassign_methods(h, best))) return rc;
    // the cell-sum strategy at this width: pieces or levels, the faster pass
    float sms[2] = {1e30f, 1e30f};
    for (int m = 0; m < 2 && !rc; ++m) {
        h->scatter_pick = m;
        rc = dtype == TFI_F32 ? time_pass<float>(h, (const float*)f, (int32_t)d, st, 5,
                                                 with_backward != 0, &sms[m])
                              : time_pass<double>(h, (const double*)f, (int32_t)d, st, 5,
                                                  with_backward != 0, &sms[m]);
    }
    h->scatter_pick = sms[0] <= sms[1] ? 0 : 1;
    if (rc) return rc;
    *best_cost = best;
    return TFI_OK;
}

int tfi_autotune_fft(tfi_handle h, const void* f, int64_t d, tfi_dtype dtype, int with_backward,
                     void* stream) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!f) return fail(TFI_ERR_ARG, "tfi_autotune_fft: null pointer");
    if (d < 1 || d > (1 << 20)) return fail(TFI_ERR_ARG, "tfi_autotune_fft: need 1 <= d <= 2^20");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == TFI_F32)
        return tune_fft<float>(h, (const float*)f, (int32_t)d, st, with_backward != 0);
    if (dtype == TFI_F64)
        return tune_fft<double>(h, (const double*)f, (int32_t)d, st, with_backward != 0);
    return fail(TFI_ERR_DTYPE, "tfi_autotune_fft: unknown dtype");
}

int tfi_set_fft_params(tfi_handle h, const tfi_fft_params* p) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if (!p) return fail(TFI_ERR_ARG, "tfi_set_fft_params: null pointer");
    auto pow2_or0 = [](int32_t v, int32_t hi) { return v == 0 || (v > 0 && v <= hi && !(v & (v - 1))); };
    for (int t = 0; t < 3; ++t)
        if (!pow2_or0(p->lds_pairs[t], 64))
            return fail(TFI_ERR_ARG, "tfi_set_fft_params: lds_pairs must be 0 or a power of two <= 64");
    if (p->conv1d_min_lg < 2 || p->conv1d_min_lg > 31)
        return fail(TFI_ERR_ARG, "tfi_set_fft_params: conv1d_min_lg outside [2, 31]");
    if (!pow2_or0(p->conv1d_pairs, 16))
        return fail(TFI_ERR_ARG, "tfi_set_fft_params: conv1d_pairs must be 0 or a power of two <= 16");
    if (p->conv1d_group_mib < 0 || p->conv1d_group_mib > (1 << 20))
        return fail(TFI_ERR_ARG, "tfi_set_fft_params: conv1d_group_mib outside [0, 2^20]");
    if (p->col_lines < 1 || p->col_lines > 64 || (p->col_lines & (p->col_lines - 1)))
        return fail(TFI_ERR_ARG, "tfi_set_fft_params: col_lines must be a power of two <= 64");
    FftParams q;
    for (int t = 0; t < 3; ++t) q.lds_pairs[t] = p->lds_pairs[t];
    q.conv1d_min_lg = p->conv1d_min_lg;
    q.conv1d_pairs = p->conv1d_pairs;
    q.conv1d_group_mib = p->conv1d_group_mib;
    q.col_lines = p->col_lines;
    return apply_fft_params(h, q);
}

int tfi_get_fft_params(tfi_handle h, tfi_fft_params* p) {
    g_err.clear();
    if (!h || !p) return fail(TFI_ERR_ARG, "tfi_get_fft_params: null argument");
    for (int t = 0; t < 3; ++t) p->lds_pairs[t] = h->fp.lds_pairs[t];
    p->conv1d_min_lg = h->fp.conv1d_min_lg;
    p->conv1d_pairs = h->fp.conv1d_pairs;
    p->conv1d_group_mib = h->fp.conv1d_group_mib;
    p->col_lines = h->fp.col_lines;
    return TFI_OK;
}

int tfi_profile(tfi_handle h, int enable) {
    g_err.clear();
    if (!h) return fail(TFI_ERR_ARG, "tfi_profile: null handle");
    h->prof = enable != 0;
    return TFI_OK;
}

int64_t tfi_profile_report(tfi_handle h, char* json, size_t cap) {
    g_err.clear();
    int rc = check_handle(h, true);
    if (rc) return rc;
    if ((rc = drain_profile(h))) return rc;
    std::string s = "{";
    bool first = true;
    char buf[256];
    for (auto& kv : h->tally) {
        std::snprintf(buf, sizeof(buf),
                      "%s\"%s\":{\"launches\":%lld,\"ms\":%.6f,\"bytes\":%.1f,\"flops\":%.1f}",
                      first ? "" : ",", kv.first.c_str(), (long long)kv.second.launches,
                      kv.second.ms, kv.second.bytes, kv.second.flops);
        s += buf;
        first = false;
    }
    s += "}";
    h->tally.clear();
    if (json && cap > 0) {
        size_t n = std::min(cap - 1, s.size());
        std::memcpy(json, s.data(), n);
        json[n] = 0;
    }
    return (int64_t)s.size();
}

void tfi_destroy(tfi_handle h) { delete h; }

const char* tfi_last_error(void) { return g_err.c_str(); }

}  // extern "C"
