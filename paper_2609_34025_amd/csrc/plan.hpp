// plan.hpp -- host-side decomposition of a forest into table jobs, the
// scatter/gather incidence structure and dense leaf tiles.
//
// The recursion of algorithm "Solve" (appendix, recursion pseudocode) is
// flattened: every call's cross term depends only on the field restricted
// to that call, never on another call's output, so
//     out[v] = sum over calls S containing v of Cross_S(v)
// plus the dense value of the leaf tile that finally holds v. All calls of
// all levels therefore form one independent batch of table jobs.
//
// Per non-leaf call S with backbone P (weighted lattice coordinates x_t,
// off-backbone depths r = weighted distance to P), the aggregate table
// A_r[x] (Section 2.2) has one "A-cell" per occupied (r, x). Each A-cell is
// the union of "b-cells" (r, x, component): the component's depth profile
// b_alpha[r] (equation "stad-E"). A call job evaluates
//     G[q][s] = sum_{r, t} f(q + r + |s - t|) A[r][t]
// at its own occupied cells; a correction job evaluates
//     E_alpha[q] = sum_r f(q + r) b_alpha[r]
// at the component's b-cells (a table with X = 0). Lemma "stad-cross":
// a backbone vertex takes G_0[x], a component vertex G_{r}[x] - E[r].
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace tfi {

// Evaluation of a table job: direct sums, one FFT convolution on the padded
// lattice (lemma "stad-2d-fft"), or -- tables with several depths and
// several backbone positions only -- 1-D FFT convolutions along the
// backbone for every pair of depths (algorithm "global-anchor"), or the
// product with the Hankel matrix f(l + r) followed by walks along the
// backbone (the attention-width appendix "Hankel-GEMM"; depth H <= 127).
enum Method : int32_t { METHOD_DIRECT = 0, METHOD_FFT = 1, METHOD_FFT1D = 2, METHOD_HANKEL = 3 };
constexpr int32_t kHankelMaxDepth = 127;

struct PlanOptions {
    int32_t policy = 0;       // 0 adaptive, 1 diameter, 2 centroid, 3 channel-aware
    int32_t leaf_max = 32;    // dense tiles for subtrees up to this size
    int32_t table_method = 0; // 0 choose, 1 direct, 2 fft, 3 fft1d, 4 hankel (2-D tables)
    double fft_cost = 4.0;    // direct iff cells^2 <= fft_cost * P log2 P; a table with
                              // 0 < H <= 127 and X > 0 takes the Hankel product when
                              // (H + X + 1)(X + 1)(H + 3) is below both
    // channel-aware cost model (policy 3): a candidate backbone costs
    // cost_call per table job + chan_width x (cost_vertex per incidence,
    // cost_direct per direct cell pair, cost_fft per P log2 P of an FFT)
    int32_t chan_width = 1;
    double cost_vertex = 1.0, cost_direct = 1.0, cost_fft = 4.0, cost_call = 0.0;
};

struct Plan {
    int64_t N = 0;
    int64_t roots = 0;

    // ---- table jobs (call jobs: sign +1; correction jobs: sign -1) ------
    std::vector<int32_t> job_H, job_X, job_sign, job_method, job_level;
    std::vector<int32_t> job_lg1, job_lg2;  // log2 of padded FFT sizes
    std::vector<int64_t> job_cell_off;      // [J+1] into jc_*
    std::vector<int32_t> jc_r, jc_x;        // cell coordinates
    std::vector<int32_t> jc_val;            // value row: A-cell a, or NA + b

    // ---- scatter: b-cells are runs of incidences, A-cells runs of b-cells
    int64_t NA = 0, NB = 0;
    std::vector<int32_t> inc_v;             // [I] vertex per incidence
    std::vector<int64_t> b_inc_off;         // [NB+1]
    std::vector<int64_t> a_b_off;           // [NA+1]
    std::vector<int32_t> b2a;               // [NB] A-cell holding b
    std::vector<int8_t> b_corr;             // [NB] 1 if b belongs to a
                                            // component (has a correction)

    // ---- gather: per vertex, the b-cells that hold it ---------------------
    std::vector<int64_t> v_off;             // [N+1]
    std::vector<int32_t> v_b;               // b-cell ids

    // ---- dense leaf tiles --------------------------------------------------
    std::vector<int64_t> leaf_off;          // [NL+1] into leaf_v
    std::vector<int32_t> leaf_v;            // vertices, ascending per tile
    std::vector<int64_t> leaf_doff;         // [NL+1] into leaf_D
    std::vector<int32_t> leaf_D;            // row-major n x n distances

    // ---- statistics ----------------------------------------------------------
    int64_t kernel_len = 1;   // entries of f read by any stage
    int64_t max_backbone = 0; // longest backbone or leaf-tile distance
    int32_t leaf_max = 0;     // dense-tile size the plan was built with
    int64_t calls = 0, leaf_calls = 0, singleton_calls = 0;
    int64_t diam_choices = 0, centroid_choices = 0;
    int32_t levels = 0;
    int64_t incidences = 0;   // sum over table calls of |V(S)|
    int64_t sum_cells = 0;    // sum of A-cells + b-cells
    int64_t sum_M = 0;        // sum of (H+1)(X+1) over call jobs
    int64_t sum_P = 0;        // padded FFT cells over FFT jobs
    int64_t leaf_pairs = 0;   // sum of n^2 over leaf tiles
    int32_t root_m = 0, root_X = 0, root_H = 0, root_choice = -1;
    std::vector<int32_t> root_comp_sizes;
    double root_score_diam = 0, root_score_cent = 0;
};

// Returns 0 or a negative tfi_status; err receives a message.
int build_plan(const int64_t* parent, const int32_t* weight, int64_t N,
               const PlanOptions& opt, Plan& plan, std::string& err);

// Per-job evaluation method (direct sums or FFT) from the cost rule
// cells^2 <= fft_cost * P log2 P, or forced by opt.table_method.
void assign_methods(Plan& plan, const PlanOptions& opt);

// 64-bit FNV-1a hash of the plan's shape (job sizes and depths), the key of
// tuned settings.
uint64_t plan_fingerprint(const Plan& p);

// Score of equation "stad-score" with natural logarithms.
double backbone_score(int64_t nS, int64_t M, const std::vector<int64_t>& compH,
                      const std::vector<int64_t>& compN);

std::string plan_stats_json(const Plan& p);

}  // namespace tfi
