// plan.cpp -- host planner: adaptive backbone recursion flattened into
// table jobs, incidence (scatter/gather) arrays and dense leaf tiles.
//
// Follows Section 2 and the appendix pseudocode: "ChooseBackbone"
// (diameter by two traversals, centroid by subtree sizes, score of
// equation "stad-score", centroid only if strictly cheaper),
// "DecomposeOffPathComponents" (components, anchors, projections, depths)
// and the recursion "Solve". Distances are weighted: the backbone
// coordinate of p_t is its weighted distance from p_1 and the depth of a
// vertex is its weighted distance to the backbone, so the lemma
// "stad-distance" reads dist(u, v) = d(u) + |x_s - x_t| + d(v) on the
// integer lattice (an edge of length w behaves as w unit edges whose
// interior points carry no field).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <map>
#include <numeric>
#include <sstream>
#include <utility>

namespace tfi {

namespace {

constexpr int kOk = 0, kErrArg = -1, kErrTree = -2, kErrWeight = -3,
              kErrOom = -5;
constexpr int64_t kMaxCoord = std::numeric_limits<int32_t>::max() / 4;

struct Forest {
    int64_t n = 0;
    std::vector<int64_t> off;
    std::vector<int32_t> nbr, len;
};

int make_forest(const int64_t* parent, const int32_t* weight, int64_t n,
                Forest& t, std::vector<int32_t>& roots, std::string& err) {
    if (n < 1 || !parent || !weight) {
        err = "tfi_build: need N >= 1 and non-null parent/weight";
        return kErrArg;
    }
    if (n > std::numeric_limits<int32_t>::max() / 2) {
        err = "tfi_build: N too large for 32-bit vertex ids";
        return kErrArg;
    }
    t.n = n;
    t.off.assign(n + 1, 0);
    int64_t edges = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t p = parent[v];
        if (p < -1 || p >= n || p == v) {
            err = "tfi_build: parent[" + std::to_string(v) + "] = " +
                  std::to_string(p) + " is out of range or a self loop";
            return kErrTree;
        }
        if (p < 0) {
            roots.push_back((int32_t)v);
            continue;
        }
        if (weight[v] < 1) {
            err = "tfi_build: weight[" + std::to_string(v) + "] = " +
                  std::to_string(weight[v]) + " must be >= 1";
            return kErrWeight;
        }
        t.off[v + 1]++;
        t.off[p + 1]++;
        edges++;
    }
    for (int64_t v = 0; v < n; ++v) t.off[v + 1] += t.off[v];
    t.nbr.resize(2 * edges);
    t.len.resize(2 * edges);
    std::vector<int64_t> fill(t.off.begin(), t.off.end() - 1);
    for (int64_t v = 0; v < n; ++v) {
        int64_t p = parent[v];
        if (p < 0) continue;
        t.nbr[fill[v]] = (int32_t)p;
        t.len[fill[v]++] = weight[v];
        t.nbr[fill[p]] = (int32_t)v;
        t.len[fill[p]++] = weight[v];
    }
    // every vertex must be reached exactly once from the roots
    std::vector<int8_t> seen(n, 0);
    std::vector<int32_t> stack;
    int64_t count = 0;
    for (int32_t r : roots) {
        seen[r] = 1;
        stack.push_back(r);
        while (!stack.empty()) {
            int32_t x = stack.back();
            stack.pop_back();
            ++count;
            for (int64_t k = t.off[x]; k < t.off[x + 1]; ++k) {
                int32_t y = t.nbr[k];
                if (!seen[y]) {
                    seen[y] = 1;
                    stack.push_back(y);
                }
            }
        }
    }
    if (count != n || edges != n - (int64_t)roots.size()) {
        err = "tfi_build: parent pointers contain a cycle";
        return kErrTree;
    }
    return kOk;
}

struct Decomp {
    std::vector<int32_t> P;       // backbone p_1..p_m
    std::vector<int64_t> px;      // lattice coordinate of p_t
    int64_t H = 0, X = 0;
    std::vector<int64_t> cH, cN;  // per component: depth, size
    std::vector<int32_t> cAnchor; // index t of the anchor p_t
    std::vector<int64_t> cOff;    // [k+1] into cv / cr
    std::vector<int32_t> cv;      // component vertices
    std::vector<int64_t> cr;      // their depths
    void clear() {
        P.clear(); px.clear(); H = X = 0;
        cH.clear(); cN.clear(); cAnchor.clear(); cOff.clear();
        cv.clear(); cr.clear();
    }
};

int64_t next_pow2(int64_t x);
int32_t ilog2(int64_t p);

class Planner {
  public:
    Planner(const Forest& t, const PlanOptions& o, Plan& p)
        : T(t), opt(o), plan(p), stamp(t.n, -1), pstamp(t.n, -1),
          dist(t.n, 0), from(t.n, -1), sz(t.n, 0), cmax(t.n, 0),
          loc(t.n, -1) {}

    int run(const std::vector<int32_t>& roots, std::string& err);

  private:
    const Forest& T;
    const PlanOptions& opt;
    Plan& plan;
    std::vector<int32_t> stamp, pstamp;
    int32_t cur = -1, curp = -1;
    std::vector<int64_t> dist;
    std::vector<int32_t> from, order, stk;
    std::vector<int64_t> sz, cmax;
    std::vector<int32_t> loc;
    bool overflow = false;
    Decomp dA, dB;
    std::vector<std::pair<int32_t, int32_t>> vinc;  // (vertex, b-cell)
    struct Rec { int32_t x, r, c, v; };
    std::vector<Rec> recs;
    std::vector<int64_t> keys, rk;  // scratch of chan_score

    // Traverse the current call from src (entered from `par`, starting
    // distance d0), skipping backbone vertices when skipP. Fills `order`
    // (appending) and dist/from for the visited vertices.
    void walk(int32_t src, int32_t par, int64_t d0, bool skipP) {
        stk.clear();
        stk.push_back(src);
        from[src] = par;
        dist[src] = d0;
        while (!stk.empty()) {
            int32_t x = stk.back();
            stk.pop_back();
            order.push_back(x);
            for (int64_t k = T.off[x]; k < T.off[x + 1]; ++k) {
                int32_t y = T.nbr[k];
                if (y == from[x] || stamp[y] != cur) continue;
                if (skipP && pstamp[y] == curp) continue;
                from[y] = x;
                int64_t dy = dist[x] + T.len[k];
                if (dy > kMaxCoord) overflow = true;
                dist[y] = dy;
                stk.push_back(y);
            }
        }
    }

    int32_t farthest(const std::vector<int32_t>& ord) const {
        int32_t best = ord[0];
        for (int32_t v : ord)
            if (dist[v] > dist[best] || (dist[v] == dist[best] && v < best))
                best = v;
        return best;
    }

    void diameter_path(const std::vector<int32_t>& S, std::vector<int32_t>& P) {
        int32_t start = *std::min_element(S.begin(), S.end());
        order.clear();
        walk(start, -1, 0, false);
        int32_t a = farthest(order);
        order.clear();
        walk(a, -1, 0, false);
        int32_t b = farthest(order);
        P.clear();
        for (int32_t v = b; v != -1; v = from[v]) P.push_back(v);
        std::reverse(P.begin(), P.end());  // p_1 = a
    }

    int32_t centroid(const std::vector<int32_t>& S) {
        int32_t start = *std::min_element(S.begin(), S.end());
        order.clear();
        walk(start, -1, 0, false);
        int64_t n = (int64_t)S.size();
        for (int32_t v : order) sz[v] = 1, cmax[v] = 0;
        for (size_t i = order.size(); i-- > 1;) {
            int32_t v = order[i], p = from[v];
            sz[p] += sz[v];
            cmax[p] = std::max(cmax[p], sz[v]);
        }
        int32_t best = -1;
        int64_t bestv = std::numeric_limits<int64_t>::max();
        for (int32_t v : order) {
            int64_t m = std::max(cmax[v], n - sz[v]);
            if (m < bestv || (m == bestv && v < best)) {
                bestv = m;
                best = v;
            }
        }
        return best;
    }

    // "DecomposeOffPathComponents" with weighted depths.
    void decompose(const std::vector<int32_t>& P, Decomp& D) {
        D.clear();
        D.P = P;
        ++curp;
        for (int32_t p : P) pstamp[p] = curp;
        D.px.resize(P.size());
        int64_t x = 0;
        for (size_t t = 0; t < P.size(); ++t) {
            if (t > 0) {
                // length of edge (p_{t-1}, p_t)
                int32_t a = P[t - 1], b = P[t];
                int64_t w = 0;
                for (int64_t k = T.off[a]; k < T.off[a + 1]; ++k)
                    if (T.nbr[k] == b) { w = T.len[k]; break; }
                x += w;
                if (x > kMaxCoord) overflow = true;
            }
            D.px[t] = x;
        }
        D.X = x;
        D.cOff.push_back(0);
        for (size_t t = 0; t < P.size(); ++t) {
            int32_t p = P[t];
            for (int64_t k = T.off[p]; k < T.off[p + 1]; ++k) {
                int32_t y = T.nbr[k];
                if (stamp[y] != cur || pstamp[y] == curp) continue;
                order.clear();
                walk(y, p, T.len[k], true);
                int64_t h = 0;
                for (int32_t u : order) {
                    D.cv.push_back(u);
                    D.cr.push_back(dist[u]);
                    h = std::max(h, dist[u]);
                }
                D.cH.push_back(h);
                D.cN.push_back((int64_t)order.size());
                D.cAnchor.push_back((int32_t)t);
                D.cOff.push_back((int64_t)D.cv.size());
                D.H = std::max(D.H, h);
            }
        }
    }

    double score(const std::vector<int32_t>& S, const Decomp& D) const {
        int64_t M = (D.H + 1) * (D.X + 1);
        return backbone_score((int64_t)S.size(), M, D.cH, D.cN);
    }

    // Per-channel cost of one table: the cheaper of direct sums over its
    // occupied cells and an FFT of its padded shape.
    double table_cost(int64_t cells, int64_t H, int64_t X) const {
        const double P = (double)(next_pow2(2 * H + 1) * next_pow2(2 * X + 1));
        const double direct = opt.cost_direct * (double)cells * (double)cells;
        const double fft = opt.cost_fft * P * std::log2(std::max(P, 2.0));
        return std::min(direct, fft);
    }

    // Channel-aware cost of a candidate (appendix "Channel-aware backbone
    // selection"): cost_call per table job of the call (its own and one
    // correction per component) plus C times the per-channel work -- the
    // call's incidences, the call's table and every correction table (each
    // at its cheaper evaluator, over its exact occupied cells), and the
    // recursion proxy n log2(n + 1) of every component (the last term of
    // equation "stad-score"), priced like incidences.
    double chan_score(const std::vector<int32_t>& S, const Decomp& D) {
        keys.clear();
        for (int64_t x : D.px) keys.push_back(x << 32);  // backbone cells: r = 0
        const size_t k = D.cN.size();
        double corr = 0, rec = 0;
        for (size_t c = 0; c < k; ++c) {
            const int64_t x = D.px[D.cAnchor[c]];
            rk.clear();
            for (int64_t i = D.cOff[c]; i < D.cOff[c + 1]; ++i) {
                keys.push_back((x << 32) | D.cr[i]);
                rk.push_back(D.cr[i]);
            }
            std::sort(rk.begin(), rk.end());
            const int64_t nb = std::unique(rk.begin(), rk.end()) - rk.begin();
            corr += table_cost(nb, D.cH[c], 0);
            rec += (double)D.cN[c] * std::log2((double)D.cN[c] + 1.0);
        }
        std::sort(keys.begin(), keys.end());
        const int64_t cells = std::unique(keys.begin(), keys.end()) - keys.begin();
        const double chan =
            opt.cost_vertex * ((double)S.size() + rec) + table_cost(cells, D.H, D.X) + corr;
        return opt.cost_call * (double)(1 + k) + (double)opt.chan_width * chan;
    }

    void emit_leaf(const std::vector<int32_t>& S);
    void emit_table(const Decomp& D, int32_t level);
};

void Planner::emit_leaf(const std::vector<int32_t>& S0) {
    std::vector<int32_t> S(S0);
    std::sort(S.begin(), S.end());
    int64_t n = (int64_t)S.size();
    plan.leaf_calls++;
    if (n == 1) plan.singleton_calls++;
    for (int64_t i = 0; i < n; ++i) loc[S[i]] = (int32_t)i;
    for (int32_t v : S) plan.leaf_v.push_back(v);
    plan.leaf_off.push_back((int64_t)plan.leaf_v.size());
    size_t base = plan.leaf_D.size();
    plan.leaf_D.resize(base + n * n);
    for (int64_t i = 0; i < n; ++i) {
        order.clear();
        walk(S[i], -1, 0, false);
        for (int32_t u : order) {
            plan.leaf_D[base + i * n + loc[u]] = (int32_t)dist[u];
            plan.kernel_len = std::max(plan.kernel_len, dist[u] + 1);
            plan.max_backbone = std::max(plan.max_backbone, dist[u]);
        }
    }
    plan.leaf_doff.push_back((int64_t)plan.leaf_D.size());
    plan.leaf_pairs += n * n;
}

void Planner::emit_table(const Decomp& D, int32_t level) {
    // incidence records sorted by (x, r, component, vertex)
    recs.clear();
    for (size_t t = 0; t < D.P.size(); ++t)
        recs.push_back({(int32_t)D.px[t], 0, -1, D.P[t]});
    for (size_t c = 0; c + 1 < D.cOff.size(); ++c) {
        int32_t x = (int32_t)D.px[D.cAnchor[c]];
        for (int64_t i = D.cOff[c]; i < D.cOff[c + 1]; ++i)
            recs.push_back({x, (int32_t)D.cr[i], (int32_t)c, D.cv[i]});
    }
    std::sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) {
        if (a.x != b.x) return a.x < b.x;
        if (a.r != b.r) return a.r < b.r;
        if (a.c != b.c) return a.c < b.c;
        return a.v < b.v;
    });
    const int64_t k = (int64_t)D.cH.size();
    std::vector<std::vector<int32_t>> compCells(k);
    // call job header
    plan.job_H.push_back((int32_t)D.H);
    plan.job_X.push_back((int32_t)D.X);
    plan.job_sign.push_back(1);
    plan.job_level.push_back(level);
    size_t i = 0;
    while (i < recs.size()) {
        // one A-cell: same (x, r)
        int32_t x = recs[i].x, r = recs[i].r;
        int64_t a = plan.NA++;
        plan.jc_r.push_back(r);
        plan.jc_x.push_back(x);
        plan.jc_val.push_back((int32_t)a);
        while (i < recs.size() && recs[i].x == x && recs[i].r == r) {
            int32_t c = recs[i].c;
            int64_t b = plan.NB++;
            plan.b2a.push_back((int32_t)a);
            plan.b_corr.push_back(c >= 0 ? 1 : 0);
            if (c >= 0) compCells[c].push_back((int32_t)b);
            while (i < recs.size() && recs[i].x == x && recs[i].r == r &&
                   recs[i].c == c) {
                plan.inc_v.push_back(recs[i].v);
                vinc.emplace_back(recs[i].v, (int32_t)b);
                ++i;
            }
            plan.b_inc_off.push_back((int64_t)plan.inc_v.size());
        }
        plan.a_b_off.push_back(plan.NB);
    }
    plan.job_cell_off.push_back((int64_t)plan.jc_r.size());
    // correction jobs: one per component, cells = its b-cells (X = 0)
    for (int64_t c = 0; c < k; ++c) {
        plan.job_H.push_back((int32_t)D.cH[c]);
        plan.job_X.push_back(0);
        plan.job_sign.push_back(-1);
        plan.job_level.push_back(level);
        for (int32_t b : compCells[c]) {
            // depth of the b-cell = r of its A-cell
            plan.jc_r.push_back(-1);  // filled below
            plan.jc_x.push_back(0);
            plan.jc_val.push_back(-(b + 1));  // fixed up to NA + b at the end
        }
        plan.job_cell_off.push_back((int64_t)plan.jc_r.size());
    }
    plan.incidences += (int64_t)recs.size();
    plan.sum_M += (D.H + 1) * (D.X + 1);
    plan.max_backbone = std::max(plan.max_backbone, D.X);
}

int Planner::run(const std::vector<int32_t>& roots, std::string& err) {
    plan.job_cell_off.assign(1, 0);
    plan.b_inc_off.assign(1, 0);
    plan.a_b_off.assign(1, 0);
    plan.leaf_off.assign(1, 0);
    plan.leaf_doff.assign(1, 0);
    const int32_t leaf_max = std::max<int32_t>(1, opt.leaf_max);

    // components of the forest are the level-0 calls
    std::vector<std::vector<int32_t>> level_calls, next;
    {
        std::vector<int32_t> S;
        ++cur;
        for (int32_t r : roots) {
            S.clear();
            std::vector<int32_t> st{r};
            stamp[r] = cur;
            while (!st.empty()) {
                int32_t x = st.back();
                st.pop_back();
                S.push_back(x);
                for (int64_t k = T.off[x]; k < T.off[x + 1]; ++k) {
                    int32_t y = T.nbr[k];
                    if (stamp[y] != cur) {
                        stamp[y] = cur;
                        st.push_back(y);
                    }
                }
            }
            level_calls.push_back(S);
        }
    }
    bool first = true;
    int32_t level = 0;
    while (!level_calls.empty()) {
        next.clear();
        for (auto& S : level_calls) {
            ++cur;
            for (int32_t v : S) stamp[v] = cur;
            plan.calls++;
            if ((int64_t)S.size() <= leaf_max) {
                emit_leaf(S);
                if (overflow) {
                    err = "tfi_build: a weighted distance exceeds the 32-bit "
                          "lattice range";
                    return kErrWeight;
                }
                continue;
            }
            // candidates (algorithm "ChooseBackbone")
            std::vector<int32_t> Pd, Pc;
            double sd = 0, sc = 0;
            int choice;
            if (opt.policy == 1) {
                diameter_path(S, Pd);
                decompose(Pd, dA);
                choice = 0;
            } else if (opt.policy == 2) {
                Pc.assign(1, centroid(S));
                decompose(Pc, dA);
                choice = 1;
            } else {
                diameter_path(S, Pd);
                decompose(Pd, dA);
                sd = opt.policy == 3 ? chan_score(S, dA) : score(S, dA);
                Pc.assign(1, centroid(S));
                decompose(Pc, dB);
                sc = opt.policy == 3 ? chan_score(S, dB) : score(S, dB);
                // the centroid only if strictly cheaper; diameter wins ties
                choice = (sc < sd) ? 1 : 0;
                if (choice == 1) std::swap(dA, dB);
            }
            if (overflow) {
                err = "tfi_build: a weighted distance exceeds the 32-bit "
                      "lattice range";
                return kErrWeight;
            }
            if (choice == 0) plan.diam_choices++; else plan.centroid_choices++;
            if (first) {
                plan.root_m = (int32_t)dA.P.size();
                plan.root_X = (int32_t)dA.X;
                plan.root_H = (int32_t)dA.H;
                plan.root_choice = choice;
                plan.root_score_diam = sd;
                plan.root_score_cent = sc;
                for (int64_t c : dA.cN) plan.root_comp_sizes.push_back((int32_t)c);
                first = false;
            }
            emit_table(dA, level);
            for (size_t c = 0; c + 1 < dA.cOff.size(); ++c)
                next.emplace_back(dA.cv.begin() + dA.cOff[c],
                                  dA.cv.begin() + dA.cOff[c + 1]);
        }
        level_calls.swap(next);
        ++level;
    }
    plan.levels = level;

    // fix up correction-job cells: value rows live after the A-cells
    for (size_t j = 0; j < plan.jc_val.size(); ++j)
        if (plan.jc_val[j] < 0)
            plan.jc_val[j] = (int32_t)(plan.NA + (-plan.jc_val[j] - 1));
    // depth of a b-cell = depth of its A-cell
    {
        std::vector<int32_t> a_r(plan.NA);
        const int64_t J = (int64_t)plan.job_H.size();
        for (int64_t j = 0; j < J; ++j) {
            if (plan.job_sign[j] < 0) continue;
            for (int64_t c = plan.job_cell_off[j]; c < plan.job_cell_off[j + 1]; ++c)
                a_r[plan.jc_val[c]] = plan.jc_r[c];
        }
        for (size_t j = 0; j < plan.jc_val.size(); ++j)
            if (plan.jc_r[j] < 0)
                plan.jc_r[j] = a_r[plan.b2a[plan.jc_val[j] - plan.NA]];
    }
    // vertex-major gather lists
    plan.v_off.assign(T.n + 1, 0);
    for (auto& e : vinc) plan.v_off[e.first + 1]++;
    for (int64_t v = 0; v < T.n; ++v) plan.v_off[v + 1] += plan.v_off[v];
    plan.v_b.resize(vinc.size());
    {
        std::vector<int64_t> fill(plan.v_off.begin(), plan.v_off.end() - 1);
        for (auto& e : vinc) plan.v_b[fill[e.first]++] = e.second;
    }
    vinc.clear();
    vinc.shrink_to_fit();
    return kOk;
}

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

int32_t ilog2(int64_t p) {
    int32_t l = 0;
    while ((int64_t(1) << l) < p) ++l;
    return l;
}

}  // namespace

double backbone_score(int64_t nS, int64_t M, const std::vector<int64_t>& compH,
                      const std::vector<int64_t>& compN) {
    double s = (double)nS + (double)M * std::log((double)std::max<int64_t>(M, 2));
    for (int64_t h : compH) s += (double)h * std::log((double)h + 1.0);
    for (int64_t c : compN) s += (double)c * std::log((double)c + 1.0);
    return s;
}

void assign_methods(Plan& plan, const PlanOptions& opt) {
    const int64_t J = (int64_t)plan.job_H.size();
    plan.job_method.resize(J);
    plan.sum_P = 0;
    for (int64_t j = 0; j < J; ++j) {
        const int64_t P = (int64_t)1 << (plan.job_lg1[j] + plan.job_lg2[j]);
        const int64_t nc = plan.job_cell_off[j + 1] - plan.job_cell_off[j];
        const double direct = (double)nc * (double)nc;
        const double fft = opt.fft_cost * (double)P * std::log2((double)std::max<int64_t>(P, 2));
        int32_t m;
        if (opt.table_method == 1) m = METHOD_DIRECT;
        else if (opt.table_method == 2) m = METHOD_FFT;
        else if (opt.table_method == 3)
            m = (plan.job_H[j] > 0 && plan.job_X[j] > 0) ? METHOD_FFT1D : METHOD_FFT;
        else if (opt.table_method == 4)
            m = (plan.job_H[j] > 0 && plan.job_X[j] > 0 && plan.job_H[j] <= kHankelMaxDepth)
                    ? METHOD_HANKEL
                    : METHOD_FFT;
        else {
            m = (direct <= fft) ? METHOD_DIRECT : METHOD_FFT;
            // tables with several depths and backbone positions: the Hankel
            // product and walks when their multiply-adds, (H + X + 1)(H + 1)
            // (X + 1) plus two walks over B, undercut both
            const int64_t H = plan.job_H[j], X = plan.job_X[j];
            if (H > 0 && X > 0 && H <= kHankelMaxDepth) {
                const double hank = (double)(H + X + 1) * (double)(X + 1) * (double)(H + 3);
                if (hank < std::min(direct, fft)) m = METHOD_HANKEL;
            }
        }
        plan.job_method[j] = m;
        if (m == METHOD_FFT || m == METHOD_FFT1D) plan.sum_P += P;
    }
}

uint64_t plan_fingerprint(const Plan& p) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)p.N);
    mix((uint64_t)p.NA);
    mix((uint64_t)p.NB);
    mix((uint64_t)p.leaf_D.size());
    for (size_t j = 0; j < p.job_H.size(); ++j) {
        mix((uint64_t)p.job_H[j]);
        mix((uint64_t)p.job_X[j]);
        mix((uint64_t)(p.job_cell_off[j + 1] - p.job_cell_off[j]));
    }
    return h;
}

int build_plan(const int64_t* parent, const int32_t* weight, int64_t N,
               const PlanOptions& opt, Plan& plan, std::string& err) {
    plan = Plan();
    if (opt.policy < 0 || opt.policy > 3 || opt.table_method < 0 ||
        opt.table_method > 4 || opt.leaf_max < 0 || !(opt.fft_cost > 0.0) ||
        opt.chan_width < 1 || !(opt.cost_vertex >= 0.0) || !(opt.cost_direct > 0.0) ||
        !(opt.cost_fft > 0.0) || !(opt.cost_call >= 0.0)) {
        err = "tfi_build: invalid option";
        return kErrArg;
    }
    Forest T;
    std::vector<int32_t> roots;
    int rc = make_forest(parent, weight, N, T, roots, err);
    if (rc) return rc;
    plan.N = N;
    plan.roots = (int64_t)roots.size();
    plan.leaf_max = opt.leaf_max;
    try {
        Planner pl(T, opt, plan);
        rc = pl.run(roots, err);
        if (rc) return rc;
    } catch (const std::bad_alloc&) {
        err = "tfi_build: host allocation failed while planning";
        return kErrOom;
    }
    // padded FFT sizes per job; the kernel table covers the reach of every
    // job's FFT bucket, so that re-assigning methods (autotuning) never
    // changes the number of entries of f that may be read
    const int64_t J = (int64_t)plan.job_H.size();
    plan.job_lg1.resize(J);
    plan.job_lg2.resize(J);
    std::map<std::pair<int32_t, int32_t>, std::pair<int64_t, int64_t>> bucket_hx;
    for (int64_t j = 0; j < J; ++j) {
        const int64_t H = plan.job_H[j], X = plan.job_X[j];
        plan.job_lg1[j] = ilog2(next_pow2(2 * H + 1));
        plan.job_lg2[j] = ilog2(next_pow2(2 * X + 1));
        auto& hx = bucket_hx[{plan.job_lg1[j], plan.job_lg2[j]}];
        hx.first = std::max(hx.first, H);
        hx.second = std::max(hx.second, X);
    }
    for (auto& kv : bucket_hx)
        plan.kernel_len = std::max(plan.kernel_len,
                                   2 * kv.second.first + kv.second.second + 1);
    assign_methods(plan, opt);
    plan.sum_cells = plan.NA + plan.NB;
    return kOk;
}

std::string plan_stats_json(const Plan& p) {
    std::ostringstream o;
    const int64_t J = (int64_t)p.job_H.size();
    int64_t calljobs = 0, corrjobs = 0, direct = 0, fft = 0, direct_pairs = 0;
    std::map<std::pair<int32_t, int32_t>, std::pair<int64_t, int64_t>> buckets;
    for (int64_t j = 0; j < J; ++j) {
        if (p.job_sign[j] > 0) calljobs++; else corrjobs++;
        int64_t nc = p.job_cell_off[j + 1] - p.job_cell_off[j];
        if (p.job_method[j] == METHOD_DIRECT) {
            direct++;
            direct_pairs += nc * nc;
        } else {
            fft++;
            auto& b = buckets[{p.job_lg1[j], p.job_lg2[j]}];
            b.first++;
            b.second += nc;
        }
    }
    o << "{\"N\":" << p.N << ",\"roots\":" << p.roots
      << ",\"calls\":" << p.calls << ",\"leaf_max\":" << p.leaf_max
      << ",\"leaf_calls\":" << p.leaf_calls
      << ",\"singleton_calls\":" << p.singleton_calls
      << ",\"diameter_choices\":" << p.diam_choices
      << ",\"centroid_choices\":" << p.centroid_choices
      << ",\"levels\":" << p.levels << ",\"incidences\":" << p.incidences
      << ",\"a_cells\":" << p.NA << ",\"b_cells\":" << p.NB
      << ",\"sum_M\":" << p.sum_M << ",\"sum_P\":" << p.sum_P
      << ",\"leaf_pairs\":" << p.leaf_pairs
      << ",\"table_jobs\":" << J << ",\"call_jobs\":" << calljobs
      << ",\"correction_jobs\":" << corrjobs
      << ",\"direct_jobs\":" << direct << ",\"direct_pairs\":" << direct_pairs
      << ",\"fft_jobs\":" << fft
      << ",\"kernel_length\":" << p.kernel_len << ",\"max_backbone\":" << p.max_backbone
      << ",\"root\":{\"m\":" << p.root_m << ",\"X\":" << p.root_X
      << ",\"H\":" << p.root_H << ",\"choice\":\""
      << (p.root_choice == 1 ? "centroid" : p.root_choice == 0 ? "diameter" : "leaf")
      << "\",\"score_diameter\":" << p.root_score_diam
      << ",\"score_centroid\":" << p.root_score_cent << ",\"components\":[";
    for (size_t i = 0; i < p.root_comp_sizes.size() && i < 64; ++i)
        o << (i ? "," : "") << p.root_comp_sizes[i];
    o << "]},\"fft_buckets\":[";
    bool firstb = true;
    for (auto& kv : buckets) {
        o << (firstb ? "" : ",") << "[" << (1 << kv.first.first) << ","
          << (1 << kv.first.second) << "," << kv.second.first << ","
          << kv.second.second << "]";
        firstb = false;
    }
    o << "]";
    return o.str();  // caller appends its own fields and the closing brace
}

}  // namespace tfi
