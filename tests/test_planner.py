"""Host planner tests (CPU only; host-only handles, no device).

The plan replay below evaluates, in FP64 on the host, exactly the arrays
the GPU kernels consume (cells, table jobs, scatter runs, gather lists,
leaf tiles), with every interaction table computed by direct sums. It is a
test of the planner, not a second oracle: its result is compared with the
oracle, which shares nothing with it.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2609_34025_amd import synth as S
from paper_2609_34025_amd import TreeIntegrator
from paper_2609_34025_amd._lib import TFIError

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def plan_arrays(t):
    names = ["job_H", "job_X", "job_sign", "job_cell_off", "jc_r", "jc_x", "jc_val",
             "inc_v", "b_inc_off", "a_b_off", "b2a", "b_corr", "v_off", "v_b",
             "leaf_off", "leaf_v", "leaf_doff", "leaf_D", "job_method", "job_lg1", "job_lg2"]
    return {n: t.export(n) for n in names}


def replay(t, f, F):
    """FP64 evaluation of the plan by direct table sums."""
    a = plan_arrays(t)
    NA = len(a["a_b_off"]) - 1
    NB = len(a["b2a"])
    F = F.reshape(len(F), -1)
    d = F.shape[1]
    val = np.zeros((NA + NB, d))
    for b in range(NB):
        vs = a["inc_v"][a["b_inc_off"][b]:a["b_inc_off"][b + 1]]
        val[NA + b] = F[vs].sum(0)
    for c in range(NA):
        val[c] = val[NA + a["a_b_off"][c]:NA + a["a_b_off"][c + 1]].sum(0)
    g = np.full((NA + NB, d), np.nan)
    off = a["job_cell_off"]
    for j in range(len(a["job_H"])):
        cb, ce = off[j], off[j + 1]
        r = a["jc_r"][cb:ce]
        x = a["jc_x"][cb:ce]
        vi = a["jc_val"][cb:ce]
        assert r.max() <= a["job_H"][j] and x.max() <= a["job_X"][j]
        dist = r[:, None] + r[None, :] + np.abs(x[:, None] - x[None, :])
        g[vi] = f[dist] @ val[vi]
    out = np.zeros((len(F), d))
    for v in range(len(F)):
        for b in a["v_b"][a["v_off"][v]:a["v_off"][v + 1]]:
            out[v] += g[a["b2a"][b]]
            if a["b_corr"][b]:
                out[v] -= g[NA + b]
    for L in range(len(a["leaf_off"]) - 1):
        vs = a["leaf_v"][a["leaf_off"][L]:a["leaf_off"][L + 1]]
        n = len(vs)
        D = a["leaf_D"][a["leaf_doff"][L]:a["leaf_doff"][L + 1]].reshape(n, n)
        out[vs] += f[D] @ F[vs]
    return out


def trees_for_replay():
    rng = np.random.default_rng(7)
    out = []
    p, _ = S.random_recursive(300, rng)
    out.append(("rrt300_w8", p, S.uniform_weights(p, 1, 8, rng)))
    out.append(("grid12_w16", *S.grid_mst(12, 16, rng)))
    out.append(("cater40_w5", S.caterpillar(40, 3)[0],
                S.uniform_weights(S.caterpillar(40, 3)[0], 1, 5, rng)))
    out.append(("chp8", *S.caterpillar_hanging_paths(8)))
    out.append(("spider6x9", *S.spider(6, 9)))
    out.append(("binary3", *S.balanced_kary(2, 5)))
    out.append(("broom40", *S.broom(40)))
    out.append(("star30", *S.star(30)))
    out.append(("path50_w3", S.path(50)[0], S.uniform_weights(S.path(50)[0], 1, 3, rng)))
    t1 = S.random_recursive(60, rng)
    t2 = S.grid_mst(6, 9, rng)
    fp, fw, _ = S.forest([(t1[0], S.uniform_weights(t1[0], 1, 4, rng)), t2, S.path(1)])
    out.append(("forest", fp, fw))
    return out


@pytest.mark.parametrize("policy", ["adaptive", "diameter", "centroid", "channel"])
@pytest.mark.parametrize("leaf_max", [1, 5, 32])
def test_plan_replay_matches_oracle(policy, leaf_max):
    rng = np.random.default_rng(17)
    for name, p, w in trees_for_replay():
        t = TreeIntegrator(p, w, device=None, policy=policy, leaf_max=leaf_max)
        K = t.kernel_length
        assert K >= oracle.diameter(p, w) + 1
        f = rng.standard_normal(K)
        F = rng.standard_normal((len(p), 2))
        np.testing.assert_allclose(replay(t, f, F), oracle.integrate(p, w, f, F),
                                   rtol=1e-10, atol=1e-10, err_msg=name)


def test_distance_lemma_on_every_cross_pair():
    # Lemma "stad-distance": u, v not in the same component of a call ->
    # dist = r_u + |x_u - x_v| + r_v (weighted lattice form).
    rng = np.random.default_rng(23)
    for name, p, w in trees_for_replay()[:4]:
        D = oracle.distances(p, w)
        for policy in ("adaptive", "diameter", "centroid"):
            t = TreeIntegrator(p, w, device=None, policy=policy, leaf_max=1)
            a = plan_arrays(t)
            NA = len(a["a_b_off"]) - 1
            NB = len(a["b2a"])
            comp = -np.ones(NB, dtype=np.int64)
            off = a["job_cell_off"]
            cell_r = np.zeros(NA, dtype=np.int64)
            cell_x = np.zeros(NA, dtype=np.int64)
            for j in range(len(a["job_H"])):
                vi = a["jc_val"][off[j]:off[j + 1]]
                if a["job_sign"][j] < 0:
                    comp[vi - NA] = j
                else:
                    cell_r[vi] = a["jc_r"][off[j]:off[j + 1]]
                    cell_x[vi] = a["jc_x"][off[j]:off[j + 1]]
            for j in range(len(a["job_H"])):
                if a["job_sign"][j] < 0:
                    continue
                cells = a["jc_val"][off[j]:off[j + 1]]
                us, rs, xs, cs = [], [], [], []
                for c in cells:
                    for b in range(a["a_b_off"][c], a["a_b_off"][c + 1]):
                        for v in a["inc_v"][a["b_inc_off"][b]:a["b_inc_off"][b + 1]]:
                            us.append(v)
                            rs.append(cell_r[c])
                            xs.append(cell_x[c])
                            cs.append(comp[b])
                us, rs, xs, cs = map(np.array, (us, rs, xs, cs))
                cross = (cs[:, None] != cs[None, :]) | (cs[:, None] < 0) | (cs[None, :] < 0)
                lemma = rs[:, None] + rs[None, :] + np.abs(xs[:, None] - xs[None, :])
                assert np.array_equal(D[np.ix_(us, us)][cross], lemma[cross]), name


def test_backbones_and_leaves_partition_vertices():
    rng = np.random.default_rng(29)
    for name, p, w in trees_for_replay():
        for leaf_max in (1, 8):
            t = TreeIntegrator(p, w, device=None, leaf_max=leaf_max)
            a = plan_arrays(t)
            count = np.zeros(len(p), dtype=np.int64)
            for b in np.flatnonzero(a["b_corr"] == 0):
                count[a["inc_v"][a["b_inc_off"][b]:a["b_inc_off"][b + 1]]] += 1
            np.add.at(count, a["leaf_v"], 1)
            assert np.all(count == 1), name


def _call_sizes(a):
    NA = len(a["a_b_off"]) - 1
    off = a["job_cell_off"]
    sizes = []
    for j in range(len(a["job_H"])):
        if a["job_sign"][j] < 0:
            continue
        n = 0
        for c in a["jc_val"][off[j]:off[j + 1]]:
            b0, b1 = a["a_b_off"][c], a["a_b_off"][c + 1]
            n += a["b_inc_off"][b1] - a["b_inc_off"][b0]
        sizes.append((j, n))
    return sizes


@pytest.mark.parametrize("maker", [
    lambda r: S.random_recursive(800, r), lambda r: S.random_mst_topology(300, r),
    lambda r: S.preferential_attachment(800, r), lambda r: S.balanced_kary(2, 8),
    lambda r: S.balanced_kary(3, 6), lambda r: S.caterpillar(200, 3),
    lambda r: S.caterpillar_hanging_paths(24), lambda r: S.comb(200), lambda r: S.broom(320),
    lambda r: S.double_broom(320), lambda r: S.spider(20, 20), lambda r: S.spider(100, 2),
    lambda r: S.spider(8, 160), lambda r: S.star(400), lambda r: S.path(400)])
def test_adaptive_invariants_unweighted(maker):
    # Unweighted adaptive plans: total incidences <= n log2(n+1)
    # (proof of the backbone-geometry theorem), table size
    # M_S <= (3 + 1/ln 2)|V(S)| (proof of lemma "stad-selection"), and
    # sum_alpha H_alpha <= |V(S)| - m (eq. "stad-component-depth-volume").
    p, w = maker(np.random.default_rng(3))
    n = len(p)
    t = TreeIntegrator(p, w, device=None, leaf_max=1)
    st = t.stats()
    assert st["incidences"] <= n * math.log2(n + 1)
    a = plan_arrays(t)
    sizes = dict(_call_sizes(a))
    J = len(a["job_H"])
    j = 0
    while j < J:
        assert a["job_sign"][j] > 0
        H, X = a["job_H"][j], a["job_X"][j]
        nS = sizes[j]
        assert (H + 1) * (X + 1) <= (3 + 1 / math.log(2)) * nS
        k = j + 1
        sumH = 0
        while k < J and a["job_sign"][k] < 0:
            sumH += a["job_H"][k]
            k += 1
        assert sumH <= nS - (X + 1)
        j = k


def test_diameter_backbone_depth_bound():
    # A diameter backbone of an unweighted tree has H <= (m - 1) / 2.
    rng = np.random.default_rng(31)
    for _ in range(10):
        p, w = S.random_recursive(int(rng.integers(20, 400)), rng)
        t = TreeIntegrator(p, w, device=None, policy="diameter", leaf_max=1)
        a = plan_arrays(t)
        for j in np.flatnonzero(a["job_sign"] > 0):
            assert 2 * a["job_H"][j] <= a["job_X"][j]


def test_golden_plan_pins_from_paper():
    pins = json.load(open(os.path.join(GOLDEN, "plan_pins.json")))
    g = pins["caterpillar_hanging_paths_32"]
    p, w = S.caterpillar_hanging_paths(32)
    assert len(p) == g["N"]
    r = TreeIntegrator(p, w, device=None, policy="diameter").stats()["root"]
    assert (r["m"], r["H"]) == (g["diameter_root"]["m"], g["diameter_root"]["H"])
    assert r["components"] == [32] * 30
    r = TreeIntegrator(p, w, device=None).stats()["root"]
    ga = g["adaptive_root"]
    assert (r["m"], r["H"], r["choice"]) == (ga["m"], ga["H"], ga["choice"])
    assert sorted(r["components"]) == sorted(ga["components"])
    # scores recomputed from equation "stad-score" (natural logarithms)
    assert abs(r["score_diameter"] - 33306.09) < 0.05
    assert abs(r["score_centroid"] - 8222.57) < 0.05

    g = pins["spider_8x500"]
    p, w = S.spider(8, 500)
    assert len(p) == g["N"]
    r = TreeIntegrator(p, w, device=None, policy="diameter").stats()["root"]
    assert (r["m"], r["H"]) == (g["diameter_root"]["m"], g["diameter_root"]["H"])
    assert r["m"] * (r["H"] + 1) == g["diameter_root"]["table_cells"]
    r = TreeIntegrator(p, w, device=None).stats()["root"]
    ga = g["adaptive_root"]
    assert (r["m"], r["H"], r["choice"]) == (ga["m"], ga["H"], ga["choice"])
    assert r["m"] * (r["H"] + 1) == ga["table_cells"]
    assert r["components"] == [500] * 8

    g = pins["path_800"]
    r = TreeIntegrator(*S.path(800), device=None).stats()["root"]
    ga = g["adaptive_root"]
    assert (r["m"], r["H"], r["choice"]) == (ga["m"], ga["H"], ga["choice"])


def test_equal_arm_spider_corollary():
    # Corollary "stad-adaptive-equal-spider": hub first, then every arm is
    # taken whole as a path backbone.
    for s, h in [(3, 10), (8, 40), (30, 25)]:
        t = TreeIntegrator(*S.spider(s, h), device=None, leaf_max=1)
        st = t.stats()
        assert st["root"]["choice"] == "centroid" and st["root"]["H"] == h
        a = plan_arrays(t)
        calls = np.flatnonzero(a["job_sign"] > 0)
        assert len(calls) == 1 + s
        assert all(a["job_H"][j] == 0 and a["job_X"][j] == h - 1 for j in calls[1:])


def test_build_errors():
    ok_p = np.array([-1, 0, 1], dtype=np.int64)
    ok_w = np.array([0, 1, 1], dtype=np.int32)
    ones = np.ones(3, dtype=np.int32)
    with pytest.raises(TFIError, match="TREE"):
        TreeIntegrator(np.array([1, 2, 0]), ones, device=None)   # cycle
    with pytest.raises(TFIError, match="TREE"):
        TreeIntegrator(np.array([-1, 2, 1]), ones, device=None)  # cycle off the root
    with pytest.raises(TFIError, match="TREE"):
        TreeIntegrator(np.array([-1, 7, 0]), ones, device=None)  # out of range
    with pytest.raises(TFIError, match="TREE"):
        TreeIntegrator(np.array([-1, 1, 0]), ones, device=None)  # self loop
    with pytest.raises(TFIError, match="WEIGHT"):
        TreeIntegrator(ok_p, np.array([0, 0, 1]), device=None)   # zero weight
    with pytest.raises(TFIError, match="WEIGHT"):
        big = np.array([0, 2 ** 30, 2 ** 30], dtype=np.int32)
        TreeIntegrator(ok_p, big, device=None)                   # lattice overflow
    with pytest.raises(TFIError, match="ARG"):
        TreeIntegrator(np.zeros(0, np.int64), np.zeros(0, np.int32), device=None)
    with pytest.raises(TFIError, match="ARG"):
        TreeIntegrator(ok_p, ok_w, device=None, policy=7)
    t = TreeIntegrator(ok_p, ok_w, device=None)
    with pytest.raises(TFIError, match="ARG"):
        t.export("no_such_array")


def test_channel_policy_trades_call_cost_against_channel_width():
    # Eight-arm spider, 500-edge arms (the paper's long-arm spider): the
    # diameter backbone leaves 6 components (7 table jobs), the hub 8 (9
    # jobs), but the diameter's per-channel work is larger (a 1501-cell table
    # against 501). With a per-job cost of 1e7 units the diameter wins at one
    # channel and the hub at 4160 (appendix "Channel-aware backbone
    # selection": the product C x C_chan decides at wide channels).
    p, w = S.spider(8, 500)
    cm = {"vertex": 1.0, "direct": 1.0, "fft": 4.0, "call": 1e7}
    narrow = TreeIntegrator(p, w, device=None, policy="channel", channel_width=1,
                            cost_model=cm).stats()["root"]
    wide = TreeIntegrator(p, w, device=None, policy="channel", channel_width=4160,
                          cost_model=cm).stats()["root"]
    assert (narrow["choice"], narrow["m"], narrow["H"]) == ("diameter", 1001, 500)
    assert (wide["choice"], wide["m"], wide["H"]) == ("centroid", 1, 500)
    # a dominant per-job cost alone picks the candidate with fewer jobs
    calls = TreeIntegrator(p, w, device=None, policy="channel",
                           cost_model={"vertex": 1, "direct": 1, "fft": 4, "call": 1e9}
                           ).stats()["root"]
    assert calls["choice"] == "diameter"


def test_channel_policy_rejects_bad_cost_model():
    p, w = S.path(10)
    with pytest.raises(TFIError):
        TreeIntegrator(p, w, device=None, policy="channel",
                       cost_model={"vertex": 1, "direct": -1, "fft": 4})
    with pytest.raises(TFIError):
        TreeIntegrator(p, w, device=None, policy="channel", channel_width=-3)


def test_fft1d_method_assignment():
    """table_method 'fft1d' gives the per-depth-pair method (2) to exactly the
    tables with several depths and several backbone positions, FFT (1) to
    the others; with 'hankel' (4) the tables of depth <= 127 among them get
    the Hankel product (3); a method outside [0, 4] is refused."""
    p, w = S.caterpillar_hanging_paths(20)
    t = TreeIntegrator(p, w, device=None, policy="diameter", table_method="fft1d")
    H, X, m = t.export("job_H"), t.export("job_X"), t.export("job_method")
    two_d = (H > 0) & (X > 0)
    assert two_d.any() and (~two_d).any()
    assert np.array_equal(m, np.where(two_d, 2, 1))
    t = TreeIntegrator(p, w, device=None, policy="diameter", table_method="hankel")
    assert np.array_equal(t.export("job_method"), np.where(two_d & (H <= 127), 3, 1))
    with pytest.raises(TFIError, match="table_method"):
        TreeIntegrator(p, w, device=None, table_method=5)
