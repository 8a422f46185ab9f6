"""CPU: the pieces of the cell-sum kernel (k_cells and k_cells_combine in
kernels_cells.hpp), replayed on the host with the kernel's index arithmetic
in numpy, followed by the tables by their direct-sum definition and the
gather, and compared with the FP64 oracle. Every index the kernels would
use is checked against the bounds of the array or LDS rows it reads, and
every cell row must be written exactly once, so a planning mistake fails
here rather than on the device.

The replay follows the kernels: a piece sums its segments (at most 16
incidences of one b-cell) from the field rows, a b-cell row is the sum of
its segment rows in order and an A-cell row the sum of its b-cell rows in
order; cells whole in the piece go to the value matrix, cells cut by the
piece's ends to partial rows, which the combine launch adds in piece
order."""
import zlib

import numpy as np
import pytest

import oracle
from paper_2609_34025_amd import TreeIntegrator
from paper_2609_34025_amd import synth as S

REC = 8
SEG = 16
BE = 4
AE = 4
PIECE_SEGS = 64


def plan_arrays(t):
    names = ["job_sign", "job_cell_off", "jc_r", "jc_x", "jc_val", "inc_v", "b_inc_off",
             "a_b_off", "b2a", "b_corr", "v_off", "v_b", "leaf_off", "leaf_v", "leaf_doff",
             "leaf_D"]
    P = {n: t.export(n) for n in names}
    for n in ["piece", "seg", "bent", "aent", "comb"]:
        P["c_" + n] = t.export("cells_" + n)
    return P


def replay(P, f, F):
    NA = len(P["a_b_off"]) - 1
    NB = len(P["b_inc_off"]) - 1
    N, d = F.shape
    inc_v = P["inc_v"]
    piece = P["c_piece"].reshape(-1, REC)
    seg = P["c_seg"].reshape(-1, 2)
    bent = P["c_bent"].reshape(-1, BE)
    aent = P["c_aent"].reshape(-1, AE)
    comb = P["c_comb"].reshape(-1, 4)
    jc_r, jc_x, jc_val = P["jc_r"], P["jc_x"], P["jc_val"]
    val = np.full(((NA + NB), d), np.nan)
    nparts = int((comb[:, 2] + comb[:, 3]).max()) if len(comb) else 1
    part = np.full((max(nparts, 1), d), np.nan)
    written = np.zeros(NA + NB, int)

    def put(row, out, v):
        if out < 0:
            val[row] = v
            written[row] += 1
        else:
            assert 0 <= out < len(part) and np.isnan(part[out]).all()
            part[out] = v

    for t in piece:
        s0, s1, e0, e1, q0, q1 = (int(x) for x in t[:6])
        assert 0 <= s0 < s1 <= len(seg) and s1 - s0 <= PIECE_SEGS
        assert 0 <= e0 < e1 <= len(bent) and 0 <= q0 < q1 <= len(aent)
        nseg, nb = s1 - s0, e1 - e0
        srow = np.zeros((nseg, d))
        for s in range(s0, s1):
            beg, ln = int(seg[s, 0]), int(seg[s, 1])
            assert 1 <= ln <= SEG and 0 <= beg and beg + ln <= len(inc_v)
            srow[s - s0] = F[inc_v[beg:beg + ln]].sum(0)
        brow = np.zeros((nb, d))
        for k in range(e0, e1):
            b, lo, hi, out = (int(x) for x in bent[k])
            assert 0 <= lo < hi <= nseg and 0 <= b < NB
            brow[k - e0] = srow[lo:hi].sum(0)
            put(NA + b, out, brow[k - e0])
        for k in range(q0, q1):
            a, lo, hi, out = (int(x) for x in aent[k])
            assert 0 <= lo < hi <= nb and 0 <= a < NA
            assert np.all(P["b2a"][bent[e0 + lo:e0 + hi, 0]] == a)
            put(a, out, brow[lo:hi].sum(0))
    # the combine launch: each cut cell's partial rows in piece order
    for ck, idx, pf, n in comb:
        assert n >= 2 and pf + n <= len(part)
        v = part[pf:pf + n].sum(0)
        assert not np.isnan(v).any()
        put(int(idx) if ck else NA + int(idx), -1, v)
    assert np.all(written == 1)
    # tables by the direct-sum definition from the value rows
    g = np.full(((NA + NB), d), np.nan)
    jco = P["job_cell_off"]
    for j in range(len(P["job_sign"])):
        cells = np.arange(jco[j], jco[j + 1])
        src = val[jc_val[cells]]
        for i in cells:
            idx = jc_r[i] + jc_r[cells] + np.abs(jc_x[i] - jc_x[cells])
            g[jc_val[i]] = f[idx] @ src
    # gather onto the dense leaf values
    out = np.zeros((N, d))
    lo_, lv, ld, lD = P["leaf_off"], P["leaf_v"], P["leaf_doff"], P["leaf_D"]
    for k in range(len(lo_) - 1):
        vs = lv[lo_[k]:lo_[k + 1]]
        n = len(vs)
        D = lD[ld[k]:ld[k + 1]].reshape(n, n)
        out[vs] = f[D] @ F[vs]
    voff, vb = P["v_off"], P["v_b"]
    for v in range(N):
        for k in range(voff[v], voff[v + 1]):
            b = vb[k]
            out[v] += g[P["b2a"][b]]
            if P["b_corr"][b]:
                out[v] -= g[NA + b]
    return out, len(piece), len(comb)


CASES = [
    ("rrt1500_w8", lambda r: (lambda p: (p, S.uniform_weights(p, 1, 8, r)))(
        S.random_recursive(1500, r)[0]), {}),
    ("rrt3000_leaf64", lambda r: (lambda p: (p, S.uniform_weights(p, 1, 8, r)))(
        S.random_recursive(3000, r)[0]), {"leaf_max": 64}),
    ("rrt2000_leaf1", lambda r: (lambda p: (p, S.uniform_weights(p, 1, 4, r)))(
        S.random_recursive(2000, r)[0]), {"leaf_max": 1}),
    ("spider8x60_diam", lambda r: S.spider(8, 60), {"policy": "diameter"}),
    ("grid40_w16", lambda r: S.grid_mst(40, 16, r), {}),
    ("star300", lambda r: S.star(300), {"leaf_max": 1}),
    ("cater200_fft", lambda r: (lambda p: (p, S.uniform_weights(p, 1, 8, r)))(
        S.caterpillar(200, 3)[0]), {"table_method": "fft"}),
    ("broom3000", lambda r: S.broom(1000), {"leaf_max": 1}),
    ("forest", lambda r: S.forest([S.path(40), S.star(7), S.grid_mst(9, 5, r),
                                   (lambda p: (p, S.uniform_weights(p, 1, 3, r)))(
                                       S.random_recursive(600, r)[0])])[:2], {}),
]


@pytest.mark.parametrize("name,gen,opts", CASES, ids=[c[0] for c in CASES])
def test_cell_pieces_replay_matches_oracle(name, gen, opts):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    p, w = gen(rng)
    t = TreeIntegrator(p, w, device=None, **opts)
    K = t.kernel_length
    f = np.exp(-0.03 * np.arange(K)) + 0.5 / (1.0 + np.arange(K))
    F = rng.standard_normal((len(p), 3))
    P = plan_arrays(t)
    out, npieces, ncut = replay(P, f, F)
    ref = oracle.integrate(p, w, f, F)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    print(f"{name}: pieces {npieces}, cut cells {ncut}, err {err:.1e}")
    assert err <= 1e-12, err


def test_cell_pieces_of_the_100k_vertex_tree():
    # the 100k-vertex tree with leaf tiles of 64: pieces of up to 64 segments
    # (of any calls), whose cut cells the combine launch adds up
    W = S.workload("rrt100k")
    t = TreeIntegrator(W["parent"], W["weight"], device=None, leaf_max=64)
    piece = t.export("cells_piece").reshape(-1, REC)
    seg = t.export("cells_seg").reshape(-1, 2)
    comb = t.export("cells_comb").reshape(-1, 4)
    assert np.all(piece[:, 1] - piece[:, 0] <= PIECE_SEGS)
    assert len(comb) > 0 and np.all(comb[:, 3] >= 2)
    assert np.all(seg[:, 1] <= SEG) and seg[:, 1].sum() == t.stats()["incidences"]
