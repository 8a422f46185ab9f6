"""The Hankel-product path (table_method 'hankel', the attention-width
appendix "Hankel-GEMM"): a table with depths 0..H and backbone positions
0..X is evaluated as B = F A with the Hankel matrix F[l][r] = f(l + r),
then G_q[s] = sum_t B[q + |s - t|][t] by one running sum per antidiagonal
and per diagonal of B. Checked against the oracle and the 2-D FFT path,
forward and adjoint, in FP64 on the paper's families, in FP32 at several
channel chunks, and on a tree whose tables need several buffer groups."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import TreeIntegrator, synth as S

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _families():
    fam = {name: (p, w) for name, p, w in S.paper_families(seed=5)}
    rng = np.random.default_rng(51)
    out = [(n, *fam[n]) for n in ("caterpillar_hanging_paths", "uniform_spider", "complete_3ary",
                                   "random_recursive", "comb")]
    p, _ = S.random_recursive(3000, rng)
    out.append(("rrt3000_w", p, S.uniform_weights(p, 1, 5, rng)))
    return out


def _run(p, w, meth, ftab_fn, F, G, dtype):
    t = TreeIntegrator(p, w, device=0, policy="diameter", table_method=meth)
    K = t.kernel_length
    ftab = ftab_fn(K)
    f = torch.tensor(ftab, dtype=dtype, device=DEV)
    Ft = torch.tensor(F, dtype=dtype, device=DEV)
    Gt = torch.tensor(G, dtype=dtype, device=DEV)
    t.profile(True)
    y = t.integrate(f, Ft)
    dF, df = t.backward(f, Ft, Gt)
    torch.cuda.synchronize()
    st = t.profile_report()
    t.profile(False)
    return (y.double().cpu().numpy(), dF.double().cpu().numpy(), df.cpu().numpy(), st, ftab,
            t.stats())


def _ftab(K):
    return np.exp(-0.06 * np.arange(K)) + 0.4 / (1.0 + np.arange(K)) ** 2


@pytest.mark.parametrize("case", _families(), ids=lambda c: c[0])
def test_hankel_matches_oracle_and_fft(case):
    name, p, w = case
    rng = np.random.default_rng(52)
    F = rng.standard_normal((len(p), 3))
    G = rng.standard_normal((len(p), 3))
    y1, dF1, df1, st1, ftab, stats = _run(p, w, "hankel", _ftab, F, G, torch.float64)
    y2, dF2, df2, st2, _, _ = _run(p, w, "fft", _ftab, F, G, torch.float64)
    assert stats["hankel_jobs"] > 0 and "hankel" in st1, sorted(st1)
    e = [relerr(y1, y2), relerr(dF1, dF2), relerr(df1, df2)]
    ref = oracle.integrate(p, w, ftab, F)
    refg = oracle.integrate(p, w, ftab, G)
    eo = [relerr(y1, ref), relerr(dF1, refg)]
    print(f"{name}: N={len(p)} hankel jobs {stats['hankel_jobs']}: vs FFT {e}, vs oracle {eo}",
          flush=True)
    assert max(e) <= 1e-12
    assert max(eo) <= 1e-10


def test_hankel_fp32_channel_chunks():
    """130 channels: two full chunks of 64 and one of 2."""
    p, w = S.caterpillar_hanging_paths(40)
    rng = np.random.default_rng(53)
    F = rng.standard_normal((len(p), 130))
    G = rng.standard_normal((len(p), 130))
    y, dF, df, st, ftab, _ = _run(p, w, "hankel", _ftab, F, G, torch.float32)
    rows = np.sort(rng.choice(len(p), 48, replace=False))
    e = [relerr(y[rows], oracle.integrate(p, w, ftab, F, rows=rows)),
         relerr(dF[rows], oracle.integrate(p, w, ftab, G, rows=rows))]
    print(f"caterpillar_hanging_paths(40) fp32 d=130: {e}", flush=True)
    assert max(e) <= 1e-4


def test_hankel_buffer_groups():
    """A 256 x 256 patch-grid spanning tree under the diameter policy: the
    Hankel tables' B rows exceed one buffer group, so the product and the
    walks run group by group. FP32 at d = 8 against the 2-D FFT path."""
    p, w = S.patch_grid_tree("random", 256, np.random.default_rng(54))
    rng = np.random.default_rng(55)
    F = rng.standard_normal((len(p), 8))
    G = rng.standard_normal((len(p), 8))
    y1, dF1, df1, _, ftab, stats = _run(p, w, "hankel", _ftab, F, G, torch.float32)
    y2, dF2, df2, _, _, _ = _run(p, w, "fft", _ftab, F, G, torch.float32)
    t = TreeIntegrator(p, w, device=None, policy="diameter", table_method="hankel")
    m, H, X = t.export("job_method"), t.export("job_H"), t.export("job_X")
    rows = int((((H + X + 1) * (X + 1)).astype(np.int64) * (m == 3)).sum())
    print(f"random256 diameter: hankel jobs {stats['hankel_jobs']}, B rows {rows}", flush=True)
    assert rows > (1 << 21)
    e = [relerr(y1, y2), relerr(dF1, dF2), relerr(df1, df2)]
    print(f"random256 diameter fp32: vs FFT {e}", flush=True)
    assert max(e) <= 1e-5
    sel = np.sort(rng.choice(len(p), 32, replace=False))
    assert relerr(y1[sel], oracle.integrate(p, w, ftab, F, rows=sel)) <= 1e-4
