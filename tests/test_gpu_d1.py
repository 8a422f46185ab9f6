"""The per-depth-pair path (table_method 'fft1d', algorithm "global-anchor"):
a table with depths 0..H and backbone positions 1..m is evaluated as 1-D
FFT convolutions along the backbone, one per depth pair (q, r), instead of
one 2-D convolution (lemma "stad-2d-fft"). With the diameter policy it is
the paper's Diameter-1D variant. Checked against the oracle and against the
2-D path on the paper's families, forward and adjoint."""
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
    fam = {name: (p, w) for name, p, w in S.paper_families(seed=4)}
    rng = np.random.default_rng(41)
    out = [(n, *fam[n]) for n in ("caterpillar_hanging_paths", "uniform_spider", "complete_3ary",
                                   "random_recursive", "random_mst_topology")]
    p, _ = S.random_recursive(3000, rng)
    out.append(("rrt3000_w", p, S.uniform_weights(p, 1, 5, rng)))
    return out


@pytest.mark.parametrize("case", _families(), ids=lambda c: c[0])
def test_fft1d_matches_oracle_and_2d(case):
    name, p, w = case
    d = 3
    rng = np.random.default_rng(42)
    F = rng.standard_normal((len(p), d))
    G = rng.standard_normal((len(p), d))
    res = {}
    for meth in ("fft1d", "fft"):
        t = TreeIntegrator(p, w, device=0, policy="diameter", table_method=meth)
        K = t.kernel_length
        ftab = np.exp(-0.07 * np.arange(K)) + 0.5 / (1.0 + np.arange(K)) ** 2
        f = torch.tensor(ftab, dtype=torch.float64, device=DEV)
        t.profile(True)
        y = t.integrate(f, torch.tensor(F, device=DEV))
        dF, df = t.backward(f, torch.tensor(F, device=DEV), torch.tensor(G, device=DEV))
        torch.cuda.synchronize()
        st = t.profile_report()
        t.profile(False)
        res[meth] = (y.cpu().numpy(), dF.cpu().numpy(), df.cpu().numpy(), st, ftab)
    y1, dF1, df1, st1, ftab = res["fft1d"]
    y2, dF2, df2, st2, _ = res["fft"]
    assert "fft1d_global" in st1, sorted(st1)
    assert "fft1d_global" not in st2
    e = [relerr(y1, y2), relerr(dF1, dF2), relerr(df1, df2)]
    ref = oracle.integrate(p, w, ftab, F)
    refg = oracle.integrate(p, w, ftab, G)
    eo = [relerr(y1, ref), relerr(dF1, refg)]
    print(f"{name}: N={len(p)} vs 2-D {e}, vs oracle {eo}", flush=True)
    assert max(e) <= 1e-12
    assert max(eo) <= 1e-10


def test_fft1d_fp32_wide():
    """FP32 at 64 channels (32 channel pairs per table) on the hanging-path
    caterpillar (root backbone m = 32 with H = 32): the oracle at 1e-4."""
    p, w = S.caterpillar_hanging_paths(48)
    rng = np.random.default_rng(43)
    F = rng.standard_normal((len(p), 64)).astype(np.float32)
    t = TreeIntegrator(p, w, device=0, policy="diameter", table_method="fft1d")
    K = t.kernel_length
    ftab = np.exp(-0.03 * np.arange(K))
    f = torch.tensor(ftab, dtype=torch.float32, device=DEV)
    y = t.integrate(f, torch.tensor(F, device=DEV)).cpu().numpy()
    rows = np.sort(rng.choice(len(p), 64, replace=False))
    ref = oracle.integrate(p, w, ftab, F.astype(np.float64), rows=rows)
    e = relerr(y[rows].astype(np.float64), ref)
    print(f"caterpillar_hanging_paths(48) fp32 d=64: {e:.2e}", flush=True)
    assert e <= 1e-4
