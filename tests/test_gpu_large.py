"""N = 2,000,000 trees with a 64 GB device budget: a caterpillar (spine of
N/4, three leaves per spine vertex) and a binary random recursive tree,
weights U{1..8}, F[N x 32] FP32, f = exp(-0.01 d). Forward and dF are
checked on 512 sampled rows against the traversal oracle and on all rows
against the exp-kernel tree recursion."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import TreeIntegrator, synth as S

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BUDGET = 64 << 30


def relerr(y, ref):
    return np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["cater2m", "binary2m"])
def test_two_million_vertices(name):
    t0 = time.time()
    W = S.workload(name)
    p, w, F = W["parent"], W["weight"], W["F"]
    t1 = time.time()
    t = TreeIntegrator(p, w, device=0, memory_budget=BUDGET)
    t2 = time.time()
    K = t.kernel_length
    lam = np.exp(-0.01)
    f = torch.tensor(lam ** np.arange(K), dtype=torch.float32, device=DEV)
    Ft = torch.tensor(F, device=DEV)
    G = torch.tensor(np.random.default_rng(55).standard_normal(F.shape), dtype=torch.float32,
                     device=DEV)
    out = t.integrate(f, Ft)
    dF, _ = t.backward(f, Ft, G, need_df=False)
    torch.cuda.synchronize()
    t3 = time.time()
    out = t.integrate(f, Ft)
    torch.cuda.synchronize()
    t4 = time.time()
    st = t.stats()
    print(f"{name}: gen {t1 - t0:.1f}s plan {t2 - t1:.1f}s first fwd+bwd {t3 - t2:.2f}s "
          f"fwd {1e3 * (t4 - t3):.1f} ms device {st['device_bytes'] / 2**30:.1f} GiB "
          f"K={K}", flush=True)
    assert st["device_bytes"] <= BUDGET
    y, yd = out.cpu().numpy(), dF.cpu().numpy()
    Fd, Gd = F.astype(np.float64), G.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(5).choice(len(p), 512, replace=False)
    ftab = lam ** np.arange(K)
    e1 = relerr(y[rows], oracle.integrate(p, w, ftab, Fd, rows=rows))
    e2 = relerr(yd[rows], oracle.integrate(p, w, ftab, Gd, rows=rows))
    e3 = relerr(y, oracle.expdp(p, w, [1.0], [lam], Fd))
    e4 = relerr(yd, oracle.expdp(p, w, [1.0], [lam], Gd))
    print(f"{name}: rows fwd {e1:.2e} dF {e2:.2e}; all rows fwd {e3:.2e} dF {e4:.2e}", flush=True)
    assert max(e1, e2, e3, e4) <= 1e-4
