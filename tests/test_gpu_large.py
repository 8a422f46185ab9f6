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


def test_cater2m_under_a_4gib_budget():
    """The 2M-vertex caterpillar at d = 32 needs about 13 GiB; under a 4 GiB
    budget the forward and the adjoint run on channel tiles that fit (each
    tile a full pass that forms the kernel spectra again). Checked like the
    unbudgeted case, and the handle never holds more than the budget."""
    W = S.workload("cater2m")
    p, w, F = W["parent"], W["weight"], W["F"]
    budget = 4 << 30
    t = TreeIntegrator(p, w, device=0, memory_budget=budget)
    K = t.kernel_length
    lam = np.exp(-0.01)
    f = torch.tensor(lam ** np.arange(K), dtype=torch.float32, device=DEV)
    Ft = torch.tensor(F, device=DEV)
    G = torch.tensor(np.random.default_rng(56).standard_normal(F.shape), dtype=torch.float32,
                     device=DEV)
    t0 = time.time()
    out = t.integrate(f, Ft)
    dF, _ = t.backward(f, Ft, G, need_df=False)
    torch.cuda.synchronize()
    st = t.stats()
    print(f"cater2m 4 GiB: fwd+dF {time.time() - t0:.2f} s, device "
          f"{st['device_bytes'] / 2**30:.2f} GiB", flush=True)
    assert st["device_bytes"] <= budget
    y, yd = out.cpu().numpy(), dF.cpu().numpy()
    Fd, Gd = F.astype(np.float64), G.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(6).choice(len(p), 256, replace=False)
    ftab = lam ** np.arange(K)
    e1 = relerr(y[rows], oracle.integrate(p, w, ftab, Fd, rows=rows))
    e2 = relerr(yd[rows], oracle.integrate(p, w, ftab, Gd, rows=rows))
    e3 = relerr(y, oracle.expdp(p, w, [1.0], [lam], Fd))
    e4 = relerr(yd, oracle.expdp(p, w, [1.0], [lam], Gd))
    print(f"cater2m 4 GiB: rows fwd {e1:.2e} dF {e2:.2e}; all rows fwd {e3:.2e} dF {e4:.2e}",
          flush=True)
    assert max(e1, e2, e3, e4) <= 1e-4


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_channel_tiles_with_df(dtype):
    """A budget between the plan's own bytes and a whole call's: forward,
    dF and df on channel tiles equal the unbudgeted handle's (df summed over
    the tiles), and the budgeted handle stays within its budget."""
    rng = np.random.default_rng(71)
    p, _ = S.random_recursive(20000, rng)
    w = S.uniform_weights(p, 1, 6, rng)
    d = 24
    F = rng.standard_normal((len(p), d))
    G = rng.standard_normal((len(p), d))
    ftab = lambda K: np.exp(-0.03 * np.arange(K))
    free = TreeIntegrator(p, w, device=0, table_method="fft")
    K = free.kernel_length
    f = torch.tensor(ftab(K), dtype=dtype, device=DEV)
    Ft = torch.tensor(F, dtype=dtype, device=DEV)
    Gt = torch.tensor(G, dtype=dtype, device=DEV)
    plan_bytes = free.stats()["device_bytes"]
    y0 = free.integrate(f, Ft)
    dF0, df0 = free.backward(f, Ft, Gt)
    torch.cuda.synchronize()
    whole = free.stats()["device_bytes"] - plan_bytes
    budget = plan_bytes + whole // 3
    t = TreeIntegrator(p, w, device=0, table_method="fft", memory_budget=budget)
    assert t.stats()["device_bytes"] == plan_bytes
    y1 = t.integrate(f, Ft)
    dF1, df1 = t.backward(f, Ft, Gt)
    torch.cuda.synchronize()
    assert t.stats()["device_bytes"] <= budget
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    e = [relerr(a.cpu().numpy(), b.cpu().numpy()) for a, b in ((y1, y0), (dF1, dF0), (df1, df0))]
    print(f"channel tiles {dtype}: budget {budget / 2**20:.1f} MiB of "
          f"{(plan_bytes + whole) / 2**20:.1f} MiB; errs {e}", flush=True)
    assert max(e) <= tol, e
    rows = np.sort(rng.choice(len(p), 64, replace=False))
    ref = oracle.integrate(p, w, ftab(K), F, rows=rows)
    assert relerr(y1.cpu().numpy()[rows], ref) <= (1e-10 if dtype == torch.float64 else 1e-4)
