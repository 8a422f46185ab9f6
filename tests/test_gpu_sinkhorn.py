"""Sinkhorn on the sphere kNN MST (N = 50,000, lengths in units of 1/64,
f(k) = exp(-k / 3.2), i.e. exp(-d / 0.05)): 200 iterations, every device
product (FP32) checked against the FP64 exp-kernel tree recursion applied
to the same rounded input vector."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import TreeIntegrator, synth as S
from paper_2609_34025_amd.sinkhorn import sinkhorn

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_sinkhorn_sphere50k_every_product_matches_oracle():
    W = S.workload("sphere50k")
    p, w = W["parent"], W["weight"]
    t = TreeIntegrator(p, w, device=0)
    K = t.kernel_length
    lam = np.exp(-1.0 / 3.2)
    f = torch.tensor(lam ** np.arange(K), dtype=torch.float32, device=DEV)
    errs = []

    def check(xin, y):
        x = xin.double().cpu().numpy()
        ref = oracle.expdp(p, w, [1.0], [lam], x)
        errs.append(np.linalg.norm(y.double().cpu().numpy() - ref) / np.linalg.norm(ref))

    a = torch.tensor(W["a"], device=DEV)
    b = torch.tensor(W["b"], device=DEV)
    u, v, res = sinkhorn(t, f, a, b, iters=200, on_product=check)
    assert len(errs) == 400 + 2 * len(res)
    print(f"sinkhorn: {len(errs)} products, max rel err {max(errs):.2e}, "
          f"residuals {res[0][1]:.3e} -> {res[-1][1]:.3e}")
    # the criterion: every FP32 product against the FP64 oracle on the same
    # rounded input; the FP32 trajectory itself is not compared (the scaling
    # vectors span many orders of magnitude)
    assert max(errs) <= 1e-4
    assert torch.isfinite(u).all() and torch.isfinite(v).all()


def test_sinkhorn_fp64_products_follow_cpu_trajectory():
    W = S.workload("sphere50k")
    p, w = W["parent"], W["weight"]
    t = TreeIntegrator(p, w, device=0)
    lam = np.exp(-1.0 / 3.2)
    f = torch.tensor(lam ** np.arange(t.kernel_length), dtype=torch.float64, device=DEV)
    a = torch.tensor(W["a"], device=DEV)
    b = torch.tensor(W["b"], device=DEV)
    iters = 41
    u, v, res = sinkhorn(t, f, a, b, iters=iters)
    # CPU FP64 Sinkhorn with the oracle's exp-kernel recursion as K
    Kc = lambda x: oracle.expdp(p, w, [1.0], [lam], x)
    uc, vc = np.ones(len(p)), np.ones(len(p))
    rc = []
    for it in range(1, iters + 1):
        uc = W["a"] / (Kc(vc) + 1e-30)
        vc = W["b"] / (Kc(uc) + 1e-30)
        if it == 1 or (it - 1) % 20 == 0:
            rc.append(max(np.abs(uc * Kc(vc) - W["a"]).max(), np.abs(vc * Kc(uc) - W["b"]).max()))
    print(f"sinkhorn fp64: residuals {[r for _, r in res]} cpu {rc}")
    # FP64 products differ from the recursion's by ~1e-15; the iteration
    # amplifies that (u, v span ~1e-13 .. 1e5 after 40 iterations)
    assert np.linalg.norm(u.cpu().numpy() - uc) / np.linalg.norm(uc) < 1e-5
    assert np.linalg.norm(v.cpu().numpy() - vc) / np.linalg.norm(vc) < 1e-5
    np.testing.assert_allclose([r for _, r in res], rc, rtol=1e-5)
    assert res[-1][1] < res[0][1]


def test_sinkhorn_through_backbone_sweeps():
    """f = exp(-k / 3.2) is one exponential: the products may run through
    the backbone sweeps (f given as (c, lam)). Every FP32 product against the
    FP64 recursion, and the FP64 sweep trajectory equals the FP64 table
    trajectory to the iteration's amplification of rounding."""
    W = S.workload("sphere50k")
    p, w = W["parent"], W["weight"]
    t = TreeIntegrator(p, w, device=0)
    lam = np.exp(-1.0 / 3.2)
    a = torch.tensor(W["a"], device=DEV)
    b = torch.tensor(W["b"], device=DEV)
    errs = []

    def check(xin, y):
        ref = oracle.expdp(p, w, [1.0], [lam], xin.double().cpu().numpy())
        errs.append(np.linalg.norm(y.double().cpu().numpy() - ref) / np.linalg.norm(ref))

    cl32 = (torch.ones(1, device=DEV), torch.full((1,), lam, dtype=torch.float32, device=DEV))
    sinkhorn(t, cl32, a, b, iters=60, on_product=check)
    print(f"sinkhorn sweeps fp32: {len(errs)} products, max rel err {max(errs):.2e}")
    assert max(errs) <= 1e-4
    cl64 = (torch.ones(1, dtype=torch.float64, device=DEV),
            torch.full((1,), lam, dtype=torch.float64, device=DEV))
    f64 = torch.tensor(lam ** np.arange(t.kernel_length), dtype=torch.float64, device=DEV)
    u1, v1, r1 = sinkhorn(t, cl64, a, b, iters=41)
    u2, v2, r2 = sinkhorn(t, f64, a, b, iters=41)
    assert np.linalg.norm((u1 - u2).cpu().numpy()) / np.linalg.norm(u2.cpu().numpy()) < 1e-5
    np.testing.assert_allclose([r for _, r in r1], [r for _, r in r2], rtol=1e-5)
