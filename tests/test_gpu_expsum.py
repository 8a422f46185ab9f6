"""GPU sweep evaluator for kernels given as sums of exponentials,
f(k) = sum_l c_l lam_l^k (appendix "Specialized Kernels"): forward and dF
against the oracle with the tabulated f, the moments s0/s1 against the
oracle's pair histogram, and the autograd function against finite
differences and against the table path."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import synth as S
from paper_2609_34025_amd import TreeIntegrator, TreeIntegrate, ExpSumIntegrate, expsum_table

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relerr(y, ref):
    n = np.linalg.norm(ref)
    return np.linalg.norm(np.asarray(y, np.float64) - ref) / (n if n > 0 else 1.0)


def table(c, lam, K):
    k = np.arange(K)
    return (np.asarray(c)[None, :] * np.asarray(lam)[None, :] ** k[:, None]).sum(1)


def trees():
    rng = np.random.default_rng(31)
    out = []
    p, _ = S.random_recursive(500, rng)
    out.append(("rrt500_w6", p, S.uniform_weights(p, 1, 6, rng)))
    out.append(("grid18_w16", *S.grid_mst(18, 16, rng)))
    out.append(("path400_w3", S.path(400)[0], S.uniform_weights(S.path(400)[0], 1, 3, rng)))
    out.append(("chp12", *S.caterpillar_hanging_paths(12)))
    out.append(("spider6x40", *S.spider(6, 40)))
    cp = S.caterpillar(60, 3)[0]
    out.append(("cater60_w4", cp, S.uniform_weights(cp, 1, 4, rng)))
    fp, fw, _ = S.forest([S.grid_mst(9, 5, rng), S.path(1), S.star(7), S.path(30)])
    out.append(("forest", fp, fw))
    return out


@pytest.mark.parametrize("policy", ["adaptive", "diameter", "centroid"])
@pytest.mark.parametrize("nterm", [1, 3, 8, 16])
def test_expsum_fp64_forward_backward_moments(policy, nterm):
    # diameter backbones give jobs with many positions (full sweeps);
    # centroid backbones one position per job
    rng = np.random.default_rng(7 + nterm)
    c = rng.standard_normal(nterm)
    lam = rng.uniform(0.55, 0.99, nterm)
    for name, p, w in trees():
        for leaf in (1, 32):
            t = TreeIntegrator(p, w, device=0, policy=policy, leaf_max=leaf)
            K = t.kernel_length
            d = 3
            F = rng.standard_normal((len(p), d))
            G = rng.standard_normal((len(p), d))
            ct = torch.tensor(c, device=DEV)
            lt = torch.tensor(lam, device=DEV)
            Ft = torch.tensor(F, device=DEV)
            y = t.integrate_expsum(ct, lt, Ft).cpu().numpy()
            dF, s0, s1 = t.backward_expsum(ct, lt, Ft, torch.tensor(G, device=DEV))
            ftab = table(c, lam, K)
            e1 = relerr(y, oracle.integrate(p, w, ftab, F))
            e2 = relerr(dF.cpu().numpy(), oracle.integrate(p, w, ftab, G))
            h = oracle.pair_hist(p, w, G, F, K)
            k = np.arange(K)
            r0 = np.array([(lam[l] ** k * h).sum() for l in range(nterm)])
            r1 = np.array([(k * lam[l] ** k * h).sum() for l in range(nterm)])
            e3, e4 = relerr(s0.cpu().numpy(), r0), relerr(s1.cpu().numpy(), r1)
            assert max(e1, e2, e3, e4) <= 1e-10, (name, leaf, e1, e2, e3, e4)


@pytest.mark.parametrize("d", [1, 2, 5, 16, 33, 64, 100])
def test_expsum_fp32_channel_counts(d):
    rng = np.random.default_rng(40 + d)
    p, w, _ = S.forest([S.grid_mst(int(s), 16, rng) for s in (12, 15, 9)])
    for policy in ("adaptive", "diameter"):
        t = TreeIntegrator(p, w, device=0, policy=policy)
        K = t.kernel_length
        c = rng.standard_normal(8)
        lam = np.exp(-rng.uniform(0.01, 0.5, 8))
        F = rng.standard_normal((len(p), d))
        G = rng.standard_normal((len(p), d))
        ct = torch.tensor(c, dtype=torch.float32, device=DEV)
        lt = torch.tensor(lam, dtype=torch.float32, device=DEV)
        Ft = torch.tensor(F, dtype=torch.float32, device=DEV)
        Gt = torch.tensor(G, dtype=torch.float32, device=DEV)
        y = t.integrate_expsum(ct, lt, Ft).cpu().numpy()
        dF, s0, s1 = t.backward_expsum(ct, lt, Ft, Gt)
        # the oracle takes the same FP32-rounded parameters and fields
        c32, l32 = ct.double().cpu().numpy(), lt.double().cpu().numpy()
        F32, G32 = Ft.double().cpu().numpy(), Gt.double().cpu().numpy()
        ftab = table(c32, l32, K)
        assert relerr(y, oracle.integrate(p, w, ftab, F32)) <= 1e-4
        assert relerr(dF.cpu().numpy(), oracle.integrate(p, w, ftab, G32)) <= 1e-4
        h = oracle.pair_hist(p, w, G32, F32, K)
        k = np.arange(K)
        r0 = np.array([(l32[l] ** k * h).sum() for l in range(8)])
        r1 = np.array([(k * l32[l] ** k * h).sum() for l in range(8)])
        assert relerr(s0.cpu().numpy(), r0) <= 1e-4
        assert relerr(s1.cpu().numpy(), r1) <= 1e-4


@pytest.mark.parametrize("policy", ["adaptive", "centroid"])
def test_expsum_fp64_wide_rows(policy):
    """d > 32: a one-position job's cell walk is the same in every lane (the
    cell's row and weights pass through scalar registers, two halves per
    double)."""
    rng = np.random.default_rng(77)
    p, w, _ = S.forest([S.grid_mst(14, 16, rng), S.spider(5, 30)])
    d = 40
    print(f"expsum fp64 wide rows policy={policy} N={len(p)} d={d}", flush=True)
    t = TreeIntegrator(p, w, device=0, policy=policy)
    K = t.kernel_length
    c = rng.standard_normal(8)
    lam = rng.uniform(0.55, 0.99, 8)
    F = rng.standard_normal((len(p), d))
    G = rng.standard_normal((len(p), d))
    ct, lt = torch.tensor(c, device=DEV), torch.tensor(lam, device=DEV)
    Ft = torch.tensor(F, device=DEV)
    y = t.integrate_expsum(ct, lt, Ft).cpu().numpy()
    dF, s0, s1 = t.backward_expsum(ct, lt, Ft, torch.tensor(G, device=DEV))
    ftab = table(c, lam, K)
    h = oracle.pair_hist(p, w, G, F, K)
    k = np.arange(K)
    r0 = np.array([(lam[l] ** k * h).sum() for l in range(8)])
    r1 = np.array([(k * lam[l] ** k * h).sum() for l in range(8)])
    errs = (relerr(y, oracle.integrate(p, w, ftab, F)),
            relerr(dF.cpu().numpy(), oracle.integrate(p, w, ftab, G)),
            relerr(s0.cpu().numpy(), r0), relerr(s1.cpu().numpy(), r1))
    assert max(errs) <= 1e-10, errs


@pytest.mark.parametrize("dtype,d", [(torch.float32, 64), (torch.float64, 3)])
def test_expsum_kept_cells_bitwise(dtype, d):
    """The backward that reads the forward's cell sums equals the one that
    forms them again, also when the handle ran another field in between: dF
    bit for bit, the moments to the rounding of the leaf pair histogram
    (binned with atomics); misuse of the cells argument is an error."""
    rng = np.random.default_rng(91)
    cp = S.caterpillar(40, 3)[0]
    p, w, _ = S.forest([S.grid_mst(16, 16, rng), (cp, S.uniform_weights(cp, 1, 4, rng))])
    print(f"expsum kept cells N={len(p)} d={d} {dtype}", flush=True)
    t = TreeIntegrator(p, w, device=0)
    ct = torch.tensor(rng.standard_normal(8), dtype=dtype, device=DEV)
    lt = torch.tensor(np.exp(-rng.uniform(0.01, 0.5, 8)), dtype=dtype, device=DEV)
    F1 = torch.tensor(rng.standard_normal((len(p), d)), dtype=dtype, device=DEV)
    F2 = torch.tensor(rng.standard_normal((len(p), d)), dtype=dtype, device=DEV)
    G = torch.tensor(rng.standard_normal((len(p), d)), dtype=dtype, device=DEV)
    ref = t.integrate_expsum(ct, lt, F1)
    out, cells = t.integrate_expsum(ct, lt, F1, keep_cells=True)
    assert torch.equal(out, ref)
    t.integrate_expsum(ct, lt, F2)  # the handle's own buffers now hold F2
    for _ in range(2):  # eager, then graph replay
        a = t.backward_expsum(ct, lt, F1, G)
        b = t.backward_expsum(ct, lt, F1, G, cells=cells)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0])
        tol = 1e-5 if dtype == torch.float32 else 1e-12
        for x, y in zip(a[1:], b[1:]):
            assert relerr(y.cpu().numpy(), x.cpu().numpy()) <= tol
    with pytest.raises(ValueError):
        t.backward_expsum(ct, lt, F1, G, cells=cells[1:])


@pytest.mark.parametrize("policy", ["adaptive", "diameter"])
@pytest.mark.parametrize("d", [5, 40])
def test_expsum_fused_backward_dF_bitwise(policy, d):
    """With moments and dF together, one launch per one-position job writes
    both; its dF equals the forward integration of gout bit for bit, as does
    the dF-only backward."""
    rng = np.random.default_rng(5 + d)
    p, w, _ = S.forest([S.grid_mst(15, 16, rng), S.spider(4, 25), S.path(60)])
    print(f"expsum fused backward policy={policy} N={len(p)} d={d}", flush=True)
    t = TreeIntegrator(p, w, device=0, policy=policy)
    ct = torch.tensor(rng.standard_normal(8), dtype=torch.float32, device=DEV)
    lt = torch.tensor(np.exp(-rng.uniform(0.01, 0.5, 8)), dtype=torch.float32, device=DEV)
    F = torch.tensor(rng.standard_normal((len(p), d)), dtype=torch.float32, device=DEV)
    G = torch.tensor(rng.standard_normal((len(p), d)), dtype=torch.float32, device=DEV)
    ref = t.integrate_expsum(ct, lt, G)
    for _ in range(2):  # eager, then graph replay
        dF, s0, s1 = t.backward_expsum(ct, lt, F, G)
        dF2, _, _ = t.backward_expsum(ct, lt, F, G, need_moments=False)
        torch.cuda.synchronize()
        assert torch.equal(dF, ref) and torch.equal(dF2, ref)
    K = t.kernel_length
    c32, l32 = ct.double().cpu().numpy(), lt.double().cpu().numpy()
    h = oracle.pair_hist(p, w, G.double().cpu().numpy(), F.double().cpu().numpy(), K)
    k = np.arange(K)
    r0 = np.array([(l32[l] ** k * h).sum() for l in range(8)])
    assert relerr(s0.cpu().numpy(), r0) <= 1e-4


def test_expsum_autograd_matches_fd_and_table_path():
    rng = np.random.default_rng(55)
    p, w, _ = S.forest([S.grid_mst(s, 16, rng) for s in (6, 8, 7)])
    n = len(p)
    t = TreeIntegrator(p, w, device=0)
    K = t.kernel_length
    a = torch.tensor(rng.standard_normal(8), device=DEV, requires_grad=True)
    b = torch.tensor(rng.uniform(0.01, 0.5, 8), device=DEV, requires_grad=True)
    F = torch.tensor(rng.standard_normal((n, 4)), device=DEV, requires_grad=True)
    Wt = torch.tensor(rng.standard_normal((n, 4)), device=DEV)

    def loss(a_, b_, F_):
        return (Wt * ExpSumIntegrate.apply(t, F_, a_, b_)).sum()

    L = loss(a, b, F)
    L.backward()
    with torch.no_grad():
        for theta, g in ((a, a.grad), (b, b.grad)):
            for k in range(8):
                h = 1e-6 * max(1.0, abs(theta[k].item()))
                old = theta[k].item()
                theta[k] = old + h
                lp = loss(a, b, F).item()
                theta[k] = old - h
                lm = loss(a, b, F).item()
                theta[k] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[k].item()) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k].item())
    # the table path gives the same forward and gradients
    a2 = a.detach().clone().requires_grad_(True)
    b2 = b.detach().clone().requires_grad_(True)
    F2 = F.detach().clone().requires_grad_(True)
    L2 = (Wt * TreeIntegrate.apply(t, F2, expsum_table(a2, b2, K))).sum()
    L2.backward()
    assert abs(L.item() - L2.item()) <= 1e-10 * max(1.0, abs(L2.item()))
    for g1, g2 in ((a.grad, a2.grad), (b.grad, b2.grad), (F.grad, F2.grad)):
        assert relerr(g1.cpu().numpy(), g2.cpu().numpy()) <= 1e-10


def test_expsum_graph_replay_and_errors():
    rng = np.random.default_rng(57)
    W = S.workload("small")
    p, w = W["parent"], W["weight"]
    t = TreeIntegrator(p, w, device=0)
    c = torch.tensor([1.0, -0.3], dtype=torch.float64, device=DEV)
    lam = torch.tensor([0.9, 0.7], dtype=torch.float64, device=DEV)
    F = torch.tensor(rng.standard_normal((len(p), 4)), device=DEV)
    ref = t.integrate_expsum(c, lam, F).clone()
    for _ in range(3):
        torch.cuda.synchronize()
        y = t.integrate_expsum(c, lam, F)
        assert torch.equal(y, ref)
    # new parameter values in the same buffers are picked up by the replay
    with torch.no_grad():
        lam.copy_(torch.tensor([0.8, 0.6], dtype=torch.float64, device=DEV))
    y2 = t.integrate_expsum(c, lam, F).cpu().numpy()
    ftab = table([1.0, -0.3], [0.8, 0.6], t.kernel_length)
    assert relerr(y2, oracle.integrate(p, w, ftab, F.cpu().numpy())) <= 1e-10
    with pytest.raises(ValueError):
        t.integrate_expsum(c[:1], lam, F)
    with pytest.raises(ValueError):
        t.integrate_expsum(torch.zeros(17, device=DEV, dtype=torch.float64),
                           torch.ones(17, device=DEV, dtype=torch.float64), F)


def test_grid512_timed_configuration():
    # The batched training step at full size, as the benchmark times it:
    # 512 grid-MST trees, d = 64, f = 8 exponentials, loss sum(W * out);
    # the sweep evaluator and the table path (rule autotuned on forward +
    # adjoint passes). out and dF on sampled rows against the oracle; da and
    # db against the oracle's exp-kernel recursion (da_k = <W, K_k F>, db_k
    # by a central difference of it in b_k).
    W = S.workload("grid512")
    p, w, F = W["parent"], W["weight"], W["F"]
    n, d = F.shape
    rng = np.random.default_rng(34)
    t = TreeIntegrator(p, w, device=0)
    K = t.kernel_length
    t.autotune(torch.tensor(W["kernels"][0][1](K), dtype=torch.float32, device=DEV), d,
               backward=True)
    Wt = torch.tensor(rng.standard_normal((n, d)), dtype=torch.float32, device=DEV)
    a = torch.tensor(W["a"], dtype=torch.float32, device=DEV, requires_grad=True)
    b = torch.tensor(W["b"], dtype=torch.float32, device=DEV, requires_grad=True)
    Ft = torch.tensor(F, device=DEV, requires_grad=True)
    rows = np.random.default_rng(35).choice(n, 256, replace=False)
    A = a.detach().double().cpu().numpy()
    B = b.detach().double().cpu().numpy()
    ftab = table(A, np.exp(-B), K)
    Fd = F.astype(np.float64)
    Wd = Wt.double().cpu().numpy()
    ref_out = oracle.integrate(p, w, ftab, Fd, rows=rows)
    ref_dF = oracle.integrate(p, w, ftab, Wd, rows=rows)
    da_ref = np.array([np.sum(Wd * oracle.expdp(p, w, [1.0], [np.exp(-B[k])], Fd))
                       for k in range(len(A))])
    # db_k = -a_k sum_{v,w} D e^{-b_k D} <W_v, F_w> = a_k dL_k/db_k with
    # L_k(b) = <W, K_b F> and K_b the single exponential e^{-b D}: a central
    # difference of the oracle's exp-kernel recursion in b (step 1e-5; its
    # truncation error is orders below the 1e-4 bar)
    hb = 1e-5
    db_ref = np.array([A[k] * (np.sum(Wd * oracle.expdp(p, w, [1.0], [np.exp(-B[k] - hb)], Fd))
                               - np.sum(Wd * oracle.expdp(p, w, [1.0], [np.exp(-B[k] + hb)],
                                                          Fd))) / (2 * hb)
                       for k in range(len(A))])
    paths = {"sweep": lambda: ExpSumIntegrate.apply(t, Ft, a, b),
             "table": lambda: TreeIntegrate.apply(t, Ft, expsum_table(a, b, K))}
    for name, fwd in paths.items():
        for rep in range(2):
            a.grad = b.grad = Ft.grad = None
            out = fwd()
            (Wt * out).sum().backward()
            torch.cuda.synchronize()
            errs = {"out": relerr(out.detach().cpu().numpy()[rows], ref_out),
                    "dF": relerr(Ft.grad.cpu().numpy()[rows], ref_dF),
                    "da": relerr(a.grad.cpu().numpy(), da_ref),
                    "db": relerr(b.grad.cpu().numpy(), db_ref)}
            print(f"grid512 {name} step {rep}: {errs}", flush=True)
            assert max(errs.values()) <= 1e-4, (name, rep, errs)
