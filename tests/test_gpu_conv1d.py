"""GPU parity of the 1-D FFT convolution kernels (tables with H = 0 beyond
LDS: long paths taken whole as their own backbone) against the FP64 oracle
on sampled rows. Error metric and bars as in test_gpu_parity.

Plans made only of such paths run in whole-path mode (stage
"fft_conv1d_path": field rows in, output rows out); a forest that also holds
a bushy tree keeps the scatter/gather around the same kernels (stage
"fft_conv1d")."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import synth as S
from paper_2609_34025_amd import TreeIntegrator

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-4}
DEV = "cuda:0"


def relerr(y, ref):
    return np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref)


def wavy(K):
    k = np.arange(K, dtype=np.float64)
    return np.exp(-0.0005 * k) * (1.0 + 0.5 * np.cos(0.01 * k))


def run(p, w, ftab, F, dtype, rows):
    """Profiled (eager) run checked against the oracle, then two graph
    replays that must reproduce it bit for bit."""
    t = TreeIntegrator(p, w, device=0)
    K = t.kernel_length
    f = torch.tensor(ftab(K), dtype=dtype, device=DEV)
    Ft = torch.tensor(F, dtype=dtype, device=DEV)
    t.profile(True)
    out = t.integrate(f, Ft)
    torch.cuda.synchronize()
    stages = t.profile_report()
    t.profile(False)
    for _ in range(2):
        again = t.integrate(f, Ft)
        torch.cuda.synchronize()
        assert torch.equal(again, out)
    ref = oracle.integrate(p, w, ftab(K), F, rows=rows)
    return relerr(out.cpu().numpy()[rows], ref), stages


@pytest.mark.parametrize("d", [1, 2, 5, 16, 33, 130])
def test_long_path_fp32(d):
    n = 20000
    print(f"conv1d path n={n} d={d} fp32", flush=True)
    p, w = S.path(n)
    rng = np.random.default_rng(d)
    F = rng.standard_normal((n, d))
    rows = np.sort(rng.choice(n, 256, replace=False))
    e, st = run(p, w, wavy, F, torch.float32, rows)
    print(f"  err {e:.2e}", flush=True)
    assert "fft_conv1d_path" in st, st
    assert e <= TOL[torch.float32], e


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("d", [3, 20])
def test_long_path_beside_bushy_tree(dtype, d):
    rng = np.random.default_rng(40 + d)
    pa, wa = S.path(25000)
    pb, _ = S.random_recursive(3000, rng)
    wb = S.uniform_weights(pb, 1, 4, rng)
    p, w, _ = S.forest([(pa, wa), (pb, wb)])
    N = len(p)
    print(f"conv1d path+tree forest N={N} d={d} {dtype}", flush=True)
    F = rng.standard_normal((N, d))
    rows = np.sort(np.concatenate([rng.choice(25000, 200, replace=False),
                                   25000 + rng.choice(3000, 56, replace=False)]))
    e, st = run(p, w, wavy, F, dtype, rows)
    print(f"  err {e:.2e}", flush=True)
    assert "fft_conv1d" in st and "fft_conv1d_path" not in st, st
    assert e <= TOL[dtype], e


def test_weighted_path_forest_fp64():
    rng = np.random.default_rng(7)
    trees = []
    for n in (6000, 7000, 9000):
        p, _ = S.path(n)
        trees.append((p, S.uniform_weights(p, 1, 3, rng)))
    p, w, _ = S.forest(trees)
    N = len(p)
    print(f"conv1d weighted path forest N={N} d=3 fp64", flush=True)
    F = rng.standard_normal((N, 3))
    rows = np.sort(rng.choice(N, 256, replace=False))
    e, st = run(p, w, wavy, F, torch.float64, rows)
    print(f"  err {e:.2e}", flush=True)
    assert "fft_conv1d_path" in st, st
    assert e <= TOL[torch.float64], e


def test_serpentine_attention_payload_fp32():
    side = 150
    print(f"conv1d serpentine side={side} payload r=2 dh=8 fp32", flush=True)
    p, w = S.patch_grid_tree("serpentine", side)
    rng = np.random.default_rng(11)
    phi, v = S.attention_features(len(p), 2, 8, rng)
    F = S.attention_payload(phi, v).astype(np.float64)
    rows = np.sort(rng.choice(len(p), 256, replace=False))
    mask = lambda K: S.topo_mask_table(K, -1e-5, -0.01, 0.5)
    e, st = run(p, w, mask, F, torch.float32, rows)
    print(f"  err {e:.2e}", flush=True)
    assert "fft_conv1d_path" in st, st
    assert e <= TOL[torch.float32], e


def test_long_path_backward_dF_fp32():
    n = 30000
    print(f"conv1d path backward n={n} d=8 fp32", flush=True)
    p, w = S.path(n)
    rng = np.random.default_rng(3)
    F = rng.standard_normal((n, 8))
    G = rng.standard_normal((n, 8))
    t = TreeIntegrator(p, w, device=0)
    K = t.kernel_length
    f = torch.tensor(wavy(K), dtype=torch.float32, device=DEV)
    dF, _ = t.backward(f, torch.tensor(F, dtype=torch.float32, device=DEV),
                       torch.tensor(G, dtype=torch.float32, device=DEV),
                       need_dF=True, need_df=False)
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(n, 256, replace=False))
    ref = oracle.integrate(p, w, wavy(K), G, rows=rows)
    e = relerr(dF.cpu().numpy()[rows], ref)
    print(f"  err {e:.2e}", flush=True)
    assert e <= TOL[torch.float32], e


def test_long_path_backward_dF_and_df_fp64():
    """df needs the cell sums, so this backward leaves whole-path mode."""
    n = 20000
    print(f"conv1d path backward dF+df n={n} d=2 fp64", flush=True)
    p, w = S.path(n)
    rng = np.random.default_rng(5)
    F = rng.standard_normal((n, 2))
    G = rng.standard_normal((n, 2))
    t = TreeIntegrator(p, w, device=0)
    K = t.kernel_length
    f = torch.tensor(wavy(K), dtype=torch.float64, device=DEV)
    dF, df = t.backward(f, torch.tensor(F, device=DEV), torch.tensor(G, device=DEV))
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(n, 256, replace=False))
    e1 = relerr(dF.cpu().numpy()[rows], oracle.integrate(p, w, wavy(K), G, rows=rows))
    h = oracle.pair_hist(p, w, G, F, K)
    e2 = relerr(df.cpu().numpy(), h)
    print(f"  err dF {e1:.2e} df {e2:.2e}", flush=True)
    assert e1 <= 1e-10 and e2 <= 1e-10, (e1, e2)


@pytest.mark.parametrize("dtype,d", [(torch.float64, 5), (torch.float32, 33)])
def test_one_column_tables(dtype, d):
    """Centroid calls and corrections are one-column tables (a single
    backbone position, G(q) = sum_r f(q + r) A_r): the hub of a long-arm
    spider has depth 1000, so its table and the arms' corrections take the
    channel-tiled kernels with reflected sources."""
    p, w = S.spider(8, 1000)
    rng = np.random.default_rng(21 + d)
    print(f"conv1d one-column spider 8x1000 d={d} {dtype}", flush=True)
    F = rng.standard_normal((len(p), d))
    rows = np.sort(rng.choice(len(p), 200, replace=False))
    t = TreeIntegrator(p, w, device=0, policy="centroid", table_method="fft")
    K = t.kernel_length
    f = torch.tensor(wavy(K), dtype=dtype, device=DEV)
    t.profile(True)
    y = t.integrate(f, torch.tensor(F, dtype=dtype, device=DEV))
    torch.cuda.synchronize()
    st = t.profile_report()
    t.profile(False)
    assert "fft_conv1d" in st, st
    ref = oracle.integrate(p, w, wavy(K), F, rows=rows)
    e = relerr(y.cpu().numpy()[rows], ref)
    print(f"  err {e:.2e}", flush=True)
    assert e <= TOL[dtype], e


@pytest.mark.parametrize("side", [384, 512])
def test_serpentine_full_size_c4160(side):
    """The masked-attention payload at full width (C = 4160, r = dh = 64) on
    the 384 x 384 and 512 x 512 serpentine paths, as the benchmark runs it:
    P = 2^19 lattice points, 16 channel pairs per slot, the 2^9-point
    high-bit passes and the 2^10-point low-bit pass in two channel halves.
    32 sampled rows x 64 sampled channels against the FP64 oracle (every
    channel is integrated on its own, so a channel subset of F gives the
    same rows of those channels), and a graph replay that reproduces the
    profiled run bit for bit."""
    W = S.workload("attn", tree="serpentine", side=side)
    p, w = W["parent"], W["weight"]
    n, C = len(p), W["d"]
    print(f"conv1d serpentine side={side} N={n} C={C} fp32", flush=True)
    t = TreeIntegrator(p, w, device=0)
    K = t.kernel_length
    tab = W["kernels"][0][1](K)
    f = torch.tensor(tab, dtype=torch.float32, device=DEV)
    phi = torch.from_numpy(W["phi"]).to(DEV)
    v = torch.from_numpy(W["v"]).to(DEV)
    F = torch.cat([(phi[:, :, None] * v[:, None, :]).reshape(n, -1), phi], 1).contiguous()
    del phi, v
    t.profile(True)
    y = t.integrate(f, F)
    torch.cuda.synchronize()
    st = t.profile_report()
    t.profile(False)
    assert "fft_conv1d_path" in st, st
    again = t.integrate(f, F)
    torch.cuda.synchronize()
    assert torch.equal(again, y)
    del again
    rng = np.random.default_rng(side)
    rows = np.sort(rng.choice(n, 32, replace=False))
    chans = np.sort(rng.choice(C, 64, replace=False))
    Fs = F[:, torch.from_numpy(chans).to(DEV)].double().cpu().numpy()
    got = y[torch.from_numpy(rows).to(DEV)][:, torch.from_numpy(chans).to(DEV)]
    got = got.double().cpu().numpy()
    ref = oracle.integrate(p, w, tab, Fs, rows=rows)
    e = relerr(got, ref)
    print(f"  err {e:.2e}", flush=True)
    assert e <= TOL[torch.float32], e
    del t, F, y
    torch.cuda.empty_cache()


def test_comb_c4160_lds_tables_in_xcd_order():
    """The masked-attention payload at full width on the 256 x 256 comb at
    the direct/FFT rule the benchmark's tuner picks (8): its FFT tables fit
    LDS, and with 2080 channel pairs every job has far more than 16 pair
    groups, so k_fft_conv_multi runs its 4096-point workgroups in the XCD
    order (job j on XCD j mod 8, the job columns padded to a multiple of 8)
    and its smaller tables take more pairs per workgroup. 32 sampled rows x
    64 sampled channels against the FP64 oracle, and a graph replay equal
    to the profiled run bit for bit."""
    W = S.workload("attn", tree="comb", side=256)
    p, w = W["parent"], W["weight"]
    n, C = len(p), W["d"]
    print(f"comb side=256 N={n} C={C} fp32 fft_cost 8", flush=True)
    t = TreeIntegrator(p, w, device=0)
    t.set_fft_cost(8.0)
    K = t.kernel_length
    tab = W["kernels"][0][1](K)
    f = torch.tensor(tab, dtype=torch.float32, device=DEV)
    phi = torch.from_numpy(W["phi"]).to(DEV)
    v = torch.from_numpy(W["v"]).to(DEV)
    F = torch.cat([(phi[:, :, None] * v[:, None, :]).reshape(n, -1), phi], 1).contiguous()
    del phi, v
    t.profile(True)
    y = t.integrate(f, F)
    torch.cuda.synchronize()
    st = t.profile_report()
    t.profile(False)
    assert "fft_lds" in st, st
    again = t.integrate(f, F)
    torch.cuda.synchronize()
    assert torch.equal(again, y)
    del again
    rng = np.random.default_rng(256)
    rows = np.sort(rng.choice(n, 32, replace=False))
    chans = np.sort(rng.choice(C, 64, replace=False))
    Fs = F[:, torch.from_numpy(chans).to(DEV)].double().cpu().numpy()
    got = y[torch.from_numpy(rows).to(DEV)][:, torch.from_numpy(chans).to(DEV)]
    got = got.double().cpu().numpy()
    ref = oracle.integrate(p, w, tab, Fs, rows=rows)
    e = relerr(got, ref)
    print(f"  err {e:.2e}", flush=True)
    assert e <= TOL[torch.float32], e
    del t, F, y
    torch.cuda.empty_cache()
