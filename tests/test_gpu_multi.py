"""Several kernels over one field in one call (tfi_integrate_multi): every
output equals the separate tfi_integrate call bit for bit, on general plans
(direct and FFT tables, leaf tiles, corrections) and in whole-path mode,
across graph replays; plus the oracle on sampled rows."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import synth as S
from paper_2609_34025_amd import TreeIntegrator

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def kernels(K, nk):
    k = np.arange(K, dtype=np.float64)
    tabs = [np.exp(-0.05 * k), 1.0 / (1.0 + k) ** 2, np.exp(-0.002 * k) * np.cos(0.01 * k),
            1.0 / (1.0 + k)]
    return tabs[:nk]


@pytest.mark.parametrize("case", ["rrt_auto_f32", "rrt_fft_f64", "grid_direct_f32",
                                  "path_f32", "forest_f64"])
def test_multi_equals_separate_calls(case):
    rng = np.random.default_rng(3)
    opts, dtype, d, nk = {}, torch.float32, 16, 2
    if case.startswith("rrt"):
        p, _ = S.random_recursive(6000, rng)
        w = S.uniform_weights(p, 1, 8, rng)
        if case == "rrt_fft_f64":
            opts, dtype, d, nk = {"table_method": "fft"}, torch.float64, 5, 3
    elif case == "grid_direct_f32":
        p, w = S.grid_mst(40, 9, rng)
        opts, d, nk = {"table_method": "direct"}, 33, 4
    elif case == "path_f32":
        p, w = S.path(20000)
        d, nk = 8, 2
    else:
        t1 = S.random_recursive(500, rng)
        p, w, _ = S.forest([(t1[0], S.uniform_weights(t1[0], 1, 4, rng)), S.path(3000),
                            S.grid_mst(9, 5, rng), S.star(7)])
        dtype, d, nk = torch.float64, 3, 3
    print(f"multi {case} N={len(p)} d={d} nk={nk}", flush=True)
    t = TreeIntegrator(p, w, device=0, **opts)
    K = t.kernel_length
    tabs = kernels(K, nk)
    fs = [torch.tensor(x, dtype=dtype, device=DEV) for x in tabs]
    for rep in range(3):
        F = torch.tensor(rng.standard_normal((len(p), d)), dtype=dtype, device=DEV)
        outs = t.integrate_many(fs, F)
        sep = [t.integrate(f, F) for f in fs]
        torch.cuda.synchronize()
        for a, b in zip(outs, sep):
            assert torch.equal(a, b), (case, rep)
    rows = np.sort(rng.choice(len(p), 64, replace=False))
    Fn = F.double().cpu().numpy()
    tol = 1e-10 if dtype == torch.float64 else 1e-4
    for tab, y in zip(tabs, outs):
        ref = oracle.integrate(p, w, tab, Fn, rows=rows)
        e = np.linalg.norm(y.double().cpu().numpy()[rows] - ref) / np.linalg.norm(ref)
        assert e <= tol, (case, e)


def test_multi_argument_errors():
    p, w = S.path(50)
    t = TreeIntegrator(p, w, device=0)
    f = torch.ones(t.kernel_length, device=DEV)
    F = torch.ones(50, 2, device=DEV)
    with pytest.raises(ValueError):
        t.integrate_many([], F)
    with pytest.raises(ValueError):
        t.integrate_many([f] * 5, F)
    with pytest.raises(TypeError):
        t.integrate_many([f, f.double()], F)


def test_tuned_leaf_size():
    """TreeIntegrator.tuned builds one plan per leaf-tile size, keeps the
    fastest, and that plan integrates like any other (oracle on rows)."""
    rng = np.random.default_rng(12)
    p, _ = S.random_recursive(5000, rng)
    w = S.uniform_weights(p, 1, 8, rng)
    d = 16
    print(f"tuned leaf sizes rrt N={len(p)} d={d}", flush=True)
    make = lambda K: [torch.tensor(t, dtype=torch.float32, device=DEV) for t in kernels(K, 2)]
    t = TreeIntegrator.tuned(p, w, make, d, leaf_sizes=(8, 64), reps=5)
    assert set(t.tuning) == {8, 64} and t.leaf_max in t.tuning
    assert t.tuning[t.leaf_max] == min(t.tuning.values())
    assert t.stats()["leaf_max"] == t.leaf_max
    F = rng.standard_normal((len(p), d))
    outs = t.integrate_many(make(t.kernel_length), torch.tensor(F, dtype=torch.float32, device=DEV))
    rows = np.sort(rng.choice(len(p), 128, replace=False))
    for tab, y in zip(kernels(t.kernel_length, 2), outs):
        ref = oracle.integrate(p, w, tab, F, rows=rows)
        e = np.linalg.norm(y.cpu().numpy()[rows] - ref) / np.linalg.norm(ref)
        assert e <= 1e-4, e


def test_preallocated_outputs():
    """out= writes the same values into the caller's tensors (one graph for
    the loop); bad out arguments are errors."""
    rng = np.random.default_rng(14)
    p, _ = S.random_recursive(3000, rng)
    w = S.uniform_weights(p, 1, 8, rng)
    d = 8
    print(f"preallocated outputs rrt N={len(p)} d={d}", flush=True)
    t = TreeIntegrator(p, w, device=0)
    fs = [torch.tensor(x, dtype=torch.float32, device=DEV) for x in kernels(t.kernel_length, 2)]
    F = torch.tensor(rng.standard_normal((len(p), d)), dtype=torch.float32, device=DEV)
    ref = t.integrate_many(fs, F)
    outs = [torch.full_like(F, float("nan")) for _ in fs]
    for _ in range(3):
        got = t.integrate_many(fs, F, out=outs)
        torch.cuda.synchronize()
        assert all(g is o for g, o in zip(got, outs))
        assert all(torch.equal(a, b) for a, b in zip(ref, outs))
    one = torch.empty_like(F)
    assert t.integrate(fs[0], F, out=one) is one and torch.equal(one, t.integrate(fs[0], F))
    with pytest.raises(ValueError):
        t.integrate(fs[0], F, out=F)
    with pytest.raises(ValueError):
        t.integrate(fs[0], F, out=one[:-1])
    with pytest.raises(ValueError):
        t.integrate_many(fs, F, out=[one, one])
    with pytest.raises(ValueError):
        t.integrate_many(fs, F, out=[one])
