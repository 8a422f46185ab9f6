"""Shapes of the FFT convolution kernels (tfi_set_fft_params, searched by
tfi_autotune_fft): pairs per LDS workgroup, the 1-D threshold, tile width and
tile groups of the 1-D kernels, columns per workgroup of the blocked global
passes. They change only how the transforms of lemma "stad-2d-fft" are
blocked, so every setting must give the default's result up to rounding and
the oracle's rows. FP64, every table forced to the FFT."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import TreeIntegrator, synth as S

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# random spanning trees of a 96 x 96 patch grid: under the diameter policy
# the FFT tables fill all three LDS tiers and three exceed LDS (blocked
# global passes); under the adaptive policy two one-column tables of 2^10
# points take the 1-D kernels
SETTINGS = [
    {"lds_pairs": [1, 1, 1]},
    {"lds_pairs": [8, 4, 2]},
    {"lds_pairs": [32, 32, 32]},
    {"conv1d_min_lg": 6},
    {"conv1d_min_lg": 15},
    {"conv1d_pairs": 1},
    {"conv1d_pairs": 2, "conv1d_group_mib": 1},
    {"col_lines": 1},
    {"col_lines": 4},
    {"col_lines": 64},
]


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(policy):
    p, w = S.patch_grid_tree("random", 96, np.random.default_rng(91))
    t = TreeIntegrator(p, w, device=0, policy=policy, table_method="fft")
    K = t.kernel_length
    ftab = np.exp(-0.05 * np.arange(K)) + 0.3 / (1.0 + np.arange(K))
    rng = np.random.default_rng(92)
    F = rng.standard_normal((len(p), 6))
    G = rng.standard_normal((len(p), 6))
    return p, w, t, ftab, F, G


def _run(t, ftab, F, G):
    f = torch.tensor(ftab, dtype=torch.float64, device=DEV)
    Ft = torch.tensor(F, device=DEV)
    Gt = torch.tensor(G, device=DEV)
    t.profile(True)
    y = t.integrate(f, Ft)
    dF, df = t.backward(f, Ft, Gt)
    torch.cuda.synchronize()
    stages = t.profile_report()
    t.profile(False)
    return y.cpu().numpy(), dF.cpu().numpy(), df.cpu().numpy(), stages


@pytest.mark.parametrize("policy", ["diameter", "adaptive"])
def test_settings_agree(policy):
    p, w, t, ftab, F, G = _case(policy)
    y0, dF0, df0, st0 = _run(t, ftab, F, G)
    paths = sorted(k for k in st0 if k.startswith("fft") or k.startswith("df_fft"))
    print(f"{policy}: default {t.fft_params()} stages {paths}", flush=True)
    if policy == "diameter":
        assert "fft_lds" in st0 and "fft_global" in st0
    else:
        assert "fft_conv1d" in st0
    rows = np.sort(np.random.default_rng(93).choice(len(p), 48, replace=False))
    ref = oracle.integrate(p, w, ftab, F, rows=rows)
    assert relerr(y0[rows], ref) <= 1e-10
    base = t.fft_params()
    for ch in SETTINGS:
        t.set_fft_params(**{**base, **ch})
        assert {k: t.fft_params()[k] for k in ch} == ch
        y, dF, df, st = _run(t, ftab, F, G)
        e = [relerr(y, y0), relerr(dF, dF0), relerr(df, df0)]
        print(f"{policy} {ch}: {e}", flush=True)
        assert max(e) <= 1e-12, (ch, e)
        assert relerr(y[rows], ref) <= 1e-10
    if policy == "adaptive":
        # 2^15 points: the one-column tables of 2^10 points stay in LDS
        t.set_fft_params(**{**base, "conv1d_min_lg": 15})
        assert "fft_conv1d" not in _run(t, ftab, F, G)[3]
    t.set_fft_params(**base)
    assert t.fft_params() == base


def test_bad_settings_refused():
    p, w, t, ftab, F, G = _case("diameter")
    for bad in ({"lds_pairs": [3, 0, 0]}, {"lds_pairs": [0, 0, 128]}, {"conv1d_min_lg": 1},
                {"conv1d_pairs": 32}, {"conv1d_group_mib": -1}, {"col_lines": 0},
                {"col_lines": 12}):
        with pytest.raises(RuntimeError, match="TFI_ERR_ARG"):
            t.set_fft_params(**bad)
    assert t.fft_params()["col_lines"] == 16


def test_autotune_forced_fft_and_cache(tmp_path):
    """Autotune with the FFT-shape search on a handle whose tables are all
    forced to the FFT keeps the method, tunes the kernel shapes, and a second
    handle restores them from the cache without timing."""
    p, w, t, ftab, F, G = _case("diameter")
    y0, dF0, df0, _ = _run(t, ftab, F, G)
    f = torch.tensor(ftab, dtype=torch.float64, device=DEV)
    cache = str(tmp_path / "tune.json")
    t.autotune(f, 6, cache=cache, backward=True, fft_shapes=True)
    tuned = t.fft_params()
    y, dF, df, _ = _run(t, ftab, F, G)
    assert max(relerr(y, y0), relerr(dF, dF0), relerr(df, df0)) <= 1e-12
    ent = list(json.load(open(cache)).values())[0]
    assert ent["fft"] == tuned
    print(f"tuned {tuned}", flush=True)
    t2 = TreeIntegrator(p, w, device=0, policy="diameter", table_method="fft")
    t2.autotune(f, 6, cache=cache, backward=True, fft_shapes=True)
    assert t2.fft_params() == tuned
    y2, _, _, _ = _run(t2, ftab, F, G)
    assert relerr(y2, y0) <= 1e-12
