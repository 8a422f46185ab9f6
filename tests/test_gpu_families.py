"""The fifteen synthetic families of the paper's benchmark at their largest
sizes (appendix table "synthetic-largest"), under each backbone policy:
FP64 scalar fields against the oracle on every row (bar 1e-10), and FP32
fields of C = 4160 channels on sampled rows x channels (bar 1e-4)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import synth as S
from paper_2609_34025_amd import TreeIntegrator

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relerr(y, ref):
    return np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("policy", ["adaptive", "diameter", "centroid"])
def test_paper_families_scalar_fp64(policy):
    for name, p, w in S.paper_families():
        print(f"family {name} N={len(p)} policy={policy} fp64 d=1", flush=True)
        t = TreeIntegrator(p, w, device=0, policy=policy)
        K = t.kernel_length
        tab = 1.0 / (1.0 + np.arange(K, dtype=np.float64))
        F = np.random.default_rng(123).standard_normal(len(p))
        y = t.integrate(torch.tensor(tab, device=DEV), torch.tensor(F, device=DEV))
        torch.cuda.synchronize()
        e = relerr(y.cpu().numpy(), oracle.integrate(p, w, tab, F))
        assert e <= 1e-10, (name, policy, e)


@pytest.mark.parametrize("policy", ["adaptive", "diameter", "centroid"])
def test_paper_families_wide_fp32(policy):
    for name, p, w in S.paper_families():
        n = len(p)
        print(f"family {name} N={n} policy={policy} fp32 C=4160", flush=True)
        rng = np.random.default_rng(5)
        phi, v = S.attention_features(n, 64, 64, rng)
        F = S.attention_payload(phi, v)
        t = TreeIntegrator(p, w, device=0, policy=policy)
        K = t.kernel_length
        tab = 1.0 / (1.0 + np.arange(K, dtype=np.float64))
        y = t.integrate(torch.tensor(tab, dtype=torch.float32, device=DEV),
                        torch.tensor(F, device=DEV))
        torch.cuda.synchronize()
        rows = np.sort(rng.choice(n, 24, replace=False))
        ch = np.sort(rng.choice(F.shape[1], 40, replace=False))
        ref = oracle.integrate(p, w, tab, F[:, ch].astype(np.float64), rows=rows)
        e = relerr(y.cpu().numpy()[rows][:, ch], ref)
        assert e <= 1e-4, (name, policy, e)


def test_calibrated_channel_policy():
    """tfi_calibrate on an adaptive plan, then a channel-aware plan built
    from the measured costs: finite positive costs, the calibrated handle
    gives bit-identical results afterwards, and the new plan matches the
    oracle."""
    fams = {name: (p, w) for name, p, w in S.paper_families()}
    for name in ("random_recursive", "caterpillar_hanging_paths", "long_arm_spider"):
        p, w = fams[name]
        n, C = len(p), 96
        print(f"calibrate {name} N={n} C={C} fp32", flush=True)
        rng = np.random.default_rng(9)
        F = torch.tensor(rng.standard_normal((n, C)), dtype=torch.float32, device=DEV)
        t = TreeIntegrator(p, w, device=0)
        K = t.kernel_length
        tab = 1.0 / (1.0 + np.arange(K, dtype=np.float64))
        f = torch.tensor(tab, dtype=torch.float32, device=DEV)
        before = t.integrate(f, F)
        cm = t.calibrate(f, C)
        after = t.integrate(f, F)
        torch.cuda.synchronize()
        assert torch.equal(before, after)
        assert cm["direct"] > 0 and cm["fft"] > 0 and cm["vertex"] >= 0, cm
        assert all(np.isfinite(v) for v in cm.values()), cm
        t2 = TreeIntegrator(p, w, device=0, policy="channel", channel_width=C, cost_model=cm)
        K2 = t2.kernel_length
        tab2 = 1.0 / (1.0 + np.arange(K2, dtype=np.float64))
        y = t2.integrate(torch.tensor(tab2, dtype=torch.float32, device=DEV), F)
        torch.cuda.synchronize()
        rows = np.sort(rng.choice(n, 64, replace=False))
        ref = oracle.integrate(p, w, tab2, F.double().cpu().numpy(), rows=rows)
        e = relerr(y.cpu().numpy()[rows], ref)
        assert e <= 1e-4, (name, e)
