"""GPU: tfi_integrate_noalloc, the forward whose scratch lives in a fixed
device array, against tfi_integrate (same kernels, so equal bit for bit)
and against the FP64 oracle, on two calls in a row with the second input
smaller than the first (the array keeps the first call's contents)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2609_34025_amd import TreeIntegrator, _lib
from paper_2609_34025_amd import synth as S
from paper_2609_34025_amd._lib import TFIError

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {torch.float64: 1e-10, torch.float32: 1e-4}


def relerr(y, ref):
    return np.linalg.norm(np.asarray(y, np.float64) - ref) / np.linalg.norm(ref)


def noalloc(t, f, F, out):
    """The entry point through the C ABI."""
    d = 1 if F.dim() == 1 else F.shape[1]
    dt = _lib.TFI_F32 if F.dtype == torch.float32 else _lib.TFI_F64
    stream = torch.cuda.current_stream().cuda_stream
    _lib.check(_lib.load().tfi_integrate_noalloc(t._h, f.data_ptr(), F.data_ptr(), d, dt,
                                                 out.data_ptr(), stream))
    return out


def case(p, w, ftab, F, dtype, rows, **opts):
    t = TreeIntegrator(p, w, device=0, **opts)
    K = t.kernel_length
    f = torch.tensor(ftab(K), dtype=dtype, device=DEV)
    Ft = torch.tensor(F, dtype=dtype, device=DEV)
    ref_gpu = t.integrate(f, Ft)
    out = torch.full_like(Ft, float("nan"))
    noalloc(t, f, Ft, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_gpu)
    ref = oracle.integrate(p, w, ftab(K), F, rows=rows)
    e = relerr(out.cpu().numpy()[rows], ref)
    assert e <= TOL[dtype], e
    return t, e


def test_noalloc_matches_integrate_large_then_small():
    W = S.workload("rrt100k")
    p, w, F = W["parent"], W["weight"], W["F"]
    rows = np.sort(np.random.default_rng(1).choice(len(p), 256, replace=False))
    print("noalloc rrt100k N=100000 d=16 fp32 leaf 64", flush=True)
    _, e1 = case(p, w, W["kernels"][1][1], F, torch.float32, rows, leaf_max=64)
    Ws = S.workload("small")
    print("noalloc small N=2000 d=4 fp64", flush=True)
    _, e2 = case(Ws["parent"], Ws["weight"], Ws["kernels"][0][1], Ws["F"], torch.float64,
                 np.arange(2000))
    print(f"  errs {e1:.2e} {e2:.2e}", flush=True)


def test_noalloc_fft_paths_large_then_small():
    # whole-path mode (the 1-D convolution slots in the scratch array), then
    # a smaller forest whose tables go through the LDS and global FFT passes
    rng = np.random.default_rng(3)
    p, w = S.path(30000)
    F = rng.standard_normal((len(p), 8))
    wavy = lambda K: np.exp(-0.0005 * np.arange(K)) * (1 + 0.5 * np.cos(0.01 * np.arange(K)))
    print("noalloc path N=30000 d=8 fp32", flush=True)
    _, e1 = case(p, w, wavy, F, torch.float32,
                 np.sort(rng.choice(len(p), 256, replace=False)))
    p2, w2 = S.spider(8, 300)
    F2 = rng.standard_normal((len(p2), 3))
    print("noalloc spider 8x300 d=3 fp64 fft tables", flush=True)
    _, e2 = case(p2, w2, wavy, F2, torch.float64, np.arange(len(p2)), policy="diameter",
                 table_method="fft")
    print(f"  errs {e1:.2e} {e2:.2e}", flush=True)


def test_noalloc_rejects_too_much_scratch():
    # d = 1024 on the 100k-vertex tree needs far more than the fixed array:
    # refused on the host before any launch, and the handle still works
    W = S.workload("rrt100k")
    p, w = W["parent"], W["weight"]
    t = TreeIntegrator(p, w, device=0)
    f = torch.tensor(W["kernels"][0][1](t.kernel_length), dtype=torch.float32, device=DEV)
    F = torch.zeros((len(p), 1024), dtype=torch.float32, device=DEV)
    out = torch.empty_like(F)
    with pytest.raises(TFIError) as ei:
        noalloc(t, f, F, out)
    assert ei.value.code == -6 and b"scratch" in _lib.load().tfi_last_error()
    F1 = torch.ones((len(p), 2), dtype=torch.float32, device=DEV)
    y = noalloc(t, f, F1, torch.empty_like(F1))
    torch.cuda.synchronize()
    assert torch.equal(y, t.integrate(f, F1))
