"""User-facing tree field integrator on one MI355X GPU.

``TreeIntegrator`` owns a plan built once per forest (``tfi_build``) and
integrates fields on the GPU: ``out[v] = sum_w f(dist(v, w)) F[w]``.
``TreeIntegrate`` is the autograd function with the hand-written adjoint
(dF = f(D) gout since f(D) is symmetric; df from pair histograms), and
``expsum_table`` materialises the learnable kernel
``f(k) = sum_j a_j exp(-b_j k)`` as a table so autograd carries df to da, db.

PyTorch supplies device memory and the current stream; all arithmetic runs
in libtfi.so.
"""
from __future__ import annotations

import ctypes as C
import json
import time
import os

import numpy as np
import torch

from . import _lib

EXPSUM_MAX_TERMS = 16

_DTYPES = {torch.float32: _lib.TFI_F32, torch.float64: _lib.TFI_F64}


class TreeIntegrator:
    """Plan of one forest, uploaded to one GPU.

    parent  int64[N], -1 at roots; weight int32[N] >= 1 (edge to parent).
    policy  'adaptive' (paper's score), 'diameter', 'centroid', or 'channel'
            (the channel-aware cost model of ``channel_width`` channels and
            ``cost_model``, e.g. from ``calibrate``).
    leaf_max  subtrees up to this size are integrated densely (0 = default).
    device  CUDA/HIP device index, or None for a host-only plan (stats and
            plan inspection only).
    table_method  'auto', 'direct' or 'fft' for every interaction table, or
            'fft1d': tables with several depths and backbone positions as one
            1-D FFT convolution along the backbone per pair of depths (with
            policy 'diameter', the paper's Diameter-1D variant), the others
            by FFT; or 'hankel': such tables of depth <= 127 by the product
            with the Hankel matrix f(l + r) and walks along the backbone, the
            others by FFT.
    memory_budget  cap in bytes on device memory held by the handle (0 = no cap);
            an integration or adjoint whose scratch would exceed it runs on
            tiles of channels that fit.
    graphs  replay captured hipGraphs (True) or launch kernels directly.
    fft_cost  direct sums for a table iff cells^2 <= fft_cost * P log2 P
            (0 = default 4).
    direct_kernel  'auto' (matrix cores for FP32 with d >= 8), 'vector' or
            'mfma'.
    channel_width, cost_model  for policy 'channel': the channel count C and
            {'vertex', 'direct', 'fft', 'call'} costs in seconds per unit
            (None = defaults).
    """

    def __init__(self, parent, weight, *, policy="adaptive", leaf_max=0, device=0,
                 table_method="auto", memory_budget=0, graphs=True, fft_cost=0.0,
                 direct_kernel="auto", channel_width=0, cost_model=None):
        if device is not None and isinstance(device, torch.device):
            device = device.index or 0
        self._h = _lib.build_handle(parent, weight, policy=policy, leaf_max=leaf_max,
                                    device=device, table_method=table_method,
                                    memory_budget=memory_budget, graphs=graphs,
                                    fft_cost=fft_cost, direct_kernel=direct_kernel,
                                    channel_width=channel_width, cost_model=cost_model)
        self.device = None if device is None else torch.device("cuda", int(device))
        lib = _lib.load()
        self.num_vertices = int(lib.tfi_num_vertices(self._h))
        self.kernel_length = int(lib.tfi_kernel_length(self._h))

    @classmethod
    def tuned(cls, parent, weight, f, d, *, leaf_sizes=(16, 32, 48, 64), device=0, reps=30,
              **options):
        """Plan with the fastest dense leaf-tile size for forward integrations
        of ``d`` channels with the kernel table ``f`` (or a list of tables,
        integrated together as by ``integrate_many``; or a callable that
        returns them for a kernel length, since the length a plan needs can
        depend on its leaf tiles). One plan per size in
        ``leaf_sizes`` is built, its table rule autotuned (``autotune``) and
        ``reps`` integrations of a zero field timed; the fastest plan is
        returned with ``tuning`` = {leaf size: ms per integration}. Larger
        tiles trade incidences and table work for dense n^2 tile work, so the
        best size depends on the tree, d and the dtype. ``options`` go to the
        constructor."""
        best, times = None, {}
        for leaf in leaf_sizes:
            t = cls(parent, weight, leaf_max=int(leaf), device=device, **options)
            fs = f(t.kernel_length) if callable(f) else f
            fs = list(fs) if isinstance(fs, (list, tuple)) else [fs]
            t.autotune(fs[0], d)
            F = torch.zeros((t.num_vertices, int(d)), dtype=fs[0].dtype, device=t.device)
            outs = [torch.empty_like(F) for _ in fs]
            run = ((lambda: t.integrate_many(fs, F, out=outs)) if len(fs) > 1
                   else (lambda: t.integrate(fs[0], F, out=outs[0])))
            for _ in range(3):
                run()
            torch.cuda.synchronize(t.device)
            t0 = time.perf_counter()
            for _ in range(reps):
                run()
            torch.cuda.synchronize(t.device)
            times[int(leaf)] = 1e3 * (time.perf_counter() - t0) / reps
            del F, outs
            if best is None or times[int(leaf)] < times[best[0]]:
                if best is not None:
                    best[1].close()
                best = (int(leaf), t)
            else:
                t.close()
        best[1].tuning = times
        best[1].leaf_max = best[0]
        return best[1]

    # ------------------------------------------------------------- info --
    def stats(self):
        lib = _lib.load()
        n = _lib.check(lib.tfi_plan_stats(self._h, None, 0))
        buf = C.create_string_buffer(n + 1)
        _lib.check(lib.tfi_plan_stats(self._h, buf, n + 1))
        return json.loads(buf.value.decode())

    def export(self, name):
        lib = _lib.load()
        nbytes = _lib.check(lib.tfi_plan_export(self._h, name.encode(), None, 0))
        kind = self.stats()["arrays"][name]
        arr = np.empty(nbytes // np.dtype(_lib._EXPORT_TYPES[kind]).itemsize,
                       dtype=_lib._EXPORT_TYPES[kind])
        if arr.nbytes != nbytes:
            raise _lib.TFIError(-1, f"plan array {name}: {nbytes} bytes is not a whole number "
                                    f"of {kind} elements")
        if nbytes:
            _lib.check(lib.tfi_plan_export(self._h, name.encode(), arr.ctypes.data, arr.nbytes))
        return arr

    def autotune(self, f, d, cache=None, backward=False, fft_shapes=False):
        """Choose the per-table method rule (direct sums vs FFT) and the
        cell-sum strategy by timing passes of ``d`` channels in ``f``'s
        dtype: forward integrations, or forward + adjoint (dF and df) with
        ``backward=True``; with ``fft_shapes=True`` also the FFT kernels'
        shapes (``tfi_autotune_fft``). The fastest settings stay in effect.
        ``cache``: optional JSON file of tuned settings keyed by (plan
        fingerprint, d, dtype, pass), read before and updated after tuning.
        Returns the chosen cost constant."""
        self._check(f)
        key = (f"{self.stats()['fingerprint']}:{int(d)}:{str(f.dtype)}:"
               f"{'fwdbwd' if backward else 'fwd'}{':fft' if fft_shapes else ''}")
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fp:
                table = json.load(fp)
        lib = _lib.load()
        if key in table:
            ent = table[key]
            if not isinstance(ent, dict):
                ent = {"fft_cost": ent}
            _lib.check(lib.tfi_set_fft_cost(self._h, float(ent["fft_cost"])))
            if "scatter" in ent:
                _lib.check(lib.tfi_set_scatter(self._h, int(ent["scatter"])))
            if "fft" in ent:
                self.set_fft_params(**ent["fft"])
            return float(ent["fft_cost"])
        best = C.c_float()
        _lib.check(lib.tfi_autotune(self._h, f.data_ptr(), int(d), _DTYPES[f.dtype],
                                    1 if backward else 0, C.byref(best),
                                    self._stream(self.device)))
        if fft_shapes:
            _lib.check(lib.tfi_autotune_fft(self._h, f.data_ptr(), int(d), _DTYPES[f.dtype],
                                            1 if backward else 0, self._stream(self.device)))
        if cache:
            table[key] = {"fft_cost": best.value, "scatter": self.stats()["scatter_pick"],
                          "fft": self.fft_params()}
            tmp = f"{cache}.{os.getpid()}.tmp"
            with open(tmp, "w") as fp:
                json.dump(table, fp, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return best.value

    def fft_params(self):
        """Shapes of the FFT kernels (``tfi_fft_params``) as a dict."""
        q = _lib.FftParams()
        _lib.check(_lib.load().tfi_get_fft_params(self._h, C.byref(q)))
        return {"lds_pairs": list(q.lds_pairs), "conv1d_min_lg": q.conv1d_min_lg,
                "conv1d_pairs": q.conv1d_pairs, "conv1d_group_mib": q.conv1d_group_mib,
                "col_lines": q.col_lines}

    def set_fft_params(self, **changes):
        """Change some of the FFT kernels' shapes (keys of ``fft_params``)."""
        cur = self.fft_params()
        unknown = set(changes) - set(cur)
        if unknown:
            raise KeyError(f"unknown FFT parameters {sorted(unknown)}")
        cur.update(changes)
        q = _lib.FftParams()
        for t in range(3):
            q.lds_pairs[t] = int(cur["lds_pairs"][t])
        q.conv1d_min_lg = int(cur["conv1d_min_lg"])
        q.conv1d_pairs = int(cur["conv1d_pairs"])
        q.conv1d_group_mib = int(cur["conv1d_group_mib"])
        q.col_lines = int(cur["col_lines"])
        _lib.check(_lib.load().tfi_set_fft_params(self._h, C.byref(q)))

    def calibrate(self, f, d):
        """Measure the channel-aware cost model on this plan at ``d``
        channels of ``f``'s dtype (profiled all-direct and all-FFT passes);
        returns {'vertex', 'direct', 'fft', 'call'} in seconds per unit, the
        ``cost_model`` of policy 'channel'."""
        self._check(f)
        costs = (C.c_float * 4)()
        _lib.check(_lib.load().tfi_calibrate(self._h, f.data_ptr(), int(d), _DTYPES[f.dtype],
                                             costs, self._stream(self.device)))
        return {"vertex": costs[0], "direct": costs[1], "fft": costs[2], "call": costs[3]}

    def set_fft_cost(self, cost):
        """Apply a direct-vs-FFT cost constant without timing."""
        _lib.check(_lib.load().tfi_set_fft_cost(self._h, float(cost)))

    def set_scatter(self, method):
        """Strategy of the cell sums: 'pieces', 'levels' or 'auto' (by
        width; ``autotune`` times both and keeps the faster)."""
        m = {"auto": -1, "pieces": 0, "levels": 1}[method]
        _lib.check(_lib.load().tfi_set_scatter(self._h, m))

    def profile(self, enable=True):
        """Record per-stage HIP events and algorithmic bytes from now on."""
        _lib.check(_lib.load().tfi_profile(self._h, 1 if enable else 0))

    def profile_report(self):
        """Per-stage {launches, ms, bytes} since the last report (waits for
        the recorded events)."""
        lib = _lib.load()
        buf = C.create_string_buffer(1 << 16)
        n = _lib.check(lib.tfi_profile_report(self._h, buf, len(buf)))
        if n >= len(buf):
            raise RuntimeError("profile report truncated")
        return json.loads(buf.value.decode())

    # ---------------------------------------------------------- compute --
    def _check(self, f, *mats):
        if self.device is None:
            raise _lib.TFIError(-8, "host-only plan: build with a device to integrate")
        if f.dtype not in _DTYPES:
            raise TypeError("f must be float32 or float64")
        if f.device != self.device or f.dim() != 1 or not f.is_contiguous():
            raise ValueError(f"f must be a contiguous 1-D tensor on {self.device}")
        if f.numel() < self.kernel_length:
            raise ValueError(f"f needs at least kernel_length={self.kernel_length} entries, "
                             f"got {f.numel()}")
        for m in mats:
            if m.dtype != f.dtype:
                raise TypeError("field and kernel must share one dtype")
            if m.device != self.device or not m.is_contiguous():
                raise ValueError(f"fields must be contiguous tensors on {self.device}")
            if m.shape[0] != self.num_vertices or m.dim() not in (1, 2):
                raise ValueError(f"fields must be [N] or [N, d] with N={self.num_vertices}")

    @staticmethod
    def _stream(dev):
        return torch.cuda.current_stream(dev).cuda_stream

    @staticmethod
    def _out_like(F, out):
        """``out`` checked to be a tensor F's shape, dtype and device (and
        distinct from F), or a new one."""
        if out is None:
            return torch.empty_like(F)
        if (out.shape != F.shape or out.dtype != F.dtype or out.device != F.device
                or not out.is_contiguous()):
            raise ValueError("out must be a contiguous tensor like F")
        if out.data_ptr() == F.data_ptr():
            raise ValueError("out must not alias F")
        return out

    def integrate(self, f, F, out=None, keep_cells=False):
        """out = f(D) F for F of shape [N] or [N, d]. ``out``: optional
        preallocated result (a loop that reuses it replays one captured
        graph; a new tensor per call may need a graph per address). With
        ``keep_cells`` returns ``(out, cells)``: the cell sums of F, which
        ``backward(..., cells=cells)`` reads for df instead of forming them
        again."""
        self._check(f, F)
        d = 1 if F.dim() == 1 else F.shape[1]
        out = self._out_like(F, out)
        if d == 0:
            return (out, None) if keep_cells else out
        lib = _lib.load()
        if not keep_cells:
            _lib.check(lib.tfi_integrate(self._h, f.data_ptr(), F.data_ptr(), d,
                                         _DTYPES[f.dtype], out.data_ptr(),
                                         self._stream(self.device)))
            return out
        cells = self._new_cells(F, d)
        _lib.check(lib.tfi_integrate_cells(self._h, f.data_ptr(), F.data_ptr(), d,
                                           _DTYPES[f.dtype], out.data_ptr(), cells.data_ptr(),
                                           self._stream(self.device)))
        return out, cells

    def integrate_noalloc(self, f, F, out):
        """``integrate`` into the preallocated ``out`` without any device
        allocation by the library: its scratch comes from one fixed array per
        GPU (``_lib.NOALLOC_SCRATCH_BYTES``), shared by every such call on
        that GPU, and the kernels are launched directly (no graph). Raises
        ``TFIError`` (TFI_ERR_BUDGET) when the plan needs more scratch at
        this width than the array holds. Calls that overlap on one GPU race
        on the shared array."""
        self._check(f, F)
        d = 1 if F.dim() == 1 else F.shape[1]
        out = self._out_like(F, out)
        if d == 0:
            return out
        _lib.check(_lib.load().tfi_integrate_noalloc(self._h, f.data_ptr(), F.data_ptr(), d,
                                                     _DTYPES[f.dtype], out.data_ptr(),
                                                     self._stream(self.device)))
        return out

    def _new_cells(self, F, d):
        rows = _lib.load().tfi_cell_rows(self._h)
        _lib.check(rows if rows < 0 else 0)
        return torch.empty((rows, d), dtype=F.dtype, device=F.device)

    def _check_cells(self, cells, F, d):
        if (cells.dtype != F.dtype or cells.device != F.device or not cells.is_contiguous()
                or tuple(cells.shape) != (_lib.load().tfi_cell_rows(self._h), d)):
            raise ValueError("cells must be the tensor the forward kept for this F")

    def integrate_many(self, fs, F, out=None):
        """[f_i(D) F for f_i in fs] in one call (at most 4 kernel tables of
        one dtype): the cell sums of F are formed once for all kernels.
        ``out``: optional list of preallocated results, one per table."""
        fs = list(fs)
        if not 1 <= len(fs) <= 4:
            raise ValueError("integrate_many takes 1 to 4 kernel tables")
        if any(f.dtype != fs[0].dtype for f in fs):
            raise TypeError("kernel tables must share one dtype")
        for f in fs:
            self._check(f, F)
        d = 1 if F.dim() == 1 else F.shape[1]
        if out is not None and len(out) != len(fs):
            raise ValueError("out needs one tensor per kernel table")
        outs = [self._out_like(F, None if out is None else out[i]) for i in range(len(fs))]
        if len({o.data_ptr() for o in outs}) != len(outs):
            raise ValueError("the outputs must be distinct tensors")
        if d == 0:
            return outs
        lib = _lib.load()
        vp = C.c_void_p
        fp = (vp * len(fs))(*[f.data_ptr() for f in fs])
        op = (vp * len(fs))(*[o.data_ptr() for o in outs])
        _lib.check(lib.tfi_integrate_multi(self._h, len(fs), fp, F.data_ptr(), d,
                                           _DTYPES[fs[0].dtype], op,
                                           self._stream(self.device)))
        return outs

    def backward(self, f, F, gout, need_dF=True, need_df=True, cells=None):
        """Adjoint of ``integrate`` for L = sum(gout * out): returns
        ``(dF, df)``; df is float64 of length ``kernel_length``. ``cells``:
        the cell sums of F from ``integrate(..., keep_cells=True)``."""
        self._check(f, F, gout)
        if F.shape != gout.shape:
            raise ValueError("F and gout must have the same shape")
        d = 1 if F.dim() == 1 else F.shape[1]
        dF = torch.empty_like(F) if need_dF else None
        df = (torch.zeros(self.kernel_length, dtype=torch.float64, device=self.device)
              if need_df else None)
        lib = _lib.load()
        tail = (d, _DTYPES[f.dtype], dF.data_ptr() if dF is not None else None,
                df.data_ptr() if df is not None else None, self._stream(self.device))
        if cells is None:
            _lib.check(lib.tfi_backward(self._h, f.data_ptr(), F.data_ptr(), gout.data_ptr(),
                                        *tail))
        else:
            self._check_cells(cells, F, d)
            _lib.check(lib.tfi_backward_cells(self._h, f.data_ptr(), F.data_ptr(),
                                              cells.data_ptr(), gout.data_ptr(), *tail))
        return dF, df

    def _check_expsum(self, c, lam, F):
        self._check(F.new_zeros(self.kernel_length), F)
        for t in (c, lam):
            if t.dtype != F.dtype or t.device != self.device or t.dim() != 1 \
                    or not t.is_contiguous():
                raise ValueError("c and lam must be contiguous 1-D tensors of the field's "
                                 "dtype on the integrator's device")
        if c.numel() != lam.numel() or not 1 <= c.numel() <= EXPSUM_MAX_TERMS:
            raise ValueError(f"c and lam need the same length, 1..{EXPSUM_MAX_TERMS}")

    def integrate_expsum(self, c, lam, F, keep_cells=False):
        """out = f(D) F for f(k) = sum_l c[l] lam[l]**k (lam > 0), by backbone
        sweeps per table job instead of direct sums or FFT. With
        ``keep_cells`` returns ``(out, cells)``: the cell sums of F, which
        ``backward_expsum(..., cells=cells)`` then reads instead of forming
        them again."""
        self._check_expsum(c, lam, F)
        d = 1 if F.dim() == 1 else F.shape[1]
        out = torch.empty_like(F)
        if d == 0:
            return (out, None) if keep_cells else out
        lib = _lib.load()
        if not keep_cells:
            _lib.check(lib.tfi_integrate_expsum(
                self._h, int(c.numel()), c.data_ptr(), lam.data_ptr(), F.data_ptr(), d,
                _DTYPES[F.dtype], out.data_ptr(), self._stream(self.device)))
            return out
        cells = self._new_cells(F, d)
        _lib.check(lib.tfi_integrate_expsum_cells(
            self._h, int(c.numel()), c.data_ptr(), lam.data_ptr(), F.data_ptr(), d,
            _DTYPES[F.dtype], out.data_ptr(), cells.data_ptr(), self._stream(self.device)))
        return out, cells

    def backward_expsum(self, c, lam, F, gout, need_dF=True, need_moments=True, cells=None):
        """Adjoint of ``integrate_expsum`` for L = sum(gout * out): returns
        ``(dF, s0, s1)`` with s0[l] = sum lam[l]**dist <gout_v, F_w> and
        s1[l] = sum dist lam[l]**dist <gout_v, F_w> (float64), so that
        dL/dc = s0 and dL/dlam = c s1 / lam. ``cells``: the cell sums of F
        from ``integrate_expsum(..., keep_cells=True)`` with the same F."""
        self._check_expsum(c, lam, F)
        if F.shape != gout.shape or gout.dtype != F.dtype or not gout.is_contiguous():
            raise ValueError("gout must be a contiguous tensor like F")
        d = 1 if F.dim() == 1 else F.shape[1]
        n = int(c.numel())
        dF = torch.empty_like(F) if need_dF else None
        s0 = torch.empty(n, dtype=torch.float64, device=self.device) if need_moments else None
        s1 = torch.empty(n, dtype=torch.float64, device=self.device) if need_moments else None
        lib = _lib.load()
        ptrs = (_DTYPES[F.dtype], dF.data_ptr() if dF is not None else None,
                s0.data_ptr() if s0 is not None else None,
                s1.data_ptr() if s1 is not None else None, self._stream(self.device))
        if cells is None:
            _lib.check(lib.tfi_backward_expsum(
                self._h, n, c.data_ptr(), lam.data_ptr(), F.data_ptr(), gout.data_ptr(), d,
                *ptrs))
        else:
            self._check_cells(cells, F, d)
            _lib.check(lib.tfi_backward_expsum_cells(
                self._h, n, c.data_ptr(), lam.data_ptr(), F.data_ptr(), cells.data_ptr(),
                gout.data_ptr(), d, *ptrs))
        return dF, s0, s1

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            _lib.load().tfi_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TreeIntegrate(torch.autograd.Function):
    """``out = TreeIntegrate.apply(integrator, F, f)`` with gradients for F
    and the kernel table f."""

    @staticmethod
    def forward(ctx, integrator, F, f):
        ctx.integrator = integrator
        # df needs the cell sums of F: keep the forward's
        if ctx.needs_input_grad[2]:
            out, cells = integrator.integrate(f, F, keep_cells=True)
        else:
            out, cells = integrator.integrate(f, F), None
        ctx.save_for_backward(F, f, cells)
        return out

    @staticmethod
    def backward(ctx, gout):
        F, f, cells = ctx.saved_tensors
        need_dF, need_df = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        if not (need_dF or need_df):
            return None, None, None
        dF, df = ctx.integrator.backward(f, F, gout.contiguous(), need_dF, need_df,
                                         cells=cells if need_df else None)
        if df is not None:
            full = torch.zeros_like(f)
            k = min(f.numel(), df.numel())
            full[:k] = df[:k].to(f.dtype)
            df = full
        return None, dF, df


class ExpSumIntegrate(torch.autograd.Function):
    """``out = ExpSumIntegrate.apply(integrator, F, a, b)`` for the kernel
    f(d) = sum_l a[l] exp(-b[l] d), evaluated by backbone sweeps, with
    gradients for F, a and b from the exact moments of the adjoint."""

    @staticmethod
    def forward(ctx, integrator, F, a, b):
        lam = torch.exp(-b)
        ctx.integrator = integrator
        # the moments need the cell sums of F: keep the forward's
        keep = ctx.needs_input_grad[2] or ctx.needs_input_grad[3]
        if keep:
            out, cells = integrator.integrate_expsum(a.contiguous(), lam.contiguous(), F,
                                                     keep_cells=True)
        else:
            out, cells = integrator.integrate_expsum(a.contiguous(), lam.contiguous(), F), None
        ctx.save_for_backward(F, a, lam, cells)
        return out

    @staticmethod
    def backward(ctx, gout):
        F, a, lam, cells = ctx.saved_tensors
        need_dF = ctx.needs_input_grad[1]
        need_ab = ctx.needs_input_grad[2] or ctx.needs_input_grad[3]
        if not (need_dF or need_ab):
            return None, None, None, None
        dF, s0, s1 = ctx.integrator.backward_expsum(a.contiguous(), lam.contiguous(), F,
                                                    gout.contiguous(), need_dF, need_ab,
                                                    cells=cells)
        da = s0.to(a.dtype) if need_ab else None
        db = (-a * s1.to(a.dtype)) if need_ab else None
        return None, dF, da, db


def expsum_table(a, b, length):
    """Kernel table ``f[k] = sum_j a_j exp(-b_j k)``, k < length, built with
    torch ops so that autograd maps df to (da, db)."""
    k = torch.arange(length, dtype=a.dtype, device=a.device)
    return (a[None, :] * torch.exp(-k[:, None] * b[None, :])).sum(1)
