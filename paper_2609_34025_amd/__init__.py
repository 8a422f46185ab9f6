"""MI355X tree field integration (Structure-Adaptive Tree Field Integrators).

``out[v] = sum_w f(dist_T(v, w)) F[w]`` on weighted forests, evaluated by
the adaptive backbone/centroid decomposition with FFT or direct interaction
tables in HIP kernels for gfx950 (libtfi.so, C ABI in include/tfi.h).

Submodules: ``integrator`` (TreeIntegrator, TreeIntegrate, ExpSumIntegrate,
expsum_table), ``sinkhorn``,
``synth`` (seeded synthetic inputs), ``build`` (compiles libtfi.so).
Names are imported lazily so that ``synth`` works without torch or the
built library.
"""

__all__ = ["TreeIntegrator", "TreeIntegrate", "ExpSumIntegrate", "expsum_table"]


def __getattr__(name):
    if name in __all__:
        from . import integrator
        return getattr(integrator, name)
    raise AttributeError(name)
