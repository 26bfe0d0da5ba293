"""MI355X-native (gfx950, FP64 HIP) evaluation of thermochemical source terms
and analytical sparse/dense chemical-kinetic Jacobians for very many
independent states, after Curtis, Niemeyer & Sung, "Using SIMD and SIMT
vectorization to evaluate sparse chemical kinetic Jacobian matrices and
thermochemical source terms" (pyJac v2, arXiv:1809.01029).

Submodules:
  synth    seeded synthetic mechanisms and state batches (pure numpy)
  api      the Python binding of the C-ABI library (loads the HIP library)
"""

__all__ = ["synth", "api"]


def __getattr__(name):
    if name in ("synth", "api"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
