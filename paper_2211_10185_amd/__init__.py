"""MI355X (gfx950) imaginary-time Schroedinger solver (arXiv:2211.10185 hot path).

The compute path is the HIP library ``libqfdtd.so`` built from ``csrc/`` by
``paper_2211_10185_amd.build``; ``solver`` is its Python front end.  The
binding is imported lazily so that the build step can run before the library
exists; any use of the solver without the built library raises ImportError.
"""
__all__ = ["Solver", "batch_evolve", "batch_energies", "footprint", "build"]


def __getattr__(name):
    if name in ("Solver", "batch_evolve", "batch_energies", "footprint"):
        from . import solver
        return getattr(solver, name)
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
