"""MI355X (gfx950) implementation of the Fokker-Planck central-moment
double-distribution lattice Boltzmann method for thermal convection
(Schupbach & Premnath, arXiv 2504.09041).

The method runs in hand-written HIP kernels behind the C ABI of
``include/fpclbm.h`` (``libfpclbm.so``); this package is its Python binding.
Importing it does not load the library; the first call that needs it does,
and raises ImportError if it has not been built.
"""

__all__ = ["Simulation", "params_from_workload", "default_params", "build_library"]


def __getattr__(name):
    if name in ("Simulation", "params_from_workload", "default_params", "set_faces", "state_bytes"):
        from . import sim

        return getattr(sim, name)
    if name == "build_library":
        from .build import build_library

        return build_library
    raise AttributeError(name)
