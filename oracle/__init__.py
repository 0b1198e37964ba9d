"""FP64 CPU oracle of the Fokker-Planck central-moment thermal LBM.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written
reference that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the product package ``paper_2504_09041_amd`` never does, and the
two share no code.
"""

from . import collision, lattices, params, sim  # noqa: F401
