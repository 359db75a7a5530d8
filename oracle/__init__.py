"""CPU FP64 oracle for the coordinate-transformed Poisson multigrid
(arXiv 2602.01888).

TEST INFRASTRUCTURE ONLY.  It exists to check the GPU library: only the test
suite, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg
import it.  It shares no code with the GPU path (the package
``paper_2602_01888_amd``); the two meet only in the seeded input generators
of ``workloads``.

``oracle.core`` wraps the plain C implementation (``tomg_oracle.c``);
``oracle.direct`` assembles the discrete operator as a SciPy sparse matrix
and solves it directly, which gives the reference answer on grids small
enough for a direct solve.
"""

from .core import *  # noqa: F401,F403
