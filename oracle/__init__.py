"""Plain FP64 CPU oracle of the DUGKS step (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it.
"""
from .oracle import Oracle, build, library_path  # noqa: F401
from .oracle3d import Oracle3D  # noqa: F401
from .oracle1d import Oracle1D  # noqa: F401
