"""FP64 CPU oracle of the induced-dipole solve.  Test infrastructure only: imported by the
tests, the smoke check and the benchmark's CPU-baseline leg, never by the product library."""
from .ref import *  # noqa: F401,F403
from .ref import COULOMB, DEBYE  # noqa: F401
