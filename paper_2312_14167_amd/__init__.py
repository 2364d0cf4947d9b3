"""MI355X-native flux-reconstruction residual / RK4 hot path (HIP kernels for gfx950 behind the
C ABI declared in include/fr.h).  The binding loads libfrmi.so and fails loudly if it is absent."""
from ._lib import FrError, LIB_PATH, lib  # noqa: F401
from .solver import Solver  # noqa: F401
from .vardeg import VarDegreeSolver  # noqa: F401
