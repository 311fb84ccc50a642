"""acch: energy-stable Allen–Cahn/Cahn–Hilliard time stepping on MI355X (gfx950).

The per-time-step Newton–Krylov–Schwarz solve of scheme (2.20) runs in the HIP
library libacch.so (include/acch.h); this package only builds and binds it.
"""
from .binding import (AcchError, BatchSolver, Params, Solver, StepInfo, load_library, make_params,  # noqa: F401
                      set_option, LIB_PATH, EXPORTED)

__all__ = ["AcchError", "BatchSolver", "Params", "Solver", "StepInfo", "load_library", "make_params", "set_option",
           "LIB_PATH", "EXPORTED"]
