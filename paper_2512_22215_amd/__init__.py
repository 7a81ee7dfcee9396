"""MI355X (gfx950) LDU pressure solve: Amul/Tmul, diagonal PCG, GAMG, mixed
precision and adjoint, behind the C ABI in include/ldu.h."""
from .ldu import (  # noqa: F401
    LDU_FP64, LDU_MIXED, LIB_PATH, LduError, LduMatrix, SolveStats, gamg_opts, lib,
    pcg_opts,
)
from .autograd import LduSolve, ldu_solve  # noqa: F401
