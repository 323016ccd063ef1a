"""MI355X (gfx950) EGFEM Newton hot path: HIP kernels behind a C ABI
(include/egfem.h) with a thin ctypes binding.  See binding.py."""
from .binding import (  # noqa: F401
    Batch, BurgersOptions, BurgersStats, EgfemError, FORM_CONV, FORM_MASS, FORM_STIFF, Info, W_IQ, W_P0, W_P1, W_P2, NewtonOptions, NewtonStats, PicardOptions, PicardStats,
    Problem, Tensor,
    load_library, newton_batched, batch_autotune, stream_read, version, EXPORTS, LIB_PATH,
)
from .autograd import EGFEMSolve, solve  # noqa: F401
