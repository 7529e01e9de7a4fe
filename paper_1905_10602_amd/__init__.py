"""MI355X (gfx950) parallel inverse fast multipole method.

The compute path is the HIP library ``libifmm.so`` behind the C ABI declared
in ``include/ifmm.h``; ``paper_1905_10602_amd.ifmm`` is a thin ctypes
binding with the same names.  There is no CPU fallback: device calls fail
when the library or a gfx950 device is missing.
"""
from .ifmm import (BD, FMM, IFMM, RANK_FEATURES, IfmmError, factor_batch, fmbem_gmres, load_library,  # noqa: F401
                   library_path, rank_model_eval, rank_model_grad, rank_model_params, rank_model_train,
                   solve_batch)
