"""sdbie: regularised boundary-integral Stokes-Darcy solver on one MI355X (gfx950).

The compute path is the HIP library libsdbie.so (C ABI in include/sdbie.h);
this package is its ctypes binding.  See `binding` for the call surface.
"""
from .binding import (  # noqa: F401
    ddm_adjoint, ddm_dn_spectrum, hessenberg_eigenvalues,
    DL_RAW, DL_SUB, FP64, MIXED, SL, SYM_ALL, SYM_DEFAULT, SYM_LAPLACE, SYM_LAPLACE_F64, SYM_STOKES, SYM_STOKES_F64,
    Plan, SdbieError, darcy_solve, ddm_solve, default_opts,
    laplace_layer_apply, lib, profile_enable, profile_read, stokes_layer_apply, stokes_layer_apply_noalloc,
    stokes_solve,
    workspace_bytes,
)
from .autograd import DragFn, drag  # noqa: F401,E402
