"""Implicit-filter coarse-graining on MI355X (gfx950).

Python binding of the C-ABI library ``libifl.so`` (see ``include/ifl.h``):
mesh-only ``prepare``, per-scale ``filter`` (Jacobi-preconditioned CG on the
system of Eq. 1 discretised as in Sect. 2.1), ``spectrum``, save / load, and
a continuous-batching server. All arithmetic of the filter runs in the HIP
kernels of ``csrc/``; this package only marshals arguments.
"""
from ._ffi import (  # noqa: F401
    EXPORTED,
    Handle,
    IflError,
    Server,
    IFL_OK,
    IFL_EINVAL,
    IFL_EDEGENERATE,
    IFL_ENOMEM,
    IFL_ENOTCONV,
    IFL_EDEVICE,
    IFL_EUNSUPPORTED,
    IFL_EIO,
    IFL_ECANCELED,
    IFL_GEOM_PLANAR,
    IFL_GEOM_PERIODIC,
    IFL_GEOM_SPHERE,
    IFL_VERTEX_SCALAR,
    IFL_CELL_VECTOR,
    IFL_VORONOI_SCALAR,
    IFL_CIRCUMCENTER_SCALAR,
    IFL_VERTEX_VECTOR,
    IFL_FP64,
    IFL_MIXED,
    IFL_SOLVER_KN,
    IFL_SOLVER_SHIFTED,
    LIB_PATH,
    default_options,
    ifl_apply,
    ifl_project_cells,
    ifl_destroy,
    ifl_filter,
    ifl_last_error,
    ifl_load,
    ifl_prepare,
    ifl_save,
    ifl_spectrum,
    lib,
    prepare_mesh,
    stream_probe,
)
