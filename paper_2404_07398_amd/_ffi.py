"""ctypes binding of ``libifl.so`` (the C ABI in ``include/ifl.h``).

Argument marshalling only: every step of the filter runs in the HIP
library. Field arguments may be NumPy arrays (host memory) or torch
tensors on the GPU (device memory); PyTorch is used for nothing else.
The library must have been built (``python -m paper_2404_07398_amd.build``);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libifl.so")

IFL_OK = 0
IFL_EINVAL = -1
IFL_EDEGENERATE = -2
IFL_ENOMEM = -3
IFL_ENOTCONV = -4
IFL_EDEVICE = -5
IFL_EUNSUPPORTED = -6
IFL_EIO = -7
IFL_ECANCELED = -8

STATUS_NAMES = {
    0: "IFL_OK", -1: "IFL_EINVAL", -2: "IFL_EDEGENERATE", -3: "IFL_ENOMEM", -4: "IFL_ENOTCONV",
    -5: "IFL_EDEVICE", -6: "IFL_EUNSUPPORTED", -7: "IFL_EIO", -8: "IFL_ECANCELED",
}

IFL_GEOM_PLANAR = 0
IFL_GEOM_PERIODIC = 1
IFL_GEOM_SPHERE = 2

IFL_VERTEX_SCALAR = 0
IFL_CELL_VECTOR = 1
IFL_VORONOI_SCALAR = 2
IFL_CIRCUMCENTER_SCALAR = 3
IFL_VERTEX_VECTOR = 4

IFL_FP64 = 0
IFL_MIXED = 1
IFL_SOLVER_KN = 0
IFL_SOLVER_SHIFTED = 1


class ifl_mesh(C.Structure):
    _fields_ = [
        ("n_vertices", C.c_int64),
        ("n_triangles", C.c_int64),
        ("coords", C.POINTER(C.c_double)),
        ("triangles", C.POINTER(C.c_int32)),
        ("geometry", C.c_int32),
        ("reserved0", C.c_int32),
        ("period", C.c_double * 2),
        ("wet", C.POINTER(C.c_uint8)),
    ]


class ifl_options(C.Structure):
    _fields_ = [
        ("gamma", C.c_double),
        ("rtol", C.c_double),
        ("max_iter", C.c_int32),
        ("precision", C.c_int32),
        ("cell_A", C.c_double),
        ("device", C.c_int32),
        ("batch", C.c_int32),
        ("stream", C.c_void_p),
        ("reorder", C.c_int32),
        ("profile", C.c_int32),
        ("graphs", C.c_int32),
        ("solver", C.c_int32),
    ]


class ifl_solve_stats(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32),
        ("refinements", C.c_int32),
        ("status", C.c_int32),
        ("reserved", C.c_int32),
        ("rel_residual", C.c_double),
        ("seconds", C.c_double),
        ("energy", C.c_double),
    ]


class ifl_tune(C.Structure):
    _fields_ = [
        ("batch", C.c_int32),
        ("blocks_gather", C.c_int32),
        ("blocks_update", C.c_int32),
        ("candidates", C.c_int32),
        ("us_per_column_iteration", C.c_double),
    ]


class ifl_server_info(C.Structure):
    _fields_ = [
        ("budget", C.c_size_t),
        ("tiles", C.c_size_t),
        ("used", C.c_size_t),
        ("peak_used", C.c_size_t),
        ("submitted", C.c_int64),
        ("admitted", C.c_int64),
        ("completed", C.c_int64),
        ("in_flight", C.c_int64),
        ("peak_in_flight", C.c_int64),
        ("queued", C.c_int64),
    ]


class IflError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

_PROTOS = {
    "ifl_default_options": (None, [C.POINTER(ifl_options)]),
    "ifl_prepare": (C.c_int32, [C.POINTER(ifl_mesh), C.c_int32, C.c_int32, C.POINTER(ifl_options), C.POINTER(C.c_void_p)]),
    "ifl_destroy": (None, [C.c_void_p]),
    "ifl_num_dofs": (C.c_int64, [C.c_void_p]),
    "ifl_field_length": (C.c_int64, [C.c_void_p]),
    "ifl_num_cells": (C.c_int64, [C.c_void_p]),
    "ifl_set_options": (C.c_int32, [C.c_void_p, C.POINTER(ifl_options)]),
    "ifl_get_options": (C.c_int32, [C.c_void_p, C.POINTER(ifl_options)]),
    "ifl_filter": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_void_p,
                               C.POINTER(ifl_solve_stats)]),
    "ifl_filter_noalloc": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                       C.c_void_p, C.POINTER(ifl_solve_stats)]),
    "ifl_spectrum": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ifl_apply": (C.c_int32, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "ifl_project_cells": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ifl_operator_nnz": (C.c_int64, [C.c_void_p]),
    "ifl_export_operator": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "ifl_save": (C.c_int32, [C.c_void_p, C.c_char_p]),
    "ifl_load": (C.c_int32, [C.c_char_p, C.POINTER(ifl_options), C.POINTER(C.c_void_p)]),
    "ifl_last_error": (C.c_char_p, []),
    "ifl_profile_read": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.c_int32]),
    "ifl_profile_kernel": (C.c_int32, [C.c_void_p, C.c_char_p, C.c_int32]),
    "ifl_server_cancel": (C.c_int32, [C.c_void_p]),
    "ifl_first_order_nnz": (C.c_int64, [C.c_void_p]),
    "ifl_export_first_order": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_double)]),
    "ifl_stream_probe": (C.c_int32, [C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
    "ifl_autotune": (C.c_int32, [C.c_void_p, C.POINTER(ifl_tune)]),
    "ifl_server_create": (C.c_int32, [C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)]),
    "ifl_server_add": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "ifl_submit": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_void_p,
                               C.POINTER(C.c_void_p)]),
    "ifl_wait": (C.c_int32, [C.c_void_p, C.POINTER(ifl_solve_stats)]),
    "ifl_poll": (C.c_int32, [C.c_void_p]),
    "ifl_ticket_latency": (C.c_double, [C.c_void_p]),
    "ifl_server_destroy": (None, [C.c_void_p]),
    "ifl_server_query": (C.c_int32, [C.c_void_p, C.POINTER(ifl_server_info)]),
}

EXPORTED = tuple(_PROTOS)


def lib():
    """Load ``libifl.so`` (once). Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_2404_07398_amd.build)")
        # PyTorch ships its own HIP runtime under the same soname; loading it
        # first makes the library bind to that one runtime instead of a second
        # copy from /opt/rocm (two runtimes in one process break GPU init).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != IFL_OK:
        raise IflError(st, lib().ifl_last_error().decode(errors="replace"))


def default_options(**kw) -> ifl_options:
    o = ifl_options()
    lib().ifl_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _dptr(a):
    return C.cast(a.ctypes.data, C.POINTER(C.c_double))


class _Field:
    """A field argument: host NumPy float64 or device torch float64 tensor."""

    def __init__(self, a, writable: bool = False):
        self.obj = a
        self.device = False
        if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
            import torch

            if a.dtype != torch.float64:
                raise TypeError("fields must be float64")
            if not a.is_contiguous():
                raise ValueError("fields must be contiguous")
            self.device = bool(a.is_cuda)
            self.ptr = C.c_void_p(a.data_ptr())
            if self.device:
                torch.cuda.current_stream(a.device).synchronize()
        else:
            arr = np.asarray(a)
            if arr.dtype != np.float64 or not arr.flags.c_contiguous:
                if writable:
                    raise TypeError("output arrays must be C-contiguous float64")
                arr = np.ascontiguousarray(arr, dtype=np.float64)
            self.obj = arr
            self.ptr = C.c_void_p(arr.ctypes.data)


def make_mesh(coords, tris, geometry, period=None, wet=None):
    """Build the ``ifl_mesh`` struct; returns (struct, keepalive)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    m = ifl_mesh()
    m.n_vertices = coords.shape[0]
    m.n_triangles = tris.shape[0]
    m.coords = _dptr(coords)
    m.triangles = C.cast(tris.ctypes.data, C.POINTER(C.c_int32))
    m.geometry = int(geometry)
    if period is not None:
        m.period[0], m.period[1] = float(period[0]), float(period[1])
    keep = [coords, tris]
    if wet is not None:
        wet = np.ascontiguousarray(wet, dtype=np.uint8)
        m.wet = C.cast(wet.ctypes.data, C.POINTER(C.c_uint8))
        keep.append(wet)
    return m, keep


class Handle:
    """A prepared mesh / placement / order (``ifl_handle``)."""

    def __init__(self, ptr: C.c_void_p):
        self._h = ptr

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h:
            lib().ifl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_dofs(self) -> int:
        return int(lib().ifl_num_dofs(self._h))

    @property
    def field_length(self) -> int:
        return int(lib().ifl_field_length(self._h))

    def options(self) -> ifl_options:
        o = ifl_options()
        _check(lib().ifl_get_options(self._h, C.byref(o)))
        return o

    def set_options(self, **kw):
        """Change some solver options; the others keep their current values."""
        o = self.options()
        for k, v in kw.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        _check(lib().ifl_set_options(self._h, C.byref(o)))

    def filter(self, fields, ks, out=None, raise_on_notconv: bool = True):
        """Filter ``fields`` ((F, L) or (L,)) at wavenumbers ``ks``.

        Returns ``(out, stats)``; ``out`` has shape (F, S, L) (host NumPy
        unless a device tensor is given as ``out``)."""
        ks = np.ascontiguousarray(np.atleast_1d(ks), dtype=np.float64)
        L = self.field_length
        shape_in = fields.shape
        nf = 1 if len(shape_in) == 1 else shape_in[0]
        if shape_in[-1] != L:
            raise ValueError(f"field length {shape_in[-1]} != {L}")
        fin = _Field(fields)
        if out is None:
            out = np.zeros((nf, ks.size, L))
        fout = _Field(out, writable=True)
        stats = (ifl_solve_stats * max(1, nf * ks.size))()
        st = lib().ifl_filter(self._h, nf, fin.ptr, ks.size, _dptr(ks), fout.ptr, stats)
        if st != IFL_OK and (st != IFL_ENOTCONV or raise_on_notconv):
            _check(st)
        return out, [stats[i] for i in range(nf * ks.size)]

    def filter_noalloc(self, fields, ks, out, raise_on_notconv: bool = True):
        """``ifl_filter_noalloc``: ``fields`` and ``out`` are device tensors
        ((F, L) and (F, S, L), float64, contiguous). Returns the stats."""
        ks = np.ascontiguousarray(np.atleast_1d(ks), dtype=np.float64)
        L = self.field_length
        nf = 1 if len(fields.shape) == 1 else fields.shape[0]
        if fields.shape[-1] != L:
            raise ValueError(f"field length {fields.shape[-1]} != {L}")
        if int(np.prod(out.shape)) != nf * ks.size * L:
            raise ValueError("out must hold n_fields x n_scales x L doubles")
        fin = _Field(fields)
        fout = _Field(out, writable=True)
        stats = (ifl_solve_stats * max(1, nf * ks.size))()
        st = lib().ifl_filter_noalloc(self._h, nf, fin.ptr, ks.size, _dptr(ks), fout.ptr, stats)
        if st != IFL_OK and (st != IFL_ENOTCONV or raise_on_notconv):
            _check(st)
        return [stats[i] for i in range(nf * ks.size)]

    def spectrum(self, field, ks):
        ks = np.ascontiguousarray(ks, dtype=np.float64)
        fin = _Field(field)
        e = np.zeros(ks.size)
        dens = np.zeros(max(1, ks.size - 1))
        kmid = np.zeros(max(1, ks.size - 1))
        _check(lib().ifl_spectrum(self._h, fin.ptr, ks.size, _dptr(ks), _dptr(e), _dptr(dens), _dptr(kmid)))
        return e, dens[: ks.size - 1], kmid[: ks.size - 1]

    def apply(self, k: float, x, y=None):
        fx = _Field(x)
        if y is None:
            y = np.zeros(self.field_length)
        fy = _Field(y, writable=True)
        _check(lib().ifl_apply(self._h, float(k), fx.ptr, fy.ptr))
        return y

    def project_cells(self, cells, out=None):
        """Cell velocities (F, 2) -> the vertex field M^-1 R_vc u_c (2V,)
        that ifl_filter takes on an IFL_VERTEX_VECTOR handle."""
        nc = int(lib().ifl_num_cells(self._h))
        if nc == 0:
            raise ValueError("project_cells needs an IFL_VERTEX_VECTOR handle")
        if int(np.prod(cells.shape)) != 2 * nc:
            raise ValueError(f"cell field has {int(np.prod(cells.shape))} entries, expected {2 * nc}")
        fc = _Field(cells.reshape(-1))
        if out is None:
            out = np.zeros(self.field_length)
        if int(np.prod(out.shape)) != self.field_length:
            raise ValueError(f"out has {int(np.prod(out.shape))} entries, expected {self.field_length}")
        fo = _Field(out, writable=True)
        _check(lib().ifl_project_cells(self._h, fc.ptr, fo.ptr))
        return out

    def export_operator(self):
        n = self.num_dofs
        nnz = int(lib().ifl_operator_nnz(self._h))
        rp = np.zeros(n + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz)
        mass = np.zeros(n)
        ent = np.zeros(n, np.int64)
        _check(lib().ifl_export_operator(
            self._h, C.cast(rp.ctypes.data, C.POINTER(C.c_int64)), C.cast(col.ctypes.data, C.POINTER(C.c_int32)),
            _dptr(val), _dptr(mass), C.cast(ent.ctypes.data, C.POINTER(C.c_int64))))
        return rp, col, val, mass, ent

    def export_first_order(self):
        """The first-order operator K (rows in the library's order)."""
        n = self.num_dofs
        nnz = int(lib().ifl_first_order_nnz(self._h))
        rp = np.zeros(n + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz)
        _check(lib().ifl_export_first_order(
            self._h, C.cast(rp.ctypes.data, C.POINTER(C.c_int64)), C.cast(col.ctypes.data, C.POINTER(C.c_int32)),
            _dptr(val)))
        return rp, col, val

    def save(self, path: str):
        _check(lib().ifl_save(self._h, path.encode()))

    def profile_read(self, reset: bool = False):
        n = C.c_int64()
        ms = C.c_double()
        b = C.c_double()
        _check(lib().ifl_profile_read(self._h, C.byref(n), C.byref(ms), C.byref(b), int(reset)))
        return int(n.value), float(ms.value), float(b.value)

    def profile_kernel(self) -> str:
        """Name of the SpMV kernel of the last timed launch (``ifl_profile_kernel``)."""
        buf = C.create_string_buffer(128)
        _check(lib().ifl_profile_kernel(self._h, buf, len(buf)))
        return buf.value.decode()

    def autotune(self) -> dict:
        """Time tile and grid sizes of the batched engine on this handle
        (``ifl_autotune``); returns the fastest configuration."""
        t = ifl_tune()
        _check(lib().ifl_autotune(self._h, C.byref(t)))
        return {"batch": t.batch, "blocks_gather": t.blocks_gather, "blocks_update": t.blocks_update,
                "candidates": t.candidates, "us_per_column_iteration": t.us_per_column_iteration}


def ifl_prepare(coords, tris, geometry, placement=IFL_VERTEX_SCALAR, n=1, period=None, wet=None, **opts) -> Handle:
    m, keep = make_mesh(coords, tris, geometry, period, wet)
    o = default_options(**opts)
    h = C.c_void_p()
    _check(lib().ifl_prepare(C.byref(m), int(placement), int(n), C.byref(o), C.byref(h)))
    del keep
    return Handle(h)


def ifl_load(path: str, **opts) -> Handle:
    o = default_options(**opts)
    h = C.c_void_p()
    _check(lib().ifl_load(path.encode(), C.byref(o), C.byref(h)))
    return Handle(h)


def prepare_mesh(mesh, placement=IFL_VERTEX_SCALAR, n=1, **opts) -> Handle:
    """``ifl_prepare`` from a ``workloads.Mesh``-like object (coords, tris,
    geometry, period, wet)."""
    return ifl_prepare(mesh.coords, mesh.tris, mesh.geometry, placement, n, mesh.period, mesh.wet, **opts)


def ifl_filter(h: Handle, fields, ks, out=None):
    return h.filter(fields, ks, out)


def ifl_spectrum(h: Handle, field, ks):
    return h.spectrum(field, ks)


def ifl_apply(h: Handle, k, x, y=None):
    return h.apply(k, x, y)


def ifl_project_cells(h: Handle, cells, out=None):
    return h.project_cells(cells, out)


def ifl_save(h: Handle, path: str):
    h.save(path)


def ifl_destroy(h: Handle):
    h.close()


def stream_probe(device: int = 0, mib: int = 4096, reps: int = 10):
    """Best and median GB/s of a plain device copy of ``mib`` MiB
    (``ifl_stream_probe``)."""
    best, med = C.c_double(), C.c_double()
    _check(lib().ifl_stream_probe(int(device), int(mib) << 20, int(reps), C.byref(best), C.byref(med)))
    return float(best.value), float(med.value)


def ifl_last_error() -> str:
    return lib().ifl_last_error().decode(errors="replace")


class Server:
    """Continuous-batching server (``ifl_server_*``)."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 32):
        self._s = C.c_void_p()
        _check(lib().ifl_server_create(int(hbm_budget_bytes), int(slots), C.byref(self._s)))
        self._keep = {}
        self._len = {}

    def add(self, h: Handle) -> int:
        mid = C.c_int32()
        _check(lib().ifl_server_add(self._s, h.ptr, C.byref(mid)))
        self._len[int(mid.value)] = h.field_length
        return int(mid.value)

    def submit(self, mesh_id: int, field: np.ndarray, ks, out: np.ndarray | None = None,
               spectrum_only: bool = False):
        """Queue a request; returns (ticket, out). With spectrum_only the
        filtered fields are not returned (out is None) and the energies are
        in the stats of wait(). field (and out) are kept alive here until
        wait(), as the server reads them until then."""
        field = np.ascontiguousarray(field, dtype=np.float64)
        ks = np.ascontiguousarray(ks, dtype=np.float64)
        L = self._len.get(int(mesh_id))
        if L is not None and field.size != L:
            raise ValueError(f"field has {field.size} entries, the mesh's fields have {L}")
        if spectrum_only:
            out = None
        elif out is None:
            out = np.empty((ks.size, field.size))
        elif out.size != ks.size * field.size or out.dtype != np.float64 or not out.flags.c_contiguous:
            raise ValueError("out must be a C-contiguous float64 array of n_scales x field length")
        t = C.c_void_p()
        _check(lib().ifl_submit(self._s, int(mesh_id), C.c_void_p(field.ctypes.data), ks.size, _dptr(ks),
                                C.c_void_p(out.ctypes.data if out is not None else None), C.byref(t)))
        self._keep[t.value] = (field, ks, out)
        return t, out

    def cancel(self):
        """Cancel the requests waiting for admission or for a slot
        (``ifl_server_cancel``); their wait() returns IFL_ECANCELED."""
        _check(lib().ifl_server_cancel(self._s))

    def query(self) -> dict:
        """Memory accounting and request counters (``ifl_server_query``)."""
        info = ifl_server_info()
        _check(lib().ifl_server_query(self._s, C.byref(info)))
        return {name: int(getattr(info, name)) for name, _ in ifl_server_info._fields_}

    def poll(self, ticket) -> bool:
        return bool(lib().ifl_poll(ticket))

    def latency(self, ticket) -> float:
        return float(lib().ifl_ticket_latency(ticket))

    def wait(self, ticket, n_scales: int):
        """Block until the request is done; returns (status, stats, out,
        latency in seconds from submit to completion, server clock)."""
        stats = (ifl_solve_stats * max(1, n_scales))()
        while not self.poll(ticket):  # the latency is final once the ticket is done
            time.sleep(0.0005)
        lat = float(lib().ifl_ticket_latency(ticket))
        st = lib().ifl_wait(ticket, stats)
        keep = self._keep.pop(ticket.value, None)
        return st, [stats[i] for i in range(n_scales)], (keep[2] if keep else None), lat

    def close(self):
        if self._s:
            lib().ifl_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

