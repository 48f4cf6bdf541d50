"""Python binding of ``liblt.so`` (include/lt.h): the adaptation cycle of
the h-adaptive flux-reconstruction method on linear trees, on one MI355X.

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory and the current stream.  Importing works
without a GPU; using a tree needs the built library and a HIP device, and
raises ``LtError`` if either is missing (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "liblt.so")

LT_KEYS, LT_OLD_KEYS, LT_NBR, LT_HANG, LT_MAP_SRC, LT_MAP_KIND = range(6)
LT_MAX_VORTICES = 8
LT_MAX_DEGREE = 7

STATUS = {0: "LT_OK", 1: "LT_ERR_ARG", 2: "LT_ERR_OOM", 3: "LT_ERR_HIP", 4: "LT_ERR_DEPTH",
          5: "LT_ERR_INVALID_TREE", 6: "LT_ERR_UNBALANCED", 7: "LT_ERR_STATE",
          8: "LT_ERR_INTERNAL", 9: "LT_ERR_CAPACITY"}

# Every symbol include/lt.h declares.
EXPORTS = ["lt_set_allocator", "lt_build_uniform", "lt_build", "lt_build_points", "lt_build_batch",
           "lt_flag_batch", "lt_mesh_offsets", "lt_set_mesh_degree", "lt_transfer_mixed",
           "lt_flag", "lt_adapt", "lt_balance", "lt_connect", "lt_set_connect_grid", "lt_map",
           "lt_transfer", "lt_transfer_noalloc", "lt_size",
           "lt_view", "lt_export", "lt_mlp_create", "lt_mlp_params", "lt_mlp_features",
           "lt_mlp_grads", "lt_mlp_train_step", "lt_mlp_infer", "lt_flag_mlp", "lt_vortex_field",
           "lt_flag_modal", "lt_mlp_destroy", "lt_cycle_create", "lt_cycle_run",
           "lt_cycle_stats", "lt_cycle_destroy", "lt_autotune_transfer", "lt_set_tuning",
           "lt_get_tuning", "lt_fr_face_flux", "lt_fr_residual", "lt_fr_rk3", "lt_last_error",
           "lt_destroy"]
MLP_NPARAM = 128 * 320 + 128 + 64 * 128 + 64 + 3 * 64 + 3


class LtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Geom(C.Structure):
    _fields_ = [("dim", C.c_int), ("d_min", C.c_int), ("d_max", C.c_int),
                ("periodic_mask", C.c_uint), ("balance", C.c_int)]


class FlagParams(C.Structure):
    _fields_ = [("nvort", C.c_int), ("centre", C.POINTER(C.c_double)),
                ("r_in", C.c_double), ("r_out", C.c_double), ("dist_axes", C.c_int),
                ("periodic_dist", C.c_int), ("p", C.c_int),
                ("nodes01", C.POINTER(C.c_double)), ("lo", C.c_double * 3),
                ("len", C.c_double), ("raw", C.c_int)]


class Tune(C.Structure):
    _fields_ = [("copy_elems_per_lane", C.c_int), ("interp_grid", C.c_int), ("ms", C.c_float),
                ("ms_default", C.c_float)]


class CycleDesc(C.Structure):
    _fields_ = [("p", C.c_int), ("nvar", C.c_int), ("capacity", C.c_int64), ("ld", C.c_int64),
                ("balance_passes", C.c_int), ("u", C.c_void_p * 2), ("nmesh", C.c_int),
                ("flag_template", C.POINTER(FlagParams)), ("precision", C.c_int),
                ("mlp", C.c_void_p), ("conf_min", C.c_float)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_lib = None


def lib() -> C.CDLL:
    """Load liblt.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise LtError(3, f"{SO_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(SO_PATH)
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        L.lt_set_allocator.argtypes = [ALLOC_FN, FREE_FN, P]
        L.lt_build_uniform.argtypes = [C.POINTER(Geom), i32, P, C.POINTER(P)]
        L.lt_build.argtypes = [C.POINTER(Geom), P, i64, P, C.POINTER(P)]
        L.lt_build_points.argtypes = [C.POINTER(Geom), P, i64, P, C.c_double, P, C.POINTER(P)]
        L.lt_build_batch.argtypes = [C.POINTER(Geom), i32, P, P, P, P, C.POINTER(P)]
        L.lt_flag_batch.argtypes = [P, P, i32, P, P]
        L.lt_mesh_offsets.argtypes = [P, P, P]
        L.lt_set_mesh_degree.argtypes = [P, P, P]
        L.lt_transfer_mixed.argtypes = [P, i32, P, i64, P, i64, P]
        L.lt_flag.argtypes = [P, C.POINTER(FlagParams), P, P]
        L.lt_adapt.argtypes = [P, P, P]
        L.lt_balance.argtypes = [P, P]
        L.lt_connect.argtypes = [P, P]
        L.lt_set_connect_grid.argtypes = [P, i32]
        L.lt_map.argtypes = [P, P]
        L.lt_transfer.argtypes = [P, i32, i32, P, i64, P, i64, i32, P]
        L.lt_transfer_noalloc.argtypes = [P, i32, i32, P, i64, P, i64, P]
        L.lt_size.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.lt_view.argtypes = [P, i32, C.POINTER(P), C.POINTER(i64)]
        L.lt_export.argtypes = [P, i32, P, i64, P]
        L.lt_mlp_create.argtypes = [P, C.POINTER(P)]
        L.lt_mlp_params.argtypes = [P, P, P, P]
        L.lt_mlp_features.argtypes = [P, P, i64, i32, P, i64, P, P]
        L.lt_mlp_grads.argtypes = [P, P, P, i64, P]
        L.lt_mlp_train_step.argtypes = [P, P, P, i64, C.c_float, P]
        L.lt_mlp_infer.argtypes = [P, P, i64, P, P]
        L.lt_flag_mlp.argtypes = [P, P, C.POINTER(FlagParams), P, i64, C.c_float, P, P, P]
        L.lt_vortex_field.argtypes = [P, C.POINTER(FlagParams), P, P, i64, P]
        L.lt_flag_modal.argtypes = [P, i32, P, i64, C.c_double, C.c_double, P, P]
        L.lt_mlp_destroy.argtypes = [P]
        L.lt_mlp_destroy.restype = None
        L.lt_cycle_create.argtypes = [P, C.POINTER(CycleDesc), P, C.POINTER(P)]
        L.lt_cycle_run.argtypes = [P, C.POINTER(FlagParams), P, C.POINTER(i32)]
        L.lt_cycle_stats.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.lt_autotune_transfer.argtypes = [P, i32, i32, P, i64, P, i64, i32, P, C.POINTER(Tune)]
        L.lt_set_tuning.argtypes = [P, C.POINTER(Tune)]
        L.lt_get_tuning.argtypes = [P, C.POINTER(Tune)]
        L.lt_fr_face_flux.argtypes = [P, i32, P, i64, C.c_double, P, i64, P]
        L.lt_fr_residual.argtypes = [P, i32, P, i64, C.c_double, C.c_double, P, i64, P]
        L.lt_fr_rk3.argtypes = [P, i32, P, i64, P, C.c_double, C.c_double, C.c_double, i32, P]
        L.lt_cycle_destroy.argtypes = [P]
        L.lt_cycle_destroy.restype = None
        L.lt_last_error.restype = C.c_char_p
        L.lt_destroy.argtypes = [P]
        L.lt_destroy.restype = None
        for name in EXPORTS:
            if name not in ("lt_last_error", "lt_destroy", "lt_mlp_destroy", "lt_cycle_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise LtError(rc, lib().lt_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise LtError(3, "no HIP device is available")
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class TorchAllocator:
    """torch's caching allocator behind lt_set_allocator, so that trees,
    cycles and models draw device memory from the same pool as tensors.
    ``limit`` (bytes, optional) caps what the library holds at once: a
    request beyond it is refused and the call needing it fails with
    LT_ERR_OOM.  ``held`` is what the library holds now."""

    def __init__(self, limit=None):
        import torch
        self.limit = limit
        self.held = 0
        self._live = {}

        def _alloc(nbytes, stream, ctx):
            if self.limit is not None and self.held + nbytes > self.limit:
                return None
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), stream=0)
            except RuntimeError:
                return None
            self._live[ptr] = int(nbytes)
            self.held += int(nbytes)
            return ptr

        def _free(ptr, stream, ctx):
            self.held -= self._live.pop(ptr, 0)
            torch.cuda.caching_allocator_delete(ptr)

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)


# Every allocator ever registered stays referenced: the objects created while
# it was registered call it until they are destroyed.
_ALLOCATORS = []


def set_allocator(a=None):
    """Register ``a`` (a TorchAllocator) for the trees, cycles and models
    created from now on; None restores hipMalloc / hipFree."""
    _torch()
    if a is None:
        _check(lib().lt_set_allocator(ALLOC_FN(), FREE_FN(), None))
    else:
        _ALLOCATORS.append(a)
        _check(lib().lt_set_allocator(a._a, a._f, None))


def _dptr(t) -> C.c_void_p:
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _flag_params(dim, centres, r_in, r_out, nodes01, lo, length, dist_axes=None,
                 periodic_dist=False, raw=False):
    """lt_flag_params and the ctypes arrays it points to (keep them alive)."""
    cen = (C.c_double * (3 * len(centres)))()
    for v, c in enumerate(centres):
        for a in range(len(c)):
            cen[3 * v + a] = float(c[a])
    nodes = (C.c_double * len(nodes01))(*[float(x) for x in nodes01])
    lo3 = (C.c_double * 3)(*([float(x) for x in lo] + [0.0] * (3 - len(lo))))
    fp = FlagParams(len(centres), C.cast(cen, C.POINTER(C.c_double)), float(r_in), float(r_out),
                    int(dist_axes or dim), int(bool(periodic_dist)), len(nodes01) - 1,
                    C.cast(nodes, C.POINTER(C.c_double)), lo3, float(length), int(bool(raw)))
    return fp, (cen, nodes)


class Tree:
    """One linear quadtree / octree in device memory (owns an lt_tree)."""

    def __init__(self, handle: C.c_void_p, geom: Geom):
        self._h = handle
        self.geom = geom
        self.dim = geom.dim

    # ---- construction
    @classmethod
    def uniform(cls, dim, d_min, d_max, depth=None, periodic_mask=None, balance=2) -> "Tree":
        g = Geom(dim, d_min, d_max, (1 << dim) - 1 if periodic_mask is None else periodic_mask,
                 balance)
        h = C.c_void_p()
        _stream()
        _check(lib().lt_build_uniform(C.byref(g), d_min if depth is None else depth, _stream(),
                                      C.byref(h)))
        return cls(h, g)

    @classmethod
    def from_keys(cls, keys, dim, d_min, d_max, periodic_mask=None, balance=2) -> "Tree":
        """keys: device int64 tensor holding the uint64 Morton IDs."""
        torch = _torch()
        k = keys.to(device="cuda", dtype=torch.int64).contiguous()
        g = Geom(dim, d_min, d_max, (1 << dim) - 1 if periodic_mask is None else periodic_mask,
                 balance)
        h = C.c_void_p()
        _check(lib().lt_build(C.byref(g), _dptr(k), k.numel(), _stream(), C.byref(h)))
        return cls(h, g)

    @classmethod
    def from_points(cls, points, dim, d_min, d_max, lo, length, periodic_mask=None,
                    balance=2) -> "Tree":
        """Bottom-up construction (lt_build_points): points is an (n, dim)
        float64 tensor (moved to the device); the tree is not balanced."""
        torch = _torch()
        pts = points.to(device="cuda", dtype=torch.float64).contiguous()
        g = Geom(dim, d_min, d_max, (1 << dim) - 1 if periodic_mask is None else periodic_mask,
                 balance)
        lo3 = (C.c_double * 3)(*([float(x) for x in lo] + [0.0] * (3 - len(lo))))
        h = C.c_void_p()
        _check(lib().lt_build_points(C.byref(g), _dptr(pts) if pts.numel() else None,
                                     pts.shape[0] if pts.numel() else 0, lo3, float(length),
                                     _stream(), C.byref(h)))
        return cls(h, g)

    @classmethod
    def batch(cls, dim, d_finest, d_min, d_max, depth, periodic_mask=None, balance=2) -> "Tree":
        """Ensemble of len(d_min) trees in one key array (per-mesh lists)."""
        nm = len(d_min)
        g = Geom(dim, 0, d_finest, (1 << dim) - 1 if periodic_mask is None else periodic_mask,
                 balance)
        arr = lambda v: (C.c_int * nm)(*[int(x) for x in v])
        h = C.c_void_p()
        _check(lib().lt_build_batch(C.byref(g), nm, arr(d_min), arr(d_max), arr(depth), _stream(),
                                    C.byref(h)))
        t = cls(h, g)
        t.nmesh = nm
        return t

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lt_destroy(h)
            self._h = None

    # ---- sizes
    def sizes(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().lt_size(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def size(self) -> int:
        return self.sizes()[0]

    # ---- cycle
    def flag(self, centres, r_in, r_out, nodes01, lo, length, dist_axes=None,
             periodic_dist=False, out=None, raw=False):
        torch = _torch()
        n = self.size()
        if out is None:
            out = torch.empty(n, dtype=torch.int8, device="cuda")
        fp, _keep = _flag_params(self.dim, centres, r_in, r_out, nodes01, lo, length, dist_axes,
                                 periodic_dist, raw)
        _check(lib().lt_flag(self._h, C.byref(fp), _dptr(out), _stream()))
        return out

    def flag_batch(self, per_mesh, out=None):
        """per_mesh: list of dicts with keys centres, r_in, r_out, nodes01, lo, length,
        dist_axes, periodic_dist (one per mesh)."""
        torch = _torch()
        n = self.size()
        if out is None:
            out = torch.empty(n, dtype=torch.int8, device="cuda")
        keep = []
        fps = (FlagParams * len(per_mesh))()
        for m, a in enumerate(per_mesh):
            fps[m], k = _flag_params(self.dim, **a)
            keep.append(k)
        _check(lib().lt_flag_batch(self._h, C.cast(fps, C.c_void_p), len(per_mesh), _dptr(out),
                                   _stream()))
        return out

    def set_mesh_degree(self, degrees):
        """Per-mesh degrees (lt_set_mesh_degree) for transfer_mixed / mixed cycles."""
        arr = (C.c_int * len(degrees))(*[int(x) for x in degrees])
        _check(lib().lt_set_mesh_degree(self._h, arr, _stream()))
        self.degrees = [int(x) for x in degrees]

    def transfer_mixed(self, u_old, u_new=None):
        """u_old: (nvar, NPM, ld_old) with NPM the largest (p+1)^3 -> (nvar, NPM, n_cur)."""
        torch = _torch()
        nvar, npm, ld_old = u_old.shape
        if u_new is None:
            u_new = torch.empty((nvar, npm, self.size()), dtype=torch.float64, device="cuda")
        _check(lib().lt_transfer_mixed(self._h, nvar, _dptr(u_old), ld_old, _dptr(u_new),
                                       u_new.shape[2], _stream()))
        return u_new

    def mesh_offsets(self):
        nm = getattr(self, "nmesh", 1)
        offs = (C.c_int64 * (nm + 1))()
        _check(lib().lt_mesh_offsets(self._h, C.cast(offs, C.c_void_p), _stream()))
        return [int(x) for x in offs]

    def vortex_field(self, centres, strengths, nodes01, lo, length, ld=None, out=None):
        """Isentropic-vortex conserved variables at the solution points."""
        torch = _torch()
        n = self.size()
        p = len(nodes01) - 1
        npts = (p + 1) ** self.dim
        nvar = 5 if self.dim == 3 else 4
        if out is None:
            out = torch.empty((nvar, npts, ld or n), dtype=torch.float64, device="cuda")
        fp, keep = _flag_params(self.dim, centres, 0.0, 0.0, nodes01, lo, length)
        st = (C.c_double * len(strengths))(*[float(a) for a in strengths])
        _check(lib().lt_vortex_field(self._h, C.byref(fp), C.cast(st, C.c_void_p), _dptr(out),
                                     out.shape[2], _stream()))
        return out

    def flag_mlp(self, mlp, u, centres, r_in, r_out, nodes01, lo, length, conf_min=0.9,
                 dist_axes=None, periodic_dist=False):
        """Learned flags with the geometric criterion as the fallback; returns
        (flags, top softmax probability)."""
        torch = _torch()
        n = self.size()
        flags = torch.empty(n, dtype=torch.int8, device="cuda")
        conf = torch.empty(n, dtype=torch.float32, device="cuda")
        fp, _keep = _flag_params(self.dim, centres, r_in, r_out, nodes01, lo, length, dist_axes,
                                 periodic_dist)
        _check(lib().lt_flag_mlp(self._h, mlp._h, C.byref(fp), _dptr(u), u.shape[2],
                                 float(conf_min), _dptr(flags), _dptr(conf), _stream()))
        return flags, conf

    def flag_modal(self, p, u, tau_refine, tau_coarsen, out=None):
        """Modal-energy flags from the density (variable 0) of u (nvar, n_p, ld)."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.size(), dtype=torch.int8, device="cuda")
        _check(lib().lt_flag_modal(self._h, int(p), _dptr(u), u.shape[2], float(tau_refine),
                                   float(tau_coarsen), _dptr(out), _stream()))
        return out

    def adapt(self, flags):
        torch = _torch()
        f = flags.to(device="cuda", dtype=torch.int8).contiguous()
        if f.numel() != self.size():
            raise LtError(1, "flags must have one entry per leaf")
        _check(lib().lt_adapt(self._h, _dptr(f), _stream()))

    def balance(self):
        _check(lib().lt_balance(self._h, _stream()))

    def connect(self):
        _check(lib().lt_connect(self._h, _stream()))

    def set_connect_grid(self, blocks):
        """Cap the face search's workgroups (0: one lane per face); see lt.h."""
        _check(lib().lt_set_connect_grid(self._h, int(blocks)))

    def map(self):
        _check(lib().lt_map(self._h, _stream()))

    def transfer(self, p, u_old, u_new=None, precision=0):
        """u_old: (nvar, n_p, ld_old) float64 device tensor -> (nvar, n_p, n_cur)."""
        torch = _torch()
        assert u_old.dtype == torch.float64 and u_old.is_cuda and u_old.is_contiguous()
        nvar, npts, ld_old = u_old.shape
        if npts != (p + 1) ** self.dim:
            raise LtError(1, "u_old has the wrong number of points per element")
        n = self.size()
        if u_new is None:
            u_new = torch.empty((nvar, npts, n), dtype=torch.float64, device="cuda")
        _check(lib().lt_transfer(self._h, p, nvar, _dptr(u_old), ld_old, _dptr(u_new),
                                 u_new.shape[2], precision, _stream()))
        return u_new

    def transfer_noalloc(self, p, u_old, u_new):
        """lt_transfer_noalloc: the FP64 transfer into the caller's u_new
        (nvar, n_p, ld_new) with no device allocation; needs map() first."""
        torch = _torch()
        assert u_old.dtype == torch.float64 and u_new.dtype == torch.float64
        _check(lib().lt_transfer_noalloc(self._h, int(p), u_old.shape[0], _dptr(u_old), u_old.shape[2],
                                         _dptr(u_new), u_new.shape[2], _stream()))
        return u_new

    # ---- flux reconstruction (Euler, periodic)
    def fr_face_flux(self, p, u, gamma=1.4):
        """Common normal fluxes at every face: (2 dim, dim+2, (p+1)^(dim-1), n)."""
        torch = _torch()
        n = self.size()
        nfp = (p + 1) ** (self.dim - 1)
        out = torch.empty((2 * self.dim, self.dim + 2, nfp, n), dtype=torch.float64, device="cuda")
        _check(lib().lt_fr_face_flux(self._h, int(p), _dptr(u), u.shape[2], float(gamma), _dptr(out),
                                     n, _stream()))
        return out

    def fr_residual(self, p, u, length, gamma=1.4, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((u.shape[0], u.shape[1], self.size()), dtype=torch.float64,
                              device="cuda")
        _check(lib().lt_fr_residual(self._h, int(p), _dptr(u), u.shape[2], float(gamma),
                                    float(length), _dptr(out), out.shape[2], _stream()))
        return out

    def fr_rk3(self, p, u, work, dt, length, gamma=1.4, steps=1):
        """steps RK3 steps in place on u (work: same shape)."""
        assert work.shape == u.shape
        _check(lib().lt_fr_rk3(self._h, int(p), _dptr(u), u.shape[2], _dptr(work), float(dt),
                               float(gamma), float(length), int(steps), _stream()))
        return u

    # ---- results
    def autotune_transfer(self, p, u_old, u_new, precision=0):
        """Time every transfer launch shape on the current mapping and keep the
        fastest; returns the lt_tune record (as a dict)."""
        tn = Tune()
        _check(lib().lt_autotune_transfer(self._h, int(p), u_old.shape[0], _dptr(u_old), u_old.shape[2],
                                          _dptr(u_new), u_new.shape[2], int(precision), _stream(),
                                          C.byref(tn)))
        return {"copy_elems_per_lane": tn.copy_elems_per_lane, "interp_grid": tn.interp_grid,
                "ms": tn.ms, "ms_default": tn.ms_default}

    def set_tuning(self, copy_elems_per_lane=2, interp_grid=2048):
        tn = Tune(int(copy_elems_per_lane), int(interp_grid), -1.0, -1.0)
        _check(lib().lt_set_tuning(self._h, C.byref(tn)))

    def tuning(self):
        tn = Tune()
        _check(lib().lt_get_tuning(self._h, C.byref(tn)))
        return {"copy_elems_per_lane": tn.copy_elems_per_lane, "interp_grid": tn.interp_grid}

    def export(self, what: int):
        torch = _torch()
        n, n_old, n_hang = self.sizes()
        nf = 2 * self.dim
        w = 2 + (1 << (self.dim - 1))
        shapes = {LT_KEYS: ((n,), torch.int64), LT_OLD_KEYS: ((max(n_old, 0),), torch.int64),
                  LT_NBR: ((n, nf), torch.int32), LT_HANG: ((max(n_hang, 0), w), torch.int32),
                  LT_MAP_SRC: ((n,), torch.int32), LT_MAP_KIND: ((n,), torch.int8)}
        shape, dt = shapes[what]
        out = torch.empty(shape, dtype=dt, device="cuda")
        ptr = _dptr(out) if out.numel() else C.c_void_p()
        _check(lib().lt_export(self._h, what, ptr, out.numel(), _stream()))
        return out

    def keys(self):
        return self.export(LT_KEYS)

    def old_keys(self):
        return self.export(LT_OLD_KEYS)

    def nbr(self):
        return self.export(LT_NBR)

    def hang(self):
        return self.export(LT_HANG)

    def mapping(self):
        return self.export(LT_MAP_SRC), self.export(LT_MAP_KIND)


class MLP:
    """Learned refinement indicator (320 -> 128 -> 64 -> 3) on the device."""

    def __init__(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_NPARAM
        h = C.c_void_p()
        _torch()
        _check(lib().lt_mlp_create(p.ctypes.data_as(C.c_void_p), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lt_mlp_destroy(h)
            self._h = None

    def params(self, grads=False):
        import numpy as np
        p = np.zeros(MLP_NPARAM, dtype=np.float32)
        g = np.zeros(MLP_NPARAM, dtype=np.float32) if grads else None
        _check(lib().lt_mlp_params(self._h, p.ctypes.data_as(C.c_void_p),
                                   g.ctypes.data_as(C.c_void_p) if grads else None, _stream()))
        return (p, g) if grads else p

    def features(self, u, rows=None):
        """u: (5, 64, ld) float64 device tensor -> (n, 320) bfloat16 device tensor."""
        torch = _torch()
        n = rows.numel() if rows is not None else u.shape[2]
        X = torch.empty((n, 320), dtype=torch.bfloat16, device="cuda")
        r = _dptr(rows.to(torch.int32).contiguous()) if rows is not None else None
        _check(lib().lt_mlp_features(self._h, _dptr(u), u.shape[2], u.shape[0], r, n, _dptr(X),
                                     _stream()))
        return X

    def grads(self, X, labels):
        _check(lib().lt_mlp_grads(self._h, _dptr(X), _dptr(labels), X.shape[0], _stream()))

    def train_step(self, X, labels, lr):
        _check(lib().lt_mlp_train_step(self._h, _dptr(X), _dptr(labels), X.shape[0], float(lr),
                                       _stream()))

    def logits(self, X):
        torch = _torch()
        out = torch.empty((X.shape[0], 3), dtype=torch.float32, device="cuda")
        _check(lib().lt_mlp_infer(self._h, _dptr(X), X.shape[0], _dptr(out), _stream()))
        return out


class Cycle:
    """The whole plain cycle captured in a hipGraph over a tree (lt_cycle_*).

    ``u`` is a pair of device FP64 arrays (nvar, n_p, ld >= capacity); ``flag`` maps a
    cycle to the flag arguments of ``Tree.flag`` (a dict per mesh for an
    ensemble).  ``run(cycle)`` returns the index of the array now holding the
    solution."""

    def __init__(self, tree, p, nvar, capacity, u, flag_args, balance_passes=4, precision=0,
                 mlp=None, conf_min=0.9):
        self.tree = tree
        self._u = u
        per = flag_args if isinstance(flag_args, (list, tuple)) else [flag_args]
        self._keep = []
        arr = (FlagParams * len(per))()
        for m, a in enumerate(per):
            fp, keep = _flag_params(tree.dim, **a)
            arr[m] = fp
            self._keep.append(keep)
        d = CycleDesc()
        d.p, d.nvar, d.capacity, d.balance_passes = int(p), int(nvar), int(capacity), int(balance_passes)
        d.ld = int(u[0].shape[2])
        assert u[1].shape == u[0].shape
        d.u[0], d.u[1] = _dptr(u[0]), _dptr(u[1])
        d.nmesh = len(per)
        d.flag_template = arr
        d.precision = int(precision)
        d.mlp = mlp._h.value if mlp is not None else None
        d.conf_min = float(conf_min)
        self._mlp = mlp
        h = C.c_void_p()
        _check(lib().lt_cycle_create(tree._h, C.byref(d), _stream(), C.byref(h)))
        self._h = h

    def run(self, flag_args):
        per = flag_args if isinstance(flag_args, (list, tuple)) else [flag_args]
        arr = (FlagParams * len(per))()
        keep = []
        for m, a in enumerate(per):
            fp, k = _flag_params(self.tree.dim, **a)
            arr[m] = fp
            keep.append(k)
        ui = C.c_int(-1)
        _check(lib().lt_cycle_run(self._h, arr, _stream(), C.byref(ui)))
        return ui.value

    def stats(self):
        """(runs, runs finished eagerly, recaptures)."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().lt_cycle_stats(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lt_cycle_destroy(h)
            self._h = None
