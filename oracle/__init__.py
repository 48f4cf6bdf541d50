"""ctypes binding of the CPU oracle (``liblt_oracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports it.  It shares no code with the GPU library.

Every call mirrors one step of the adaptation cycle (Section 4.1 procedure,
Section 3.2 balance, Section 3.3 connectivity, Section 4.2 mapping and
transfer); see ``lt_oracle.h`` for argument meanings.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblt_oracle.so")
_SRC = os.path.join(_HERE, "lt_oracle.cpp")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP contraction off, as the flag criterion needs)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", _SO + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        i64, i32, u32, dbl = C.c_int64, C.c_int, C.c_uint, C.c_double
        L.lto_create.restype = P
        L.lto_create.argtypes = [i32, i32, i32, u32, i32, P, i64]
        L.lto_create_uniform.restype = P
        L.lto_create_uniform.argtypes = [i32, i32, i32, u32, i32, i32]
        L.lto_create_points.restype = P
        L.lto_create_points.argtypes = [i32, i32, i32, u32, i32, P, i64, P, dbl]
        L.lto_point_cells.argtypes = [i32, i32, P, i64, P, dbl, P]
        L.lto_destroy.argtypes = [P]
        L.lto_size.restype = i64
        L.lto_size.argtypes = [P]
        L.lto_old_size.restype = i64
        L.lto_old_size.argtypes = [P]
        L.lto_keys.argtypes = [P, P]
        L.lto_old_keys.argtypes = [P, P]
        L.lto_encode.restype = C.c_uint64
        L.lto_encode.argtypes = [i32, i32, i32, P]
        L.lto_decode.argtypes = [i32, i32, C.c_uint64, P, P]
        L.lto_flag.argtypes = [P, i32, P, dbl, dbl, i32, i32, P, i32, P, dbl, P]
        L.lto_flag_keys.argtypes = [i32, i32, i32, P, i64, i32, P, dbl, dbl, i32, i32, P, i32, P,
                                    dbl, P]
        L.lto_adapt.argtypes = [P, P]
        L.lto_balance.argtypes = [P, i32]
        L.lto_is_balanced.argtypes = [P]
        L.lto_connect.argtypes = [P, i32, P, P, i64, P]
        L.lto_map.argtypes = [P, P, P]
        L.lto_transfer.argtypes = [P, i32, i32, P, i64, P, i64]
        L.lto_gauss_legendre.argtypes = [i32, P, P]
        L.lto_operators.argtypes = [i32, i32, P, P]
        L.lto_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        raise OracleError(lib().lto_last_error().decode())


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def encode(dim: int, d_max: int, depth: int, anchor) -> int:
    a = np.zeros(3, dtype=np.int64)
    a[: len(anchor)] = anchor
    return int(lib().lto_encode(dim, d_max, depth, _ptr(a)))


def decode(dim: int, d_max: int, key: int):
    d = C.c_int(0)
    a = np.zeros(3, dtype=np.int64)
    _check(lib().lto_decode(dim, d_max, C.c_uint64(key), C.byref(d), _ptr(a)))
    return d.value, a[:dim].copy()


def gauss_legendre(npts: int):
    x = np.zeros(npts)
    w = np.zeros(npts)
    _check(lib().lto_gauss_legendre(npts, _ptr(x), _ptr(w)))
    return x, w


def operators(dim: int, p: int):
    np_ = (p + 1) ** dim
    nc = 1 << dim
    I = np.zeros((nc, np_, np_))
    P = np.zeros((nc, np_, np_))
    _check(lib().lto_operators(dim, p, _ptr(I), _ptr(P)))
    return I, P


def flag_keys(dim, d_min, d_max, keys, centres, r_in, r_out, nodes01, lo, length, dist_axes=None,
              periodic_dist=False) -> np.ndarray:
    """The geometric criterion (Section 5.2) for arbitrary leaf keys: what
    Tree.flag gives each of them in any tree with depth limits d_min..d_max."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    c = np.zeros((len(centres), 3))
    for v, cc in enumerate(centres):
        c[v, : len(cc)] = cc
    nodes = np.ascontiguousarray(nodes01, dtype=np.float64)
    lo3 = np.zeros(3)
    lo3[: len(lo)] = lo
    out = np.zeros(len(k), dtype=np.int8)
    _check(lib().lto_flag_keys(dim, d_min, d_max, _ptr(k), len(k), len(centres), _ptr(c),
                               float(r_in), float(r_out), int(dist_axes or dim),
                               int(bool(periodic_dist)), _ptr(nodes), len(nodes) - 1, _ptr(lo3),
                               float(length), _ptr(out)))
    return out


def point_cells(dim, d_max, pts, lo, length) -> np.ndarray:
    """Finest cells (n, dim) of points (n, dim) in [lo, lo+length)^dim."""
    p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, dim)
    lo3 = np.zeros(3)
    lo3[:dim] = lo
    out = np.zeros(p.shape, dtype=np.int64)
    _check(lib().lto_point_cells(dim, d_max, _ptr(p), len(p), _ptr(lo3), float(length), _ptr(out)))
    return out


class Tree:
    """Pointer-tree oracle of one linear tree (host memory)."""

    def __init__(self, dim, d_min, d_max, periodic_mask=None, balance=2, keys=None,
                 start_depth=None, points=None, lo=None, length=None):
        if periodic_mask is None:
            periodic_mask = (1 << dim) - 1
        self.dim, self.d_min, self.d_max = dim, d_min, d_max
        if points is not None:
            pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, dim)
            lo3 = np.zeros(3)
            lo3[:dim] = lo
            h = lib().lto_create_points(dim, d_min, d_max, periodic_mask, balance,
                                        _ptr(pts) if len(pts) else None, len(pts), _ptr(lo3),
                                        float(length))
        elif keys is None:
            sd = d_min if start_depth is None else start_depth
            h = lib().lto_create_uniform(dim, d_min, d_max, periodic_mask, balance, sd)
        else:
            k = np.ascontiguousarray(keys, dtype=np.uint64)
            h = lib().lto_create(dim, d_min, d_max, periodic_mask, balance, _ptr(k), len(k))
        if not h:
            raise OracleError(lib().lto_last_error().decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().lto_destroy(h)
            self._h = None

    def size(self) -> int:
        return int(lib().lto_size(self._h))

    def old_size(self) -> int:
        return int(lib().lto_old_size(self._h))

    def keys(self) -> np.ndarray:
        out = np.zeros(self.size(), dtype=np.uint64)
        _check(lib().lto_keys(self._h, _ptr(out)))
        return out

    def old_keys(self) -> np.ndarray:
        out = np.zeros(self.old_size(), dtype=np.uint64)
        _check(lib().lto_old_keys(self._h, _ptr(out)))
        return out

    def flag(self, centres, r_in, r_out, nodes01, lo, length, dist_axes=None,
             periodic_dist=False) -> np.ndarray:
        c = np.zeros((len(centres), 3))
        for v, cc in enumerate(centres):
            c[v, : len(cc)] = cc
        nodes = np.ascontiguousarray(nodes01, dtype=np.float64)
        lo3 = np.zeros(3)
        lo3[: len(lo)] = lo
        out = np.zeros(self.size(), dtype=np.int8)
        _check(lib().lto_flag(self._h, len(centres), _ptr(c), float(r_in), float(r_out),
                              int(dist_axes or self.dim), int(bool(periodic_dist)),
                              _ptr(nodes), len(nodes) - 1, _ptr(lo3), float(length), _ptr(out)))
        return out

    def adapt(self, flags):
        f = np.ascontiguousarray(flags, dtype=np.int8)
        assert len(f) == self.size()
        _check(lib().lto_adapt(self._h, _ptr(f)))

    def balance(self, brute=False):
        _check(lib().lto_balance(self._h, int(bool(brute))))

    def is_balanced(self) -> bool:
        return bool(lib().lto_is_balanced(self._h))

    def connect(self, brute=False):
        n = self.size()
        nf = 2 * self.dim
        w = 2 + (1 << (self.dim - 1))
        nbr = np.zeros(n * nf, dtype=np.int32)
        cnt = C.c_int64(0)
        _check(lib().lto_connect(self._h, int(bool(brute)), _ptr(nbr), None, 0, C.byref(cnt)))
        hang = np.zeros((max(cnt.value, 1), w), dtype=np.int32)
        _check(lib().lto_connect(self._h, int(bool(brute)), _ptr(nbr), _ptr(hang),
                                 cnt.value, C.byref(cnt)))
        return nbr.reshape(n, nf), hang[: cnt.value]

    def map(self):
        n = self.size()
        src = np.zeros(n, dtype=np.int32)
        kind = np.zeros(n, dtype=np.int8)
        _check(lib().lto_map(self._h, _ptr(src), _ptr(kind)))
        return src, kind

    def transfer(self, p: int, u_old: np.ndarray) -> np.ndarray:
        """u_old: (nvar, n_p, N_old) float64 -> (nvar, n_p, N_new)."""
        u_old = np.ascontiguousarray(u_old, dtype=np.float64)
        nvar, np_, ld_old = u_old.shape
        assert np_ == (p + 1) ** self.dim
        n = self.size()
        u_new = np.zeros((nvar, np_, n))
        _check(lib().lto_transfer(self._h, p, nvar, _ptr(u_old), ld_old, _ptr(u_new), n))
        return u_new
