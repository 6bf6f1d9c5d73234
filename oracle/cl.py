"""ctypes wrapper of celllist.c (FP64 cell-list oracle) -- TEST INFRASTRUCTURE ONLY.

`CellModel` has the interface of potential.Model (energy, forces, hvp and the same
constants), so the path functions of path.py run unchanged on top of it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .potential import Model

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "celllist.c")


def build(force=False):
    """Compile celllist.c into liboracle.so (gcc, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", SRC_PATH,
                               "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Sys(C.Structure):
    _fields_ = [
        ("Q", C.c_int), ("box", C.c_double * 3), ("rc", C.c_double),
        ("type", C.POINTER(C.c_int)), ("ntypes", C.c_int),
        ("c6", C.POINTER(C.c_double)), ("c12", C.POINTER(C.c_double)),
        ("q", C.POINTER(C.c_double)), ("fq", C.c_double),
        ("krf", C.c_double), ("crf", C.c_double),
        ("excl_start", C.POINTER(C.c_int)), ("excl", C.POINTER(C.c_int)),
        ("nbonds", C.c_int), ("bonds", C.POINTER(C.c_int)),
        ("r0", C.POINTER(C.c_double)), ("kb", C.POINTER(C.c_double)),
        ("ewald", C.c_int), ("beta", C.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.oracle_eval.restype = C.c_int
        _lib.oracle_eval.argtypes = [C.POINTER(_Sys), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.POINTER(C.c_double), C.c_int]
        _lib.oracle_max_threads.restype = C.c_int
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class CellModel(Model):
    """Model whose energy / forces / hvp run in celllist.c (pair terms and bonds); for PME
    systems the reciprocal part and the constant terms come from pme.py as in Model."""

    def __init__(self, system, nthreads=0):
        super().__init__(system)
        self.nthreads = int(nthreads)
        Q = self.Q
        ex = self.excluded
        ii, jj = (ex // Q).astype(np.int64), (ex % Q).astype(np.int64)
        a = np.concatenate([ii, jj])
        b = np.concatenate([jj, ii])
        order = np.lexsort((b, a))
        a, b = a[order], b[order]
        self._excl_start = np.zeros(Q + 1, np.int32)
        np.add.at(self._excl_start, a + 1, 1)
        self._excl_start = np.cumsum(self._excl_start).astype(np.int32)
        self._excl = b.astype(np.int32)
        self._type = self.type.astype(np.int32)
        self._c6 = np.ascontiguousarray(self.c6, np.float64)
        self._c12 = np.ascontiguousarray(self.c12, np.float64)
        self._q = np.ascontiguousarray(self.q, np.float64)
        self._bonds = np.ascontiguousarray(self.bonds, np.int32).reshape(-1)
        self._r0 = np.ascontiguousarray(self.bond_r0, np.float64)
        self._kb = np.ascontiguousarray(self.bond_k, np.float64)
        if self._excl.size == 0:
            self._excl = np.zeros(1, np.int32)
        if self._bonds.size == 0:
            self._bonds, self._r0, self._kb = np.zeros(2, np.int32), np.zeros(1), np.zeros(1)
        s = _Sys()
        s.Q = Q
        s.box[:] = list(self.box)
        s.rc = self.rc
        s.type = _ptr(self._type, C.c_int)
        s.ntypes = int(self.c6.shape[0])
        s.c6, s.c12 = _ptr(self._c6, C.c_double), _ptr(self._c12, C.c_double)
        s.q = _ptr(self._q, C.c_double)
        s.fq = self.fq
        s.krf, s.crf = self.krf, self.crf
        s.excl_start, s.excl = _ptr(self._excl_start, C.c_int), _ptr(self._excl, C.c_int)
        s.nbonds = int(len(self.bonds))
        s.bonds = _ptr(self._bonds, C.c_int)
        s.r0, s.kb = _ptr(self._r0, C.c_double), _ptr(self._kb, C.c_double)
        s.ewald = 1 if self.pme is not None else 0
        s.beta = self.beta if self.pme is not None else 0.0
        self._s = s

    def eval(self, X, V=None, forces=True, energy=True):
        lib = _load()
        X = np.ascontiguousarray(X, np.float64)
        F = np.zeros((self.Q, 3)) if forces else None
        HV = np.zeros((self.Q, 3)) if V is not None else None
        Vc = np.ascontiguousarray(V, np.float64) if V is not None else None
        u = C.c_double(0.0)
        lib.oracle_eval(C.byref(self._s), X.ctypes.data,
                        Vc.ctypes.data if Vc is not None else None,
                        F.ctypes.data if F is not None else None,
                        HV.ctypes.data if HV is not None else None,
                        C.byref(u) if energy else None, self.nthreads)
        e = u.value
        if self.pme is not None:
            if energy:
                e += self.pme.energy(X) + self.e_const
            if F is not None:
                F += self.pme.forces(X)
            if HV is not None:
                HV += self.pme.hvp(X, Vc)
        return e, F, HV

    def energy(self, X):
        return self.eval(X, forces=False)[0]

    def forces(self, X):
        return self.eval(X, energy=False)[1]

    def hvp(self, X, V):
        return self.eval(X, V=V, forces=False, energy=False)[2]


def max_threads():
    return int(_load().oracle_max_threads())
