"""Loader for the oracle's plain C Wilson operator (wilson_ref.c).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import wilson

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wilson_ref.c")
_LIB = os.path.join(_HERE, "libwilson_ref.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp"])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        _lib.wilson_ref_apply.restype = None
    return _lib


_PM = np.ascontiguousarray(wilson.PROJ_MINUS, dtype=np.complex128)
_PP = np.ascontiguousarray(wilson.PROJ_PLUS, dtype=np.complex128)


def apply_D(U, psi, m: float, antiperiodic_t: bool = True):
    """Same operator as ``wilson.apply_D`` for a single spinor field."""
    lib = _load()
    U = np.ascontiguousarray(U, dtype=np.complex128)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    Lt, Lz, Ly, Lx = psi.shape[-6:-2]
    assert psi.shape[-2:] == (4, 3) and U.shape == (4, Lt, Lz, Ly, Lx, 3, 3)
    L = (ctypes.c_int * 4)(Lx, Ly, Lz, Lt)
    out = np.empty_like(psi)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    lib.wilson_ref_apply(L, p(U), p(psi), p(out), ctypes.c_double(m), ctypes.c_int(int(antiperiodic_t)),
                         p(_PM), p(_PP))
    return out
