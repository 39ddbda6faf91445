"""The C implementation of the oracle's lattice operations (test-only).

`clattice.c` is a second, independent FP64 implementation of what
`lattice.py` computes (streaming with the boundary rules of Sec. 2.1, the
moments of Eq. 2 and the Guo-forced BGK collision of Eqs. 4, 7, 8), in plain
C with OpenMP over z-planes, so that oracle runs over thousands of steps of
the 256x192x192 box finish in minutes.  This module compiles it with gcc
(on first use, or when the source is newer than the library) and exposes the
same call signatures as `lattice.py`, so `sim.Sim(..., lattice="c")` can use
either.  tests/test_oracle_clattice.py checks it against lattice.py and the
closed forms.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "clattice.c")
LIB = os.path.join(HERE, "libclattice.so")

PERIODIC, WALL, VELOCITY, PRESSURE, ZH_VELOCITY, ZH_PRESSURE = 0, 1, 2, 3, 4, 5

_lib = None


def build(force=False):
    """Compile clattice.c into libclattice.so (IEEE arithmetic: no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        i = C.c_int
        lib.ora_stream.argtypes = [dp, dp, i, i, i, ip, dp, C.c_double]
        lib.ora_moments.argtypes = [dp, dp, dp, i, i, i]
        lib.ora_collide.argtypes = [dp, dp, dp, dp, C.c_double, dp, i, i, i]
        lib.ora_equilibrium.argtypes = [dp, dp, dp, i, i, i]
        lib.ora_set_threads.argtypes = [i]
        for fn in (lib.ora_stream, lib.ora_moments, lib.ora_collide, lib.ora_equilibrium, lib.ora_set_threads):
            fn.restype = None
        _lib = lib
    return _lib


def set_threads(n):
    """Threads of the C lattice's parallel loops."""
    _load().ora_set_threads(int(n))


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(a, lead):
    if a.ndim != 3 + lead:
        raise ValueError("expected a (..., nz, ny, nx) array")
    nz, ny, nx = a.shape[-3:]
    return nx, ny, nz


def stream(S, bc, u_in, rho_out):
    """Same as lattice.stream."""
    S = _c(S)
    nx, ny, nz = _dims(S, 1)
    f = np.empty_like(S)
    b = (C.c_int * 6)(*[int(v) for v in bc])
    u = np.ascontiguousarray(u_in if u_in is not None else [0.0, 0.0, 0.0], dtype=np.float64)
    _load().ora_stream(_p(S), _p(f), nx, ny, nz, b, _p(u), float(rho_out))
    return f


def moments(f):
    """Same as lattice.moments: (rho, momentum)."""
    f = _c(f)
    nx, ny, nz = _dims(f, 1)
    rho = np.empty(f.shape[1:])
    mom = np.empty((3,) + f.shape[1:])
    _load().ora_moments(_p(f), _p(rho), _p(mom), nx, ny, nz)
    return rho, mom


def collide(f, rho, u, F, tau):
    """Same as lattice.collide."""
    f, rho, u, F = _c(f), _c(rho), _c(u), _c(F)
    nx, ny, nz = _dims(f, 1)
    out = np.empty_like(f)
    _load().ora_collide(_p(f), _p(rho), _p(u), _p(F), float(tau), _p(out), nx, ny, nz)
    return out


def equilibrium(rho, u):
    """Same as lattice.equilibrium for (nz, ny, nx) fields."""
    rho, u = _c(rho), _c(u)
    nx, ny, nz = _dims(rho, 0)
    out = np.empty((19,) + rho.shape)
    _load().ora_equilibrium(_p(rho), _p(u), _p(out), nx, ny, nz)
    return out
