"""The C part of the oracle (oracle/c/*.c), compiled with gcc into one shared
library -- test infrastructure.  Floating-point contraction is off so that
the C routines round exactly like their Python counterparts."""
from __future__ import annotations

import ctypes
import glob
import os
import subprocess
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = sorted(glob.glob(os.path.join(_HERE, "c", "*.c")))
_LIB = os.path.join(_HERE, "c", "liboracle.so")
_lock = threading.Lock()
_lib = None


def build_c() -> str:
    """Compile the oracle's C sources (called by the build step and lazily on
    first use)."""
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", _LIB, *_SRCS, "-lm"])
    return _LIB


def load():
    global _lib
    with _lock:
        if _lib is None:
            stale = (not os.path.exists(_LIB)) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS)
            if stale:
                build_c()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_cuthill_mckee.restype = ctypes.c_int
            lib.oracle_cuthill_mckee.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            lib.oracle_ilut.restype = ctypes.c_int
            lib.oracle_ilut.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            lib.oracle_ilutp.restype = ctypes.c_int
            lib.oracle_ilutp.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
            lib.oracle_greedy_colour.restype = ctypes.c_int
            lib.oracle_greedy_colour.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p]
            _lib = lib
    return _lib
