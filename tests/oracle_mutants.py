"""Copies of the oracle with one planted mistake, for showing that a pin fails when the
oracle is wrong.

``build`` applies exact text substitutions to ``oracle/oracle.c`` (each must match once),
compiles the result with the oracle's own flags into a temporary directory and loads
it. The oracle's source and library are left untouched; nothing outside ``tests/``
uses this module."""
import ctypes as C
import os
import subprocess

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")

_dp = C.POINTER(C.c_double)


def build(tmpdir, subs):
    """The oracle compiled with every (old, new) substitution of subs applied."""
    with open(os.path.join(ORACLE_DIR, "oracle.c")) as fh:
        src = fh.read()
    for old, new in subs:
        assert src.count(old) == 1, f"substitution target must occur once: {old!r}"
        src = src.replace(old, new)
    path = os.path.join(str(tmpdir), "oracle_mutant.c")
    with open(path, "w") as fh:
        fh.write(src)
    so = os.path.join(str(tmpdir), "liboracle_mutant.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    f"-I{ORACLE_DIR}", "-o", so, path, "-lm"], check=True)
    return C.CDLL(so)


def normal_fn(lib):
    """or_normal of a (mutant) oracle library as normal(c27, method) -> m."""
    lib.or_normal.restype = None
    lib.or_normal.argtypes = [_dp, C.c_int, _dp]

    def normal(c27, method=1):
        a = np.ascontiguousarray(np.asarray(c27, dtype=np.float64).reshape(27))
        out = np.zeros(3)
        lib.or_normal(a.ctypes.data_as(_dp), int(method), out.ctypes.data_as(_dp))
        return out

    return normal


def alpha_n_fn(lib):
    """or_alpha of a (mutant) oracle library over arrays: alpha_n(m (n, 3), c (n,))."""
    lib.or_alpha.restype = C.c_double
    lib.or_alpha.argtypes = [_dp, C.c_double]

    def alpha_n(m, c):
        m = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
        out = np.empty(len(c))
        for i in range(len(c)):
            row = np.ascontiguousarray(m[i])
            out[i] = lib.or_alpha(row.ctypes.data_as(_dp), float(c[i]))
        return out

    return alpha_n
