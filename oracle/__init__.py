"""Oracle for the SyMBA kick/encounter step -- test infrastructure only.

Python front end (ctypes) of the plain single-threaded FP64 C oracle in
symba_oracle.c, and of its all-core build (symba_oracle_omp.c), which the
benchmark times for context.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the GPU library and its binding never do.

Every function takes host numpy arrays (float64 SoA, int32 pair lists) and
follows the paper's Sec. 2: trapezoid pair loop, close-encounter check and
grouping of encounter pairs.  See symba_oracle.c for the readings of the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsymba_oracle.so")
SRC_PATH = os.path.join(_HERE, "symba_oracle.c")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-mfma", "-fno-fast-math", "-fPIC", "-shared"]


OMP_LIB_PATH = os.path.join(_HERE, "libsymba_oracle_omp.so")
OMP_SRC_PATH = os.path.join(_HERE, "symba_oracle_omp.c")


def build(out_path: str = LIB_PATH, src_path: str = SRC_PATH, extra=()) -> str:
    """Compile the oracle with gcc (FP contraction off; fma() is explicit),
    and its all-core build (OpenMP) for the benchmark's CPU context."""
    cmd = ["gcc", *CFLAGS, *extra, "-o", out_path, src_path, "-lm"]
    subprocess.run(cmd, check=True)
    if out_path == LIB_PATH:
        build_omp()
    return out_path


def build_omp(out_path: str = OMP_LIB_PATH) -> str:
    cmd = ["gcc", *CFLAGS, "-fopenmp", "-o", out_path, OMP_SRC_PATH, SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


_D = ctypes.c_double
_I64 = ctypes.c_int64
_P = ctypes.c_void_p


def _declare(lib):
    lib.oracle_accel.restype = ctypes.c_int
    lib.oracle_accel.argtypes = [_I64, _I64] + [_P] * 7
    lib.oracle_accel_body.restype = ctypes.c_int
    lib.oracle_accel_body.argtypes = [_I64, _I64, _I64] + [_P] * 5
    lib.oracle_encounter.restype = ctypes.c_int
    lib.oracle_encounter.argtypes = [_D] * 16
    lib.oracle_encounter_list.restype = ctypes.c_int
    lib.oracle_encounter_list.argtypes = [_I64] + [_P] * 7 + [_D, _D, _I64, _P, _P, _P]
    lib.oracle_pairs.restype = _I64
    lib.oracle_pairs.argtypes = [_I64, _I64] + [_P] * 7 + [_D, _D, _P, _P, _I64]
    lib.oracle_partners.restype = _I64
    lib.oracle_partners.argtypes = [_I64, _I64, _I64] + [_P] * 7 + [_D, _D, _P, _I64]
    lib.oracle_groups.restype = _I64
    lib.oracle_groups.argtypes = [_I64, _I64, _P, _P, _P]
    lib.oracle_kick_encounter.restype = _I64
    lib.oracle_kick_encounter.argtypes = ([_I64, _I64] + [_P] * 8 + [_D, _D] + [_P] * 5
                                          + [_I64, _P, _P])
    lib.oracle_helio.restype = ctypes.c_int
    lib.oracle_helio.argtypes = [_I64, _I64] + [_P] * 10
    return lib


def load_omp(path: str = OMP_LIB_PATH):
    """The all-core build (OpenMP; the paper's Sec. 2 scheme), compiled first
    only if it is not built."""
    if not os.path.exists(path):
        build_omp(path)
    L = _declare(ctypes.CDLL(path))
    L.oracle_kick_encounter_omp.restype = _I64
    L.oracle_kick_encounter_omp.argtypes = ([_I64, _I64] + [_P] * 8 + [_D, _D] + [_P] * 5
                                            + [_I64, _P, _P, _P])
    return L


def load(path: str = LIB_PATH):
    """Load the oracle library, compiling it first only if it is not built."""
    if not os.path.exists(path):
        build(path)
    return _declare(ctypes.CDLL(path))


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data


class Oracle:
    """Bound to one compiled oracle library (the default one, or a test build)."""

    def __init__(self, library=None):
        self.L = library if library is not None else lib()

    def accel(self, s, n_m):
        x, y, z, m = (_f64(s[k]) for k in ("x", "y", "z", "m"))
        n = x[0].size
        out = [np.zeros(n) for _ in range(3)]
        rc = self.L.oracle_accel(n, n_m, x[1], y[1], z[1], m[1], *(o.ctypes.data for o in out))
        if rc != 0:
            raise ValueError("oracle_accel: invalid arguments")
        return np.stack(out, axis=1)

    def accel_body(self, s, n_m, k):
        x, y, z, m = (_f64(s[key]) for key in ("x", "y", "z", "m"))
        out = np.zeros(3)
        rc = self.L.oracle_accel_body(int(k), x[0].size, n_m, x[1], y[1], z[1], m[1], out.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_accel_body: invalid arguments")
        return out

    def encounter(self, bi, bj, dt, f):
        """bi, bj: (x, y, z, vx, vy, vz, rh) of the two bodies."""
        return bool(self.L.oracle_encounter(*map(float, bi), *map(float, bj), float(dt), float(f)))

    def encounter_list(self, s, pi, pj, dt, f):
        """The predicate on each listed pair (pi[k], pj[k]) of state s: bool array."""
        arrs = [_f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "rh")]
        pi, pj = _i32(pi), _i32(pj)
        flag = np.zeros(pi[0].size, np.uint8)
        rc = self.L.oracle_encounter_list(arrs[0][0].size, *(a[1] for a in arrs), float(dt), float(f),
                                          pi[0].size, pi[1], pj[1], flag.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_encounter_list: invalid arguments")
        return flag.astype(bool)

    def pairs(self, s, n_m, dt, f, cap=None):
        arrs = [_f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "rh")]
        n = arrs[0][0].size
        if cap is None:
            cap = max(4 * n, 4096)
        while True:
            pi = np.zeros(cap, np.int32)
            pj = np.zeros(cap, np.int32)
            cnt = self.L.oracle_pairs(n, n_m, *(a[1] for a in arrs), float(dt), float(f),
                                      pi.ctypes.data, pj.ctypes.data, cap)
            if cnt < 0:
                raise ValueError("oracle_pairs: invalid arguments")
            if cnt <= cap:
                return pi[:cnt].copy(), pj[:cnt].copy()
            cap = int(cnt)

    def partners(self, s, n_m, i, dt, f):
        arrs = [_f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "rh")]
        n = arrs[0][0].size
        cap = 1024
        while True:
            out = np.zeros(cap, np.int32)
            cnt = self.L.oracle_partners(int(i), n, n_m, *(a[1] for a in arrs), float(dt), float(f),
                                         out.ctypes.data, cap)
            if cnt < 0:
                raise ValueError("oracle_partners: invalid arguments")
            if cnt <= cap:
                return out[:cnt].copy()
            cap = int(cnt)

    def groups(self, n, pi, pj):
        pi, pi_p = _i32(pi)
        pj, pj_p = _i32(pj)
        gid = np.zeros(n, np.int32)
        ng = self.L.oracle_groups(n, pi.size, pi_p, pj_p, gid.ctypes.data)
        if ng < 0:
            raise ValueError("oracle_groups: invalid arguments")
        return gid, int(ng)

    def kick_encounter(self, s, n_m, dt, f, cap=None):
        """Whole step: returns dict(acc[N,3], pair_i, pair_j, group_id, n_groups)."""
        arrs = [_f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rh")]
        n = arrs[0][0].size
        if cap is None:
            cap = max(4 * n, 4096)
        while True:
            acc = [np.zeros(n) for _ in range(3)]
            pi = np.zeros(cap, np.int32)
            pj = np.zeros(cap, np.int32)
            gid = np.zeros(n, np.int32)
            ng = ctypes.c_int64(0)
            cnt = self.L.oracle_kick_encounter(
                n, n_m, *(a[1] for a in arrs), float(dt), float(f),
                *(a.ctypes.data for a in acc), pi.ctypes.data, pj.ctypes.data, cap,
                gid.ctypes.data, ctypes.addressof(ng))
            if cnt < 0:
                raise ValueError("oracle_kick_encounter: invalid arguments")
            if cnt <= cap:
                return dict(acc=np.stack(acc, axis=1), pair_i=pi[:cnt].copy(),
                            pair_j=pj[:cnt].copy(), group_id=gid, n_groups=int(ng.value))
            cap = int(cnt)

    def kick_encounter_omp(self, s, n_m, dt, f, cap=None):
        """The whole step on every core (needs the library from load_omp()):
        the paper's Sec. 2 scheme, thread-private accumulators summed in
        thread order.  Returns kick_encounter's dict plus `threads`."""
        arrs = [_f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rh")]
        n = arrs[0][0].size
        if cap is None:
            cap = max(4 * n, 4096)
        while True:
            acc = [np.zeros(n) for _ in range(3)]
            pi = np.zeros(cap, np.int32)
            pj = np.zeros(cap, np.int32)
            gid = np.zeros(n, np.int32)
            ng = ctypes.c_int64(0)
            th = ctypes.c_int32(0)
            cnt = self.L.oracle_kick_encounter_omp(
                n, n_m, *(a[1] for a in arrs), float(dt), float(f),
                *(a.ctypes.data for a in acc), pi.ctypes.data, pj.ctypes.data, cap,
                gid.ctypes.data, ctypes.addressof(ng), ctypes.addressof(th))
            if cnt == -1:
                raise ValueError("oracle_kick_encounter_omp: invalid arguments")
            if cnt < 0:
                raise MemoryError("oracle_kick_encounter_omp: out of host memory")
            if cnt <= cap:
                return dict(acc=np.stack(acc, axis=1), pair_i=pi[:cnt].copy(), pair_j=pj[:cnt].copy(),
                            group_id=gid, n_groups=int(ng.value), threads=int(th.value))
            cap = int(cnt)

    def helio(self, s, n_m, acc):
        x, y, z, m = (_f64(s[k]) for k in ("x", "y", "z", "m"))
        n = x[0].size
        a = [_f64(acc[:, c]) for c in range(3)]
        out = [np.zeros(n) for _ in range(3)]
        rc = self.L.oracle_helio(n, n_m, x[1], y[1], z[1], m[1], *(t[1] for t in a),
                                 *(o.ctypes.data for o in out))
        if rc != 0:
            raise ValueError("oracle_helio: invalid arguments")
        return np.stack(out, axis=1)


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
