"""CPU FP64 oracle for the cuROB test functions (arXiv 1407.7737) -- test infrastructure.

This package is the correctness reference for the GPU library.  It is a ctypes binding to
``curob_oracle.c``: plain FP64 loops that evaluate each definition of the paper literally
(shift, dense rotation, formula, bias).  It shares no code with ``paper_1407_7737_amd`` and is
only imported by ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py``.  The product path never calls it.

Parity status per part is listed at the top of ``curob_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "curob_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Tab. 1 ids
SPHERE, ELLIPSOID, ELLIPTIC, DISCUS, CIGAR, POWERS, SHARPV = range(7)
STEP, WEIERSTRASS, GRIEWANK, RASTRIGIN_U, RASTRIGIN, SCHAFFERSF7 = range(7, 13)
GRIE_ROSEN, ROSENBROCK, SCHWEFEL_U, SCHWEFEL, KATSUURA, LUNACEK = range(13, 19)
ACKLEY, HAPPYCAT, HGBAT, SCHAFFERSF6 = range(19, 23)

# (scale s, offset c, rotated) read off each function's "where" clause, Secs. 3-4
XFORM = {
    0: (1.0, 0.0, True), 1: (1.0, 0.0, True), 2: (1.0, 0.0, True), 3: (1.0, 0.0, True),
    4: (1.0, 0.0, True), 5: (0.01, 0.0, True), 6: (1.0, 0.0, True), 7: (1.0, 0.0, True),
    8: (0.005, 0.0, True), 9: (6.0, 0.0, True), 10: (0.0512, 0.0, False), 11: (0.0512, 0.0, True),
    12: (1.0, 0.0, True), 13: (0.05, 1.0, True), 14: (0.02048, 1.0, True), 15: (10.0, 0.0, False),
    16: (10.0, 0.0, True), 17: (0.05, 0.0, True), 18: (0.1, 2.5, True), 19: (1.0, 0.0, True),
    20: (0.05, -1.0, True), 21: (0.05, -1.0, True), 22: (1.0, 0.0, True),
}


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain -O2, no fast-math; OpenMP only for timing)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
             "-Wall", "-Wextra", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, u32, u64, i64, f64 = ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_long, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_uint64)
        sig = {
            "orc_problem_basic": (P, [i32, i32, u64]),
            "orc_problem_custom_basic": (P, [i32, i32, i32, u64, f64, f64, i32]),
            "orc_problem_hybrid": (P, [i32, i32, u64, i32, ip, dp]),
            "orc_problem_composition": (P, [i32, i32, u64, i32, ip, dp, dp, dp]),
            "orc_problem_paper_hybrid": (P, [i32, i32, u64]),
            "orc_problem_paper_composition": (P, [i32, i32, u64]),
            "orc_problem_fid": (P, [i32, i32, u64]),
            "orc_problem_free": (None, [P]),
            "orc_evaluate": (i32, [P, dp, i64, dp, i32]),
            "orc_problem_dim": (i32, [P]),
            "orc_problem_kind": (i32, [P]),
            "orc_problem_ncomp": (i32, [P]),
            "orc_problem_shift": (i32, [P, i32, dp]),
            "orc_problem_rotation": (i32, [P, i32, dp]),
            "orc_problem_hybrid_parts": (i32, [P, ip, ip, dp]),
            "orc_problem_transform": (i32, [P, dp, dp]),
            "orc_g": (f64, [i32, i32, dp]),
            "orc_stream_u64": (None, [u64, i32, u32, u32, i64, up]),
            "orc_stream_normal": (None, [u64, i32, u32, u32, i64, dp]),
            "orc_splitmix64_from_state": (u64, [u64, i64]),
            "orc_orthonormalise": (None, [i32, dp]),
            "orc_num_threads_available": (i32, []),
            "orc_table_xform": (i32, [i32, dp, dp, ip]),
            "orc_table_hybrid": (i32, [i32, dp, ip]),
            "orc_table_composition": (i32, [i32, dp, dp, ip]),
            "orc_problem_basic_params": (i32, [P, ip, dp, dp, ip]),
            "orc_problem_group_bases": (i32, [P, ip]),
            "orc_problem_blend_params": (i32, [P, dp, dp, dp]),
            "orc_problem_component": (P, [P, i32]),
            "orc_de_run": (f64, [P, i32, f64, f64, u64, u64, i32, dp, dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class Problem:
    """One oracle problem (basic, hybrid or composition).  A component of a composition is a
    borrowed view: it keeps its composition alive and never frees the handle itself."""

    def __init__(self, handle, owner=None):
        if not handle:
            raise ValueError("oracle rejected the problem definition")
        self._h = handle
        self._owner = owner
        self.dim = lib().orc_problem_dim(handle)
        self.kind = lib().orc_problem_kind(handle)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None and getattr(self, "_owner", None) is None:
            _lib.orc_problem_free(h)
        self._h = None

    def ncomp(self) -> int:
        """Components (composition), groups (hybrid) or 1 (basic)."""
        return int(lib().orc_problem_ncomp(self._h))

    def component(self, i: int) -> "Problem":
        """Component i of a composition (a basic or hybrid problem)."""
        h = lib().orc_problem_component(self._h, int(i))
        if not h:
            raise IndexError(i)
        return Problem(h, owner=self)

    def basic_params(self):
        """(formula id, s, c, rotated) a basic problem was built with."""
        b, r = ctypes.c_int(), ctypes.c_int()
        s, c = ctypes.c_double(), ctypes.c_double()
        assert lib().orc_problem_basic_params(self._h, ctypes.byref(b), ctypes.byref(s), ctypes.byref(c),
                                              ctypes.byref(r)) == 0
        return b.value, s.value, c.value, bool(r.value)

    def group_bases(self) -> list:
        out = np.zeros(16, dtype=np.int32)
        n = lib().orc_problem_group_bases(self._h, _ip(out))
        assert n > 0
        return [int(v) for v in out[:n]]

    def blend_params(self):
        """(sigma, lambda, bias) arrays of a composition."""
        a = [np.zeros(16) for _ in range(3)]
        n = lib().orc_problem_blend_params(self._h, *[_dp(v) for v in a])
        assert n > 0
        return tuple(v[:n].copy() for v in a)

    def __call__(self, x, threads: int = 1) -> np.ndarray:
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        if x.ndim == 1:
            x = x[None, :]
        assert x.shape[1] == self.dim
        f = np.empty(x.shape[0], dtype=np.float64)
        lib().orc_evaluate(self._h, _dp(x), x.shape[0], _dp(f), int(threads))
        return f

    def shift(self, comp: int = 0) -> np.ndarray:
        o = np.empty(self.dim)
        assert lib().orc_problem_shift(self._h, comp, _dp(o)) == 0
        return o

    def rotation(self, comp: int = 0) -> np.ndarray:
        R = np.empty((self.dim, self.dim))
        assert lib().orc_problem_rotation(self._h, comp, _dp(R)) == 0
        return R

    def hybrid_parts(self):
        perm = np.empty(self.dim, dtype=np.int32)
        sizes = np.zeros(16, dtype=np.int32)
        blocks = np.empty(self.dim * self.dim)
        ng = lib().orc_problem_hybrid_parts(self._h, _ip(perm), _ip(sizes), _dp(blocks))
        assert ng > 0
        sizes = sizes[:ng].copy()
        out, off = [], 0
        for n in sizes:
            out.append(blocks[off:off + n * n].reshape(n, n).copy())
            off += n * n
        return perm, sizes, out

    def de_run(self, pop, fit, F: float, CR: float, seed: int, gen0: int, generations: int) -> float:
        """DE/rand/1/bin for `generations` generations from generation gen0, updating the (np, D)
        array pop and the (np,) array fit in place; returns the closest selection margin."""
        assert pop.dtype == np.float64 and pop.flags.c_contiguous and fit.dtype == np.float64
        return float(lib().orc_de_run(self._h, pop.shape[0], F, CR, seed, gen0, generations, _dp(pop), _dp(fit)))

    def transform(self, x) -> np.ndarray:
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        z = np.empty(self.dim)
        assert lib().orc_problem_transform(self._h, _dp(x), _dp(z)) == 0
        return z


def basic(fid: int, dim: int, seed: int) -> Problem:
    """Tab. 1 function 0..22 with the transform its section states."""
    return Problem(lib().orc_problem_basic(fid, dim, seed))


def fid_problem(fid: int, dim: int, seed: int) -> Problem:
    """Any Tab. 1 id 0..36 (hybrids and compositions use the paper's fixed tables)."""
    return Problem(lib().orc_problem_fid(fid, dim, seed))


def custom_basic(pid: int, base: int, dim: int, seed: int, scale: float, offset: float, rotated: bool) -> Problem:
    return Problem(lib().orc_problem_custom_basic(pid, base, dim, seed, scale, offset, int(rotated)))


def hybrid(pid: int, dim: int, seed: int, bases, p) -> Problem:
    b = np.ascontiguousarray(bases, dtype=np.int32)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    return Problem(lib().orc_problem_hybrid(pid, dim, seed, len(b), _ip(b), _dp(pp)))


def composition(pid: int, dim: int, seed: int, bases, sigma, lam, bias) -> Problem:
    b = np.ascontiguousarray(bases, dtype=np.int32)
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    lm = np.ascontiguousarray(lam, dtype=np.float64)
    bi = np.ascontiguousarray(bias, dtype=np.float64)
    return Problem(lib().orc_problem_composition(pid, dim, seed, len(b), _ip(b), _dp(s), _dp(lm), _dp(bi)))


def table_xform(fid: int):
    """(s, c, rotated) as transcribed in the oracle's table for Tab. 1 function fid."""
    s, c, r = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    assert lib().orc_table_xform(int(fid), ctypes.byref(s), ctypes.byref(c), ctypes.byref(r)) == 0
    return s.value, c.value, bool(r.value)


def table_hybrid(fid: int):
    """(p, G ids) as transcribed in the oracle's table for hybrid fid (23..28)."""
    p = np.zeros(16)
    g = np.zeros(16, dtype=np.int32)
    n = lib().orc_table_hybrid(int(fid), _dp(p), _ip(g))
    assert n > 0
    return [float(v) for v in p[:n]], [int(v) for v in g[:n]]


def table_composition(fid: int):
    """(sigma, lambda, G ids) as transcribed in the oracle's table for composition fid (29..36)."""
    s, lm = np.zeros(16), np.zeros(16)
    g = np.zeros(16, dtype=np.int32)
    n = lib().orc_table_composition(int(fid), _dp(s), _dp(lm), _ip(g))
    assert n > 0
    return [float(v) for v in s[:n]], [float(v) for v in lm[:n]], [int(v) for v in g[:n]]


def g(fid: int, z) -> float:
    """Formula g(z) of Tab. 1 function 0..22 on a given z, without the bias."""
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    return float(lib().orc_g(fid, z.shape[0], _dp(z)))


def stream_u64(seed: int, dim: int, key: int, purpose: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    lib().orc_stream_u64(seed, dim, key, purpose, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def stream_normal(seed: int, dim: int, key: int, purpose: int, n: int) -> np.ndarray:
    out = np.empty(n)
    lib().orc_stream_normal(seed, dim, key, purpose, n, _dp(out))
    return out


def splitmix64_from_state(state: int, k: int) -> int:
    return int(lib().orc_splitmix64_from_state(state, k))


def orthonormalise(A) -> np.ndarray:
    A = np.ascontiguousarray(np.array(A, dtype=np.float64))
    lib().orc_orthonormalise(A.shape[0], _dp(A))
    return A


def threads_available() -> int:
    return int(lib().orc_num_threads_available())
