"""Plain FP64 CPU oracle for the HELIOS-K opacity / k-distribution method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It wraps
``liboracle.so`` (plain C, see ``oracle.c``) with ctypes and shares no code
with the GPU library; the product path never imports it.

Every function follows the paper (Grimm & Heng 2015, arXiv:1503.03806) in its
own notation; the section and equation are named in ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

# -O3 without fast-math and without floating-point contraction: every
# expression is evaluated as written, in the order written, so the results
# are the same bits whatever the instruction set.  The in-tree library
# targets x86-64-v2 (it may run on another host than the one that built it);
# the timed baseline builds a -march=native copy on the host it runs on.
_FLAGS = ["-std=gnu11", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False, native: bool = False, path: str | None = None) -> str:
    """Compile the oracle with gcc (see _FLAGS): ``liboracle.so`` for
    x86-64-v2, or with native=True a copy for this host's own CPU at `path`."""
    src = os.path.join(_HERE, "oracle.c")
    so = path or _SO
    if native or force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        tmp = so + ".tmp%d" % os.getpid()
        arch = "-march=native" if native else "-march=x86-64-v2"
        subprocess.run(["gcc"] + _FLAGS + [arch, "-o", tmp, src, "-lm"], check=True)
        os.replace(tmp, so)
    return so


def use_native(path: str) -> None:
    """Build a -march=native copy of the oracle at `path` and use it for
    every later call of this module (the timed CPU baseline)."""
    global _lib, _SO
    build(native=True, path=path)
    _SO = path
    _lib = None


class _Lines(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, C.POINTER(C.c_double)) for f in (
        "nu", "S_ref", "E_lower", "gamma_air", "n_air", "gamma_self", "delta", "A21")]


class _Cond(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("T0", "mass_amu", "T", "P", "P_self", "q_ratio")]


class _Grid(C.Structure):
    _fields_ = [("nu_min", C.c_double), ("dnu", C.c_double),
                ("n_points", C.c_int64), ("cutoff", C.c_double), ("cutoff_lorentz", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        build()  # rebuilds when oracle.c is newer than the library
        L = C.CDLL(_SO)
        d, i64, i32 = C.c_double, C.c_int64, C.c_int
        pd = C.POINTER(C.c_double)
        pi64 = C.POINTER(C.c_int64)
        L.ora_const.argtypes = [i32]; L.ora_const.restype = d
        L.ora_line_strength.argtypes = [d] * 6; L.ora_line_strength.restype = d
        L.ora_doppler_hwhm.argtypes = [d] * 3; L.ora_doppler_hwhm.restype = d
        L.ora_lorentz_hwhm.argtypes = [d] * 8; L.ora_lorentz_hwhm.restype = d
        for f in ("ora_voigt_H", "ora_voigt_series", "ora_voigt_gh3", "ora_voigt_gh1"):
            getattr(L, f).argtypes = [d, d]; getattr(L, f).restype = d
        L.ora_erfcx.argtypes = [d]; L.ora_erfcx.restype = d
        L.ora_voigt_vec.argtypes = [i32, i64, pd, pd, pd]; L.ora_voigt_vec.restype = i32
        L.ora_window.argtypes = [d, d, d, d, i64, pi64, pi64]; L.ora_window.restype = i64
        L.ora_opacity.argtypes = [C.POINTER(_Lines), C.POINTER(_Cond), C.POINTER(_Grid),
                                  i64, i64, pd]
        L.ora_opacity.restype = i64
        L.ora_eval_counts.argtypes = [C.POINTER(_Lines), C.POINTER(_Cond), C.POINTER(_Grid), pi64]
        L.ora_eval_counts.restype = i32
        L.ora_gauss_legendre.argtypes = [i32, pd, pd]; L.ora_gauss_legendre.restype = i32
        L.ora_kdist_bin.argtypes = [pd, i64, i32, pd, i32, pd, pd]; L.ora_kdist_bin.restype = i32
        L.ora_kdist.argtypes = [pd, i64, i64, i32, pd, i32, pd]; L.ora_kdist.restype = i32
        L.ora_num_threads.argtypes = []; L.ora_num_threads.restype = i32
        L.ora_set_num_threads.argtypes = [i32]; L.ora_set_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def const(name: str) -> float:
    return lib().ora_const({"c": 0, "kB": 1, "h": 2, "amu": 3, "c2": 4}[name])


def num_threads() -> int:
    return lib().ora_num_threads()


def set_num_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the count."""
    return lib().ora_set_num_threads(int(n))


# ---- §2.3 ------------------------------------------------------------------

def line_strength(S0, E_lower, nu, T, T0=296.0, q_ratio=1.0):
    f = lib().ora_line_strength
    return np.vectorize(lambda s, e, n: f(s, e, n, T, T0, q_ratio))(S0, E_lower, nu)


def doppler_hwhm(nu, T, mass_amu):
    f = lib().ora_doppler_hwhm
    return np.vectorize(lambda n: f(n, T, mass_amu))(nu)


def lorentz_hwhm(A21, n_coll, gamma_air, gamma_self, T, T0, P, P_self):
    f = lib().ora_lorentz_hwhm
    return np.vectorize(lambda A, n, ga, gs: f(A, n, ga, gs, T, T0, P, P_self))(
        A21, n_coll, gamma_air, gamma_self)


# ---- §2.4 ------------------------------------------------------------------

def _voigt(which, a, u):
    a, u = np.broadcast_arrays(_f64(a), _f64(u))
    a, u = _f64(a).ravel(), _f64(u).ravel()
    out = np.empty_like(a)
    rc = lib().ora_voigt_vec(which, a.size, _p(a), _p(u), _p(out))
    assert rc == 0
    return out


def voigt_H(a, u):
    """Three-region scheme of §2.4 for H_V(a, u)."""
    return _voigt(0, a, u)


def voigt_series(a, u):
    return _voigt(1, a, u)


def voigt_gh3(a, u):
    return _voigt(2, a, u)


def voigt_gh1(a, u):
    return _voigt(3, a, u)


def erfcx(t):
    f = lib().ora_erfcx
    return np.vectorize(f)(t)


def window(nu0_shifted, cutoff, nu_min, dnu, n_points):
    lo, hi = C.c_int64(), C.c_int64()
    n = lib().ora_window(nu0_shifted, cutoff, nu_min, dnu, n_points, C.byref(lo), C.byref(hi))
    return int(lo.value), int(hi.value), int(n)


# ---- opacity grid -------------------------------------------------------------

def _structs(lines, cond, grid):
    keep = {}

    def arr(k):
        v = lines.get(k)
        if v is None:
            return None
        keep[k] = _f64(v)
        return _p(keep[k])

    n = len(lines["nu"])
    Ls = _Lines(n, *[arr(k) for k in ("nu", "S_ref", "E_lower", "gamma_air", "n_air",
                                       "gamma_self", "delta", "A21")])
    cs = _Cond(cond.get("T0", 296.0), cond["mass_amu"], cond["T"], cond["P"],
               cond.get("P_self", 0.5 * cond["P"]), cond.get("q_ratio", 1.0))
    gs = _Grid(grid["nu_min"], grid["dnu"], int(grid["n_points"]), grid["cutoff"],
               float(grid.get("cutoff_lorentz", 0.0)))
    return Ls, cs, gs, keep


def opacity(lines: dict, cond: dict, grid: dict, j_begin: int = 0, j_end: int | None = None):
    """kappa_j (cm^2/molecule) for j in [j_begin, j_end); returns (kappa, evals)."""
    Ls, cs, gs, keep = _structs(lines, cond, grid)
    if j_end is None:
        j_end = gs.n_points
    out = np.empty(max(j_end - j_begin, 1), dtype=np.float64)
    n = lib().ora_opacity(C.byref(Ls), C.byref(cs), C.byref(gs), j_begin, j_end, _p(out))
    if n < 0:
        raise ValueError("ora_opacity rejected its input (%d)" % n)
    return out[: j_end - j_begin], int(n)


def eval_counts(lines: dict, cond: dict, grid: dict):
    """(total, core, gh3, gh1) line-point evaluation counts."""
    Ls, cs, gs, keep = _structs(lines, cond, grid)
    cnt = (C.c_int64 * 4)()
    rc = lib().ora_eval_counts(C.byref(Ls), C.byref(cs), C.byref(gs), cnt)
    if rc != 0:
        raise ValueError("ora_eval_counts rejected its input")
    return tuple(int(v) for v in cnt)


# ---- §2.2 ------------------------------------------------------------------

def gauss_legendre(n: int):
    x = np.empty(n); w = np.empty(n)
    assert lib().ora_gauss_legendre(n, _p(x), _p(w)) == 0
    return x, w


def g_nodes(n: int = 20):
    """Gauss-Legendre nodes mapped to (0, 1): g = (1 + xi)/2."""
    x, w = gauss_legendre(n)
    return 0.5 * (1.0 + x), 0.5 * w


def kdist_bin(kappa, g, rule: int = 0):
    """k(g) of one bin: rule 0 step, rule 1 midpoint-linear (oracle.h)."""
    kappa = _f64(kappa); g = _f64(g)
    out = np.empty(len(g)); srt = np.empty(len(kappa))
    rc = lib().ora_kdist_bin(_p(kappa), kappa.size, len(g), _p(g), int(rule), _p(out), _p(srt))
    if rc != 0:
        raise ValueError("ora_kdist_bin rejected its input")
    return out, srt


def kdist(kappa, points_per_bin: int, g, rule: int = 0):
    kappa = _f64(kappa); g = _f64(g)
    n_bins = -(-kappa.size // points_per_bin)
    out = np.empty((n_bins, len(g)))
    rc = lib().ora_kdist(_p(kappa), kappa.size, points_per_bin, len(g), _p(g), int(rule), _p(out))
    if rc != 0:
        raise ValueError("ora_kdist rejected its input")
    return out
