"""Python binding of libhk, the MI355X line-by-line opacity and
k-distribution library (Grimm & Heng 2015, HELIOS-K, arXiv:1503.03806).

Argument marshalling only: every numerical step runs in the HIP kernels of
``libhk.so`` behind the C ABI of ``include/hk.h``; the functions below carry
the same names.  PyTorch supplies device memory and streams.  There is no CPU
fallback: importing this package fails if ``libhk.so`` has not been built
(``python -m paper_1503_03806_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["HK_OK", "HK_EINVAL", "HK_ENOMEM", "HK_EDEVICE", "HK_EUNSUPPORTED", "HK_ENOTREADY",
           "HK_F64", "HK_F32_KAHAN", "HK_MAX_G", "HK_RULE_STEP", "HK_RULE_LINEAR", "HKError", "lib",
           "hk_version", "hk_create",
           "hk_destroy", "hk_set_stream", "hk_sync", "hk_last_error", "hk_load_lines",
           "hk_opacity", "hk_kdist", "hk_kdist_noalloc", "HK_KDIST_NOALLOC_SCRATCH_BYTES",
           "hk_gauss_legendre", "hk_stats", "hk_set_timing",
           "hk_get_timing", "hk_set_option", "hk_get_option", "hk_tables", "HK_F32_SURROGATE",
           "HK_SURR_N_PARAMS", "HK_SURR_CELLS_X", "HK_SURR_CELLS_Y", "hk_train_cfg",
           "hk_surrogate_labels", "hk_surrogate_set_params", "hk_surrogate_get_params",
           "hk_surrogate_grad", "hk_surrogate_train", "hk_surrogate_eval", "hk_surrogate_certify",
           "hk_surrogate_save", "hk_surrogate_load",
           "hk_resample", "hk_transmission", "hk_transmission_direct", "HK_MAX_COEF",
           "HK_TRANSMISSION_NODES", "hk_opacity_stream", "hk_read_par", "HK_MAX_CHUNKS", "Context",
           "LIB_PATH"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhk.so")

HK_OK, HK_EINVAL, HK_ENOMEM, HK_EDEVICE, HK_EUNSUPPORTED, HK_ENOTREADY = 0, -1, -2, -3, -4, -5
HK_F64, HK_F32_KAHAN, HK_F32_SURROGATE = 0, 1, 2
HK_SURR_N_PARAMS, HK_SURR_MAX_BATCH = 12737, 65536
HK_SURR_CELLS_X, HK_SURR_CELLS_Y = 80, 40
HK_MAX_COEF, HK_MAX_COLUMNS, HK_TRANSMISSION_NODES = 32, 1 << 20, 100
HK_MAX_G = 64
HK_RULE_STEP, HK_RULE_LINEAR = 0, 1
HK_MAX_POINTS = 1 << 30
HK_MAX_CHUNKS = 65536
HK_KDIST_NOALLOC_SCRATCH_BYTES = 64 << 20

_pd = C.POINTER(C.c_double)


LINE_FIELDS = ("nu", "S_ref", "E_lower", "gamma_air", "n_air", "gamma_self", "delta", "A21")


class hk_lines(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, _pd) for f in LINE_FIELDS]


class hk_lines_out(C.Structure):
    _fields_ = [("capacity", C.c_int64)] + [(f, _pd) for f in LINE_FIELDS]


class hk_species(C.Structure):
    _fields_ = [("T_ref", C.c_double), ("mass_amu", C.c_double)]


class hk_state(C.Structure):
    _fields_ = [("T", C.c_double), ("P", C.c_double), ("P_self", C.c_double),
                ("q_ratio", C.c_double), ("abundance", C.c_double)]


class hk_grid(C.Structure):
    _fields_ = [("nu_min", C.c_double), ("dnu", C.c_double), ("n_points", C.c_int64),
                ("cutoff", C.c_double), ("cutoff_lorentz", C.c_double)]


class hk_bins(C.Structure):
    _fields_ = [("points_per_bin", C.c_int64), ("n_g", C.c_int32), ("g", _pd), ("rule", C.c_int32)]


class hk_run_stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in ("evals", "evals_core", "evals_gh3", "evals_gh1",
                                         "n_lines", "evals_surrogate")]


HK_STAGE_LINE_PREP, HK_STAGE_OPACITY, HK_STAGE_KDIST, HK_STAGE_CORE, HK_N_STAGES = 0, 1, 2, 3, 4
STAGE_NAMES = ("line_prep", "opacity", "kdist", "core")


class hk_timing(C.Structure):
    _fields_ = [("ms", C.c_double * HK_N_STAGES), ("calls", C.c_int64 * HK_N_STAGES)]


class HKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libhk error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load libhk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhk.so is not built; run `python -m paper_1503_03806_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int, C.c_int64
        L.hk_version.argtypes = []; L.hk_version.restype = i32
        L.hk_create.argtypes = [i32, C.POINTER(vp)]; L.hk_create.restype = i32
        L.hk_destroy.argtypes = [vp]; L.hk_destroy.restype = i32
        L.hk_set_stream.argtypes = [vp, vp]; L.hk_set_stream.restype = i32
        L.hk_sync.argtypes = [vp]; L.hk_sync.restype = i32
        L.hk_last_error.argtypes = [vp]; L.hk_last_error.restype = C.c_char_p
        L.hk_load_lines.argtypes = [vp, C.POINTER(hk_lines), C.POINTER(hk_species), i32]
        L.hk_load_lines.restype = i32
        L.hk_opacity.argtypes = [vp, C.POINTER(hk_state), C.POINTER(hk_grid), i32, vp, vp, i32]
        L.hk_opacity.restype = i32
        L.hk_opacity_stream.argtypes = [vp, C.POINTER(hk_lines), C.c_int32, C.POINTER(hk_species),
                                        C.POINTER(hk_state), C.POINTER(hk_grid), i32, vp, i32]
        L.hk_opacity_stream.restype = i32
        L.hk_read_par.argtypes = [C.c_char_p, i64, C.c_int32, C.POINTER(hk_lines_out),
                                  C.POINTER(i64), C.POINTER(i64)]
        L.hk_read_par.restype = i32
        L.hk_kdist.argtypes = [vp, vp, i32, i64, C.POINTER(hk_bins), vp, vp]
        L.hk_kdist.restype = i32
        L.hk_kdist_noalloc.argtypes = [vp, vp, i32, i64, C.POINTER(hk_bins), vp, vp]
        L.hk_kdist_noalloc.restype = i32
        L.hk_gauss_legendre.argtypes = [C.c_int32, _pd, _pd]; L.hk_gauss_legendre.restype = i32
        L.hk_stats.argtypes = [vp, C.POINTER(hk_run_stats)]; L.hk_stats.restype = i32
        L.hk_set_timing.argtypes = [vp, i32]; L.hk_set_timing.restype = i32
        L.hk_set_option.argtypes = [vp, C.c_char_p, i64]; L.hk_set_option.restype = i32
        L.hk_get_option.argtypes = [vp, C.c_char_p, C.POINTER(i64)]; L.hk_get_option.restype = i32
        L.hk_tables.argtypes = [vp, C.POINTER(hk_state), C.c_int32, C.POINTER(hk_grid),
                                C.POINTER(hk_bins), i32, vp]
        L.hk_tables.restype = i32
        L.hk_surrogate_labels.argtypes = [vp, vp, vp, i64, vp]
        L.hk_surrogate_set_params.argtypes = [vp, vp]
        L.hk_surrogate_get_params.argtypes = [vp, vp]
        L.hk_surrogate_grad.argtypes = [vp, vp, vp, vp, i64, C.c_double, vp, vp]
        L.hk_surrogate_train.argtypes = [vp, vp, vp, vp, i64, C.POINTER(hk_train_cfg), vp]
        L.hk_surrogate_eval.argtypes = [vp, vp, vp, i64, vp, vp]
        L.hk_surrogate_certify.argtypes = [vp, C.c_double, vp, C.POINTER(C.c_int32)]
        L.hk_surrogate_save.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        L.hk_surrogate_load.argtypes = [vp, vp, C.c_size_t]
        L.hk_resample.argtypes = [vp, vp, i32, i64, i64, C.c_int32, vp]
        L.hk_transmission.argtypes = [vp, vp, i64, C.c_int32, vp, C.c_int32, vp]
        L.hk_transmission_direct.argtypes = [vp, vp, i32, i64, i64, vp, C.c_int32, vp]
        for f in ("hk_resample", "hk_transmission", "hk_transmission_direct"):
            getattr(L, f).restype = i32
        for f in ("labels", "set_params", "get_params", "grad", "train", "eval", "certify", "save", "load"):
            getattr(L, "hk_surrogate_" + f).restype = i32
        L.hk_get_timing.argtypes = [vp, C.POINTER(hk_timing)]; L.hk_get_timing.restype = i32
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != HK_OK:
        raise HKError(rc, hk_last_error(ctx))
    return rc


def _ptr(t):
    """Raw pointer of a tensor / numpy array (None -> NULL)."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data


def hk_version() -> int:
    return lib().hk_version()


def hk_last_error(ctx=None) -> str:
    s = lib().hk_last_error(ctx)
    return s.decode() if s else ""


def hk_create(device: int = 0):
    h = C.c_void_p()
    _check(lib().hk_create(device, C.byref(h)))
    return h


def hk_destroy(ctx):
    return lib().hk_destroy(ctx)


def hk_set_stream(ctx, stream_ptr):
    _check(lib().hk_set_stream(ctx, stream_ptr), ctx)


def hk_sync(ctx):
    _check(lib().hk_sync(ctx), ctx)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _lines(lines: dict):
    """(hk_lines, the arrays it points into: keep them alive)."""
    keep = {k: _f64(lines.get(k)) for k in LINE_FIELDS}
    n = len(keep["nu"])
    for k, v in keep.items():
        if v is not None and len(v) != n:
            raise ValueError("line field %s has %d values, expected %d" % (k, len(v), n))
    fld = [None if v is None else v.ctypes.data_as(_pd) for v in keep.values()]
    return hk_lines(n, *fld), keep


def _species(species: dict) -> hk_species:
    return hk_species(float(species.get("T_ref", 296.0)), float(species["mass_amu"]))


def _lines_device(lines: dict):
    """hk_lines over device tensors (contiguous float64, one length)."""
    ptrs, n = [], None
    for k in LINE_FIELDS:
        v = lines.get(k)
        if v is None:
            ptrs.append(None)
            continue
        if str(v.dtype) != "torch.float64" or not v.is_contiguous() or v.dim() != 1:
            raise ValueError("device line field %s must be a contiguous 1-D float64 tensor" % k)
        if n is None:
            n = v.numel()
        elif v.numel() != n:
            raise ValueError("line field %s has %d values, expected %d" % (k, v.numel(), n))
        ptrs.append(C.cast(C.c_void_p(v.data_ptr()), _pd))
    return hk_lines(n or 0, *ptrs)


def _on_device(lines: dict) -> bool:
    v = lines.get("nu")
    return hasattr(v, "is_cuda") and bool(v.is_cuda)


def hk_load_lines(ctx, lines: dict, species: dict):
    """lines: dict of arrays (nu, S_ref, E_lower, gamma_air, n_air and
    optional gamma_self, delta, A21), all host arrays or all device tensors
    (float64; then lines_on_device = 1); species: {T_ref, mass_amu}."""
    sp = _species(species)
    if _on_device(lines):
        s = _lines_device(lines)
        _check(lib().hk_load_lines(ctx, C.byref(s), C.byref(sp), 1), ctx)
    else:
        s, keep = _lines(lines)
        _check(lib().hk_load_lines(ctx, C.byref(s), C.byref(sp), 0), ctx)


def hk_opacity_stream(ctx, chunks, species: dict, state: dict, grid: dict, precision: int, kappa,
                      accumulate: bool = False):
    """chunks: a sequence of line dicts (as hk_load_lines takes)."""
    made = [_lines(c) for c in chunks]
    arr = (hk_lines * max(len(made), 1))(*[m[0] for m in made])
    sp, st, gr = _species(species), _state(state), _grid(grid)
    _check(lib().hk_opacity_stream(ctx, arr if made else None, len(made), C.byref(sp), C.byref(st),
                                   C.byref(gr), int(precision), _ptr(kappa), 1 if accumulate else 0),
           ctx)


def hk_read_par(path: str, first: int = 0, capacity: int = 1 << 20, molecule: int = 0):
    """Read up to `capacity` HITRAN-format records from record `first`:
    (dict of float64 arrays, n_read, next)."""
    arrays = {k: np.empty(max(int(capacity), 1)) for k in LINE_FIELDS}
    out = hk_lines_out(int(capacity), *[arrays[k].ctypes.data_as(_pd) for k in LINE_FIELDS])
    n_read, nxt = C.c_int64(0), C.c_int64(0)
    _check(lib().hk_read_par(os.fsencode(path), int(first), int(molecule), C.byref(out),
                             C.byref(n_read), C.byref(nxt)))
    n = n_read.value
    return {k: v[:n].copy() for k, v in arrays.items()}, n, nxt.value


def _state(st: dict) -> hk_state:
    P = float(st["P"])
    return hk_state(float(st["T"]), P, float(st.get("P_self", 0.5 * P)),
                    float(st.get("q_ratio", 1.0)), float(st.get("abundance", 1.0)))


def _grid(g: dict) -> hk_grid:
    return hk_grid(float(g["nu_min"]), float(g["dnu"]), int(g["n_points"]), float(g["cutoff"]),
                   float(g.get("cutoff_lorentz", 0.0)))


def hk_opacity(ctx, state: dict, grid: dict, precision: int, kappa, comp=None,
               accumulate: bool = False):
    st, gr = _state(state), _grid(grid)
    _check(lib().hk_opacity(ctx, C.byref(st), C.byref(gr), int(precision), _ptr(kappa),
                            _ptr(comp), 1 if accumulate else 0), ctx)


def hk_kdist(ctx, kappa, precision: int, n_points: int, points_per_bin: int, g, k_out,
             sorted_out=None, rule: int = 0):
    gg = _f64(g)
    b = hk_bins(int(points_per_bin), len(gg), gg.ctypes.data_as(_pd), int(rule))
    _check(lib().hk_kdist(ctx, _ptr(kappa), int(precision), int(n_points), C.byref(b),
                          _ptr(k_out), _ptr(sorted_out)), ctx)


def hk_kdist_noalloc(ctx, kappa, precision: int, n_points: int, points_per_bin: int, g, k_out,
                     sorted_out=None, rule: int = 0):
    """hk_kdist that allocates nothing (a fixed device array serves large
    bins; see hk.h)."""
    gg = _f64(g)
    b = hk_bins(int(points_per_bin), len(gg), gg.ctypes.data_as(_pd), int(rule))
    _check(lib().hk_kdist_noalloc(ctx, _ptr(kappa), int(precision), int(n_points), C.byref(b),
                                  _ptr(k_out), _ptr(sorted_out)), ctx)


def hk_tables(ctx, states, grid: dict, points_per_bin: int, g, precision: int, k_out,
              rule: int = 0):
    """states: sequence of state dicts; k_out: device tensor
    [len(states)][n_bins][len(g)] of float64."""
    arr = (hk_state * max(len(states), 1))(*[_state(s) for s in states])
    gr = _grid(grid)
    gg = _f64(g)
    b = hk_bins(int(points_per_bin), len(gg), gg.ctypes.data_as(_pd), int(rule))
    _check(lib().hk_tables(ctx, arr, len(states), C.byref(gr), C.byref(b), int(precision),
                           _ptr(k_out)), ctx)


class hk_train_cfg(C.Structure):
    _fields_ = [("batch", C.c_int32), ("steps", C.c_int32), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("wscale", C.c_double)]


def hk_surrogate_labels(ctx, x, y, z):
    _check(lib().hk_surrogate_labels(ctx, _ptr(x), _ptr(y), _numel(x, y), _ptr(z)), ctx)


def hk_surrogate_set_params(ctx, theta):
    t = np.ascontiguousarray(theta, dtype=np.float32)
    if t.shape != (HK_SURR_N_PARAMS,):
        raise ValueError("theta must hold %d values" % HK_SURR_N_PARAMS)
    _check(lib().hk_surrogate_set_params(ctx, t.ctypes.data), ctx)


def hk_surrogate_get_params(ctx) -> np.ndarray:
    t = np.empty(HK_SURR_N_PARAMS, dtype=np.float32)
    _check(lib().hk_surrogate_get_params(ctx, t.ctypes.data), ctx)
    return t


def hk_surrogate_grad(ctx, x, y, z, grad, loss=None, wscale: float = 0.0):
    _check(lib().hk_surrogate_grad(ctx, _ptr(x), _ptr(y), _ptr(z), _numel(x, y, z), float(wscale),
                                   _ptr(grad), _ptr(loss)), ctx)


def hk_surrogate_train(ctx, x, y, z, batch: int, steps: int, lr: float, beta1: float = 0.9,
                       beta2: float = 0.999, eps: float = 1e-8, wscale: float = 0.0, loss_hist=None):
    cfg = hk_train_cfg(int(batch), int(steps), float(lr), float(beta1), float(beta2), float(eps),
                       float(wscale))
    _check(lib().hk_surrogate_train(ctx, _ptr(x), _ptr(y), _ptr(z), _numel(x, y, z), C.byref(cfg),
                                    _ptr(loss_hist)), ctx)


def hk_surrogate_eval(ctx, x, y, z, K=None):
    _check(lib().hk_surrogate_eval(ctx, _ptr(x), _ptr(y), _numel(x, y), _ptr(z), _ptr(K)), ctx)


def hk_surrogate_certify(ctx, budget: float):
    err = np.empty((HK_SURR_CELLS_Y, HK_SURR_CELLS_X))
    cnt = C.c_int32(0)
    _check(lib().hk_surrogate_certify(ctx, float(budget), err.ctypes.data, C.byref(cnt)), ctx)
    return err, int(cnt.value)


def hk_surrogate_save(ctx) -> bytes:
    """The trained (and, if done, certified) surrogate as a byte string."""
    n = C.c_size_t(0)
    _check(lib().hk_surrogate_save(ctx, None, 0, C.byref(n)), ctx)
    buf = C.create_string_buffer(n.value)
    _check(lib().hk_surrogate_save(ctx, buf, n.value, C.byref(n)), ctx)
    return buf.raw[:n.value]


def hk_surrogate_load(ctx, blob: bytes):
    b = bytes(blob)
    _check(lib().hk_surrogate_load(ctx, C.c_char_p(b), len(b)), ctx)


def _count(a) -> int:
    return int(a.numel() if hasattr(a, "numel") else len(a))


def _numel(*arrays) -> int:
    n = {int(a.numel() if hasattr(a, "numel") else len(a)) for a in arrays}
    if len(n) != 1:
        raise ValueError("arrays differ in length: %s" % sorted(n))
    for a in arrays:
        if hasattr(a, "dtype") and str(a.dtype) not in ("torch.float32", "float32"):
            raise ValueError("surrogate arrays are float32 (got %s)" % a.dtype)
    return n.pop()


def hk_resample(ctx, sorted_kappa, precision: int, n_points: int, points_per_bin: int, n_coef: int,
                coef_out):
    _check(lib().hk_resample(ctx, _ptr(sorted_kappa), int(precision), int(n_points),
                             int(points_per_bin), int(n_coef), _ptr(coef_out)), ctx)


def hk_transmission(ctx, coef, n_bins: int, n_coef: int, m_col, T_out):
    _check(lib().hk_transmission(ctx, _ptr(coef), int(n_bins), int(n_coef), _ptr(m_col),
                                 _count(m_col), _ptr(T_out)), ctx)


def hk_transmission_direct(ctx, sorted_kappa, precision: int, n_points: int, points_per_bin: int,
                           m_col, T_out):
    _check(lib().hk_transmission_direct(ctx, _ptr(sorted_kappa), int(precision), int(n_points),
                                        int(points_per_bin), _ptr(m_col), _count(m_col),
                                        _ptr(T_out)), ctx)


def hk_gauss_legendre(n: int):
    g = np.empty(n); w = np.empty(n)
    _check(lib().hk_gauss_legendre(int(n), g.ctypes.data_as(_pd), w.ctypes.data_as(_pd)))
    return g, w


def hk_stats(ctx) -> dict:
    s = hk_run_stats()
    _check(lib().hk_stats(ctx, C.byref(s)), ctx)
    return {f: int(getattr(s, f)) for f, _ in hk_run_stats._fields_}


def hk_set_option(ctx, name: str, value: int):
    _check(lib().hk_set_option(ctx, name.encode(), int(value)), ctx)


def hk_get_option(ctx, name: str) -> int:
    v = C.c_int64(0)
    _check(lib().hk_get_option(ctx, name.encode(), C.byref(v)), ctx)
    return int(v.value)


def hk_set_timing(ctx, enable: bool):
    _check(lib().hk_set_timing(ctx, 1 if enable else 0), ctx)


def hk_get_timing(ctx) -> dict:
    t = hk_timing()
    _check(lib().hk_get_timing(ctx, C.byref(t)), ctx)
    return {name: (float(t.ms[i]), int(t.calls[i])) for i, name in enumerate(STAGE_NAMES)}


class Context:
    """A libhk context bound to a CUDA/HIP device and torch's current stream.

    Allocates outputs as torch tensors; everything else is the C ABI."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.device = device
        self.h = hk_create(device)
        self.use_current_stream()

    def use_current_stream(self):
        torch = self._torch
        with torch.cuda.device(self.device):
            hk_set_stream(self.h, torch.cuda.current_stream().cuda_stream)

    def close(self):
        if self.h is not None:
            hk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_lines(self, lines: dict, mass_amu: float, T_ref: float = 296.0):
        hk_load_lines(self.h, lines, {"T_ref": T_ref, "mass_amu": mass_amu})

    def opacity_stream(self, chunks, mass_amu: float, state: dict, grid: dict,
                       precision: int = HK_F64, out=None, accumulate: bool = False,
                       T_ref: float = 296.0):
        torch = self._torch
        n = int(grid["n_points"])
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda:%d" % self.device)[:n]
        hk_opacity_stream(self.h, chunks, {"T_ref": T_ref, "mass_amu": mass_amu}, state, grid,
                          precision, out, accumulate)
        return out

    def opacity(self, state: dict, grid: dict, precision: int = HK_F64, out=None, comp=None,
                accumulate: bool = False):
        torch = self._torch
        n = int(grid["n_points"])
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda:%d" % self.device)[:n]
        hk_opacity(self.h, state, grid, precision, out, comp, accumulate)
        return out

    def kdist(self, kappa, points_per_bin: int, g, precision: int = HK_F64, sorted_out=None,
              rule: int = 0):
        torch = self._torch
        n = kappa.numel()
        n_bins = -(-n // points_per_bin)
        k = torch.empty((max(n_bins, 1), len(g)), dtype=torch.float64,
                        device="cuda:%d" % self.device)[:n_bins]
        hk_kdist(self.h, kappa, precision, n, points_per_bin, g, k, sorted_out, rule)
        return k

    def tables(self, states, grid: dict, points_per_bin: int, g, precision: int = HK_F32_KAHAN,
               out=None, rule: int = 0):
        torch = self._torch
        n = int(grid["n_points"])
        n_bins = -(-n // points_per_bin)
        if out is None:
            out = torch.empty((len(states), n_bins, len(g)), dtype=torch.float64,
                              device="cuda:%d" % self.device)
        hk_tables(self.h, states, grid, points_per_bin, g, precision, out, rule)
        return out

    # -- resampling and transmission (float64 device tensors) --
    def resample(self, sorted_kappa, points_per_bin: int, n_coef: int = 20, precision: int = HK_F64):
        torch = self._torch
        n = sorted_kappa.numel()
        n_bins = -(-n // points_per_bin)
        coef = torch.empty((n_bins, n_coef), dtype=torch.float64, device=sorted_kappa.device)
        hk_resample(self.h, sorted_kappa, precision, n, points_per_bin, n_coef, coef)
        return coef

    def transmission(self, coef, m_col):
        torch = self._torch
        T = torch.empty((coef.shape[0], m_col.numel()), dtype=torch.float64, device=coef.device)
        hk_transmission(self.h, coef, coef.shape[0], coef.shape[1], m_col, T)
        return T

    def transmission_direct(self, sorted_kappa, points_per_bin: int, m_col, precision: int = HK_F64):
        torch = self._torch
        n = sorted_kappa.numel()
        T = torch.empty((-(-n // points_per_bin), m_col.numel()), dtype=torch.float64,
                        device=sorted_kappa.device)
        hk_transmission_direct(self.h, sorted_kappa, precision, n, points_per_bin, m_col, T)
        return T

    # -- learned surrogate (float32 device tensors) --
    def surrogate_labels(self, x, y):
        z = self._torch.empty_like(x)
        hk_surrogate_labels(self.h, x, y, z)
        return z

    def surrogate_set_params(self, theta):
        hk_surrogate_set_params(self.h, theta)

    def surrogate_params(self):
        return hk_surrogate_get_params(self.h)

    def surrogate_grad(self, x, y, z, wscale: float = 0.0):
        torch = self._torch
        g = torch.empty(HK_SURR_N_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        hk_surrogate_grad(self.h, x, y, z, g, loss, wscale)
        return g, loss

    def surrogate_train(self, x, y, z, batch: int, steps: int, lr: float, **kw):
        torch = self._torch
        hist = torch.empty(max(steps, 1), dtype=torch.float32, device=x.device)
        hk_surrogate_train(self.h, x, y, z, batch, steps, lr, loss_hist=hist, **kw)
        return hist[:steps]

    def surrogate_eval(self, x, y):
        z = self._torch.empty_like(x)
        K = self._torch.empty_like(x)
        hk_surrogate_eval(self.h, x, y, z, K)
        return z, K

    def surrogate_save(self) -> bytes:
        return hk_surrogate_save(self.h)

    def surrogate_load(self, blob: bytes):
        hk_surrogate_load(self.h, blob)

    def surrogate_certify(self, budget: float):
        return hk_surrogate_certify(self.h, budget)

    def sync(self):
        hk_sync(self.h)

    def stats(self) -> dict:
        return hk_stats(self.h)

    def set_option(self, name: str, value: int):
        hk_set_option(self.h, name, value)

    def get_option(self, name: str) -> int:
        return hk_get_option(self.h, name)

    def set_timing(self, enable: bool = True):
        hk_set_timing(self.h, enable)

    def timing(self) -> dict:
        return hk_get_timing(self.h)
