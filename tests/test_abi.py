"""Host-side checks of the C ABI: the library loads and exports every symbol
include/hk.h declares, argument validation rejects bad input before any
device work, and the host helpers match their definitions.  No GPU needed."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1503_03806_amd as hk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hk.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hk_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "hk_opacity" in names and "hk_kdist" in names and len(names) >= 11
    L = C.CDLL(hk.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", hk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (hk_[a-z0-9_]+)\b", out))
    assert set(names) <= exported


def test_header_compiles_as_c():
    src = '#include "hk.h"\nint main(void){hk_ctx* c = 0; return hk_sync(c) == HK_EINVAL ? 0 : 1;}\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I",
                        os.path.dirname(HEADER), "-x", "c", "-"], input=src, text=True,
                       capture_output=True)
    assert r.returncode == 0, r.stderr


def test_version_and_last_error():
    assert hk.hk_version() >= 100
    assert isinstance(hk.hk_last_error(None), str)


GOOD_STATE = {"T": 1500.0, "P": 1.0, "P_self": 0.5, "q_ratio": 0.1}
GOOD_GRID = {"nu_min": 0.0, "dnu": 0.01, "n_points": 1000, "cutoff": 25.0}


def _opacity_rc(state, grid, precision=hk.HK_F64, kappa=1, comp=None):
    st, gr = hk._state(state), hk._grid(grid)
    return hk.lib().hk_opacity(None, C.byref(st), C.byref(gr), precision, kappa, comp, 0)


@pytest.mark.parametrize("field,value,msg", [
    ("T", 0.0, "T must"), ("T", float("nan"), "T must"), ("P", -1.0, "P must"),
    ("P_self", 2.0, "P_self"), ("q_ratio", 0.0, "q_ratio"), ("abundance", -0.5, "abundance"),
    ("abundance", float("inf"), "abundance")])
def test_opacity_rejects_bad_state(field, value, msg):
    st = dict(GOOD_STATE); st[field] = value
    assert _opacity_rc(st, GOOD_GRID) == hk.HK_EINVAL
    assert msg in hk.hk_last_error(None)


@pytest.mark.parametrize("field,value,msg", [
    ("dnu", 0.0, "dnu"), ("dnu", -0.01, "dnu"), ("n_points", -1, "n_points"),
    ("n_points", (1 << 30) + 1, "n_points"), ("cutoff", -1.0, "cutoff"),
    ("nu_min", float("inf"), "nu_min")])
def test_opacity_rejects_bad_grid(field, value, msg):
    g = dict(GOOD_GRID); g[field] = value
    assert _opacity_rc(GOOD_STATE, g) == hk.HK_EINVAL
    assert msg in hk.hk_last_error(None)


def test_opacity_rejects_bad_precision_and_buffers():
    assert _opacity_rc(GOOD_STATE, GOOD_GRID, precision=7) == hk.HK_EINVAL
    assert _opacity_rc(GOOD_STATE, GOOD_GRID, kappa=None) == hk.HK_EINVAL
    assert "kappa" in hk.hk_last_error(None)
    # valid arguments reach the context check
    assert _opacity_rc(GOOD_STATE, GOOD_GRID) == hk.HK_EINVAL
    assert "context" in hk.hk_last_error(None)


def test_kdist_rejects_bad_bins():
    g = np.array([0.1, 0.5])

    def rc(ppb, gv, n_points=100, rule=hk.HK_RULE_STEP):
        gg = np.ascontiguousarray(gv, dtype=np.float64)
        b = hk.hk_bins(ppb, len(gg), gg.ctypes.data_as(C.POINTER(C.c_double)), rule)
        return hk.lib().hk_kdist(None, 1, hk.HK_F64, n_points, C.byref(b), 1, None)
    assert rc(0, g) == hk.HK_EINVAL and "points_per_bin" in hk.hk_last_error(None)
    assert rc(10, [0.0, 0.5]) == hk.HK_EINVAL and "(0, 1)" in hk.hk_last_error(None)
    assert rc(10, [0.5, 1.0]) == hk.HK_EINVAL
    assert rc(10, np.full(65, 0.5)) == hk.HK_EINVAL and "n_g" in hk.hk_last_error(None)
    assert rc(10, g, n_points=-1) == hk.HK_EINVAL
    assert rc(10, g, rule=2) == hk.HK_EINVAL and "rule 2" in hk.hk_last_error(None)
    assert rc(10, g, rule=-1) == hk.HK_EINVAL and "rule -1" in hk.hk_last_error(None)
    assert rc(10, g) == hk.HK_EINVAL and "context" in hk.hk_last_error(None)
    assert rc(10, g, rule=hk.HK_RULE_LINEAR) == hk.HK_EINVAL and "context" in hk.hk_last_error(None)


def test_load_lines_rejects_bad_lists():
    base = {"nu": np.array([100.0, 200.0]), "S_ref": np.array([1e-20, 1e-21]),
            "E_lower": np.array([10.0, 20.0]), "gamma_air": np.array([0.05, 0.06]),
            "n_air": np.array([0.5, 0.6])}
    for k, v, msg in [("nu", [0.0, 1.0], "nu[0]"), ("nu", [1.0, float("nan")], "nu[1]"),
                      ("S_ref", [-1.0, 1.0], "S_ref"), ("gamma_air", [0.1, -0.1], "gamma_air"),
                      ("E_lower", [np.inf, 1.0], "E_lower")]:
        L = dict(base); L[k] = np.array(v)
        with pytest.raises(hk.HKError) as e:
            hk.hk_load_lines(None, L, {"mass_amu": 18.0})
        assert e.value.code == hk.HK_EINVAL and msg in str(e.value)
    with pytest.raises(hk.HKError) as e:
        hk.hk_load_lines(None, base, {"mass_amu": 0.0})
    assert "mass_amu" in str(e.value)
    with pytest.raises(hk.HKError) as e:
        hk.hk_load_lines(None, base, {"mass_amu": 18.0})
    assert "context" in str(e.value)


def test_load_lines_scan_of_large_lists():
    """Lists long enough for the threaded one-pass check: every value rule,
    also of the optional fields, and the first offending line in input order
    when several lines, in different threads' shares, break rules."""
    import synth
    base = synth.line_list(200_000, 3000.0, seed=4)
    base = dict(base, gamma_self=base["gamma_air"] * 1.5, delta=np.full(200_000, -0.002),
                A21=np.full(200_000, 10.0))
    cases = [("n_air", 150_000, np.inf, "n_air[150000]"), ("E_lower", 3, np.nan, "E_lower[3]"),
             ("gamma_self", 199_999, -1e-9, "gamma_self[199999]"), ("delta", 77_777, np.nan, "delta[77777]"),
             ("A21", 123_456, np.inf, "A21[123456]"), ("nu", 100_000, -np.inf, "nu[100000]")]
    for k, i, v, msg in cases:
        L = {f: a.copy() for f, a in base.items()}
        L[k][i] = v
        with pytest.raises(hk.HKError) as e:
            hk.hk_load_lines(None, L, {"mass_amu": 18.0})
        assert e.value.code == hk.HK_EINVAL and msg in str(e.value), (k, str(e.value))
    L = {f: a.copy() for f, a in base.items()}
    L["S_ref"][190_000] = -1.0
    L["gamma_air"][60_000] = np.nan
    with pytest.raises(hk.HKError) as e:
        hk.hk_load_lines(None, L, {"mass_amu": 18.0})
    assert "gamma_air[60000]" in str(e.value)
    # a valid list, unordered or not, reaches the context check
    for L in (base, {f: a[::-1].copy() for f, a in base.items()}):
        with pytest.raises(hk.HKError) as e:
            hk.hk_load_lines(None, L, {"mass_amu": 18.0})
        assert "context" in str(e.value)


def test_opacity_stream_reports_chunks_in_order():
    """Every chunk is checked before any work: the first failing chunk in
    chunk order decides the error, be it a value or a shape rule."""
    good = [_chunk(5, 0), _chunk(70_000, 1), _chunk(7, 2)]
    bad_value = {k: v.copy() for k, v in good[1].items()}
    bad_value["gamma_air"][69_000] = -1.0
    missing = hk.hk_lines(5, None, None, None, None, None, None, None, None)
    sp = hk.hk_species(296.0, 18.0)
    st, gr = hk._state(GOOD_STATE), hk._grid(GOOD_GRID)

    def rc(chunks):
        pairs = [(c, None) if isinstance(c, hk.hk_lines) else hk._lines(c) for c in chunks]
        arr = (hk.hk_lines * len(pairs))(*[m for m, _ in pairs])
        return hk.lib().hk_opacity_stream(None, arr, len(pairs), C.byref(sp), C.byref(st), C.byref(gr),
                                          hk.HK_F64, 1, 0)

    assert rc([good[0], bad_value, missing]) == hk.HK_EINVAL
    assert hk.hk_last_error(None).startswith("chunk 1: gamma_air[69000]")
    assert rc([good[0], missing, bad_value]) == hk.HK_EINVAL
    assert hk.hk_last_error(None).startswith("chunk 1: nu, S_ref")
    assert rc([good[0], good[1], missing]) == hk.HK_EINVAL
    assert hk.hk_last_error(None).startswith("chunk 2: nu, S_ref")
    assert rc(good) == hk.HK_EINVAL and "context" in hk.hk_last_error(None)


def test_null_context_calls():
    for f in ("hk_sync", "hk_set_stream"):
        fn = getattr(hk.lib(), f)
        rc = fn(None) if f == "hk_sync" else fn(None, None)
        assert rc == hk.HK_EINVAL
    assert hk.lib().hk_destroy(None) == hk.HK_OK
    s = hk.hk_run_stats()
    assert hk.lib().hk_stats(None, C.byref(s)) == hk.HK_EINVAL


def test_gauss_legendre_helper_matches_numpy():
    for n in (1, 2, 3, 7, 20, 64):
        g, w = hk.hk_gauss_legendre(n)
        x, wr = np.polynomial.legendre.leggauss(n)
        assert np.max(np.abs(g - 0.5 * (1 + x))) < 2e-15
        assert np.max(np.abs(w - 0.5 * wr)) < 2e-15
    with pytest.raises(hk.HKError):
        hk.hk_gauss_legendre(0)


def _tables_rc(states, n_states=None, grid=GOOD_GRID, ppb=100, g=(0.25, 0.75),
               precision=hk.HK_F32_KAHAN, k_out=1, rule=hk.HK_RULE_STEP):
    arr = (hk.hk_state * max(len(states), 1))(*[hk._state(s) for s in states])
    gg = np.ascontiguousarray(g, dtype=np.float64)
    b = hk.hk_bins(ppb, len(gg), gg.ctypes.data_as(C.POINTER(C.c_double)), rule)
    gr = hk._grid(grid)
    n = len(states) if n_states is None else n_states
    return hk.lib().hk_tables(None, arr, n, C.byref(gr), C.byref(b), precision, k_out)


def test_tables_rejects_bad_arguments():
    bad = dict(GOOD_STATE, T=-5.0)
    assert _tables_rc([GOOD_STATE], n_states=-1) == hk.HK_EINVAL
    assert "n_states" in hk.hk_last_error(None)
    assert _tables_rc([GOOD_STATE, GOOD_STATE, bad]) == hk.HK_EINVAL
    assert "states[2]" in hk.hk_last_error(None) and "T must" in hk.hk_last_error(None)
    assert _tables_rc([GOOD_STATE], ppb=0) == hk.HK_EINVAL
    assert _tables_rc([GOOD_STATE], precision=5) == hk.HK_EINVAL
    assert _tables_rc([GOOD_STATE], rule=7) == hk.HK_EINVAL and "rule 7" in hk.hk_last_error(None)
    assert _tables_rc([GOOD_STATE], grid=dict(GOOD_GRID, dnu=1e-7, cutoff=1.0)) == hk.HK_EINVAL
    assert "2^23" in hk.hk_last_error(None)
    assert _tables_rc([GOOD_STATE], k_out=None) == hk.HK_EINVAL
    assert "k_out" in hk.hk_last_error(None)
    # valid arguments reach the context check
    assert _tables_rc([GOOD_STATE]) == hk.HK_EINVAL and "context" in hk.hk_last_error(None)


def test_options_need_a_context_and_valid_values():
    v = C.c_int64(0)
    assert hk.lib().hk_get_option(None, b"tables_batch", C.byref(v)) == hk.HK_EINVAL
    assert hk.lib().hk_set_option(None, b"tables_autotune", 2) == hk.HK_EINVAL
    assert hk.lib().hk_set_option(None, b"tables_batch", -1) == hk.HK_EINVAL
    assert hk.lib().hk_set_option(None, b"no_such_option", 1) == hk.HK_EINVAL
    # binary64 points form groups of four within a lane
    assert hk.lib().hk_set_option(None, b"f64_points_per_lane", 2) == hk.HK_EINVAL
    assert "4 or 8" in hk.hk_last_error(None)
    assert hk.lib().hk_set_option(None, b"f32_points_per_lane", 3) == hk.HK_EINVAL
    assert hk.lib().hk_set_option(None, b"f64_points_per_lane", 8) == hk.HK_EINVAL
    assert "context" in hk.hk_last_error(None)
    assert hk.lib().hk_set_option(None, b"wing_edge_paths", 2) == hk.HK_EINVAL
    assert "0 or 1" in hk.hk_last_error(None)
    assert hk.lib().hk_set_option(None, b"tables_overlap", -1) == hk.HK_EINVAL
    assert "0 or 1" in hk.hk_last_error(None)


def test_surrogate_calls_validate_arguments():
    L = hk.lib()
    assert L.hk_surrogate_labels(None, None, None, 5, None) == hk.HK_EINVAL
    assert "x and y" in hk.hk_last_error(None)
    assert L.hk_surrogate_labels(None, 1, 1, -1, 1) == hk.HK_EINVAL
    theta = np.zeros(hk.HK_SURR_N_PARAMS, dtype=np.float32)
    theta[17] = np.nan
    assert L.hk_surrogate_set_params(None, theta.ctypes.data) == hk.HK_EINVAL
    assert "theta[17]" in hk.hk_last_error(None)
    assert L.hk_surrogate_grad(None, 1, 1, 1, 0, 0.0, 1, None) == hk.HK_EINVAL
    assert L.hk_surrogate_grad(None, 1, 1, 1, hk.HK_SURR_MAX_BATCH + 1, 0.0, 1, None) == hk.HK_EINVAL
    assert L.hk_surrogate_grad(None, 1, 1, 1, 64, -1.0, 1, None) == hk.HK_EINVAL
    assert "wscale" in hk.hk_last_error(None)
    cfg = hk.hk_train_cfg(0, 10, 1e-3, 0.9, 0.999, 1e-8, 0.0)
    assert L.hk_surrogate_train(None, 1, 1, 1, 100, C.byref(cfg), None) == hk.HK_EINVAL
    assert "batch" in hk.hk_last_error(None)
    cfg = hk.hk_train_cfg(64, 10, 1e-3, 1.0, 0.999, 1e-8, 0.0)
    assert L.hk_surrogate_train(None, 1, 1, 1, 100, C.byref(cfg), None) == hk.HK_EINVAL
    assert L.hk_surrogate_certify(None, 0.0, None, None) == hk.HK_EINVAL
    assert L.hk_surrogate_certify(None, 1e-5, None, None) == hk.HK_EINVAL
    assert "context" in hk.hk_last_error(None)
    # the saved-surrogate blob: header and size are checked before anything
    # else; the layout is 32 + 4 * N_PARAMS (+ 8 * cells when certified)
    assert L.hk_surrogate_load(None, None, 0) == hk.HK_EINVAL
    assert L.hk_surrogate_load(None, b"HKSURR01", 8) == hk.HK_EINVAL
    assert "header" in hk.hk_last_error(None)
    n_cells = hk.HK_SURR_CELLS_X * hk.HK_SURR_CELLS_Y
    head = np.zeros(1, dtype=[("m", "S8"), ("p", "<i4"), ("c", "<i4"), ("cert", "<i4"), ("r", "<i4"),
                              ("b", "<f8")])
    head["m"], head["p"], head["c"], head["cert"], head["b"] = b"HKSURR0X", hk.HK_SURR_N_PARAMS, n_cells, 0, 0.0
    body = np.zeros(hk.HK_SURR_N_PARAMS, dtype="<f4").tobytes()
    assert L.hk_surrogate_load(None, head.tobytes() + body, 32 + len(body)) == hk.HK_EINVAL
    assert "magic" in hk.hk_last_error(None)
    head["m"] = b"HKSURR01"
    assert L.hk_surrogate_load(None, head.tobytes() + body[:-4], 28 + len(body)) == hk.HK_EINVAL
    assert "expected" in hk.hk_last_error(None)
    head["p"] = 100
    assert L.hk_surrogate_load(None, head.tobytes() + body, 32 + len(body)) == hk.HK_EINVAL
    assert "layout" in hk.hk_last_error(None)
    head["p"] = hk.HK_SURR_N_PARAMS
    # a well-formed blob reaches the context check
    assert L.hk_surrogate_load(None, head.tobytes() + body, 32 + len(body)) == hk.HK_EINVAL
    assert "context" in hk.hk_last_error(None)
    size = C.c_size_t(0)
    assert L.hk_surrogate_save(None, None, 0, C.byref(size)) == hk.HK_EINVAL


def test_resample_and_transmission_validate_arguments():
    L = hk.lib()
    assert L.hk_resample(None, 1, 0, 100, 10, 20, 1) == hk.HK_EINVAL  # bins of 10 < 20 coefficients
    assert "n_coef" in hk.hk_last_error(None)
    assert L.hk_resample(None, 1, 0, 105, 100, 20, 1) == hk.HK_EINVAL  # ragged bin of 5
    assert L.hk_resample(None, 1, 0, 100, 100, 33, 1) == hk.HK_EINVAL
    assert L.hk_resample(None, 1, 7, 100, 100, 20, 1) == hk.HK_EINVAL
    assert L.hk_resample(None, 1, 0, 100, 100, 20, 1) == hk.HK_EINVAL and "context" in hk.hk_last_error(None)
    assert L.hk_transmission(None, 1, 3, 20, 1, -1, 1) == hk.HK_EINVAL
    assert L.hk_transmission(None, None, 3, 20, 1, 5, 1) == hk.HK_EINVAL
    assert L.hk_transmission_direct(None, 1, 0, 100, 0, 1, 5, 1) == hk.HK_EINVAL


def _stream_rc(chunks, n_chunks=None, species=(296.0, 18.0), state=GOOD_STATE, grid=GOOD_GRID,
               precision=hk.HK_F64):
    made = [hk._lines(c) for c in chunks]
    arr = (hk.hk_lines * max(len(made), 1))(*[m[0] for m in made])
    sp = hk.hk_species(*species)
    st, gr = hk._state(state), hk._grid(grid)
    n = len(made) if n_chunks is None else n_chunks
    return hk.lib().hk_opacity_stream(None, arr if made else None, n, C.byref(sp), C.byref(st),
                                      C.byref(gr), precision, 1, 0)


def _chunk(n, seed):
    import synth
    return synth.line_list(n, 10.0, seed=seed)


def test_opacity_stream_rejects_bad_input():
    good = [_chunk(5, 0), _chunk(7, 1)]
    assert _stream_rc(good, n_chunks=-1) == hk.HK_EINVAL and "n_chunks" in hk.hk_last_error(None)
    assert _stream_rc([], n_chunks=2) == hk.HK_EINVAL and "chunks is NULL" in hk.hk_last_error(None)
    assert _stream_rc(good, species=(296.0, 0.0)) == hk.HK_EINVAL
    assert "mass_amu" in hk.hk_last_error(None)
    bad = _chunk(7, 1)
    bad["S_ref"][2] = -1.0
    assert _stream_rc([good[0], bad]) == hk.HK_EINVAL
    assert hk.hk_last_error(None).startswith("chunk 1: S_ref[2]")
    assert _stream_rc(good, precision=7) == hk.HK_EINVAL and "precision" in hk.hk_last_error(None)
    wide = dict(GOOD_GRID, dnu=1e-9, cutoff=1.0)
    assert _stream_rc(good, grid=wide, precision=hk.HK_F32_KAHAN) == hk.HK_EINVAL
    assert "2^23" in hk.hk_last_error(None)
    lor = dict(GOOD_GRID, dnu=1e-7, cutoff_lorentz=1e6)
    assert _stream_rc(good, grid=lor, precision=hk.HK_F32_KAHAN) == hk.HK_EINVAL
    assert hk.hk_last_error(None).startswith("chunk 0: binary32")
    # valid arguments reach the context check (NULL context)
    assert _stream_rc(good) == hk.HK_EINVAL and "context" in hk.hk_last_error(None)
