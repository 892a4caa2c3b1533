"""Batched opacity tables (hk_tables) through the C ABI.

Each state's k(g) table must equal, bit for bit, the library's own
single-state path (hk_opacity then hk_kdist), whatever the batch size and
the tile shape the autotuner picks; and it must match the FP64 CPU oracle
within 1e-6 (binary64) or 1e-4 (binary32 + compensated sums) relative.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hk = pytest.importorskip("paper_1503_03806_amd")

TOL = {0: 1e-6, 1: 1e-4}  # by precision (HK_F64, HK_F32_KAHAN)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = hk.Context(0)
    yield c
    c.close()


def state_of(cond):
    return {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}


# five states spanning the table workload's corners and middle
SMALL_STATES = [(300.0, 1e-6), (3000.0, 100.0), (1500.0, 1.0), (700.0, 0.01), (2200.0, 30.0)]


def small_setup():
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines = w.lines()
    grid = dict(w.grid(), n_points=200_003)  # ragged last bin and last tile
    conds = [synth.conditions(T, P) for T, P in SMALL_STATES]
    return w, lines, grid, conds


def single_state(ctx, lines, cond, grid, ppb, g, precision):
    k = ctx.opacity(state_of(cond), grid, precision)
    return ctx.kdist(k, ppb, g).cpu().numpy(), k.cpu().numpy()


@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_tables_match_single_state_path_and_oracle(ctx, precision):
    w, lines, grid, conds = small_setup()
    ppb = 10_000
    g, _ = oracle.g_nodes(w.n_g)
    ctx.load_lines(lines, conds[0]["mass_amu"], conds[0]["T0"])
    say("tables precision", precision, "states", SMALL_STATES)
    tab = ctx.tables([state_of(c) for c in conds], grid, ppb, g, precision)
    torch.cuda.synchronize()
    tab = tab.cpu().numpy()
    shape = ctx.get_option("tables_points_per_lane")
    say("  autotuned points per lane:", shape)
    assert shape in (2, 4, 8)
    st = ctx.stats()
    total = 0
    for s, cond in enumerate(conds):
        ctx.set_option("f64_points_per_lane" if precision == hk.HK_F64 else "f32_points_per_lane",
                       4 if precision == hk.HK_F64 else 2)
        ref_k, kap = single_state(ctx, lines, cond, grid, ppb, g, precision)
        total += ctx.stats()["evals"]
        assert np.array_equal(tab[s].view(np.uint64), ref_k.view(np.uint64)), s
        # oracle: the whole grid of this small case
        ora, _ = oracle.opacity(lines, cond, grid)
        kd = oracle.kdist(ora, ppb, g)
        e = np.abs(tab[s] / kd - 1).max()
        say("  state %d (T=%g, P=%g atm): k(g) max rel err vs oracle %.2e" % (s, cond["T"], cond["P"], e))
        assert e <= TOL[precision]
    assert st["evals"] == total


@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_tables_linear_rule_matches_single_state_path(ctx, precision):
    w, lines, grid, conds = small_setup()
    ppb = 10_000
    g, _ = oracle.g_nodes(w.n_g)
    ctx.load_lines(lines, conds[0]["mass_amu"], conds[0]["T0"])
    say("tables linear rule, precision", precision)
    tab = ctx.tables([state_of(c) for c in conds[:3]], grid, ppb, g, precision,
                     rule=hk.HK_RULE_LINEAR).cpu().numpy()
    for s, cond in enumerate(conds[:3]):
        k = ctx.opacity(state_of(cond), grid, precision)
        ref = ctx.kdist(k, ppb, g, rule=hk.HK_RULE_LINEAR).cpu().numpy()
        assert np.array_equal(tab[s].view(np.uint64), ref.view(np.uint64)), s
        # against the oracle's own opacity and linear rule
        ora, _ = oracle.opacity(lines, cond, grid)
        e = np.abs(tab[s] / oracle.kdist(ora, ppb, g, rule=1) - 1).max()
        say("  state %d: linear-rule k(g) max rel err vs oracle %.2e" % (s, e))
        assert e <= TOL[precision]


def test_tables_batches_and_shapes_are_bitwise_identical(ctx):
    w, lines, grid, conds = small_setup()
    ppb = 10_000
    g, _ = oracle.g_nodes(w.n_g)
    states = [state_of(c) for c in conds]
    ctx.load_lines(lines, conds[0]["mass_amu"], conds[0]["T0"])
    ref = ctx.tables(states, grid, ppb, g, hk.HK_F32_KAHAN).cpu().numpy()
    try:
        ctx.set_option("tables_batch", 2)  # batches of 2, 2 and 1 -> evened to 2, 2, 1
        b2 = ctx.tables(states, grid, ppb, g, hk.HK_F32_KAHAN).cpu().numpy()
        assert np.array_equal(ref.view(np.uint64), b2.view(np.uint64))
        ctx.set_option("tables_autotune", 0)
        for ppl in (2, 4, 8):
            ctx.set_option("f32_points_per_lane", ppl)
            t = ctx.tables(states, grid, ppb, g, hk.HK_F32_KAHAN).cpu().numpy()
            assert ctx.get_option("tables_points_per_lane") == ppl
            assert np.array_equal(ref.view(np.uint64), t.view(np.uint64)), ppl
    finally:
        ctx.set_option("tables_batch", 0)
        ctx.set_option("tables_autotune", 1)
        ctx.set_option("f32_points_per_lane", 4)


def test_tables_overlap_is_bitwise_identical(ctx):
    """The series beside the wing on a second stream, or before it on the
    caller's stream: the same tables, bit for bit, in both precisions."""
    w, lines, grid, conds = small_setup()
    g, _ = oracle.g_nodes(w.n_g)
    states = [state_of(c) for c in conds]
    ctx.load_lines(lines, conds[0]["mass_amu"], conds[0]["T0"])
    assert ctx.get_option("tables_overlap") == 0
    try:
        for precision in (hk.HK_F64, hk.HK_F32_KAHAN):
            a = ctx.tables(states, grid, 10_000, g, precision).cpu().numpy()
            ctx.set_option("tables_overlap", 1)
            b = ctx.tables(states, grid, 10_000, g, precision).cpu().numpy()
            ctx.set_option("tables_overlap", 0)
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), precision
    finally:
        ctx.set_option("tables_overlap", 0)


def test_tables_edge_cases(ctx):
    w, lines, grid, conds = small_setup()
    g, _ = oracle.g_nodes(4)
    ctx.load_lines(lines, conds[0]["mass_amu"], conds[0]["T0"])
    # no states: nothing written, no error
    out = torch.full((1, 1, 4), -1.0, dtype=torch.float64, device="cuda")
    hk.hk_tables(ctx.h, [], grid, 1000, g, hk.HK_F32_KAHAN, out)
    torch.cuda.synchronize()
    assert float(out[0, 0, 0]) == -1.0
    # an empty line list gives zero tables
    empty = {k: v[:0] for k, v in lines.items()}
    ctx.load_lines(empty, conds[0]["mass_amu"], conds[0]["T0"])
    t = ctx.tables([state_of(c) for c in conds[:2]], dict(grid, n_points=5000), 1000, g,
                   hk.HK_F32_KAHAN)
    torch.cuda.synchronize()
    assert t.shape == (2, 5, 4) and bool((t == 0).all())
    # one bin, one state, grid smaller than a tile
    ctx.load_lines(lines, conds[0]["mass_amu"], conds[0]["T0"])
    small = dict(grid, nu_min=1000.0, n_points=777)
    t = ctx.tables([state_of(conds[2])], small, 777, g, hk.HK_F64).cpu().numpy()
    ora, _ = oracle.opacity(lines, conds[2], small)
    kd = oracle.kdist(ora, 777, g)
    assert np.abs(t[0] / kd - 1).max() <= 1e-6


def test_tables200_full_size_sampled(ctx):
    """The table workload at full size: 1e6 lines, 3e6 points, 20 x 10
    (T, P) states, binary32 profiles; oracle k(g) on 16 (state, bin) pairs
    drawn with seed 3, plus the table's corners (coldest/lowest pressure,
    hottest/highest)."""
    from parity_util import SAMPLE_SEED, near_lines
    w = synth.WORKLOADS["lines1e6_tables200"]
    lines, grid = w.lines(), w.grid()
    conds = [synth.conditions(T, P) for T, P in w.states]
    ppb = w.points_per_bin
    g, _ = oracle.g_nodes(w.n_g)
    say("workload", w.name, "states", len(conds))
    ctx.load_lines(lines, conds[0]["mass_amu"], conds[0]["T0"])
    tab = ctx.tables([state_of(c) for c in conds], grid, ppb, g, hk.HK_F32_KAHAN)
    torch.cuda.synchronize()
    tab = tab.cpu().numpy()
    say("  autotuned points per lane:", ctx.get_option("tables_points_per_lane"))
    assert tab.shape == (200, w.n_bins, w.n_g)
    assert np.all(np.isfinite(tab)) and np.all(tab >= 0)
    assert np.all(np.diff(tab, axis=2) >= 0)  # k(g) is monotone in g
    rng = np.random.default_rng(SAMPLE_SEED)
    pairs = [(0, 0), (199, 299)] + [(int(s), int(b)) for s, b in
                                    zip(rng.choice(200, 16, replace=False), rng.choice(w.n_bins, 16))]
    for s, b in pairs:
        j0, j1 = b * ppb, (b + 1) * ppb
        ref, _ = oracle.opacity(near_lines(lines, grid, j0, j1), conds[s], grid, j0, j1)
        kr, _ = oracle.kdist_bin(ref, g)
        e = np.abs(tab[s, b] / kr - 1).max()
        say("  state %d (T=%.0f K, P=%.2e atm) bin %d: k(g) max rel err %.2e"
            % (s, conds[s]["T"], conds[s]["P"], b, e))
        assert e <= TOL[hk.HK_F32_KAHAN]
