"""Line lists that crowd into few grid tiles (a wavenumber-ordered piece of a
list, a dense band): the wing stage splits those tiles' lines at fixed
line-index segments.  Checked: the split happens (and does not on an even
list), results against the FP64 oracle, bitwise independence of the tile
shape, and hk_tables bitwise equal to single-state calls."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hk = pytest.importorskip("paper_1503_03806_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = hk.Context(0)
    yield c
    c.set_option("f64_points_per_lane", 4)
    c.set_option("f32_points_per_lane", 4)
    c.close()


GRID = {"nu_min": 0.0, "dnu": 0.01, "n_points": 300000, "cutoff": 25.0}
COND = synth.conditions(1500.0, 1.0)
STATE = {k: COND[k] for k in ("T", "P", "P_self", "q_ratio")}


def crowded():
    """3e4 lines in [1000, 1100) cm^-1 of a 0-3000 cm^-1 grid."""
    L = synth.line_list(30_000, 100.0, seed=21)
    L["nu"] = L["nu"] + 1000.0
    return L


def banded():
    """2e4 lines spread over 0-3000 cm^-1 plus 2e4 in [1500, 1510)."""
    a = synth.line_list(20_000, 3000.0, seed=22)
    b = synth.line_list(20_000, 10.0, seed=23)
    b["nu"] = b["nu"] + 1500.0
    return {k: np.concatenate([a[k], b[k]]) for k in a}


def bits(t):
    return t.cpu().numpy().view(np.uint64)


def rel(got, ref):
    nz = ref > 0
    assert np.all(got[~nz] == 0)
    return np.abs(got[nz] / ref[nz] - 1).max()


@pytest.mark.parametrize("which", ["crowded", "banded"])
def test_split_lists_match_the_oracle(ctx, which):
    lines = {"crowded": crowded, "banded": banded}[which]()
    ctx.load_lines(lines, COND["mass_amu"], COND["T0"])
    ref, n_evals = oracle.opacity(lines, COND, GRID)
    for prec, bar in ((hk.HK_F64, 1e-6), (hk.HK_F32_KAHAN, 1e-4)):
        k = ctx.opacity(STATE, GRID, prec).cpu().numpy()
        items, seg = ctx.get_option("wing_items"), ctx.get_option("wing_segment_lines")
        e = rel(k, ref)
        say("%s, precision %d: %d items, segments of %d lines, max rel err %.2e" % (which, prec, items, seg, e))
        assert seg >= 64 and items > 586
        assert e <= bar
    assert ctx.stats()["evals"] == n_evals


@pytest.mark.parametrize("prec", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_split_results_do_not_depend_on_the_tile_shape(ctx, prec):
    ctx.load_lines(crowded(), COND["mass_amu"], COND["T0"])
    name = "f64_points_per_lane" if prec == hk.HK_F64 else "f32_points_per_lane"
    shapes = (4, 8) if prec == hk.HK_F64 else (2, 4, 8)
    outs = []
    for ppl in shapes:
        ctx.set_option(name, ppl)
        outs.append(bits(ctx.opacity(STATE, GRID, prec)))
        say("points per lane %d: %d items" % (ppl, ctx.get_option("wing_items")))
    ctx.set_option(name, shapes[0])
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


@pytest.mark.parametrize("prec", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_tables_equal_single_state_calls_when_split(ctx, prec):
    lines = banded()
    ctx.load_lines(lines, COND["mass_amu"], COND["T0"])
    states = [STATE, {k: v for k, v in synth.conditions(600.0, 0.01).items() if k in STATE}, STATE]
    g, _ = hk.hk_gauss_legendre(20)
    tab = ctx.tables(states, GRID, 100000, g, prec).cpu().numpy()
    for i, st in enumerate(states):
        k = ctx.opacity(st, GRID, prec)
        one = ctx.kdist(k, 100000, g).cpu().numpy()
        assert np.array_equal(one.view(np.uint64), tab[i].view(np.uint64)), i


def test_even_list_is_not_split(ctx):
    lines = synth.line_list(300_000, 30000.0, seed=24)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 3_000_000, "cutoff": 25.0}
    ctx.load_lines(lines, COND["mass_amu"], COND["T0"])
    k = ctx.opacity(STATE, grid, hk.HK_F64)
    tile_points = 64 * 4 * ctx.get_option("f64_points_per_lane")  # four wavefronts per tile
    n_tiles = -(-grid["n_points"] // tile_points)
    assert ctx.get_option("wing_segment_lines") == 0 and ctx.get_option("wing_items") == n_tiles
    j = np.random.default_rng(3).choice(grid["n_points"], 16, replace=False)
    for a in j:
        ref, _ = oracle.opacity(lines, COND, grid, int(a), int(a) + 1)
        v = k[int(a)].item()
        assert (ref[0] == 0 and v == 0) or abs(v / ref[0] - 1) <= 1e-6


def test_large_grid_reads_the_plan_back(ctx):
    """A grid of 4e7 points (its plans' partial-sum bound passes 1 GiB, so
    the plans are read back): sampled points against the oracle, binary64
    and binary32, with a crowded list so that tiles are split."""
    L = synth.line_list(20_000, 40.0, seed=25)
    L["nu"] = L["nu"] + 20000.0
    grid = {"nu_min": 0.0, "dnu": 0.001, "n_points": 40_000_000, "cutoff": 5.0}
    ctx.load_lines(L, COND["mass_amu"], COND["T0"])
    j = np.concatenate([np.random.default_rng(7).integers(19_990_000, 20_050_000, 24), [0, 39_999_999]])
    for prec, bar in ((hk.HK_F64, 1e-6), (hk.HK_F32_KAHAN, 1e-4)):
        k = ctx.opacity(STATE, grid, prec)
        assert ctx.get_option("wing_segment_lines") > 0
        for a in j:
            ref, _ = oracle.opacity(L, COND, grid, int(a), int(a) + 1)
            v = k[int(a)].item()
            assert (ref[0] == 0 and v == 0) or abs(v / ref[0] - 1) <= bar, (prec, int(a))
        del k
