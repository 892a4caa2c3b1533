"""Parity of the binary32 + compensated-sum path (HK_F32_KAHAN) with the FP64
CPU oracle, through the C ABI.

Bar: 1e-4 relative per grid point and per k(g) entry (the workloads' bar for
the binary32 path).  Error budget: profile arithmetic in binary32 with the
hardware reciprocal (a few ulps, ~5e-7), binary32 block sums of <= 256
positive terms (<= 1.5e-5 worst case), Kahan sum of blocks (~1e-7), the
series in binary32 (~2e-6), and the region ties of the binary64 path.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hk = pytest.importorskip("paper_1503_03806_amd")

TOL = 1e-4


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


def run(ctx, lines, cond, grid, precision=hk.HK_F32_KAHAN, out=None, accumulate=False):
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    k = ctx.opacity(state_of(cond), grid, precision, out=out, accumulate=accumulate)
    torch.cuda.synchronize()
    return k


def rel_err(got, ref):
    got = np.asarray(got); ref = np.asarray(ref)
    zero = ref == 0
    assert np.all(got[zero] == 0)
    e = np.zeros_like(ref)
    e[~zero] = np.abs(got[~zero] / ref[~zero] - 1.0)
    return e


from test_gpu_parity import CASES  # noqa: E402  (same edge cases as the binary64 path)


@pytest.mark.parametrize("name", sorted(CASES))
def test_f32_small_cases_against_oracle(ctx, name):
    lines, cond, grid = CASES[name]
    say("f32 case", name)
    k = run(ctx, lines, cond, grid).cpu().numpy()
    ref, n_ref = oracle.opacity(lines, cond, grid)
    e = rel_err(k, ref)
    say("  max rel err %.3e" % (e.max() if e.size else 0.0))
    assert e.size == 0 or e.max() <= TOL
    assert ctx.stats()["evals"] == n_ref


def test_f32_lines1e4_grid3e5_full_and_tile_shapes(ctx):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    k = run(ctx, lines, cond, grid)
    kk = k.cpu().numpy()
    ref, _ = oracle.opacity(lines, cond, grid)
    e = rel_err(kk, ref)
    ppb = w.points_per_bin
    say("per-bin max rel err:", ["%.2e" % e[b * ppb:(b + 1) * ppb].max() for b in range(3)])
    assert e.max() <= TOL
    g, _ = oracle.g_nodes(w.n_g)
    kd = ctx.kdist(k, ppb, g).cpu().numpy()
    kd_ref = oracle.kdist(ref, ppb, g)
    assert np.max(np.abs(kd / kd_ref - 1)) <= TOL
    for ppl in (2, 4, 8):
        ctx.set_option("f32_points_per_lane", ppl)
        k2 = run(ctx, lines, cond, grid).cpu().numpy()
        assert np.array_equal(kk.view(np.uint64), k2.view(np.uint64)), ppl
    ctx.set_option("f32_points_per_lane", 4)


def test_f32_ragged_grid_end_does_not_depend_on_the_tile_shape(ctx):
    """One line whose 3-node interval starts inside the last, cut-short run
    of a ragged grid at 8 points per lane but covers that run whole at 2 and
    4: the points there whose pair partner lies beyond the grid are evaluated
    alone in every tile shape (the line's terms are the whole sum there, so
    any difference in rounding would show)."""
    cond = synth.conditions(1500.0, 0.01)
    grid = {"nu_min": 1900.0, "dnu": 0.01, "n_points": 10_000 + 37, "cutoff": 25.0}
    # the 3-node interval's lower edge (a^2 + u^2 = 1e6, a ~ 0) at point 9850:
    # nu0 - 1000 alpha(nu0) = nu_9850, alpha proportional to nu0
    c_alpha = oracle.doppler_hwhm(1.0, cond["T"], cond["mass_amu"])[()] / math.sqrt(math.log(2.0))
    nu0 = (grid["nu_min"] + 9850 * grid["dnu"]) / (1.0 - 1000.0 * c_alpha)
    lines = {"nu": np.array([nu0]), "S_ref": np.array([1e-20]), "E_lower": np.array([500.0]),
             "gamma_air": np.array([0.05]), "n_air": np.array([0.5])}
    outs = []
    for ppl in (2, 4, 8):
        ctx.set_option("f32_points_per_lane", ppl)
        outs.append(run(ctx, lines, cond, grid).cpu().numpy())
    ctx.set_option("f32_points_per_lane", 4)
    for o in outs[1:]:
        assert np.array_equal(outs[0].view(np.uint64), o.view(np.uint64))
    ref, _ = oracle.opacity(lines, cond, grid)
    assert rel_err(outs[0], ref).max() <= TOL


def test_f32_accumulate_chunks(ctx):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    whole = run(ctx, lines, cond, grid).cpu().numpy()
    order = np.argsort(lines["nu"], kind="stable")
    out = torch.zeros(grid["n_points"], dtype=torch.float64, device="cuda")
    for part in np.array_split(order, 3):
        run(ctx, {k: v[part] for k, v in lines.items()}, cond, grid, out=out, accumulate=True)
    e = rel_err(out.cpu().numpy(), whole)
    assert e.max() <= 2e-5


def test_f32_rejects_too_wide_windows(ctx):
    lines, cond, grid = CASES["ragged_grid"]
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    g = dict(grid); g["dnu"] = 1e-7; g["cutoff"] = 1.0
    out = torch.empty(10, dtype=torch.float64, device="cuda")
    g["n_points"] = 10
    with pytest.raises(hk.HKError) as ex:
        ctx.opacity(state_of(cond), g, hk.HK_F32_KAHAN, out=out)
    assert ex.value.code == hk.HK_EINVAL and "2^23" in str(ex.value)


def test_f32_lines1e7_seeded_bins(ctx):
    """The precision workload at full size (1e7 lines, 2000 K, 0.1 bar) in
    the benchmark's launch configuration: 16 whole bins drawn with seed 3,
    kappa and k(g) against the oracle at 1e-4 (the oracle is given the lines
    that can reach each bin); per-bin max and p99.9 errors printed."""
    from parity_util import near_lines, rel_errors, seeded_bins
    w = synth.WORKLOADS["lines1e7_fp32"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    say("workload", w.name)
    k = run(ctx, lines, cond, grid)
    kk = k.cpu().numpy()
    assert np.all(np.isfinite(kk)) and np.all(kk > 0)
    ppb = w.points_per_bin
    g, _ = oracle.g_nodes(w.n_g)
    kd = ctx.kdist(k, ppb, g).cpu().numpy()
    worst = 0.0
    for b in seeded_bins(w.n_bins):
        j0, j1 = b * ppb, (b + 1) * ppb
        ref, _ = oracle.opacity(near_lines(lines, grid, j0, j1), cond, grid, j0, j1)
        e = rel_errors(kk[j0:j1], ref)
        kr, _ = oracle.kdist_bin(ref, g)
        ek = np.abs(kd[b] / kr - 1).max()
        say("  bin %d: kappa max %.2e p99.9 %.2e, k(g) max %.2e" % (b, e.max(), np.quantile(e, 0.999), ek))
        worst = max(worst, e.max(), ek)
    assert worst <= TOL
