"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerance: 1e-6 relative per grid point and per k(g) entry for the binary64
path.  Every opacity here is a sum of positive terms, so a per-term relative
difference bounds the per-point one; the kernel and the oracle differ only in
rounding (reciprocal-multiply vs division, recurrences vs exp() per series
term, fma), in summation association, and in which region a point whose
a^2+u^2 lies within rounding of 100 or 1e6 falls into (the scheme's own error
there is <= 5.7e-6 of one term, and such ties are ~1e-13 rare).
Integer outputs (evaluation counts, k(g) of identical inputs) are compared
exactly.
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

TOL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = hk.Context(0)
    yield c
    c.close()


def state_of(cond):
    return {"T": cond["T"], "P": cond["P"], "P_self": cond["P_self"], "q_ratio": cond["q_ratio"]}


def gpu_opacity(ctx, lines, cond, grid, out=None, accumulate=False):
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    k = ctx.opacity(state_of(cond), grid, hk.HK_F64, out=out, accumulate=accumulate)
    torch.cuda.synchronize()
    return k


def assert_close(got, ref, tol=TOL, what=""):
    got = np.asarray(got); ref = np.asarray(ref)
    assert got.shape == ref.shape
    zero = ref == 0
    assert np.all(got[zero] == 0), (what, "nonzero where the oracle is zero")
    if (~zero).any():
        err = np.abs(got[~zero] / ref[~zero] - 1.0)
        i = int(err.argmax())
        assert err.max() <= tol, (what, float(err.max()), int(np.flatnonzero(~zero)[i]))


# ---- small and edge cases, full grid against the oracle ----

def _one(nu, S=1e-20, E=100.0, g=0.05, n=0.5):
    return {"nu": np.array([nu], float), "S_ref": np.array([S]), "E_lower": np.array([E]),
            "gamma_air": np.array([g]), "n_air": np.array([n])}


def _cases():
    L = synth.line_list(500, 60.0, seed=21)
    hi = synth.line_list(300, 50.0, seed=22); hi["nu"] = hi["nu"] + 29950.0
    cases = {
        "ragged_grid": (L, synth.conditions(1500, 1.0),
                        {"nu_min": 0.0, "dnu": 0.01, "n_points": 6000 + 17, "cutoff": 5.0}),
        "tiny_grid": (L, synth.conditions(800, 0.3),
                      {"nu_min": 20.0, "dnu": 0.01, "n_points": 37, "cutoff": 5.0}),
        "high_nu_cores": (hi, synth.conditions(2500, 0.05),
                          {"nu_min": 29950.0, "dnu": 0.01, "n_points": 5000, "cutoff": 25.0}),
        "low_pressure": (hi, synth.conditions(1000, 1e-6),
                         {"nu_min": 29960.0, "dnu": 0.01, "n_points": 3000, "cutoff": 10.0}),
        "zero_pressure": (hi, synth.conditions(1000, 0.0),
                          {"nu_min": 29960.0, "dnu": 0.01, "n_points": 3000, "cutoff": 10.0}),
        "high_pressure": (L, synth.conditions(300, 100.0),
                          {"nu_min": 0.0, "dnu": 0.01, "n_points": 6000, "cutoff": 30.0}),
        "zero_cutoff": (L, synth.conditions(1500, 1.0),
                        {"nu_min": 0.0, "dnu": 0.0625, "n_points": 960, "cutoff": 0.0}),
        "offgrid_lines": (L, synth.conditions(1500, 1.0),
                          {"nu_min": 25.0, "dnu": 0.01, "n_points": 1000, "cutoff": 20.0}),
        "single_line_on_point": (_one(1000.0), synth.conditions(1500, 1.0),
                                 {"nu_min": 990.0, "dnu": 0.0078125, "n_points": 2561,
                                  "cutoff": 10.0}),
        "empty_list": ({k: np.zeros(0) for k in L}, synth.conditions(1500, 1.0),
                       {"nu_min": 0.0, "dnu": 0.01, "n_points": 1000, "cutoff": 5.0}),
    }
    # optional fields: self broadening, pressure shift, natural width
    rng = np.random.default_rng(23)
    L2 = dict(L)
    L2["gamma_self"] = rng.uniform(0.1, 0.5, 500)
    L2["delta"] = rng.uniform(-0.02, 0.02, 500)
    L2["A21"] = 10.0 ** rng.uniform(0, 8, 500)
    cases["self_shift_natural"] = (L2, synth.conditions(1200, 2.0),
                                   {"nu_min": 0.0, "dnu": 0.01, "n_points": 6000, "cutoff": 8.0})
    # lines within 1e-5 cm^-1 of zero: Doppler widths below 1e-11, so their
    # points are not grouped for a shared reciprocal (each takes its own)
    L3 = synth.line_list(300, 3.0, seed=26)
    L3["nu"][:100] = 10.0 ** rng.uniform(-7, -5, 100)
    cases["near_zero_lines"] = (L3, synth.conditions(1500, 1.0),
                                {"nu_min": 0.0, "dnu": 0.001, "n_points": 4000, "cutoff": 2.0})
    return cases


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_small_cases_against_oracle(ctx, name):
    lines, cond, grid = CASES[name]
    say("case", name, "lines", len(lines["nu"]), "points", grid["n_points"])
    k = gpu_opacity(ctx, lines, cond, grid).cpu().numpy()
    ref, n_ref = oracle.opacity(lines, cond, grid)
    assert_close(k, ref, what=name)
    st = ctx.stats()
    assert st["evals"] == n_ref
    if len(lines["nu"]):
        tot, core, g3, g1 = oracle.eval_counts(lines, cond, grid)
        assert tot == st["evals"]
        for a, b in ((core, st["evals_core"]), (g3, st["evals_gh3"]), (g1, st["evals_gh1"])):
            assert abs(a - b) <= 2  # region ties at rounding distance only


def test_ungrouped_lines_do_not_depend_on_the_tile_shape(ctx):
    lines, cond, grid = CASES["near_zero_lines"]
    outs = []
    for ppl in (8, 4):
        ctx.set_option("f64_points_per_lane", ppl)
        outs.append(gpu_opacity(ctx, lines, cond, grid).cpu().numpy().view(np.uint64))
    assert np.array_equal(outs[0], outs[1])


def test_ragged_grid_end_does_not_depend_on_the_tile_shape(ctx):
    """One line whose 3-node interval starts inside the last, cut-short run
    at 8 points per lane and covers it whole at 4: points whose group
    reaches beyond the grid are evaluated alone in both shapes."""
    cond = synth.conditions(1500.0, 0.01)
    grid = {"nu_min": 1900.0, "dnu": 0.01, "n_points": 10_000 + 37, "cutoff": 25.0}
    c_alpha = oracle.doppler_hwhm(1.0, cond["T"], cond["mass_amu"])[()] / math.sqrt(math.log(2.0))
    nu0 = (grid["nu_min"] + 9850 * grid["dnu"]) / (1.0 - 1000.0 * c_alpha)
    lines = {"nu": np.array([nu0]), "S_ref": np.array([1e-20]), "E_lower": np.array([500.0]),
             "gamma_air": np.array([0.05]), "n_air": np.array([0.5])}
    outs = []
    for ppl in (8, 4):
        ctx.set_option("f64_points_per_lane", ppl)
        outs.append(gpu_opacity(ctx, lines, cond, grid).cpu().numpy())
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    ref, _ = oracle.opacity(lines, cond, grid)
    assert_close(outs[1], ref, what="ragged end")


def test_zero_points(ctx):
    lines, cond, _ = CASES["ragged_grid"]
    g = {"nu_min": 0.0, "dnu": 0.01, "n_points": 0, "cutoff": 5.0}
    k = gpu_opacity(ctx, lines, cond, g)
    assert k.numel() == 0


# ---- the CPU-sized FP64 workload, full grid ----

def test_lines1e4_grid3e5_full(ctx):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    say("workload", w.name)
    kg = gpu_opacity(ctx, lines, cond, grid)
    k = kg.cpu().numpy()
    ref, n_ref = oracle.opacity(lines, cond, grid)
    assert np.all(ref > 0)
    assert_close(k, ref, what=w.name)
    st = ctx.stats()
    tot, core, g3, g1 = oracle.eval_counts(lines, cond, grid)
    assert st["evals"] == tot == n_ref
    assert abs(st["evals_core"] - core) <= 2 and abs(st["evals_gh1"] - g1) <= 2
    # k(g): product nodes on the GPU, the oracle's own nodes on the CPU
    g_gpu, _ = hk.hk_gauss_legendre(w.n_g)
    g_ora, _ = oracle.g_nodes(w.n_g)
    kd = ctx.kdist(kg, w.points_per_bin, g_gpu).cpu().numpy()
    kd_ref = oracle.kdist(ref, w.points_per_bin, g_ora)
    assert kd.shape == (3, 20)
    assert_close(kd, kd_ref, what="k(g)")
    assert np.all(np.diff(kd, axis=1) >= 0)


def test_deterministic_and_accumulate_chunks(ctx):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    a = gpu_opacity(ctx, lines, cond, grid).cpu().numpy()
    b = gpu_opacity(ctx, lines, cond, grid).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    # three chunks contiguous in wavenumber, accumulated: each point sums the
    # same terms; only the association of the wing and core partial sums
    # differs, so the results agree to rounding
    order = np.argsort(lines["nu"], kind="stable")
    out = torch.zeros(grid["n_points"], dtype=torch.float64, device="cuda")
    for part in np.array_split(order, 3):
        chunk = {k: v[part] for k, v in lines.items()}
        gpu_opacity(ctx, chunk, cond, grid, out=out, accumulate=True)
    c = out.cpu().numpy()
    assert_close(c, a, tol=1e-13, what="chunked")
    # and the tile shape changes nothing, bit for bit
    for ppl in (8, 4):
        ctx.set_option("f64_points_per_lane", ppl)
        d = gpu_opacity(ctx, lines, cond, grid).cpu().numpy()
        assert np.array_equal(a.view(np.uint64), d.view(np.uint64)), ppl


# ---- k-distribution: LDS and chunked/merge paths, bitwise vs the oracle ----

@pytest.mark.parametrize("n,ppb", [(1, 1), (1000, 7), (100000, 1000), (8192, 4096), (12000, 4097),
                                   (16384, 8192), (20000, 8193),
                                   (30017, 10000), (65536, 16384),
                                   (50000, 16385), (300000, 100000), (250001, 100000),
                                   (40000, 40000)])
def test_kdist_matches_oracle_bitwise(ctx, n, ppb):
    say("kdist", n, ppb)
    rng = np.random.default_rng(n + ppb)
    kap = 10.0 ** rng.uniform(-30, -18, n)
    kap[rng.integers(0, n, n // 10)] = kap[0]  # ties
    if n > 10:
        kap[:5] = 0.0
    g, _ = oracle.g_nodes(20)
    kt = torch.from_numpy(kap).cuda()
    srt = torch.empty_like(kt)
    kd = ctx.kdist(kt, ppb, g, sorted_out=srt).cpu().numpy()
    ref = oracle.kdist(kap, ppb, g)
    assert np.array_equal(kd, ref)
    s = srt.cpu().numpy()
    for b0 in range(0, n, ppb):
        assert np.array_equal(s[b0:b0 + ppb], np.sort(kap[b0:b0 + ppb]))


@pytest.mark.parametrize("run", [2, 5, 31, 32, 33, 200])
def test_kdist_runs_of_equal_high_words(ctx, run):
    """Binary64 keys are sorted by their high 32 bits first; keys equal there
    are put in order afterwards (or, past a run length of 32, by a full sort
    of all 64 bits).  Bins holding groups of `run` keys that share a high
    word and differ in the low word, among distinct keys: the sorted bins
    equal numpy's and k(g) the oracle's, bit for bit."""
    say("kdist runs", run)
    rng = np.random.default_rng(100 + run)
    ppb, n = 10000, 30000
    keys = (10.0 ** rng.uniform(-30, -18, n)).view(np.uint64).copy()
    for b0 in range(0, n, ppb):
        # a few groups per bin, each of `run` keys with one high word
        for _ in range(3):
            at = b0 + rng.integers(0, ppb)
            pos = b0 + rng.choice(ppb, run, replace=False)
            hi = keys[at] & np.uint64(0xFFFFFFFF00000000)
            lo = rng.choice(2 ** 32, run, replace=False).astype(np.uint64)
            keys[pos] = hi | lo
    kap = keys.view(np.float64)
    assert np.all(np.isfinite(kap)) and np.all(kap > 0)
    g, _ = oracle.g_nodes(20)
    kt = torch.from_numpy(kap.copy()).cuda()
    srt = torch.empty_like(kt)
    kd = ctx.kdist(kt, ppb, g, sorted_out=srt).cpu().numpy()
    assert np.array_equal(kd, oracle.kdist(kap, ppb, g))
    s = srt.cpu().numpy()
    for b0 in range(0, n, ppb):
        assert np.array_equal(s[b0:b0 + ppb].view(np.uint64), np.sort(kap[b0:b0 + ppb]).view(np.uint64))


# The midpoint-linear rule: the same binary64 expression on both sides,
# evaluated without contraction, so the results agree bit for bit; binary32
# keys enter as their exact binary64 values.
@pytest.mark.parametrize("n,ppb", [(1, 1), (3, 2), (1000, 7), (100000, 1000), (12000, 4097), (20000, 8193),
                                   (50000, 16385),
                                   (250001, 100000)])
@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_kdist_linear_rule_matches_oracle_bitwise(ctx, n, ppb, precision):
    say("kdist linear", n, ppb, precision)
    rng = np.random.default_rng(7 * n + ppb)
    kap = 10.0 ** rng.uniform(-30, -18, n)
    kap[rng.integers(0, n, n // 10)] = kap[0]  # ties
    if n > 10:
        kap[:5] = 0.0
    g = np.concatenate([oracle.g_nodes(20)[0], [1e-9, 0.5, 0.75, 1 - 1e-12]])
    if precision == hk.HK_F32_KAHAN:
        kap = kap.astype(np.float32).astype(np.float64)
        kt = torch.from_numpy(kap.astype(np.float32)).cuda()
    else:
        kt = torch.from_numpy(kap).cuda()
    kd = ctx.kdist(kt, ppb, g, precision=precision, rule=hk.HK_RULE_LINEAR).cpu().numpy()
    ref = oracle.kdist(kap, ppb, g, rule=1)
    assert np.array_equal(kd.view(np.uint64), ref.view(np.uint64))
    # and the step rule of the same call still gives the step rule's values
    kd0 = ctx.kdist(kt, ppb, g, precision=precision).cpu().numpy()
    assert np.array_equal(kd0, oracle.kdist(kap, ppb, g))


# ---- the mid-scale workload at full size (the benchmark's launch), whole grid ----

def test_lines1e6_grid3e6_full(ctx):
    """The mid-scale binary64 workload (1e6 lines, 3e6 points, 100 cm^-1
    cutoff, 1500 K, 1 atm) in the benchmark's launch configuration: every
    one of the 3e6 grid points and all 300 k(g) rows against the oracle at
    1e-6; the per-bin max and p99.9 errors are printed.  The k-distribution
    of the oracle's own grid, computed on the GPU, equals the oracle's bit
    for bit (sorting and picking involve no arithmetic)."""
    from parity_util import per_bin, rel_errors
    w = synth.WORKLOADS["lines1e6_grid3e6"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    say("workload", w.name)
    kg = gpu_opacity(ctx, lines, cond, grid)
    k = kg.cpu().numpy()
    N = grid["n_points"]
    assert np.all(np.isfinite(k)) and np.all(k > 0)
    st = ctx.stats()
    ref, n_ora = oracle.opacity(lines, cond, grid)
    assert st["evals"] == n_ora
    e = rel_errors(k, ref)
    pb = per_bin(e, w.points_per_bin)
    say("  kappa: worst bin max %.2e, worst bin p99.9 %.2e, median bin max %.2e"
        % (pb[:, 0].max(), pb[:, 1].max(), np.median(pb[:, 0])))
    assert e.max() <= TOL, ("point", int(e.argmax()), float(e.max()))
    # the tile shape changes no bit
    ctx.set_option("f64_points_per_lane", 8)
    k2 = gpu_opacity(ctx, lines, cond, grid).cpu().numpy()
    ctx.set_option("f64_points_per_lane", 4)
    assert np.array_equal(k.view(np.uint64), k2.view(np.uint64))
    g_gpu, _ = hk.hk_gauss_legendre(w.n_g)
    g_ora, _ = oracle.g_nodes(w.n_g)
    ppb = w.points_per_bin
    kd = ctx.kdist(kg, ppb, g_gpu).cpu().numpy()
    assert kd.shape == (300, 20)
    kr = oracle.kdist(ref, ppb, g_ora)
    ek = np.abs(kd / kr - 1.0)
    say("  k(g): worst bin max %.2e, median bin max %.2e" % (ek.max(), np.median(ek.max(axis=1))))
    assert ek.max() <= TOL, ("k(g) bin", int(ek.max(axis=1).argmax()), float(ek.max()))
    kd_of_ref = ctx.kdist(torch.from_numpy(ref).cuda(), ppb, g_ora).cpu().numpy()
    assert np.array_equal(kd_of_ref, kr)


def test_follows_a_non_default_torch_stream(ctx):
    """Work is ordered on whatever stream the context was given: results read
    on that stream right after the calls are complete."""
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    ref = gpu_opacity(ctx, lines, cond, grid).cpu().numpy()
    s = torch.cuda.Stream()
    c2 = hk.Context(0)
    try:
        with torch.cuda.stream(s):
            c2.use_current_stream()
            c2.load_lines(lines, cond["mass_amu"], cond["T0"])
            k = c2.opacity(state_of(cond), grid)
            kd = c2.kdist(k, w.points_per_bin, oracle.g_nodes(20)[0])
            host = k.to("cpu", non_blocking=False).numpy()
            kd_host = kd.cpu().numpy()
        assert np.array_equal(host.view(np.uint64), ref.view(np.uint64))
        assert np.all(np.diff(kd_host, axis=1) >= 0) and np.all(kd_host > 0)
    finally:
        c2.close()
