"""Line-wing cutoff in units of each line's Lorentz width (§2.4, §3.4),
and no cutoff, through the C ABI against the FP64 oracle; then the
cutoff-sensitivity comparison of the transmission function (the paper's
§3.4 experiment on synthetic lists; reported, not asserted)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import resample as R
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
    c.close()


def state_of(cond):
    return {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}


def rel_err(got, ref):
    zero = ref == 0
    assert np.all(got[zero] == 0)
    e = np.zeros_like(ref)
    e[~zero] = np.abs(got[~zero] / ref[~zero] - 1.0)
    return e


@pytest.mark.parametrize("P", [0.01, 1.0, 30.0])
def test_lorentz_cutoff_matches_oracle(ctx, P):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines = w.lines()
    cond = synth.conditions(1500.0, P)
    grid = dict(w.grid(), cutoff=0.0, cutoff_lorentz=500.0)
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    ref, n_ref = oracle.opacity(lines, cond, grid)
    k64 = ctx.opacity(state_of(cond), grid, hk.HK_F64).cpu().numpy()
    e64 = rel_err(k64, ref)
    assert ctx.stats()["evals"] == n_ref
    k32 = ctx.opacity(state_of(cond), grid, hk.HK_F32_KAHAN).cpu().numpy()
    e32 = rel_err(k32, ref)
    say("500 Gamma_L cutoff, P = %g atm: %d evals; max rel err binary64 %.2e, binary32 %.2e"
        % (P, n_ref, e64.max(), e32.max()))
    assert e64.max() <= 1e-6 and e32.max() <= 1e-4


def test_lorentz_cutoff_tables_equal_single_states(ctx):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines = w.lines()
    grid = dict(w.grid(), cutoff=0.0, cutoff_lorentz=500.0)
    conds = [synth.conditions(T, P) for T, P in ((300.0, 0.01), (1500.0, 1.0), (2500.0, 30.0))]
    ctx.load_lines(lines, conds[0]["mass_amu"], conds[0]["T0"])
    g, _ = hk.hk_gauss_legendre(20)
    ppb = w.points_per_bin
    tab = ctx.tables([state_of(c) for c in conds], grid, ppb, g, hk.HK_F32_KAHAN).cpu().numpy()
    for s, c in enumerate(conds):
        k = ctx.opacity(state_of(c), grid, hk.HK_F32_KAHAN)
        kd = ctx.kdist(k, ppb, g).cpu().numpy()
        assert np.array_equal(tab[s].view(np.uint64), kd.view(np.uint64)), s


def test_no_cutoff_matches_oracle(ctx):
    lines = synth.line_list(300, 100.0, seed=4)
    lines["nu"] = lines["nu"] + 1000.0
    cond = synth.conditions(1500.0, 1.0)
    grid = {"nu_min": 1000.0, "dnu": 0.01, "n_points": 10000, "cutoff": 1e6}  # beyond the span
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    ref, n_ref = oracle.opacity(lines, cond, grid)
    k = ctx.opacity(state_of(cond), grid, hk.HK_F64).cpu().numpy()
    assert n_ref == 300 * 10000 and ctx.stats()["evals"] == n_ref
    assert rel_err(k, ref).max() <= 1e-6


def test_cutoff_sensitivity_of_the_transmission_is_reported(ctx):
    """T(m) of the three bins of the 1e4-line workload for an absolute
    25 cm^-1 cutoff, a 500 Gamma_L cutoff and no cutoff, at 0.01, 0.1 and
    1 atm (binary64, direct transmission of the sorted bins)."""
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines = w.lines()
    ppb = w.points_per_bin
    g, _ = hk.hk_gauss_legendre(20)
    m = torch.tensor(np.logspace(-18, 30, 500), device="cuda")
    ctx.load_lines(lines, 18.0, 296.0)
    for P in (0.01, 0.1, 1.0):
        cond = synth.conditions(1500.0, P)
        T = {}
        for name, cut in (("25cm-1", {"cutoff": 25.0}), ("500GL", {"cutoff": 0.0, "cutoff_lorentz": 500.0}),
                          ("none", {"cutoff": 1e6})):
            grid = dict(w.grid(), **cut)
            k = ctx.opacity(state_of(cond), grid, hk.HK_F64)
            s = torch.empty_like(k)
            ctx.kdist(k, ppb, g, sorted_out=s)
            T[name] = ctx.transmission_direct(s, ppb, m).cpu().numpy()
        d1 = np.abs(T["25cm-1"] - T["none"]).max(axis=1)
        d2 = np.abs(T["500GL"] - T["none"]).max(axis=1)
        say("P = %g atm: max |T - T_no_cutoff| per bin: 25 cm^-1 %s, 500 Gamma_L %s"
            % (P, " ".join("%.2e" % v for v in d1), " ".join("%.2e" % v for v in d2)))
        assert np.all(np.isfinite(d1)) and np.all(np.isfinite(d2))
