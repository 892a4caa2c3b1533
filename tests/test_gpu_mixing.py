"""Species mixing (§2.1, §2.2): the opacity of a mixture is sum_s X_s
kappa_s, formed on the GPU by hk_opacity with each species' abundance X_s
and accumulation over the species' line lists, then k-distributed; against
the FP64 oracle (each species' strengths scaled by X_s).  The
correlated-k shortcut -- adding the species' k(g) tables instead -- is
compared with it and its error reported."""
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


def species():
    """Two synthetic species over 0-3000 cm^-1: water-like (18 amu, the
    workload's list) and a heavier one (44 amu, its own seed)."""
    a = synth.line_list(10_000, 3000.0, seed=0)
    b = synth.line_list(6_000, 3000.0, seed=11)
    return [(a, 18.0, 0.7), (b, 44.0, 0.3)]


def test_abundance_scales_the_opacity(ctx):
    lines, mass, _ = species()[0]
    cond = synth.conditions(1500.0, 1.0)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 300000, "cutoff": 25.0}
    ctx.load_lines(lines, mass, 296.0)
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    k1 = ctx.opacity(st, grid, hk.HK_F64).cpu().numpy()
    k3 = ctx.opacity(dict(st, abundance=0.3), grid, hk.HK_F64).cpu().numpy()
    nz = k1 > 0
    assert np.max(np.abs(k3[nz] / (0.3 * k1[nz]) - 1)) <= 1e-14
    k0 = ctx.opacity(dict(st, abundance=0.0), grid, hk.HK_F64).cpu().numpy()
    assert np.all(k0 == 0)
    k0 = ctx.opacity(dict(st, abundance=0.0), grid, hk.HK_F32_KAHAN).cpu().numpy()
    assert np.all(k0 == 0)


@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_mixture_matches_oracle(ctx, precision):
    cond = synth.conditions(1500.0, 1.0)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 300000, "cutoff": 25.0}
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    out = torch.empty(grid["n_points"], dtype=torch.float64, device="cuda")
    ref = np.zeros(grid["n_points"])
    for i, (lines, mass, X) in enumerate(species()):
        ctx.load_lines(lines, mass, 296.0)
        ctx.opacity(dict(st, abundance=X), grid, precision, out=out, accumulate=i > 0)
        scaled = dict(lines, S_ref=lines["S_ref"] * X)
        k_s, _ = oracle.opacity(scaled, dict(cond, mass_amu=mass), grid)
        ref += k_s
    got = out.cpu().numpy()
    e = np.abs(got / ref - 1).max()
    say("mixture (precision %d): max rel err vs oracle %.2e" % (precision, e))
    assert e <= (1e-6 if precision == hk.HK_F64 else 1e-4)
    g, _ = oracle.g_nodes(20)
    kd = ctx.kdist(out, 100000, g).cpu().numpy()
    assert np.abs(kd / oracle.kdist(ref, 100000, g) - 1).max() <= (1e-6 if precision == hk.HK_F64 else 1e-4)


def test_correlated_k_shortcut_is_reported(ctx):
    cond = synth.conditions(1500.0, 1.0)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 300000, "cutoff": 25.0}
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    ppb = 100000
    g, _ = hk.hk_gauss_legendre(64)
    mix = torch.empty(grid["n_points"], dtype=torch.float64, device="cuda")
    tables = []
    for i, (lines, mass, X) in enumerate(species()):
        ctx.load_lines(lines, mass, 296.0)
        ctx.opacity(dict(st, abundance=X), grid, hk.HK_F64, out=mix, accumulate=i > 0)
        k_s = ctx.opacity(dict(st, abundance=X), grid, hk.HK_F64)
        tables.append(ctx.kdist(k_s, ppb, g).cpu().numpy())
    k_mix = ctx.kdist(mix, ppb, g).cpu().numpy()
    k_sum = tables[0] + tables[1]  # the species' k(g) added at equal g
    m = np.logspace(-18, 30, 300)
    _, w = hk.hk_gauss_legendre(64)
    T_mix = np.exp(-np.einsum("bq,m->bmq", k_mix, m)) @ w
    T_sum = np.exp(-np.einsum("bq,m->bmq", k_sum, m)) @ w
    d = np.abs(T_mix - T_sum).max(axis=1)
    say("correlated-k shortcut: max |T_mixture - T_added_tables| per bin: %s" % " ".join("%.2e" % v for v in d))
    assert np.all(np.isfinite(d))
