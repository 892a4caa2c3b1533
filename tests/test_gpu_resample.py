"""Chebyshev resampling (hk_resample) and transmission (hk_transmission,
hk_transmission_direct) through the C ABI against the FP64 oracle.

Bars: both sides work in binary64 on the same sorted values; the GPU sums
Q^T d in a different order than numpy's QR solve, so coefficients agree to
1e-9 of their largest magnitude; transmissions (sums of exponentials of
the same numbers) to 1e-12.
"""
import numpy as np
import pytest

import oracle
from oracle import resample as R
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hk = pytest.importorskip("paper_1503_03806_amd")


@pytest.fixture(scope="module")
def ctx():
    c = hk.Context(0)
    yield c
    c.close()


def sorted_bins(ctx, k, ppb, g):
    s = torch.empty_like(k)
    ctx.kdist(k, ppb, g, sorted_out=s)
    torch.cuda.synchronize()
    return s


@pytest.mark.parametrize("n_points,ppb", [(300000, 100000), (250000, 100000), (300000, 10000)])
def test_resample_matches_oracle(ctx, n_points, ppb):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond = w.lines(), w.conditions()
    grid = dict(w.grid(), n_points=n_points)
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    k = ctx.opacity(st, grid, hk.HK_F64)
    g, _ = hk.hk_gauss_legendre(20)
    s = sorted_bins(ctx, k, ppb, g)
    coef = ctx.resample(s, ppb, 20).cpu().numpy()
    ref = R.fit(k.cpu().numpy(), ppb, 20)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    err = (np.abs(coef - ref) / scale).max()
    print("resample %d points, bins of %d: max coefficient error %.2e" % (n_points, ppb, err))
    assert err <= 1e-9
    # the same through binary32 keys (the values rounded to binary32 first)
    k32 = k.float()
    s32 = torch.empty_like(k32)
    ctx.kdist(k32, ppb, g, precision=hk.HK_F32_KAHAN, sorted_out=s32)
    c32 = ctx.resample(s32, ppb, 20, precision=hk.HK_F32_KAHAN).cpu().numpy()
    ref32 = R.fit(k32.double().cpu().numpy(), ppb, 20)
    assert (np.abs(c32 - ref32) / np.abs(ref32).max(axis=1, keepdims=True)).max() <= 1e-9


def test_transmission_matches_oracle(ctx):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    k = ctx.opacity(st, grid, hk.HK_F64)
    ppb = w.points_per_bin
    g, _ = hk.hk_gauss_legendre(20)
    s = sorted_bins(ctx, k, ppb, g)
    kk = k.cpu().numpy()
    ref_coef = R.fit(kk, ppb, 20)
    m = np.logspace(-18, 30, 1000)
    md = torch.tensor(m, device="cuda")
    T = ctx.transmission(torch.tensor(ref_coef, device="cuda"), md).cpu().numpy()
    Td = ctx.transmission_direct(s, ppb, md).cpu().numpy()
    for b in range(3):
        tf = R.transmission_fit(ref_coef[b], m)
        td = R.transmission_direct(np.sort(kk[b * ppb:(b + 1) * ppb]), m)
        assert np.max(np.abs(T[b] - tf)) <= 1e-12
        assert np.max(np.abs(Td[b] - td)) <= 1e-12
        print("bin %d: max |T_fit - T_direct| on the GPU %.2e" % (b, np.abs(T[b] - Td[b]).max()))
    assert np.all(np.diff(T, axis=1) <= 1e-15)  # non-increasing in m


def test_resample_mid_workload_full(ctx):
    """The 1e6-line workload: 300 bins of 1e4 points (LDS-sorted), 20
    coefficients each, then T for 1000 column masses; every bin against the
    oracle's fit of the same values."""
    w = synth.WORKLOADS["lines1e6_grid3e6"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    k = ctx.opacity(st, grid, hk.HK_F64)
    ppb = w.points_per_bin
    g, _ = hk.hk_gauss_legendre(20)
    s = sorted_bins(ctx, k, ppb, g)
    coef = ctx.resample(s, ppb, 20)
    md = torch.tensor(np.logspace(-18, 30, 1000), device="cuda")
    T = ctx.transmission(coef, md)
    torch.cuda.synchronize()
    ref = R.fit(k.cpu().numpy(), ppb, 20)
    c = coef.cpu().numpy()
    assert (np.abs(c - ref) / np.abs(ref).max(axis=1, keepdims=True)).max() <= 1e-9
    Tn = T.cpu().numpy()
    assert np.all(np.isfinite(Tn)) and np.all((Tn >= 0) & (Tn <= 1 + 1e-12))
