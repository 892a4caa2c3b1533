"""The Gauss-Hermite kernels' window-edge paths (a run that a line's window
covers only in part, wholly in one rule's region, taken on that rule's own
path with a window mask) against the general path they stand in for: with
the option "wing_edge_paths" = 0 every such run takes the general path, and
the results must be the same bits, in both precisions and both tile shapes,
on the 1e4-line workload's grid with an absolute cutoff and with a cutoff of
500 Lorentz widths (windows of every width, ending inside runs)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hk = pytest.importorskip("paper_1503_03806_amd")


@pytest.fixture(scope="module")
def ctx():
    c = hk.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
@pytest.mark.parametrize("cut", [{"cutoff": 25.0}, {"cutoff": 0.0, "cutoff_lorentz": 500.0},
                                 {"cutoff": 0.37}])
def test_edge_paths_give_the_general_paths_bits(ctx, precision, cut):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond = w.lines(), w.conditions()
    grid = dict(w.grid(), **cut)
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    name = "f64_points_per_lane" if precision == hk.HK_F64 else "f32_points_per_lane"
    out = {}
    for ppl in ((4, 8) if precision == hk.HK_F64 else (2, 8)):
        ctx.set_option(name, ppl)
        for edges in (1, 0):
            ctx.set_option("wing_edge_paths", edges)
            out[(ppl, edges)] = ctx.opacity(st, grid, precision).cpu().numpy().view(np.uint64)
    ctx.set_option("wing_edge_paths", 1)
    ctx.set_option(name, 4 if precision == hk.HK_F64 else 2)
    ref = out[(4 if precision == hk.HK_F64 else 2, 0)]
    assert np.any(ref != 0)
    for key, v in out.items():
        assert np.array_equal(v, ref), key
