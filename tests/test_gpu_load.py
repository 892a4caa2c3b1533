"""Loading a line list: the library orders it by (nu, input index) -- the
order of a stable sort by nu -- with its threaded sort of (nu, index)
pairs, and leaves absent optional fields at their defaults.  Checked bit for
bit against lists given already in that order or with the defaults
written out."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hk = pytest.importorskip("paper_1503_03806_amd")

GRID = {"nu_min": 0.0, "dnu": 0.01, "n_points": 300000, "cutoff": 25.0}
COND = synth.conditions(1500.0, 1.0)
STATE = {k: COND[k] for k in ("T", "P", "P_self", "q_ratio")}


@pytest.fixture(scope="module")
def ctx():
    c = hk.Context(0)
    yield c
    c.close()


def bits(ctx, lines, prec=hk.HK_F64):
    ctx.load_lines(lines, COND["mass_amu"], COND["T0"])
    return ctx.opacity(STATE, GRID, prec).cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("prec", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_unordered_list_sums_in_stable_order(ctx, prec):
    L = synth.line_list(200_000, 3000.0, seed=31)
    L["nu"] = np.round(L["nu"], 1) + 0.05  # many equal centres: the tie order matters
    perm = np.random.default_rng(32).permutation(len(L["nu"]))
    shuffled = {k: v[perm] for k, v in L.items()}
    order = np.argsort(shuffled["nu"], kind="stable")
    presorted = {k: v[order] for k, v in shuffled.items()}
    assert np.array_equal(bits(ctx, shuffled, prec), bits(ctx, presorted, prec))


def test_absent_fields_equal_their_defaults(ctx):
    L = synth.line_list(20_000, 3000.0, seed=33)
    full = dict(L, gamma_self=L["gamma_air"].copy(), delta=np.zeros(len(L["nu"])), A21=np.zeros(len(L["nu"])))
    assert np.array_equal(bits(ctx, L), bits(ctx, full))
    chunks = [{k: v[i::3] for k, v in L.items()} for i in range(3)]
    full_chunks = [{k: v[i::3] for k, v in full.items()} for i in range(3)]
    a = ctx.opacity_stream(chunks, COND["mass_amu"], STATE, GRID, T_ref=COND["T0"]).cpu().numpy()
    b = ctx.opacity_stream(full_chunks, COND["mass_amu"], STATE, GRID, T_ref=COND["T0"]).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
