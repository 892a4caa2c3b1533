"""Loading a line list: the library orders it by (nu, input index) -- the
order of a stable sort by nu -- with its radix sort of nu on the device
(from host arrays or device tensors), and leaves absent optional fields at
their defaults.  Checked bit for
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


def dev_lines(L):
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda() for k, v in L.items()}


@pytest.mark.parametrize("prec", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_device_list_equals_host_list(ctx, prec):
    """A list handed over as device tensors (lines_on_device) gives the
    same bits as the same list from host memory: already ordered, and
    shuffled with many equal centres (ordered on the device by the radix
    sort, ties in input order)."""
    L = synth.line_list(150_000, 3000.0, seed=34)
    L["nu"] = np.round(L["nu"], 1) + 0.05
    order = np.argsort(L["nu"], kind="stable")
    ordered = {k: v[order] for k, v in L.items()}
    ref = bits(ctx, ordered, prec)
    assert np.array_equal(bits(ctx, dev_lines(ordered), prec), ref)
    assert np.array_equal(bits(ctx, dev_lines(L), prec), ref)
    assert np.array_equal(bits(ctx, L, prec), ref)


def test_device_list_optional_fields_and_empty(ctx):
    L = synth.line_list(30_000, 3000.0, seed=35)
    rng = np.random.default_rng(36)
    full = dict(L, gamma_self=L["gamma_air"] * rng.uniform(0.5, 2.0, 30_000),
                delta=rng.uniform(-0.01, 0.01, 30_000), A21=rng.uniform(0.0, 50.0, 30_000))
    assert np.array_equal(bits(ctx, dev_lines(full)), bits(ctx, full))
    empty = {k: v[:0] for k, v in L.items()}
    assert not bits(ctx, dev_lines(empty)).any()


def test_device_list_rejects_bad_values_and_keeps_the_old_list(ctx):
    L = synth.line_list(5000, 3000.0, seed=37)
    ref = bits(ctx, L)
    for field, value in (("nu", -1.0), ("S_ref", np.nan), ("gamma_air", -0.1), ("E_lower", np.inf)):
        bad = {k: v.copy() for k, v in L.items()}
        bad[field][1234] = value
        with pytest.raises(hk.HKError) as ex:
            ctx.load_lines(dev_lines(bad), COND["mass_amu"], COND["T0"])
        assert ex.value.code == hk.HK_EINVAL and "%s[1234]" % field in str(ex.value)
        # the context still holds the last accepted list
        assert np.array_equal(ctx.opacity(STATE, GRID).cpu().numpy().view(np.uint64), ref)


def test_large_unordered_list_loads_quickly(ctx):
    """1e7 lines in random order (the synthetic generator's order): loaded
    from host arrays and from device tensors, both ordered on the device;
    the load times are printed and the results equal those of the list
    loaded in order."""
    import time
    L = synth.line_list(10_000_000, 30000.0, seed=38)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 3_000_000, "cutoff": 25.0}
    order = np.argsort(L["nu"], kind="stable")
    ordered = {k: np.ascontiguousarray(v[order]) for k, v in L.items()}
    D = dev_lines(L)
    out = {}
    for name, lines in (("ordered host", ordered), ("unordered host", L), ("unordered device", D)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.load_lines(lines, COND["mass_amu"], COND["T0"])
        dt = time.perf_counter() - t0
        out[name] = ctx.opacity(STATE, grid).cpu().numpy().view(np.uint64)
        print("  load %s: %.1f ms" % (name, 1e3 * dt), flush=True)
    assert np.array_equal(out["unordered host"], out["ordered host"])
    assert np.array_equal(out["unordered device"], out["ordered host"])
