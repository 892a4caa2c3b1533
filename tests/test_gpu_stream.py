"""Streamed line lists (§3.5: a list in many pieces whose opacities are
added): hk_opacity_stream against the same chunks loaded and accumulated
one call at a time (bitwise), against the FP64 oracle on the whole list,
its evaluation counts, and a list read from HITRAN-format records in chunks
and streamed."""
import sys

import numpy as np
import pytest

import oracle
import synth

import par_format

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


W = synth.WORKLOADS["lines1e4_grid3e5"]


def state_of(cond):
    return {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}


def chunks_of(lines):
    """Pieces of uneven size: ν-ordered runs (as database files are), one
    piece left unordered, one empty, the largest piece last but one."""
    order = np.argsort(lines["nu"], kind="stable")
    cuts = np.array([0, 500, 2000, 2100, 2100, 6000, 9000, len(order)])
    out = []
    for i, (a, b) in enumerate(zip(cuts[:-1], cuts[1:])):
        idx = order[a:b]
        if i == 5:
            idx = idx[np.random.default_rng(1).permutation(len(idx))]
        out.append({k: v[idx] for k, v in lines.items()})
    return out


def bits(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_stream_is_bitwise_the_chunk_sequence(ctx, precision):
    lines, cond, grid = W.lines(), W.conditions(), W.grid()
    chunks = chunks_of(lines)
    say("stream: %d chunks of %s lines, precision %d" % (len(chunks), [len(c["nu"]) for c in chunks], precision))
    seq = torch.empty(grid["n_points"], dtype=torch.float64, device="cuda")
    for i, c in enumerate(chunks):
        ctx.load_lines(c, cond["mass_amu"], cond["T0"])
        ctx.opacity(state_of(cond), grid, precision, out=seq, accumulate=i > 0)
    got = ctx.opacity_stream(chunks, cond["mass_amu"], state_of(cond), grid, precision, T_ref=cond["T0"])
    torch.cuda.synchronize()
    assert np.array_equal(bits(got), bits(seq))
    ref, n_evals = oracle.opacity(lines, cond, grid)
    nz = ref > 0
    e = np.abs(got.cpu().numpy()[nz] / ref[nz] - 1).max()
    say("stream vs oracle on the whole list: max rel err %.2e" % e)
    assert e <= (1e-6 if precision == hk.HK_F64 else 1e-4)
    st = ctx.stats()
    assert st["evals"] == n_evals and st["n_lines"] == len(lines["nu"])
    # the loaded list is now the last chunk
    last = ctx.opacity(state_of(cond), grid, precision)
    ctx.load_lines(chunks[-1], cond["mass_amu"], cond["T0"])
    assert np.array_equal(bits(last), bits(ctx.opacity(state_of(cond), grid, precision)))


def test_stream_accumulates_and_empty_streams(ctx):
    lines, cond, grid = W.lines(), W.conditions(), W.grid()
    chunks = chunks_of(lines)
    base = torch.full((grid["n_points"],), 1e-22, dtype=torch.float64, device="cuda")
    ctx.opacity_stream(chunks[:3], cond["mass_amu"], state_of(cond), grid, out=base, accumulate=True,
                       T_ref=cond["T0"])
    ctx.opacity_stream(chunks[3:], cond["mass_amu"], state_of(cond), grid, out=base, accumulate=True,
                       T_ref=cond["T0"])
    whole = ctx.opacity_stream(chunks, cond["mass_amu"], state_of(cond), grid, T_ref=cond["T0"])
    got, ref = base.cpu().numpy() - 1e-22, whole.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max() + 1e-36
    z = torch.full((grid["n_points"],), 3.0, dtype=torch.float64, device="cuda")
    ctx.opacity_stream([], cond["mass_amu"], state_of(cond), grid, out=z, accumulate=True)
    assert torch.all(z == 3.0)
    ctx.opacity_stream([], cond["mass_amu"], state_of(cond), grid, out=z)
    assert torch.all(z == 0.0)


@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_stream_many_chunks_both_buffers(ctx, precision):
    """34 pieces (the paper's count for its largest list), so each of the two
    device buffers, staging buffers and lanes (records, plans and sums, whose
    chunks run on two streams) is reused many times; sizes grow."""
    lines = synth.line_list(60_000, 3000.0, seed=3)
    cond = synth.conditions(1500.0, 1.0)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 300000, "cutoff": 25.0}
    order = np.argsort(lines["nu"], kind="stable")
    sizes = np.linspace(200, 3300, 34).astype(int)
    sizes[-1] += len(order) - sizes.sum()
    cuts = np.concatenate([[0], np.cumsum(sizes)])
    chunks = [{k: v[order[a:b]] for k, v in lines.items()} for a, b in zip(cuts[:-1], cuts[1:])]
    say("stream: 34 chunks, precision %d" % precision)
    got = ctx.opacity_stream(chunks, cond["mass_amu"], state_of(cond), grid, precision, T_ref=cond["T0"])
    seq = torch.empty_like(got)
    for i, c in enumerate(chunks):
        ctx.load_lines(c, cond["mass_amu"], cond["T0"])
        ctx.opacity(state_of(cond), grid, precision, out=seq, accumulate=i > 0)
    assert np.array_equal(bits(got), bits(seq))
    tol = 1e-6 if precision == hk.HK_F64 else 1e-4
    j = np.random.default_rng(5).choice(grid["n_points"], 64, replace=False)
    for a in j[:8]:
        ref, _ = oracle.opacity(lines, cond, grid, int(a), int(a) + 1)
        v = got[int(a)].item()
        assert (ref[0] == 0 and v == 0) or abs(v / ref[0] - 1) <= tol


@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_stream_on_a_non_default_torch_stream(ctx, precision):
    """A context given a caller's stream: the pieces' work, spread over that
    stream and the context's own two, ends on the caller's stream, so the
    grid read there right after the call is complete, and bitwise the same
    as on the default stream."""
    lines, cond, grid = W.lines(), W.conditions(), W.grid()
    chunks = chunks_of(lines)
    ref = ctx.opacity_stream(chunks, cond["mass_amu"], state_of(cond), grid, precision,
                             T_ref=cond["T0"]).cpu().numpy()
    s = torch.cuda.Stream()
    c2 = hk.Context(0)
    try:
        with torch.cuda.stream(s):
            c2.use_current_stream()
            for _ in range(2):  # twice: the second call reuses both lanes of device state
                k = c2.opacity_stream(chunks, cond["mass_amu"], state_of(cond), grid, precision,
                                      T_ref=cond["T0"])
                host = k.to("cpu", non_blocking=False).numpy()
                assert np.array_equal(host.view(np.uint64), ref.view(np.uint64))
    finally:
        c2.close()


def test_read_par_then_stream(ctx, tmp_path):
    """Input -> Line -> kappa: records written in the HITRAN layout, read in
    chunks of 1500 records, streamed; against the oracle on the values read."""
    lines = synth.line_list(10_000, 3000.0, seed=8)
    path = str(tmp_path / "w.par")
    par_format.write(path, {k: v[np.argsort(lines["nu"])] for k, v in lines.items()}, seed=2)
    chunks, first = [], 0
    while True:
        got, n, first = hk.hk_read_par(path, first=first, capacity=1500)
        if n == 0:
            break
        chunks.append(got)
    assert len(chunks) == 7
    cond = synth.conditions(1500.0, 1.0)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 300000, "cutoff": 25.0}
    k = ctx.opacity_stream(chunks, cond["mass_amu"], state_of(cond), grid, T_ref=cond["T0"]).cpu().numpy()
    whole = {f: np.concatenate([c[f] for c in chunks]) for f in chunks[0]}
    ref, n_evals = oracle.opacity(whole, cond, grid)
    nz = ref > 0
    e = np.abs(k[nz] / ref[nz] - 1).max()
    say("HITRAN-format records, 7 chunks: max rel err vs oracle %.2e" % e)
    assert e <= 1e-6 and np.all(k[~nz] == 0)
    assert ctx.stats()["evals"] == n_evals
