"""The learned K(x, y) surrogate through the C ABI, against the FP64 oracle.

Bars, derived from the arithmetic (bfloat16 operands, binary32 sums):
* labels: the GPU computes them in binary64 and stores binary32, so
  |dz| <= 1e-6 + 2^-23 |z|;
* forward output: binary32 sums and SiLU against binary64 shift each hidden
  value by ~1e-7 relative; a value that lands on a bfloat16 rounding
  boundary can round the other way (one bfloat16 step, 2^-8 relative), so
  almost every output agrees to 1e-4 and all to 2e-2;
* gradient: the same effects, summed over the batch: 1e-3 in norm;
* Adam: binary32 against binary64 on the same gradient: 1e-6 absolute.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import surrogate as S
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hk = pytest.importorskip("paper_1503_03806_amd")

BUDGET = 2e-5  # certified per-evaluation relative error of K
# training recipe: Adam phases (steps, learning rate), batch 4096, loss
# weight 1/(1 + (z/5)^2)
SCHEDULE = ((20000, 5e-3), (20000, 1e-3), (20000, 2e-4))
WSCALE = 5.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = hk.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")


def test_labels_match_oracle(ctx):
    x, y = synth.surrogate_samples(200_000, seed=1)
    say("labels: 200000 samples")
    z = ctx.surrogate_labels(dev(x), dev(y)).cpu().numpy().astype(np.float64)
    ref = S.target(x.astype(np.float64), y.astype(np.float64))
    err = np.abs(z - ref)
    say("  max |dz| %.2e, series-region share %.3f" % (err.max(), np.mean(ref != 0)))
    assert np.all(err <= 1e-6 + 2.0 ** -23 * np.abs(ref))


def test_forward_matches_oracle(ctx):
    theta = synth.mlp_init(0)
    ctx.surrogate_set_params(theta)
    x, y = synth.surrogate_samples(4099, seed=2)  # ragged last wavefront
    z, K = ctx.surrogate_eval(dev(x), dev(y))
    z = z.cpu().numpy().astype(np.float64)
    K = K.cpu().numpy().astype(np.float64)
    ref, _ = S.forward(theta.astype(np.float64), x, y, emulate_bf16=True)
    d = np.abs(z - ref)
    say("forward: |dz| p99 %.2e max %.2e (|z| max %.2f)" % (np.quantile(d, 0.99), d.max(), np.abs(ref).max()))
    assert np.mean(d <= 1e-4 * (1 + np.abs(ref))) >= 0.99
    assert d.max() <= 2e-2 * (1 + np.abs(ref).max())
    # K_hat = G3 exp(tau sinh z) in binary32.  Near a node of the 3-node
    # rule (x = 0, +-sqrt(3/2)) with small y, G3 is ill-conditioned in x:
    # the binary32 node and the rounding of x shift each denominator
    # d = (x - t)^2 + y^2 by up to 2 |x - t| (|t - t_f| + ulp(x)), so the
    # bound below weights that by each term's share of G3.
    Kr = S.reconstruct(z, x, y)
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    t1 = np.sqrt(1.5)
    shift = abs(float(np.float32(t1)) - t1) + np.spacing(x).astype(np.float64)
    terms = []
    for t, wgt in ((0.0, 2.0 / 3.0), (t1, 1.0 / 6.0), (-t1, 1.0 / 6.0)):
        d = (xd - t) ** 2 + yd ** 2
        terms.append((wgt / d, 2.0 * np.abs(xd - t) * shift / d))
    total = sum(a for a, _ in terms)
    bound = sum(a * b for a, b in terms) / total + 16 * 2.0 ** -24
    rel = np.abs(K / Kr - 1)
    say("  K_hat rel err max %.2e, worst ratio to bound %.2f" % (rel.max(), (rel / bound).max()))
    assert np.all(rel <= bound)


def test_gradient_matches_oracle(ctx):
    theta = synth.mlp_init(3)
    ctx.surrogate_set_params(theta)
    x, y = synth.surrogate_samples(1000, seed=4)  # 15 full wavefronts + 40
    zt = S.target(x.astype(np.float64), y.astype(np.float64))
    g, loss = ctx.surrogate_grad(dev(x), dev(y), dev(zt), wscale=WSCALE)
    g = g.cpu().numpy().astype(np.float64)
    loss = float(loss.cpu()[0])
    lref, gref = S.loss_and_grad(theta.astype(np.float64), x, y, zt.astype(np.float32), emulate_bf16=True,
                                 wscale=WSCALE)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say("gradient: loss %.6e vs %.6e, rel norm err %.2e" % (loss, lref, rel))
    assert abs(loss / lref - 1) <= 1e-4
    assert rel <= 1e-3
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in S.SHAPES])
    for k, (name, _) in enumerate(S.SHAPES):
        a, b = offs[k], offs[k + 1]
        rk = np.linalg.norm(g[a:b] - gref[a:b]) / max(np.linalg.norm(gref[a:b]), 1e-30)
        assert rk <= 5e-3, (name, rk)


def test_adam_step_matches_oracle(ctx):
    theta = synth.mlp_init(5)
    ctx.surrogate_set_params(theta)
    x, y = synth.surrogate_samples(512, seed=6)
    zt = dev(S.target(x.astype(np.float64), y.astype(np.float64)))
    xd, yd = dev(x), dev(y)
    g, _ = ctx.surrogate_grad(xd, yd, zt)
    g = g.cpu().numpy().astype(np.float64)
    lr = 1e-3
    ctx.surrogate_train(xd, yd, zt, batch=512, steps=1, lr=lr)
    th1 = ctx.surrogate_params().astype(np.float64)
    ref, _, _ = S.adam_step(theta.astype(np.float64), np.zeros_like(g), np.zeros_like(g), g, 1, lr)
    assert np.max(np.abs(th1 - ref)) <= 1e-6


@pytest.fixture(scope="module")
def trained(ctx):
    """Train on 1e6 samples of the workload's domain, then certify."""
    n = 1_000_000
    x, y = synth.surrogate_samples(n, seed=7)
    xd, yd = dev(x), dev(y)
    zd = ctx.surrogate_labels(xd, yd)
    ctx.surrogate_set_params(synth.mlp_init(7))
    hist = []
    for steps, lr in SCHEDULE:
        say("training %d steps at lr %.0e" % (steps, lr))
        hist.append(ctx.surrogate_train(xd, yd, zd, batch=4096, steps=steps, lr=lr,
                                        wscale=WSCALE).cpu().numpy())
    hist = np.concatenate(hist)
    err, count = ctx.surrogate_certify(BUDGET)
    say("  loss first %.3e last-100 mean %.3e; certified cells %d of %d"
        % (hist[0], hist[-100:].mean(), count, err.size))
    return {"hist": hist, "err": err, "count": count, "theta": ctx.surrogate_params()}


def test_saved_surrogate_loads_into_a_new_context(ctx, trained):
    """hk_surrogate_save / hk_surrogate_load: a new context given the blob
    holds the same parameters and certification, and its surrogate opacity
    equals the training context's bit for bit."""
    blob = ctx.surrogate_save()
    n_cells = hk.HK_SURR_CELLS_X * hk.HK_SURR_CELLS_Y
    assert len(blob) == 32 + 4 * hk.HK_SURR_N_PARAMS + 8 * n_cells
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    a = ctx.opacity(st, grid, hk.HK_F32_SURROGATE).cpu().numpy()
    c2 = hk.Context(0)
    try:
        with pytest.raises(hk.HKError):  # no certification yet
            c2.load_lines(lines, cond["mass_amu"], cond["T0"])
            c2.opacity(st, grid, hk.HK_F32_SURROGATE)
        c2.surrogate_load(blob)
        assert np.array_equal(c2.surrogate_params(), trained["theta"])
        b = c2.opacity(st, grid, hk.HK_F32_SURROGATE).cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        assert c2.stats()["evals_surrogate"] == ctx.stats()["evals_surrogate"] > 0
        assert c2.surrogate_save() == blob
    finally:
        c2.close()


def test_training_reduces_the_loss(trained):
    h = trained["hist"]
    assert np.all(np.isfinite(h))
    assert h[-100:].mean() < h[:100].mean() / 10
    assert trained["count"] > 0


def test_certification_matches_oracle(ctx, trained):
    """Cell errors recomputed by the oracle (bfloat16-emulating forward,
    binary64 reconstruction, binary64 series) on sampled cells; the
    certification decision agrees wherever the oracle's error is not within
    a factor 2 of the budget."""
    theta = trained["theta"].astype(np.float64)
    err = trained["err"]
    rng = np.random.default_rng(8)
    cells = rng.choice(err.size, 200, replace=False)
    lat = np.arange(16) / 15.0  # the certification's 16x16 lattice per cell
    agree = 0
    for c in cells:
        iy, ix = divmod(int(c), hk.HK_SURR_CELLS_X)
        xs = ((ix + lat[None, :]) * 0.125 + 0 * lat[:, None]).ravel()
        ly = (-4.0 + (iy + lat[:, None]) * 0.125 + 0 * lat[None, :]).ravel()
        xs = xs.astype(np.float32).astype(np.float64)
        ys = (10.0 ** ly).astype(np.float32).astype(np.float64)
        zh, _ = S.forward(theta, xs, ys, emulate_bf16=True)
        e = np.max(np.abs(S.reconstruct(zh, xs, ys) / S.plain_K(xs, ys) - 1))
        g = err.ravel()[c]
        if e < BUDGET / 2 or e > 2 * BUDGET:
            assert (g <= BUDGET) == (e <= BUDGET), (c, g, e)
            agree += 1
    say("certification decisions compared on %d of 200 sampled cells" % agree)


def test_opacity_with_surrogate_matches_oracle(ctx, trained):
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    k_s = ctx.opacity(st, grid, hk.HK_F32_SURROGATE).cpu().numpy()
    st_s = ctx.stats()
    k_f = ctx.opacity(st, grid, hk.HK_F32_KAHAN).cpu().numpy()
    st_f = ctx.stats()
    ref, _ = oracle.opacity(lines, cond, grid)
    e = np.abs(k_s / ref - 1)
    say("surrogate opacity: max rel err vs oracle %.2e (binary32 path %.2e); the network evaluated"
        " %d of %d series-region points (%.1f%%)"
        % (e.max(), np.abs(k_f / ref - 1).max(), st_s["evals_surrogate"], st_s["evals_core"],
           100.0 * st_s["evals_surrogate"] / max(st_s["evals_core"], 1)))
    # the network ran, and changed results where it did
    assert 0 < st_s["evals_surrogate"] <= st_s["evals_core"]
    assert st_f["evals_surrogate"] == 0
    assert np.count_nonzero(k_s != k_f) > 0
    assert e.max() <= 1e-4
    g, _ = oracle.g_nodes(w.n_g)
    kd = ctx.kdist(torch.tensor(k_s, device="cuda"), w.points_per_bin, g).cpu().numpy()
    assert np.abs(kd / oracle.kdist(ref, w.points_per_bin, g) - 1).max() <= 1e-4


def test_surrogate_stream_is_bitwise_the_chunk_sequence(ctx, trained):
    """A streamed list with the surrogate: consecutive chunks run on two
    streams, their updates of kappa and of the network's evaluation count in
    chunk order; bitwise the chunks loaded and accumulated one call at a
    time, with the same count."""
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    order = np.argsort(lines["nu"], kind="stable")
    cuts = np.linspace(0, len(order), 8).astype(int)
    chunks = [{k: v[order[a:b]] for k, v in lines.items()} for a, b in zip(cuts[:-1], cuts[1:])]
    seq = torch.empty(grid["n_points"], dtype=torch.float64, device="cuda")
    used = 0
    for i, c in enumerate(chunks):
        ctx.load_lines(c, cond["mass_amu"], cond["T0"])
        ctx.opacity(st, grid, hk.HK_F32_SURROGATE, out=seq, accumulate=i > 0)
        used += ctx.stats()["evals_surrogate"]
    got = ctx.opacity_stream(chunks, cond["mass_amu"], st, grid, hk.HK_F32_SURROGATE, T_ref=cond["T0"])
    torch.cuda.synchronize()
    s = ctx.stats()
    say("surrogate stream: %d chunks, network evaluations %d" % (len(chunks), s["evals_surrogate"]))
    assert np.array_equal(got.cpu().numpy().view(np.uint64), seq.cpu().numpy().view(np.uint64))
    assert s["evals_surrogate"] == used > 0


def test_surrogate_gain_is_reported(ctx, trained):
    """What the trained network gains over the method without it: the
    binary32 path with and without the surrogate on 1e6 lines, 3e6 points,
    25 cm^-1 cutoff; the time is reported, the accuracy asserted."""
    w = synth.WORKLOADS["lines1e6_grid3e6"]
    lines, cond = w.lines(), w.conditions()
    grid = dict(w.grid(), cutoff=25.0)
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    out = {}
    for prec in (hk.HK_F32_KAHAN, hk.HK_F32_SURROGATE):
        ctx.opacity(st, grid, prec)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        for _ in range(3):
            k = ctx.opacity(st, grid, prec)
        tm = ctx.timing()
        ctx.set_timing(False)
        out[prec] = (k.cpu().numpy(), tm["core"][0] / 3, sum(v[0] for v in tm.values()) / 3, ctx.stats())
    e = np.abs(out[hk.HK_F32_SURROGATE][0] / out[hk.HK_F32_KAHAN][0] - 1).max()
    ss = out[hk.HK_F32_SURROGATE][3]
    say("gain: series-kernel ms %.3f -> %.3f with the surrogate; whole opacity ms %.3f -> %.3f;"
        " certified cells %d; network share of series-region points %.1f%%; max rel diff %.2e"
        % (out[hk.HK_F32_KAHAN][1], out[hk.HK_F32_SURROGATE][1], out[hk.HK_F32_KAHAN][2],
           out[hk.HK_F32_SURROGATE][2], trained["count"],
           100.0 * ss["evals_surrogate"] / max(ss["evals_core"], 1), e))
    assert ss["evals_surrogate"] > 0 and out[hk.HK_F32_KAHAN][3]["evals_surrogate"] == 0
    assert e <= 1e-4


def test_surrogate_workload_seeded_bins(ctx, trained):
    """The surrogate configuration at its full size (1e8 lines over
    0-30000 cm^-1, 3e6 points, 25 cm^-1 cutoff, 1500 K, 1 atm), in the launch
    configuration the benchmark times: 16 whole bins drawn with seed 3,
    kappa and k(g) against the oracle at 1e-4.  The oracle is given the lines
    that can reach each bin -- every other line adds exactly nothing there --
    so that it does not sort and prepare all 1e8 lines per bin."""
    from parity_util import near_lines, rel_errors, seeded_bins
    w = synth.WORKLOADS["lines1e8_surrogate"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    say("full size: %d lines, %d points" % (len(lines["nu"]), grid["n_points"]))
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    k = ctx.opacity(st, grid, hk.HK_F32_SURROGATE)
    sts = ctx.stats()
    say("  the network evaluated %d of %d series-region points (%.1f%%)"
        % (sts["evals_surrogate"], sts["evals_core"], 100.0 * sts["evals_surrogate"] / max(sts["evals_core"], 1)))
    assert sts["evals_surrogate"] > 0
    ppb = w.points_per_bin
    g, _ = oracle.g_nodes(w.n_g)
    kd = ctx.kdist(k, ppb, g).cpu().numpy()
    kk = k.cpu().numpy()
    worst = 0.0
    for b in seeded_bins(w.n_bins):
        j0, j1 = b * ppb, (b + 1) * ppb
        ref, _ = oracle.opacity(near_lines(lines, grid, j0, j1), cond, grid, j0, j1)
        e = rel_errors(kk[j0:j1], ref)
        kr, _ = oracle.kdist_bin(ref, g)
        ek = np.abs(kd[b] / kr - 1).max()
        say("  bin %d: kappa max %.2e p99.9 %.2e, k(g) max %.2e" % (b, e.max(), np.quantile(e, 0.999), ek))
        worst = max(worst, e.max(), ek)
    assert worst <= 1e-4
    del k
    ctx.load_lines(synth.line_list(10, 10.0), cond["mass_amu"], cond["T0"])  # release the list's device memory
