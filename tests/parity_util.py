"""Helpers shared by the full-size parity tests: the seeded choice of
sampled bins, the lines that can reach a bin, and per-bin error figures."""
import numpy as np

SAMPLE_SEED = 3   # bins sampled at full size are drawn with this seed
SAMPLE_BINS = 16  # ... this many of them


def seeded_bins(n_bins: int, k: int = SAMPLE_BINS, seed: int = SAMPLE_SEED):
    """k distinct bin indices of n_bins, ascending, drawn with `seed`."""
    rng = np.random.default_rng(seed)
    return sorted(int(b) for b in rng.choice(n_bins, size=min(k, n_bins), replace=False))


def near_lines(lines: dict, grid: dict, j0: int, j1: int, margin: float = 1.0) -> dict:
    """The lines whose centre lies within the cutoff (+ margin, which covers
    the rounding of the window bounds) of grid points j0 .. j1-1: every other
    line of an unshifted list adds exactly nothing there.  Input order is
    kept, so ties of equal centres keep their order."""
    lo = grid["nu_min"] + j0 * grid["dnu"] - grid["cutoff"] - margin
    hi = grid["nu_min"] + (j1 - 1) * grid["dnu"] + grid["cutoff"] + margin
    keep = (lines["nu"] >= lo) & (lines["nu"] <= hi)
    assert "delta" not in lines or lines["delta"] is None, "shifted lists need a wider margin"
    return {k: v[keep] for k, v in lines.items() if v is not None}


def rel_errors(got, ref):
    """|got/ref - 1| where ref != 0; got must be 0 exactly where ref is."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    zero = ref == 0
    assert np.all(got[zero] == 0), "nonzero where the oracle is zero"
    e = np.zeros_like(ref)
    e[~zero] = np.abs(got[~zero] / ref[~zero] - 1.0)
    return e


def per_bin(e, points_per_bin: int):
    """(max, p99.9) of the errors e of each bin of consecutive points."""
    n = len(e)
    out = []
    for b0 in range(0, n, points_per_bin):
        s = e[b0:b0 + points_per_bin]
        out.append((float(s.max()), float(np.quantile(s, 0.999))))
    return np.array(out)
