"""Writes line lists as records of the HITRAN fixed-width format (160
characters: I2 I1 F12.6 E10.3 E10.3 F5.4 F5.3 F10.4 F4.2 F8.6, then the
quantum numbers, error codes, references, flag and statistical weights,
filled here with neutral text).  Test infrastructure: the records are
synthetic, made from seeded line lists; none is a database record."""
from __future__ import annotations

import numpy as np


def _fixed(v: float, width: int, decimals: int) -> str:
    """Fortran Fw.d: drop the leading zero of |v| < 1 when the field is
    otherwise too wide (".0500", "-.001234")."""
    s = "%.*f" % (decimals, v)
    if len(s) > width:
        s = s.replace("0.", ".", 1)
    if len(s) > width:
        raise ValueError("%r does not fit F%d.%d" % (v, width, decimals))
    return s.rjust(width)


def _exp(v: float) -> str:
    s = "%10.3E" % v
    assert len(s) == 10, s
    return s


TAIL = ("%15s%15s%15s%15s" % ("0 0 0", "0 0 0", "", "")) + "000000" + " 1 1 1 1 1 1" + " " \
    + "%7.1f%7.1f" % (1.0, 1.0)
assert len(TAIL) == 93, len(TAIL)


def record(mol: int, iso: int, nu, S, A, g_air, g_self, E, n_air, delta) -> str:
    r = ("%2d%1d" % (mol, iso) + "%12.6f" % nu + _exp(S) + _exp(A) + _fixed(g_air, 5, 4)
         + _fixed(g_self, 5, 3) + "%10.4f" % E + _fixed(n_air, 4, 2) + _fixed(delta, 8, 6) + TAIL)
    assert len(r) == 160, (len(r), r)
    return r


def write(path: str, lines: dict, molecule=None, crlf: bool = False, seed: int = 0) -> list[str]:
    """Write `lines` (synth.line_list fields; gamma_self, delta and A21 are
    drawn here when absent) and return the records written."""
    n = len(lines["nu"])
    rng = np.random.default_rng(seed)
    mol = np.ones(n, dtype=int) if molecule is None else np.asarray(molecule)
    g_self = lines.get("gamma_self")
    if g_self is None:
        g_self = rng.uniform(0.1, 0.5, n)
    delta = lines.get("delta")
    if delta is None:
        delta = rng.uniform(-0.02, 0.01, n)
    A = lines.get("A21")
    if A is None:
        A = 10.0 ** rng.uniform(-6, 2, n)
    recs = [record(int(mol[i]), 1, lines["nu"][i], lines["S_ref"][i], A[i], lines["gamma_air"][i],
                   g_self[i], lines["E_lower"][i], lines["n_air"][i], delta[i]) for i in range(n)]
    end = "\r\n" if crlf else "\n"
    with open(path, "w", newline="") as f:
        for r in recs:
            f.write(r + end)
    return recs


COLUMNS = {"nu": (4, 15), "S_ref": (16, 25), "A21": (26, 35), "gamma_air": (36, 40),
           "gamma_self": (41, 45), "E_lower": (46, 55), "n_air": (56, 59), "delta": (60, 67)}


def parsed(recs: list[str]) -> dict:
    """The values of the records' fields by Python's float()."""
    return {k: np.array([float(r[a - 1:b]) for r in recs]) for k, (a, b) in COLUMNS.items()}
