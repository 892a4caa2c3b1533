"""The HITRAN-format reader (hk_read_par): synthetic records written by
tests/par_format.py are read back, field by field, to exactly what Python's
float() makes of the same columns; chunked reading, the molecule filter, CR
LF line ends and malformed files.  Host only."""
import os

import numpy as np
import pytest

import paper_1503_03806_amd as hk
import synth

import par_format


@pytest.fixture()
def par(tmp_path):
    lines = synth.line_list(3000, 3000.0, seed=4)
    mol = np.where(np.arange(3000) % 3 == 0, 2, 1)
    path = str(tmp_path / "lines.par")
    recs = par_format.write(path, lines, molecule=mol)
    return path, recs, mol, lines


def same(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def test_reads_every_field_exactly(par):
    path, recs, _, lines = par
    got, n, nxt = hk.hk_read_par(path, capacity=10000)
    assert n == len(recs) and nxt == len(recs)
    ref = par_format.parsed(recs)
    for k in par_format.COLUMNS:
        assert same(got[k], ref[k]), k
    # and the records hold the list to the format's precision
    assert np.allclose(got["nu"], lines["nu"], rtol=0, atol=5e-7)
    assert np.allclose(got["S_ref"], lines["S_ref"], rtol=5e-4, atol=0)


def test_chunks_and_filter(par):
    path, recs, mol, _ = par
    ref = par_format.parsed(recs)
    parts, first = [], 0
    while True:
        got, n, nxt = hk.hk_read_par(path, first=first, capacity=700)
        if n == 0:
            assert nxt == len(recs)
            break
        assert n <= 700 and nxt == first + n
        parts.append(got)
        first = nxt
    assert len(parts) == 5
    for k in par_format.COLUMNS:
        assert same(np.concatenate([p[k] for p in parts]), ref[k]), k
    got, n, nxt = hk.hk_read_par(path, capacity=10000, molecule=2)
    assert n == int((mol == 2).sum()) and nxt == len(recs)
    assert same(got["nu"], ref["nu"][mol == 2])
    # a filtered chunk stops after its capacity, at the next record to read
    got, n, nxt = hk.hk_read_par(path, capacity=10, molecule=2)
    assert n == 10 and nxt == int(np.flatnonzero(mol == 2)[9]) + 1


def test_crlf_and_edges(tmp_path, par):
    _, recs, _, lines = par
    p2 = str(tmp_path / "crlf.par")
    recs2 = par_format.write(p2, {k: v[:50] for k, v in lines.items()}, crlf=True)
    got, n, _ = hk.hk_read_par(p2, capacity=100)
    assert n == 50 and same(got["E_lower"], par_format.parsed(recs2)["E_lower"])
    got, n, nxt = hk.hk_read_par(p2, first=80, capacity=100)
    assert n == 0 and nxt == 50
    empty = str(tmp_path / "empty.par")
    open(empty, "w").close()
    assert hk.hk_read_par(empty)[1] == 0
    got, n, nxt = hk.hk_read_par(p2, capacity=0)
    assert n == 0 and nxt == 0


def test_malformed_files(tmp_path, par):
    path, recs, _, _ = par
    data = open(path, "rb").read()
    cut = str(tmp_path / "cut.par")
    open(cut, "wb").write(data[:-1])
    with pytest.raises(hk.HKError, match="truncated"):
        hk.hk_read_par(cut)
    short = str(tmp_path / "short.par")
    open(short, "w").write(recs[0][:159] + "\n")
    with pytest.raises(hk.HKError, match="160"):
        hk.hk_read_par(short)
    bad = str(tmp_path / "bad.par")
    rows = list(recs[:5])
    rows[3] = rows[3][:5] + "12x4.5678901" + rows[3][17:]
    rows[3] = rows[3][:160]
    open(bad, "w").write("\n".join(rows) + "\n")
    with pytest.raises(hk.HKError, match=r"record 3: field nu \(columns 4-15\)"):
        hk.hk_read_par(bad)
    with pytest.raises(hk.HKError, match="cannot open"):
        hk.hk_read_par(str(tmp_path / "missing.par"))
    with pytest.raises(hk.HKError, match="first"):
        hk.hk_read_par(path, first=-1)
