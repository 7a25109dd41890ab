"""C-ABI library: loads, exports every declared entry point, host-only logic.

No compute call reaches a GPU here: the host-only helpers (CNF validation and
DIMACS parsing) and the error paths that fail before any device work.
"""
import os
import re

import numpy as np
import pytest

from paper_2511_07737_amd import gen, tsat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "tsat.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tsat_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = tsat.lib()
    names = declared_symbols()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    # and the binding declares a signature for each of them
    bound = {n for n, _, _ in tsat._SIGS}
    assert set(names) == bound


def test_version_and_defaults():
    assert tsat.version() == 10100
    p = tsat.default_params()
    assert p.tau == 1.0 and p.lr0 == 0.1 and p.lr_decay == 0.1 and p.lr_min == 1e-15
    assert (p.beta1, p.beta2, p.eps, p.weight_decay) == (0.9, 0.999, 1e-8, 1e-2)
    assert (p.decay_every, p.restart_every, p.norm_mode) == (30, 360, tsat.MODE_MEAN)
    assert p.converge_frac == 0.99


def test_cnf_info_dedup_tautology_widths():
    stream = np.array([1, 1, 2, 0, 3, -3, 0, 0, -2, 4, -5, 0, 5, 0], dtype=np.int32)
    info = tsat.cnf_info_of(5, stream)
    assert info["num_clauses"] == 5
    assert info["num_empty"] == 1
    assert info["num_dup_removed"] == 1
    assert info["num_tautologies"] == 1
    assert info["num_lits"] == 2 + 2 + 0 + 3 + 1
    assert info["max_width"] == 3
    assert info["width_count"][:4] == [1, 1, 2, 1]


def test_cnf_info_matches_generator():
    s = gen.structured(3200, 15000, seed=7)
    info = tsat.cnf_info_of(s.num_vars, s.dimacs_stream())
    assert info["num_clauses"] == s.num_clauses and info["num_lits"] == s.num_lits
    assert info["max_width"] == s.widths().max()
    assert info["width_count"][: 13] == list(np.bincount(s.widths(), minlength=13))


@pytest.mark.parametrize("stream,V,what", [
    ([1, 2, 7, 0], 5, "exceeds num_vars"),
    ([1, 2, 0, 3], 5, "not terminated"),
    ([1, 0], 0, "num_vars"),
    (list(range(1, 34)) + [0], 40, "distinct literals"),
])
def test_cnf_info_errors(stream, V, what):
    with pytest.raises(tsat.TsatError) as e:
        tsat.cnf_info_of(V, np.array(stream, dtype=np.int32))
    assert e.value.code == tsat.E_ARG
    assert what in str(e.value)


def test_dimacs_roundtrip(tmp_path):
    cnf = gen.planted_ksat(40, 170, 3, seed=2)
    path = tmp_path / "a.cnf"
    path.write_text("c generated\n" + cnf.to_dimacs())
    V, stream = tsat.dimacs_read(str(path))
    assert V == 40 and np.array_equal(stream, cnf.dimacs_stream())
    # free-form spacing, clauses across lines, missing final terminator
    path.write_text("c x\np cnf 3 2\n1 -2\n 3 0 -1\n2")
    V, stream = tsat.dimacs_read(str(path))
    assert V == 3 and list(stream) == [1, -2, 3, 0, -1, 2, 0]


@pytest.mark.parametrize("text,what", [
    ("1 2 0\n", "header"),
    ("p cnf 3 1\n1 x 0\n", "invalid token"),
    ("p cnf 3 2\n1 2 0\n", "declares 2 clauses"),
    ("p cnf 3 1\n1 4 0\n", "out of range"),
    ("p cnf 3 1\np cnf 3 1\n1 0\n", "second header"),
    ("p dnf 3 1\n1 0\n", "malformed header"),
])
def test_dimacs_parse_errors(tmp_path, text, what):
    path = tmp_path / "bad.cnf"
    path.write_text(text)
    with pytest.raises(tsat.TsatError) as e:
        tsat.dimacs_read(str(path))
    assert e.value.code == tsat.E_PARSE and what in str(e.value)


def test_missing_file_is_arg_error():
    with pytest.raises(tsat.TsatError) as e:
        tsat.dimacs_read("/nonexistent/x.cnf")
    assert e.value.code == tsat.E_ARG


def test_pack_unpack_helpers():
    g = np.random.default_rng(0)
    b = g.integers(0, 2, size=(7, 130)).astype(np.uint8)
    p = tsat.pack_bits(b)
    assert p.shape == (7, 3)
    assert np.array_equal(tsat.unpack_bits(p, 130), b)
    assert int(p[2, 1]) >> 5 & 1 == b[2, 69]


def test_create_without_gpu_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(tsat.TsatError) as e:
        tsat.Solver()
    assert e.value.code == tsat.E_HIP
    assert "device" in tsat.last_error()
