"""The oracle against hand-derived fixtures in tests/golden/ (no GPU)."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.lstrip().startswith("#")]


def test_hdiff_unit_spike():
    n, h, c = 7, 2, 0.1
    u = np.zeros((1, n + 2 * h, n + 2 * h))
    u[0, h + 3, h + 3] = 1.0
    out = oracle.hdiff(u, h, np.full_like(u, c), h)
    expect = np.zeros((1, n, n))
    for di, dj, base, mult in _rows("hdiff_spike.txt"):
        expect[0, 3 + int(dj), 3 + int(di)] = float(base) + float(mult) * c
    assert np.abs(out - expect).max() <= 1e-15


def test_thomas_textbook_systems():
    systems, cur = {}, None
    for row in _rows("thomas_textbook.txt"):
        if row[0] == "system":
            cur = systems.setdefault(row[1], [])
        else:
            cur.append([float(v) for v in row[1:]])
    assert len(systems) == 3
    for name, rows in systems.items():
        a, b, c, d, x = (np.array(col).reshape(-1, 1, 1) for col in zip(*rows))
        got = oracle.thomas(a, 0, b, 0, c, 0, d, 0)
        assert np.abs(got - x).max() <= 1e-15, name
