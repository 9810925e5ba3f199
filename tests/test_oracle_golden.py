"""Golden values printed in the paper (fixtures under tests/golden/)."""
import os

from oracle import Grid

HERE = os.path.dirname(__file__)


def _read(name):
    out = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            out[k] = [int(x) for x in v]
    return out


def test_inside_range_of_10x10_array():
    gold = _read("inside_10x10.txt")
    n = tuple(s - 2 for s in gold["padded_size"])
    g = Grid(n)
    assert g.shape == tuple(gold["padded_size"])
    sl = g.interior()
    # 0-based start/stop -> 1-based first/last
    assert [s.start + 1 for s in sl] == gold["interior_first_1based"]
    assert [s.stop for s in sl] == gold["interior_last_1based"]
