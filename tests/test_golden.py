"""The oracle against values fixed by the paper's printed definitions
(fixtures under tests/golden/, each citing its passage)."""
import os
from fractions import Fraction

import numpy as np

from oracle import oracle as O

HERE = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line.split()


def test_bspline_values_from_the_printed_formulas():
    rows = list(_rows("bspline_values.txt"))
    assert len(rows) >= 20
    for order, x, v in rows:
        xv, want = float(Fraction(x)), float(Fraction(v))
        assert abs(O.bspline(int(order), xv) - want) <= 1e-15, (order, x, v)


def test_bspline_weights_at_nodes_from_the_printed_formulas():
    """The oracle's interpolation weights for a particle at offset x from node
    0 equal b(x - n) at nodes n, i.e. the fixture's values at the node
    distances (x = 1/4: order 2 gives b2(1/4), b2(3/4), b2(5/4) at nodes 0, 1, -1)."""
    table = {(int(o), Fraction(x)): Fraction(v) for o, x, v in _rows("bspline_values.txt")}
    x = Fraction(1, 4)
    for order, nodes in ((1, (0, 1)), (2, (-1, 0, 1))):
        w = [O.bspline(order, float(x - n)) for n in nodes]
        want = [float(table[(order, x - n)]) for n in nodes]
        assert np.allclose(w, want, rtol=0, atol=1e-15)
        assert abs(sum(w) - 1.0) <= 1e-15
