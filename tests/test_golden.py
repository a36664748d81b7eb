"""Values the paper prints, kept as cited text fixtures under tests/golden/
(CPU only): the Section 5 model matrix that the paper-design workload uses,
and the heterosis events the event tests use."""
import os

import numpy as np

from paper_1606_06659_amd import datagen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def heterosis_events():
    """Events as lists of (v, b) rows, from the Section 5 fixture."""
    rows = np.loadtxt(os.path.join(GOLDEN, "heterosis_events.txt"))
    events = []
    for e in sorted(set(rows[:, 0].astype(int))):
        sel = rows[rows[:, 0] == e]
        events.append([(list(r[1:6]), float(r[6])) for r in sel])
    return events


def test_paper_design_is_the_printed_matrix():
    X = np.loadtxt(os.path.join(GOLDEN, "paper_model_matrix.txt"))
    assert X.shape == (16, 5)
    np.testing.assert_array_equal(datagen.design_paper(4), X)
    # the paper-design workload is simulated on it
    np.testing.assert_array_equal(datagen.paper_design_16(G=10, seed=0).X, X)


def test_heterosis_fixture():
    ev = heterosis_events()
    assert len(ev) == 2 and all(len(e) == 2 for e in ev)
    assert ev[0][0] == ([0.0, 2.0, 0.0, 1.0, 0.0], 0.0)
    # the low-parent event is the mirror of the high-parent one
    for (v_hi, b_hi), (v_lo, b_lo) in zip(ev[0], ev[1]):
        assert v_lo == [-x for x in v_hi] and b_lo == b_hi == 0.0
