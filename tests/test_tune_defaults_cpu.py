"""Host logic of the built-in table's generator (paper_2301_13016_amd/tune_defaults.py):
the shapes its re-timing step compares against the tuner's forward pick."""
import re

from paper_2301_13016_amd import tune_defaults as TD


def test_neighbours_of_a_pick():
    pick = (4, 1, 64, 4, 1, 2)
    n = TD.neighbours(pick, 64)
    assert n[0] == pick                                  # the pick is timed first
    assert len(n) == len(set(n)) == 1 + 3 * 6 - 1        # its own (ry, nzc) appears once
    # every rows-per-strip and z-chunk count the tuner tries, the pick's other choices kept
    assert {(t[1], -(-64 // t[2])) for t in n} == {(ry, c) for ry in (1, 2, 4) for c in (1, 2, 3, 4, 6, 8)}
    assert all((t[0], t[3], t[4], t[5]) == (4, 4, 1, 2) for t in n)
    assert (4, 2, 32, 4, 1, 2) in n                      # the headline grid's table shape


def test_table_rows_are_generated_candidates():
    """The built-in table says it is unedited, and every forward row holds a
    rows-per-strip and z-chunk count that the generator can have chosen."""
    import os
    path = os.path.join(os.path.dirname(TD.__file__), "csrc", "pw_tune_defaults.inc")
    text = open(path).read()
    assert "unedited" in text.splitlines()[2]
    for line in text.splitlines():
        m = re.match(r"\{([^}]*)\}", line.strip())
        if not m:
            continue
        row = [int(x) for x in m.group(1).split(",")]
        if row[0] != 0:
            continue
        ry, nzc = row[6], row[7]
        assert ry in (1, 2, 4) and nzc in (1, 2, 3, 4, 6, 8), row
