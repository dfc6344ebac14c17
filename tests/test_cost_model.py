"""Pin of the algorithmic operation-count helper against the paper's printed closed form (Sec. 7)."""
import os

from paper_2401_06841_amd import model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_rhs_cost_matches_printed_closed_form():
    with open(os.path.join(GOLDEN, "cost_model.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    for k, c in rows:
        assert model.paper_rhs_flops_per_cell(int(k), f=5, cF=15) == int(c)


def test_counts():
    for k, b, v, s in [(1, 4, 8, 4), (2, 10, 27, 9), (3, 20, 64, 16)]:
        assert model.nbasis(k) == b
        assert model.nvol(k) == v
        assert model.nface(k) == s
